"""Build the HIP library libicarus.so (gfx950) in-tree with hipcc, and the
host-sanitized driver executable icarus_san (ASan + UBSan on the host code)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libicarus.so")
SOURCES = ["stage.hip", "kernels.hip", "mlp.hip", "runtime.cpp"]
ARCH = os.environ.get("ICARUS_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # keep the compiler from emitting packed fp32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         # fuse a*b+c only within an expression: FMA placement is then fixed by the
         # source, not by register pressure, so every schedule variant of a kernel
         # gives the same bits
         "-ffp-contract=on"]


def _compile(src, obj, flags, verbose):
    cmd = ["hipcc", "-x", "hip", "-c", src, "-o", obj] + flags
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the device-only feature flag; drop that note
    noise = "is not a recognized feature for this target"
    text = "\n".join(l for l in res.stdout.splitlines() if noise not in l)
    if text.strip():
        print(text, flush=True)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd)
    return obj


def _compile_all(jobs, verbose):
    """Compile (src, obj, flags) jobs side by side (one hipcc each)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1, 8)) as ex:
        return [f.result() for f in [ex.submit(_compile, s, o, fl, verbose) for s, o, fl in jobs]]


def build(verbose=False, out=None, defines=(), extra=()):
    flags = FLAGS + list(extra) + ["-D" + d for d in defines]
    objs = _compile_all([(os.path.join(CSRC, src), os.path.join(CSRC, src + ".o"), flags) for src in SOURCES],
                        verbose)
    target = out or LIB
    tmp = target + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, target)
    for o in objs:
        os.remove(o)
    return target


# Host code instrumented by AddressSanitizer and UndefinedBehaviorSanitizer,
# device code as usual (every -fsanitize= goes to the host pass only)
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_EXE = os.path.join(HERE, "icarus_san")


def build_sanitized(verbose=False):
    """The library's sources and csrc/sanitize_driver.cpp linked into one
    executable whose host code runs under the sanitizers (a driver program,
    not a Python extension: the sanitizer runtime is linked into it)."""
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_HOST
    jobs = [(os.path.join(CSRC, src), os.path.join(CSRC, src + ".san.o"), flags) for src in SOURCES]
    jobs.append((os.path.join(CSRC, "sanitize_driver.cpp"), os.path.join(CSRC, "sanitize_driver.san.o"), flags))
    objs = _compile_all(jobs, verbose)
    tmp = SAN_EXE + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}"] + SAN_HOST + ["-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SAN_EXE)
    for o in objs:
        os.remove(o)
    return SAN_EXE


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
    if "--sanitized" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
