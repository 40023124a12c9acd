"""Shared helpers of the GPU parity tests: config conversion for both sides and
the parity norm (max relative error per conserved variable)."""
import numpy as np

from synthetic import as_dict, workload


def rel_err(U_gpu, U_ora):
    """max over variables v of max|U_gpu,v - U_ora,v| / max|U_ora,v|."""
    a = np.asarray(U_gpu).reshape(U_gpu.shape[0], 8, -1)
    b = np.asarray(U_ora).reshape(U_ora.shape[0], 8, -1)
    out = 0.0
    for v in range(8):
        scale = np.abs(b[:, v]).max()
        if scale == 0.0:
            scale = 1.0
        out = max(out, float(np.abs(a[:, v] - b[:, v]).max() / scale))
    return out


def tiny_wedge():
    w = workload("tiny_wedge")
    return as_dict(w.grid), as_dict(w.wind), as_dict(w.cmes[0]), as_dict(w.amr)


def oracle_blocks_to_abi(blocks):
    return [tuple(int(x) for x in b) for b in blocks]
