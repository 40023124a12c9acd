"""Shared helpers of the GPU parity tests: config conversion for both sides and
the parity norms.

Two norms, both must meet a test's bar:
  - per variable (the R40 reading): max over variables v of
    max|U_gpu,v - U_ora,v| / max|U_ora,v| (a variable's worst error against
    its largest value anywhere);
  - per cell: rho and E relative to the cell's own value; each momentum
    component relative to sqrt(2 rho E) of the cell and each field component
    relative to sqrt(2 E) of the cell (the largest |m| and |B| the cell's
    energy allows), and the tracer's rho s (a ninth variable, when present)
    relative to the cell's rho, so an error in the tenuous outer cells of a
    wedge (rho and E fall as r^-2 and faster) is not hidden by the inner cells.
"""
import numpy as np

from synthetic import as_dict, workload


def var_err(U_gpu, U_ora):
    """max over variables v of max|U_gpu,v - U_ora,v| / max|U_ora,v|."""
    nv = U_ora.shape[1]
    a = np.asarray(U_gpu).reshape(U_gpu.shape[0], nv, -1)
    b = np.asarray(U_ora).reshape(U_ora.shape[0], nv, -1)
    out = 0.0
    for v in range(nv):
        scale = np.abs(b[:, v]).max()
        if scale == 0.0:
            scale = 1.0
        out = max(out, float(np.abs(a[:, v] - b[:, v]).max() / scale))
    return out


def cell_err(U_gpu, U_ora):
    """max over cells and variables of the error relative to the cell's own scale."""
    nv = U_ora.shape[1]
    a = np.asarray(U_gpu).reshape(U_gpu.shape[0], nv, -1)
    b = np.asarray(U_ora).reshape(U_ora.shape[0], nv, -1)
    rho, E = np.abs(b[:, 0]), np.abs(b[:, 4])
    scale = [rho, np.sqrt(2.0 * rho * E), np.sqrt(2.0 * rho * E), np.sqrt(2.0 * rho * E), E,
             np.sqrt(2.0 * E), np.sqrt(2.0 * E), np.sqrt(2.0 * E), rho][:nv]
    out = 0.0
    for v in range(nv):
        s = np.where(scale[v] > 0.0, scale[v], 1.0)
        out = max(out, float((np.abs(a[:, v] - b[:, v]) / s).max()))
    return out


def rel_err(U_gpu, U_ora):
    """The larger of the two parity norms (both bars apply)."""
    return max(var_err(U_gpu, U_ora), cell_err(U_gpu, U_ora))


def tiny_wedge():
    w = workload("tiny_wedge")
    return as_dict(w.grid), as_dict(w.wind), as_dict(w.cmes[0]), as_dict(w.amr)


def oracle_blocks_to_abi(blocks):
    return [tuple(int(x) for x in b) for b in blocks]
