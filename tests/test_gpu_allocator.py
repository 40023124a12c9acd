"""Device memory from the caller (ic_set_device_allocator): with PyTorch's
caching allocator installed the library's buffers come out of torch's pool
(torch.cuda.memory_allocated grows by the sim's pools and returns when the
sim is closed) and a refined cone-CME run with learned-flag inference gives
bit-for-bit the forest and state of the same run on hipMalloc memory; a
buffer allocated under one allocator goes back through it after the
allocator has been switched."""
import numpy as np
import pytest

from synthetic import Cme, Wind, as_dict

pytestmark = pytest.mark.gpu


def _run(ic):
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(48, 12, 24),
                block=(12, 12, 12), stretched_r=True, max_level=3, periodic=(False, False, False), gamma=1.5,
                cfl=0.4)
    cme = as_dict(Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1400.0, half_width_deg=35.0, colat_deg=90.0,
                      lon_deg=30.0, n_cm3=1500.0, T_K=0.8e6))
    sim = ic.Sim(grid, as_dict(Wind(seed=5)), [cme], dict(dlon_earth_deg=60.0, dclt_earth_deg=30.0, regrid_every=5))
    params = ic.mlp_init(3)
    sim.mlp_set(params, np.zeros(512, np.float32), np.ones(512, np.float32))
    sim.advance(1e12, 17)
    prob, _ = sim.eval_learned()
    return sim, sim.blocks(), sim.state()[1], prob


def test_torch_allocator_gives_identical_runs():
    import torch
    import paper_2211_12867_amd as ic
    ref_sim, bl0, U0, p0 = _run(ic)
    ref_sim.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ic.use_torch_allocator(True)
    try:
        sim, bl1, U1, p1 = _run(ic)
        held = torch.cuda.memory_allocated() - base
        assert held > 10 * 2 ** 20, held                  # the sim's pools live in torch's pool
        ic.use_torch_allocator(False)                    # switched while the sim still holds torch memory
        sim.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        ic.use_torch_allocator(False)
    assert bl1 == bl0 and max(b[0] for b in bl0) >= 2
    assert np.array_equal(U1, U0) and np.array_equal(p1, p0)


def test_allocator_needs_both_functions():
    import paper_2211_12867_amd as ic
    st = ic.lib.ic_set_device_allocator(ic._ALLOC_FN(lambda n, u: None), ic._FREE_FN(), None)
    assert st == ic.IC_E_INVALID
