"""Learned refinement flags through the C ABI against the oracle's network.

- features of every leaf (8 primitives x 4^3 sub-cube means) match the
  oracle's within one float32 rounding;
- the bf16 MFMA forward + backward (ic_mlp_grad) matches the oracle's
  network with the same bf16 rounding points: loss to 1e-5 relative and each
  parameter group's gradient to 5e-3 in relative L2 norm (the two sides
  differ only in fp32 accumulation order, which moves a bf16 rounding by one
  unit now and then); sizes 1 (one ragged tile), 37, 300 rows;
- element by element: on inputs whose forward sums are exact in fp32, every
  gradient element lies within the bound propagated from the bf16 rounding
  points and fp32 accumulation (tests/mlp_bounds.py);
- one Adam step of ic_mlp_train (the whole set as one batch) equals the
  oracle's Adam step on the oracle's gradient: every parameter whose
  gradient is not near zero moves by the same amount;
- training reduces the loss of a learnable synthetic task and classifies it;
- a regrid from learned flags (REFINE where p >= 1/2 on leaves that touch
  the refinement windows) gives the oracle's forest and state when the
  oracle regrids with the flags of its own network (no near-ties); the
  window mask per leaf and ic_mlp_infer match the oracle too;
- the judge: with a recall bar that cannot be met, the regrid falls back to
  the plain criterion and equals the oracle's plain regrid.
"""
import numpy as np
import pytest

from gpu_helpers import rel_err
from oracle import forest as fo, mlp, solver, units
from synthetic import Cme, Wind, as_dict

pytestmark = pytest.mark.gpu


def _ic():
    import paper_2211_12867_amd as ic
    return ic


def _wedge(max_level=2, block=(8, 8, 8), n=(32, 16, 16)):
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=n, block=block,
                stretched_r=True, max_level=max_level, periodic=(False, False, False), gamma=1.5, cfl=0.4)
    wind = as_dict(Wind(seed=3))
    cme = as_dict(Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1400.0, half_width_deg=35.0,
                      colat_deg=90.0, lon_deg=20.0, n_cm3=1500.0, T_K=0.8e6))
    amr = dict(eps_lohner=0.01, tol_refine=0.1, tol_coarsen=0.0125, w_rho=0.5, w_v=0.5,
               lon_earth_deg=0.0, clt_earth_deg=90.0, dlon_earth_deg=60.0, dclt_earth_deg=30.0,
               dlon_cme_deg=90.0, use_windows=True, regrid_every=5, buffer_blocks=1)
    return grid, wind, cme, amr


def _oracle_after(steps, **kw):
    grid, wind, cme, amr = _wedge(**kw)
    ora = solver.Solver(grid, wind, cme, amr)
    for _ in range(steps):
        ora.step()
    return ora, grid, wind, cme, amr


@pytest.mark.parametrize("block,n", [((8, 8, 8), (32, 16, 16)), ((12, 12, 12), (48, 12, 24))])
def test_features_match_oracle(block, n):
    ic = _ic()
    ora, grid, wind, cme, amr = _oracle_after(6, block=block, n=n)
    gpu = ic.Sim(grid, wind, [cme], amr)
    gpu.set_state(*ora.state(), ora.t * units.T0)
    bl, U = ora.state()
    ref = np.stack([mlp.features(U[b], ora.gamma) for b in range(len(bl))])
    got = gpu.features()
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=3e-7, atol=1e-12)
    gpu.close()


def _params(seed):
    ic = _ic()
    p = ic.mlp_init(seed)
    g = np.random.default_rng(seed + 50)
    for a, b in ((mlp.OFF_B1, mlp.OFF_W2), (mlp.OFF_B2, mlp.OFF_W3)):
        p[a:b] = g.uniform(-0.1, 0.1, b - a)
    p[mlp.OFF_B3] = 0.2
    return p


GROUPS = (("W1", mlp.OFF_W1, mlp.OFF_B1), ("b1", mlp.OFF_B1, mlp.OFF_W2), ("W2", mlp.OFF_W2, mlp.OFF_B2),
          ("b2", mlp.OFF_B2, mlp.OFF_W3), ("w3", mlp.OFF_W3, mlp.OFF_B3), ("b3", mlp.OFF_B3, mlp.NPARAM))


@pytest.mark.parametrize("n", [1, 37, 300])
def test_gradient_matches_oracle(n):
    ic = _ic()
    g = np.random.default_rng(n)
    x = g.standard_normal((n, mlp.IN)).astype(np.float32)
    y = (g.uniform(size=n) < 0.4).astype(np.uint8)
    p = _params(n)
    grad, loss = ic.mlp_grad(x, y, p, pos_weight=2.5)
    loss_o, grad_o = mlp.loss_and_grad(x.astype(np.float64), y, p.astype(np.float64), 2.5)
    assert abs(loss - loss_o) <= 1e-5 * abs(loss_o), (loss, loss_o)
    for name, a, b in GROUPS:
        ref = grad_o[a:b]
        e = np.linalg.norm(grad[a:b] - ref) / max(np.linalg.norm(ref), 1e-30)
        assert e <= 5e-3, (name, e)


@pytest.mark.parametrize("n", [1, 37, 300])
def test_gradient_matches_oracle_elementwise(n):
    """Every gradient element within the bound propagated from the bf16
    rounding points and fp32 accumulation (mlp_bounds), on inputs whose
    forward sums are exact in fp32, so both sides hold the same activations."""
    import mlp_bounds as mb
    ic = _ic()
    x, y, p = mb.exact_problem(n, seed=n)
    g, bound, amb, loss_o = mb.gradient_bound(x, y, p, 2.5)
    grad, loss = ic.mlp_grad(x, y, p, pos_weight=2.5)
    assert abs(loss - loss_o) <= 1e-5 * abs(loss_o), (loss, loss_o)
    err = np.abs(grad.astype(np.float64) - g)
    over = np.nonzero(err > bound)[0]
    assert len(over) == 0, (n, amb, [(int(q), float(err[q]), float(bound[q])) for q in over[:5]])


def test_one_adam_step_matches_oracle():
    ic = _ic()
    g = np.random.default_rng(7)
    n = 512
    raw = (g.standard_normal((n, mlp.IN)) * g.uniform(0.5, 3.0, mlp.IN) + g.uniform(-2, 2, mlp.IN)).astype(np.float32)
    y = (g.uniform(size=n) < 0.3).astype(np.uint8)
    p0 = _params(11)
    lr = 1e-3
    p1, mean, std, loss = ic.mlp_train(raw, y, p0, epochs=1, batch=n, lr=lr, seed=5, pos_weight=2.0)
    mu = raw.astype(np.float64).mean(axis=0)
    sd = raw.astype(np.float64).std(axis=0)
    np.testing.assert_allclose(mean, mu.astype(np.float32), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(std, sd.astype(np.float32), rtol=1e-6)
    x = mlp.normalise(raw, mu.astype(np.float32), sd.astype(np.float32)).astype(np.float64)
    l0, g0 = mlp.loss_and_grad(x, y, p0.astype(np.float64), 2.0)
    assert abs(loss[0] - l0) <= 1e-5 * l0
    p1o = mlp.adam_step(p0.astype(np.float64), g0, np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), 1, lr=lr)
    for name, a, b in GROUPS:
        d = np.abs(p1[a:b] - p1o[a:b])
        bad = d > 0.01 * lr
        gs = np.abs(g0[a:b])
        scale = np.sqrt(np.mean(gs ** 2)) if gs.any() else 0.0
        assert bad.mean() <= 2e-3, (name, bad.mean())
        assert np.all(gs[bad] <= 1e-2 * scale), (name, gs[bad].max(), scale)


def test_training_learns_a_separable_task():
    ic = _ic()
    g = np.random.default_rng(3)
    n = 8192
    raw = g.standard_normal((n, mlp.IN)).astype(np.float32)
    score = raw[:, :64].mean(axis=1) * 8.0 + raw[:, 300] - 0.5 * raw[:, 7]
    y = (score > 0.8).astype(np.uint8)
    p0 = ic.mlp_init(2)
    p, mean, std, loss = ic.mlp_train(raw, y, p0, epochs=6, batch=256, lr=1e-3, seed=1)
    assert loss[-1] < 0.5 * loss[0], loss
    _, prob, _ = mlp.forward(mlp.normalise(raw, mean, std).astype(np.float64), p.astype(np.float64))
    acc = np.mean((prob >= 0.5) == (y == 1))
    assert acc >= 0.9, acc


def _network_for(ora, seed):
    """A random network whose decision threshold sits in the widest gap of
    the oracle's logits over the current leaves (about half refine)."""
    bl, U = ora.state()
    raw = np.stack([mlp.features(U[b], ora.gamma) for b in range(len(bl))])
    mean = raw.astype(np.float64).mean(axis=0).astype(np.float32)
    std = np.maximum(raw.astype(np.float64).std(axis=0), 1e-3).astype(np.float32)
    p = _params(seed)
    x = mlp.normalise(raw, mean, std).astype(np.float64)
    z, _, _ = mlp.forward(x, p.astype(np.float64))
    zs = np.sort(z)
    lo, hi = len(zs) // 4, 3 * len(zs) // 4
    k = lo + int(np.argmax(np.diff(zs[lo:hi + 1])))
    thr = 0.5 * (zs[k] + zs[k + 1])
    gap = zs[k + 1] - zs[k]
    assert gap > 2e-2, "logits too close for a tie-free threshold: %g" % gap
    p[mlp.OFF_B3] -= np.float32(thr)
    z2, _, _ = mlp.forward(x, p.astype(np.float64))
    assert np.min(np.abs(z2)) > 5e-3
    win = {b: bool(ora.window(b, ora.cme).any()) for b in bl}
    flags = {b: (fo.REFINE if zz >= 0.0 and win[b] else fo.COARSEN) for b, zz in zip(bl, z2)}
    vetoed = sum(zz >= 0.0 and not win[b] for b, zz in zip(bl, z2))
    return p, mean, std, flags, z2, vetoed


def test_learned_regrid_matches_oracle():
    ic = _ic()
    ora, grid, wind, cme, amr = _oracle_after(8, max_level=3)
    # a first plain regrid so that the forest has two levels to coarsen from
    ora.regrid()
    for _ in range(3):
        ora.step()
    gpu = ic.Sim(grid, wind, [cme], dict(amr, source=ic.IC_SOURCE_LEARNED))
    gpu.set_state(*ora.state(), ora.t * units.T0)
    p, mean, std, flags, z, vetoed = _network_for(ora, 21)
    assert vetoed > 0, "no refinement vetoed by the windows"
    gpu.mlp_set(p, mean, std)
    prob, fl = gpu.eval_learned()
    assert [int(f) for f in fl] == [flags[b] for b in ora.blocks()]
    np.testing.assert_allclose(prob, 1.0 / (1.0 + np.exp(-z)), atol=2e-3)
    ora.regrid(flags)
    gpu.regrid()
    assert gpu.blocks() == ora.blocks()
    assert rel_err(gpu.state()[1], ora.state()[1]) <= 1e-13
    st = gpu.regrid_stats()
    assert st["learned"] == 1 and st["judged"] == 0 and st["fallbacks"] == 0
    gpu.close()


def test_judge_falls_back_to_plain_criterion():
    ic = _ic()
    ora, grid, wind, cme, amr = _oracle_after(8, max_level=3)
    gpu = ic.Sim(grid, wind, [cme], dict(amr, source=ic.IC_SOURCE_LEARNED_JUDGED, judge_every=1,
                                          judge_recall=1.5))
    gpu.set_state(*ora.state(), ora.t * units.T0)
    p, mean, std, _, _, _ = _network_for(ora, 22)
    gpu.mlp_set(p, mean, std)
    ties = []
    plain = ora.flags(ties)
    assert not ties
    ora.regrid(plain)
    gpu.regrid()
    assert gpu.blocks() == ora.blocks()
    assert rel_err(gpu.state()[1], ora.state()[1]) <= 1e-13
    st = gpu.regrid_stats()
    assert st["learned"] == 1 and st["judged"] == 1 and st["fallbacks"] == 1
    gpu.close()


def test_learned_flags_need_a_network():
    ic = _ic()
    grid, wind, cme, amr = _wedge()
    gpu = ic.Sim(grid, wind, [cme], amr)
    with pytest.raises(ic.ICError) as e:
        gpu.eval_learned()
    assert e.value.status == ic.IC_E_INVALID
    gpu.close()


def test_hot_labels_match_oracle():
    """ic_eval_hot (the refinement condition without the level cap, the
    source of the look-ahead labels) equals the oracle's, bit for bit."""
    ic = _ic()
    ora, grid, wind, cme, amr = _oracle_after(8, max_level=2)
    ora.regrid()
    for _ in range(3):
        ora.step()
    ties = []
    ora.flags(ties)
    assert not ties, ties[:3]
    gpu = ic.Sim(grid, wind, [cme], amr)
    gpu.set_state(*ora.state(), ora.t * units.T0)
    hot = ora.hot()
    got = gpu.eval_hot()
    assert [int(h) for h in got] == [hot[b] for b in ora.blocks()]
    assert any(b[0] == 2 and hot[b] for b in ora.blocks()), "no hot leaf at the finest level"
    gpu.close()


def test_window_mask_and_inference_match_oracle():
    ic = _ic()
    ora, grid, wind, cme, amr = _oracle_after(8, max_level=2)
    ora.regrid()
    gpu = ic.Sim(grid, wind, [cme], amr)
    gpu.set_state(*ora.state(), ora.t * units.T0)
    win = [int(ora.window(b, ora.cme).any()) for b in ora.blocks()]
    assert [int(x) for x in gpu.eval_window()] == win
    assert 0 < sum(win) < len(win)
    bl, U = ora.state()
    raw = np.stack([mlp.features(U[b], ora.gamma) for b in range(len(bl))])
    mean = raw.astype(np.float64).mean(axis=0).astype(np.float32)
    std = np.maximum(raw.astype(np.float64).std(axis=0), 1e-3).astype(np.float32)
    p = _params(31)
    prob = ic.mlp_infer(raw, p, mean, std)
    _, ref, _ = mlp.forward(mlp.normalise(raw, mean, std).astype(np.float64), p.astype(np.float64))
    np.testing.assert_allclose(prob, ref, atol=2e-3)
    gpu.close()
