"""The allocation-free inference entry point (ic_mlp_infer_noalloc) against
ic_mlp_infer: two calls in a row on device arrays, the second with fewer
rows, each bit-equal to ic_mlp_infer on the same rows; the row limit is
enforced."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _net(seed):
    import paper_2211_12867_amd as ic
    g = np.random.default_rng(seed)
    p = ic.mlp_init(seed)
    p[ic.MLP_IN * ic.MLP_HID:ic.MLP_IN * ic.MLP_HID + ic.MLP_HID] = g.uniform(-0.1, 0.1, ic.MLP_HID)
    mean = g.uniform(-1.0, 1.0, ic.MLP_IN).astype(np.float32)
    std = g.uniform(0.5, 2.0, ic.MLP_IN).astype(np.float32)
    return p.astype(np.float32), mean, std


def test_noalloc_inference_equals_mlp_infer():
    import torch
    import paper_2211_12867_amd as ic
    dev = torch.device("cuda:0")
    p, mean, std = _net(3)
    g = np.random.default_rng(9)
    tp, tm, ts = (torch.from_numpy(a).to(dev) for a in (p, mean, std))
    for n in (3001, 517):                  # the second call has fewer rows
        raw = (g.standard_normal((n, ic.MLP_IN)) * 1.5 + 0.3).astype(np.float32)
        traw = torch.from_numpy(raw).to(dev)
        prob = torch.full((ic.MLP_NOALLOC_ROWS,), -1.0, dtype=torch.float32, device=dev)
        ic.mlp_infer_noalloc(traw.data_ptr(), n, tp.data_ptr(), tm.data_ptr(), ts.data_ptr(), prob.data_ptr())
        torch.cuda.synchronize()
        got = prob.cpu().numpy()
        ref = ic.mlp_infer(raw, p, mean, std)
        assert np.array_equal(got[:n], ref), (n, np.abs(got[:n] - ref).max())
        assert np.all(got[n:] == -1.0)          # nothing written past the rows
        assert 0.0 < ref.min() and ref.max() < 1.0


def test_noalloc_inference_rejects_too_many_rows():
    import torch
    import paper_2211_12867_amd as ic
    dev = torch.device("cuda:0")
    p, mean, std = _net(4)
    n = ic.MLP_NOALLOC_ROWS + 1
    traw = torch.zeros((n, ic.MLP_IN), dtype=torch.float32, device=dev)
    prob = torch.zeros(n, dtype=torch.float32, device=dev)
    tp, tm, ts = (torch.from_numpy(a).to(dev) for a in (p, mean, std))
    with pytest.raises(ic.ICError) as ex:
        ic.mlp_infer_noalloc(traw.data_ptr(), n, tp.data_ptr(), tm.data_ptr(), ts.data_ptr(), prob.data_ptr())
    assert ex.value.status == ic.IC_E_INVALID
    assert "exceed" in str(ex.value)
