"""The allocation-free gradient entry point (static device scratch) against the entry point
with a network workspace, on two calls in a row, the second smaller; and its size limit."""

import numpy as np
import pytest

from oracle import learned as olearned
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    _t.cuda.set_device(0)
    return _t


@pytest.fixture(scope="module")
def wb():
    import paper_2508_11790_amd as _wb
    return _wb


def _batch(seed, n):
    r = np.random.default_rng(seed)
    x = (r.standard_normal((n, 64)) * 2).astype(np.float32)
    y = r.standard_normal((n, 2)).astype(np.float32)
    return x, y


def test_static_gradient_matches_workspace_entry_point(torch, wb):
    flat = (np.random.default_rng(0).standard_normal(omlp.N_PARAMS) * 0.2).astype(np.float32)
    P = torch.from_numpy(flat).cuda()
    n_big, n_small = wb.MLP_STATIC_MAX_BATCH, 37     # full scratch, then a ragged small batch
    xb, yb = _batch(1, n_big)
    xs, ys = _batch(2, n_small)
    xb_d, yb_d = torch.from_numpy(xb).cuda(), torch.from_numpy(yb).cuda()
    xs_d, ys_d = torch.from_numpy(xs).cuda(), torch.from_numpy(ys).cuda()

    mlp = wb.Mlp(n_big)
    ref_b, ref_lb = (t.clone() for t in mlp.grad(P, xb_d, yb_d))
    ref_s, ref_ls = (t.clone() for t in mlp.grad(P, xs_d, ys_d))
    torch.cuda.synchronize()
    mlp.close()

    g_b = torch.full((wb.MLP_PARAMS,), float("nan"), device="cuda")
    l_b = torch.full((1,), float("nan"), device="cuda")
    g_s = torch.full((wb.MLP_PARAMS,), float("nan"), device="cuda")
    l_s = torch.full((1,), float("nan"), device="cuda")
    torch.cuda.synchronize()
    wb.mlp_grad_static(P, xb_d, yb_d, g_b, l_b)
    wb.mlp_grad_static(P, xs_d, ys_d, g_s, l_s)    # second call, smaller, same scratch
    torch.cuda.synchronize()
    # same kernels and reduction order as the workspace entry point: identical results
    assert torch.equal(g_b, ref_b) and torch.equal(l_b, ref_lb)
    assert torch.equal(g_s, ref_s) and torch.equal(l_s, ref_ls)
    # and both agree with the FP64 oracle (weights rounded to BF16 as the kernels use them)
    pr = omlp.unflatten(olearned.bf16_round(flat))
    for g, l, x, y in ((g_b, l_b, xb, yb), (g_s, l_s, xs, ys)):
        ref_g = omlp.flatten(omlp.backward(pr, x.astype(np.float64), y.astype(np.float64)))
        assert np.max(np.abs(g.cpu().numpy() - ref_g)) < 1e-4 * np.max(np.abs(ref_g))
        ref_l = omlp.loss(pr, x, y)
        assert abs(float(l.item()) - ref_l) < 1e-4 * ref_l

    # loss is optional
    g_n = torch.empty_like(g_s)
    wb.mlp_grad_static(P, xs_d, ys_d, g_n, None)
    torch.cuda.synchronize()
    assert torch.equal(g_n, ref_s)


def test_static_gradient_rejects_batches_beyond_the_scratch(torch, wb):
    from paper_2508_11790_amd import _lib
    n = wb.MLP_STATIC_MAX_BATCH + 1
    P = torch.zeros((wb.MLP_PARAMS,), device="cuda")
    x = torch.zeros((n, 64), device="cuda")
    y = torch.zeros((n, 2), device="cuda")
    g = torch.full((wb.MLP_PARAMS,), 7.0, device="cuda")
    with pytest.raises(wb.WbmError) as e:
        wb.mlp_grad_static(P, x, y, g)
    assert e.value.status == 2 and "WBM_MLP_STATIC_MAX_BATCH" in str(e.value)
    torch.cuda.synchronize()
    assert bool((g == 7.0).all())                    # nothing was enqueued
    assert _lib.MLP_STATIC_MAX_BATCH == wb.MLP_STATIC_MAX_BATCH
