"""The allocation-free gradient entry point (static device workspace) against the entry point
that takes a caller workspace: same kernels, so the same bits, on two calls in a row (the
second smaller, so stale partials of the first call must not leak into it), plus the fp64
oracle's gradient to the tolerance of the learned-estimator tests and the size limit."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from paper_1805_09246_amd import sps

pytestmark = pytest.mark.gpu

ETAP = 1024


def _case(seed, n):
    rng = np.random.default_rng(seed)
    p = omlp.init_params(seed)
    for k in p:
        p[k] = p[k] + rng.normal(0, 0.05, p[k].shape)
    inc = rng.integers(0, 160, size=(n + 7, 10))
    x = np.minimum(np.cumsum(inc, 1), ETAP).astype(np.uint32)
    t = rng.uniform(0, 12, n + 7)
    idx = rng.permutation(n + 7)[:n].astype(np.int32)
    return p, x, t, idx


def _grad_pair(p, x, t, idx, n):
    w = torch.from_numpy(omlp.flatten(p).astype(np.float32)).cuda()
    xd = torch.from_numpy(x.view(np.int32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    idd = torch.from_numpy(idx).cuda()
    work = torch.empty(sps.sps_mlp_work_bytes(n), dtype=torch.uint8, device="cuda")
    g_ws = torch.zeros(sps.MLP_PARAMS, dtype=torch.float32, device="cuda")
    l_ws = torch.zeros(1, dtype=torch.float32, device="cuda")
    sps.sps_mlp_grad(w, xd, td, idd, n, ETAP, work, g_ws, l_ws)
    g_na = torch.full((sps.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
    l_na = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    sps.sps_mlp_grad_noalloc(w, xd, td, idd, n, ETAP, g_na, l_na)
    torch.cuda.synchronize()
    return g_ws, l_ws, g_na, l_na


def test_noalloc_grad_matches_workspace_entry_point_twice():
    for seed, n in ((11, sps.MLP_NOALLOC_MAX_N), (12, 1000)):
        print(f"no-alloc grad: seed {seed}, n {n}", flush=True)
        p, x, t, idx = _case(seed, n)
        g_ws, l_ws, g_na, l_na = _grad_pair(p, x, t, idx, n)
        assert torch.equal(g_na, g_ws), f"n={n}: gradients differ from the workspace entry point"
        assert torch.equal(l_na, l_ws), f"n={n}: loss differs from the workspace entry point"
        loss_ref, g_ref = omlp.loss_and_grad(p, omlp.encode(x[idx], ETAP), t[idx])
        gv = omlp.flatten(g_ref)
        got = g_na.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - gv) <= 1e-3 * np.linalg.norm(gv)
        assert abs(l_na.item() - loss_ref) <= 1e-4 * loss_ref


def test_noalloc_grad_rejects_batches_beyond_its_workspace():
    p, x, t, idx = _case(13, 16)
    n = sps.MLP_NOALLOC_MAX_N + 1
    w = torch.from_numpy(omlp.flatten(p).astype(np.float32)).cuda()
    xd = torch.zeros((n, 10), dtype=torch.int32, device="cuda")
    td = torch.zeros(n, dtype=torch.float32, device="cuda")
    g = torch.zeros(sps.MLP_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(sps.SpsError) as e:
        sps.sps_mlp_grad_noalloc(w, xd, td, None, n, ETAP, g)
    assert e.value.code == sps.SPS_ECAPACITY
