"""fp_mlp_loss_grad_static: the MLP loss gradient for callers that cannot
allocate device memory, with its row buffer in a fixed device array of the
library.  Called through the C ABI on a context that has no workspace, and
compared with fp_mlp_loss_grad (workspace row buffer) on two calls in a row,
the second with fewer rows (the fixed array then holds stale rows of the
first call beyond the second call's rows)."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from paper_2211_05458_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def test_static_loss_grad_matches_workspace_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_05458_amd import lib
    L = lib.load()
    w = W.config1(n_particles=10, cells=2)
    g = lib.FlexiPart(w.mesh, w.N, 16)          # context with a workspace: the existing entry point
    stream = torch.cuda.current_stream().cuda_stream
    ctx = C.c_void_p()
    assert L.fp_create(C.byref(ctx), C.c_void_p(stream)) == 0   # no mesh, no workspace
    try:
        rng = np.random.default_rng(61)
        nw = lib.FlexiPart.mlp_n_weights()
        w64 = rng.normal(scale=0.15, size=nw)
        wt = torch.tensor(w64, dtype=torch.float32, device="cuda")
        for n in (3000, 777):
            inp64 = rng.normal(size=(n, 84))
            tgt64 = rng.uniform(-1.0, 1.0, size=(n, 3))
            inp = torch.tensor(inp64, dtype=torch.float32, device="cuda")
            tgt = torch.tensor(tgt64, dtype=torch.float32, device="cuda")
            l0, g0 = g.mlp_loss_grad(wt, inp, tgt)
            g1 = torch.full((nw,), float("nan"), dtype=torch.float32, device="cuda")
            l1 = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
            rc = L.fp_mlp_loss_grad_static(ctx, _ptr(wt), n, _ptr(inp), _ptr(tgt), _ptr(g1), _ptr(l1))
            assert rc == 0, L.fp_last_error(ctx)
            torch.cuda.synchronize()
            # the same kernels with the same row order: identical gradients
            assert torch.equal(g1, g0), n
            assert abs(l1.item() - l0.item()) <= 1e-6 * abs(l0.item())
            # and the oracle's gradient to the FP32 bar of the training kernels
            lo, go = O.mlp_loss_grad(w64.astype(np.float32).astype(np.float64),
                                     inp64.astype(np.float32).astype(np.float64),
                                     tgt64.astype(np.float32).astype(np.float64))
            assert abs(l1.item() - lo) <= 1e-5 * lo
            assert np.abs(g1.cpu().numpy() - go).max() <= 1e-4 * np.abs(go).max()
        # more rows than the fixed array holds: refused before any launch
        big = torch.zeros((4097, 84), dtype=torch.float32, device="cuda")
        tb = torch.zeros((4097, 3), dtype=torch.float32, device="cuda")
        rc = L.fp_mlp_loss_grad_static(ctx, _ptr(wt), 4097, _ptr(big), _ptr(tb), _ptr(g1), _ptr(l1))
        assert rc == lib.FP_EINVAL
        assert b"FP_MLP_STATIC_ROWS" in L.fp_last_error(ctx)
    finally:
        L.fp_destroy(ctx)
