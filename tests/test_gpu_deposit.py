"""Two-way coupling source on the GPU against the FP64 oracle.

Shape-kernel deposition: every DG node within R of a particle receives
K(r) = (1 - (r/R)^2)^2 times the particle's source, normalised per particle so
that the volume-weighted sum of the source equals minus the drag force.  Cases
cover several particles-per-element chunks, curved elements, periodic images,
radii below one node spacing (particles with no node in reach contribute
nothing) and above two element widths, FP32 output and accumulation into an
existing source.
"""
import numpy as np
import pytest

import oracle as O
from paper_2211_05458_amd import workloads as W

pytestmark = pytest.mark.gpu


def _setup(w, v):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_05458_amd.lib import FlexiPart
    o = O.Oracle(w.mesh, w.N, w.U)
    o.push(w.x, v, w.d, w.elem_hint)
    g = FlexiPart(w.mesh, w.N, len(w.x))
    g.set_fluid_state(w.U)
    g.push(w.x, v, w.d, w.elem_hint)
    return o, g


def _volumes(o, w):
    n3 = (w.N + 1) ** 3
    return np.array([[o.volume(e, q) for q in range(n3)] for e in range(w.mesh.n_elem)])


def _check(So, Sg):
    np.testing.assert_allclose(Sg, So, rtol=1e-9, atol=1e-11 * np.abs(So).max())


def test_shape_dense_elements_curved_periodic():
    """About 39 particles per element (three normalisation chunks), Ngeo=4, N=5."""
    import torch
    w = W.curved_box(cells=4, N=5, n_particles=2500, n_steps=1, seed=41)
    v = w.v + 0.2
    o, g = _setup(w, v)
    R = 1.5 / 4
    per = np.array([1.0, 0.0, 1.0])
    So = o.deposit(kind=1, radius=R, period=per)
    Sg = g.deposit(kind=1, radius=R, period=per).cpu().numpy()
    _check(So, Sg)
    # conservation: volume-weighted source equals minus the total drag force
    Sn = o.deposit(kind=0)
    V = _volumes(o, w)
    tot_shape = np.einsum("ecq,eq->c", Sg, V)
    tot_near = np.einsum("ecq,eq->c", Sn, V)
    assert np.abs(tot_shape - tot_near).max() <= 1e-11 * np.abs(tot_near).max()
    # FP32 output (matrix-core path): same source to FP32 rounding
    Sf = g.deposit(kind=1, radius=R, period=per, dtype=torch.float32).cpu().numpy()
    assert np.abs(Sf - So).max() <= 2e-5 * np.abs(So).max()


@pytest.mark.parametrize("R_cells, periodic, cells", [(0.12, True, 6), (2.5, True, 8), (1.2, False, 6)])
def test_shape_radius_and_images(R_cells, periodic, cells):
    w = W.curved_box(cells=cells, N=3, n_particles=1200, n_steps=1, seed=42)
    v = w.v - 0.1
    o, g = _setup(w, v)
    R = R_cells / cells
    per = np.array([1.0, 0.0, 1.0]) if periodic else None
    So = o.deposit(kind=1, radius=R, period=per)
    Sg = g.deposit(kind=1, radius=R, period=per).cpu().numpy()
    _check(So, Sg)
    if R_cells < 0.5:
        # some particles reach no node and deposit nothing (in both codes), so
        # the volume-weighted total falls short of the total drag force
        V = _volumes(o, w)
        tot_shape = np.einsum("ecq,eq->c", So, V)
        tot_near = np.einsum("ecq,eq->c", o.deposit(kind=0), V)
        assert np.abs(So).max() > 0
        assert np.abs(tot_shape - tot_near).max() > 1e-6 * np.abs(tot_near).max()


def test_shape_accumulates_into_existing_source():
    import torch
    w = W.curved_box(cells=4, N=3, n_particles=500, n_steps=1, seed=43)
    o, g = _setup(w, w.v + 0.3)
    R = 1.5 / 4
    per = np.array([1.0, 0.0, 1.0])
    S = torch.zeros((w.mesh.n_elem, 4, (w.N + 1) ** 3), dtype=torch.float64, device="cuda")
    g.deposit(S, kind=1, radius=R, period=per)
    g.deposit(S, kind=1, radius=R, period=per)
    So = o.deposit(kind=1, radius=R, period=per)
    _check(2.0 * So, S.cpu().numpy())


def _pairs_within(o, w, R, period):
    """(particle, DG node) pairs closer than R (minimum image), by brute force,
    over the particles the push located (status active)."""
    n3 = (w.N + 1) ** 3
    xn = np.array([[o.dg_node_pos(e, q) for q in range(n3)] for e in range(w.mesh.n_elem)]).reshape(-1, 3)
    active = o.read()["status"] == O.ACTIVE
    cnt = 0
    for p in np.nonzero(active)[0]:
        d = xn - w.x[p]
        for k in range(3):
            if period is not None and period[k] > 0:
                d[:, k] -= period[k] * np.round(d[:, k] / period[k])
        cnt += int(((d ** 2).sum(1) < R * R).sum())
    return cnt


@pytest.mark.parametrize("N, n_geo, cells, n, R_cells", [(1, 1, 4, 900, 1.5), (3, 4, 4, 1500, 1.5),
                                                         (5, 4, 4, 2500, 1.5), (7, 4, 3, 1200, 1.2),
                                                         (5, 4, 6, 3000, 0.7)])
def test_shape_fp32_matrix_core_path(N, n_geo, cells, n, R_cells):
    """FP32 sources take the matrix-core kernels (kernel argument of 16 x 16
    node-particle tiles as one rank-5 product): against the FP64 oracle to
    FP32 rounding, conservative to FP32 rounding, and counting exactly the
    pairs within R (up to pairs at r = R within rounding).  Covers one partial
    node tile (N = 1), several tiles per wave (N = 7), walls, periodic images
    and radii below and above one element width."""
    import torch
    w = W.curved_box(cells=cells, N=N, n_particles=n, n_steps=1, seed=44 + N, n_geo=n_geo)
    v = w.v + 0.25
    o, g = _setup(w, v)
    R = R_cells / cells
    per = np.array([1.0, 0.0, 1.0])
    So = o.deposit(kind=1, radius=R, period=per)
    g.reset_stats()
    Sf = g.deposit(kind=1, radius=R, period=per, dtype=torch.float32).cpu().numpy().astype(np.float64)
    assert g.stats()["deposit_pairs"] == 0          # counted only when asked for
    g.set_timing(False, count_pairs=True)
    Sc = g.deposit(kind=1, radius=R, period=per, dtype=torch.float32).cpu().numpy().astype(np.float64)
    g.set_timing(False)
    # the counting variant computes the same values (float atomics from the
    # target workgroups add the normalisation sums in a run-dependent order)
    np.testing.assert_allclose(Sc, Sf, rtol=2e-6, atol=1e-6 * np.abs(Sf).max())
    err = np.abs(Sf - So).max() / np.abs(So).max()
    print("N=%d R=%.2f h: max |S32 - S64| / max |S| = %.3g" % (N, R_cells, err))
    assert err <= 2e-5
    V = _volumes(o, w)
    tot = np.einsum("ecq,eq->c", Sf, V)
    ref = np.einsum("ecq,eq->c", So, V)
    assert np.abs(tot - ref).max() <= 1e-5 * np.abs(ref).max()
    pairs = g.stats()["deposit_pairs"]
    ref_pairs = _pairs_within(o, w, R, per)
    print("pairs within R: gpu %d, brute force %d" % (pairs, ref_pairs))
    assert abs(pairs - ref_pairs) <= max(2, 1e-4 * ref_pairs)


@pytest.mark.parametrize("N, n_geo, cells, n, R_cells", [(1, 1, 4, 900, 1.5), (5, 4, 4, 2500, 1.5),
                                                         (7, 4, 3, 1200, 1.2)])
def test_shape_fp32_reuse_list(N, n_geo, cells, n, R_cells):
    """With a caller-bound reuse list the node-sum pass reads the particles the
    normalisation pass staged for each target instead of staging them again:
    the same source (to the run-to-run order of the normalisation's float
    atomics) with room for every target, and with room for only 16 rows, where
    most targets stage again; against the oracle to FP32 rounding."""
    import torch
    w = W.curved_box(cells=cells, N=N, n_particles=n, n_steps=1, seed=54 + N, n_geo=n_geo)
    v = w.v + 0.25
    o, g = _setup(w, v)
    R = R_cells / cells
    per = np.array([1.0, 0.0, 1.0])
    So = o.deposit(kind=1, radius=R, period=per)
    S0 = g.deposit(kind=1, radius=R, period=per, dtype=torch.float32).cpu().numpy().astype(np.float64)
    for cap in (4096, 16):
        g.bind_deposit_list(cap)
        for _ in range(2):   # the list is rewritten by every call
            S1 = g.deposit(kind=1, radius=R, period=per, dtype=torch.float32).cpu().numpy().astype(np.float64)
            np.testing.assert_allclose(S1, S0, rtol=2e-6, atol=1e-6 * np.abs(S0).max())
            assert np.abs(S1 - So).max() <= 2e-5 * np.abs(So).max()
    g.bind_deposit_list(0)
    S2 = g.deposit(kind=1, radius=R, period=per, dtype=torch.float32).cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(S2, S0, rtol=2e-6, atol=1e-6 * np.abs(S0).max())


def test_reuse_list_binding_errors():
    """The reuse list's memory must be 256-byte aligned and hold at least 16
    rows per element; a rejected binding leaves the source working without it."""
    import ctypes as C
    import torch
    from paper_2211_05458_amd.lib import FPError
    w = W.curved_box(cells=3, N=3, n_particles=300, n_steps=1, seed=60)
    o, g = _setup(w, w.v)
    nb = C.c_size_t(0)
    assert g.L.fp_deposit_list_bytes(g.ctx, 16, C.byref(nb)) == 0
    buf = torch.empty(nb.value + 512, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr() + (-buf.data_ptr()) % 256
    assert g.L.fp_bind_deposit_list(g.ctx, C.c_void_p(base + 4), nb.value) < 0          # misaligned
    assert g.L.fp_bind_deposit_list(g.ctx, C.c_void_p(base), nb.value - 1) < 0          # 15 rows
    assert g.L.fp_bind_deposit_list(g.ctx, C.c_void_p(base), nb.value) == 0
    assert g.L.fp_bind_deposit_list(g.ctx, None, 0) == 0
    with pytest.raises(FPError):
        g._check(g.L.fp_deposit_list_bytes(g.ctx, 0, C.byref(nb)), "fp_deposit_list_bytes")   # no rows
    R = 1.2 / 3
    So = o.deposit(kind=1, radius=R, period=np.array([1.0, 0.0, 1.0]))
    Sf = g.deposit(kind=1, radius=R, period=np.array([1.0, 0.0, 1.0]), dtype=torch.float32)
    assert np.abs(Sf.cpu().numpy() - So).max() <= 2e-5 * np.abs(So).max()
