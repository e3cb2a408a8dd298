"""The stage kernels queue a segment for tracking only if it can reach a face
of its element.  Along a path inside element e, xi_i changes by at most G_i
per unit length, where G_i bounds |grad xi_i| = |row i of J^-1| over the
element; the library takes the largest value on a (2 n_g + 2)^3 reference
lattice that includes the element's faces, edges and corners, times 1.2.  A
segment of length L from xi reaches face (i, +-1) only if L G_i >= 1 -+ xi_i.

These tests check that sampled bound with the oracle's map on the most
strongly curved meshes of the workloads (the annular passage with N_geo = 6
and the sine box with N_geo = 4): lattices twice as dense stay well inside
the margin, and straight segments just shorter than the bound allows end
inside their element.
"""
import numpy as np
import pytest

import oracle as O
from paper_2211_05458_amd import workloads as W

MARGIN = 1.2


def _grad_xi_max(o, e, S):
    g = np.zeros(3)
    t = np.linspace(-1.0, 1.0, S)
    for a in t:
        for b in t:
            for c in t:
                _, J = o.map(e, np.array([a, b, c]))
                assert np.linalg.det(J) > 0.0
                g = np.maximum(g, np.linalg.norm(np.linalg.inv(J), axis=1))
    return g


def _mesh(kind):
    if kind == "annulus":
        w = W.config4(n_particles=1)
    else:
        w = W.curved_box(cells=6, N=3, n_particles=1, n_steps=1, seed=3)
    return w, O.Oracle(w.mesh, w.N, None)


@pytest.mark.parametrize("kind", ["annulus", "sine"])
def test_denser_lattice_stays_within_margin(kind):
    w, o = _mesh(kind)
    ng = w.mesh.n_geo + 1
    rng = np.random.default_rng(7)
    for e in rng.choice(w.mesh.n_elem, 6, replace=False):
        g = _grad_xi_max(o, int(e), 2 * ng + 2)
        gd = _grad_xi_max(o, int(e), 4 * ng + 3)
        assert np.all(gd <= 1.05 * g), (e, g, gd)


def test_segments_within_the_bound_end_inside_annulus():
    w, o = _mesh("annulus")
    ng = w.mesh.n_geo + 1
    rng = np.random.default_rng(8)
    elems = rng.choice(w.mesh.n_elem, 8, replace=False)
    G = {int(e): MARGIN * _grad_xi_max(o, int(e), 2 * ng + 2) for e in elems}
    worst = 0.0
    for k in range(800):
        e = int(elems[k % len(elems)])
        xi = rng.uniform(-0.999, 0.999, 3)
        dirn = rng.normal(size=3)
        dirn /= np.linalg.norm(dirn)
        L = 0.999 * np.min((1.0 - np.abs(xi)) / G[e])
        x0, _ = o.map(e, xi)
        conv, xi1, _ = o.newton(e, x0 + L * dirn, xi)
        assert conv
        worst = max(worst, np.abs(xi1).max())
        assert np.abs(xi1).max() < 1.0, (e, xi, xi1)
    # the bound is not vacuous: some segments end close to a face
    assert worst > 0.9


def _hess_xi_max(o, e, S, h=1e-5):
    """Largest Frobenius norm of the Hessian of each xi_i on an S^3 lattice:
    Hess xi_i = -J^-T (sum_k (J^-1)_ik d2 chi_k) J^-1, the second derivatives
    of the map by central differences of the oracle's Jacobian."""
    out = np.zeros(3)
    t = np.linspace(-1.0, 1.0, S)
    for a in t:
        for b in t:
            for c in t:
                xi = np.array([a, b, c])
                _, J = o.map(e, xi)
                K = np.linalg.inv(J)
                M = np.zeros((3, 3, 3))          # M[k][p][q] = d2 chi_k / d xi_p d xi_q
                for p in range(3):
                    d = np.zeros(3)
                    d[p] = h
                    _, Jp = o.map(e, xi + d)
                    _, Jm = o.map(e, xi - d)
                    M[:, p, :] = (Jp - Jm) / (2 * h)
                for i in range(3):
                    T = np.einsum("k,kpq->pq", K[i], M)
                    H = -K.T @ (0.5 * (T + T.T)) @ K
                    out[i] = max(out[i], np.linalg.norm(H))
    return out


@pytest.mark.parametrize("kind", ["annulus", "sine"])
def test_hessian_bound_denser_lattice(kind):
    """The Hessian bound of the second-order reach test is the maximum on the
    (2 n_g + 2)^3 lattice times 2: a lattice about 1.5 times as dense stays
    well within that margin (on the (n_g + 3)^3 lattice a small component of
    the annulus's Hessian came out 32 % low)."""
    w, o = _mesh(kind)
    ng = w.mesh.n_geo + 1
    rng = np.random.default_rng(9)
    for e in rng.choice(w.mesh.n_elem, 2, replace=False):
        hs = _hess_xi_max(o, int(e), 2 * ng + 2)
        hd = _hess_xi_max(o, int(e), 3 * ng + 2)
        assert np.all(hd <= 1.25 * hs + 1e-12 * np.abs(hs).max()), (e, hs, hd)


def test_sampled_bound_misses_a_peak_between_samples():
    """A mesh built to peak between the lattice samples (workloads.peaked_box:
    the centre geometry node of one element moved so that its map is
    compressed at the centre of its face xi_1 = +1): the library's sampled
    bound (the (2 n_g + 2)^3 lattice, which skips xi = 0, times 1.2) is far
    below |grad xi_1| at xi = (1, 0, 0), while the element stays valid.  This
    is why the sampled bounds only drop internal faces (a crossing of an
    internal face that the bound misses is repaired by the location step;
    tests/test_gpu_reach_repair.py checks that on this mesh against the oracle),
    never a wall, open or periodic face."""
    w, e = W.peaked_box()
    o = O.Oracle(w.mesh, w.N, w.U)
    ng = w.mesh.n_geo + 1
    bound = MARGIN * _grad_xi_max(o, e, 2 * ng + 2)
    _, J = o.map(e, np.array([1.0, 0.0, 0.0]))
    peak = np.linalg.norm(np.linalg.inv(J), axis=1)
    dense = _grad_xi_max(o, e, 4 * ng + 7)       # a lattice with xi = 0
    print("sampled bound", bound, "at (1, 0, 0)", peak, "dense lattice", dense)
    assert np.linalg.det(J) > 0.0 and min(np.linalg.det(o.map(e, np.array([a, b, c]))[1])
                                          for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)) > 0.0
    assert peak[0] > 2.0 * bound[0]
    assert dense[0] >= peak[0]
