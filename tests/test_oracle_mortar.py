"""Pins of the oracle's tracking across non-conforming (mortar) faces
(Sec. 3.2.3): a big element face matched by two or four small faces.

Drag-free particles move on straight lines, so their final positions are
known; an independent Newton solve confirms that the final element contains
the final position; and particles must cross the mortar interface in both
directions (coarse to fine through a big face, fine to coarse through a small
one) without a single recovery by the location step.
"""
import numpy as np
import pytest

import oracle as O
from paper_2211_05458_amd import workloads as W

CASES = [(4, (2, 2)), (4, (2, 1)), (1, (2, 2)), (1, (2, 1))]


@pytest.mark.parametrize("n_geo, refine", CASES)
def test_straight_paths_through_mortar_faces(n_geo, refine):
    w = W.mortar_box(n_geo=n_geo, N=3, refine=refine, n_particles=3000, seed=52)
    n_coarse = 8
    o = O.Oracle(w.mesh, w.N, w.U)
    rng = np.random.default_rng(3)
    vel = rng.normal(size=(len(w.x), 3)) * 0.4
    vel[:, 0] += np.where(w.elem_hint < n_coarse, 1.0, -1.0)      # towards the interface
    st, _ = o.push(w.x, vel, w.d, w.elem_hint)
    assert np.all(st == O.ACTIVE)
    dt, K = 0.01, 20
    o.step(dt, K, rk=1, drag=2)
    r = o.read()
    s = o.stats()
    assert np.all(r["status"] == O.ACTIVE)
    assert s["lost"] == 0 and s["recovered"] == 0 and s["wall_hits"] > 0
    for p in range(len(w.x)):
        conv, xi, _ = o.newton(r["elem"][p], r["x"][p], o.guess(r["elem"][p], r["x"][p]))
        assert conv and np.abs(xi).max() <= 1 + 1e-9, p
    free = r["hits"] == 0
    np.testing.assert_allclose(r["x"][free], w.x[free] + vel[free] * dt * K, rtol=0, atol=1e-12)
    to_fine = free & (w.elem_hint < n_coarse) & (r["elem"] >= n_coarse)
    to_coarse = free & (w.elem_hint >= n_coarse) & (r["elem"] < n_coarse)
    assert to_fine.sum() > 50 and to_coarse.sum() > 50


@pytest.mark.parametrize("n_geo, refine", [(4, (2, 2)), (1, (2, 1))])
def test_reference_space_localisation_equals_tracking_with_mortars(n_geo, refine):
    w = W.mortar_box(n_geo=n_geo, N=3, refine=refine, n_particles=2000, seed=53, vscale=20.0)
    out = []
    for tracking in (0, 1):
        o = O.Oracle(w.mesh, w.N, w.U)
        o.push(w.x, w.v, w.d * 4, w.elem_hint)
        o.step(2e-3, 8, rk=1, drag=1, tracking=tracking)
        out.append(o.read())
    a, b = out
    for k in ("status", "elem", "hits", "x", "v"):
        np.testing.assert_array_equal(a[k], b[k])


def test_inconsistent_mortar_table_is_rejected():
    w = W.mortar_box(n_geo=1, N=1, refine=(2, 2), n_particles=1)
    bad = W.Mesh(**{**w.mesh.__dict__, "mortar": w.mesh.mortar.copy()})
    bad.mortar[0, 1] = bad.mortar[1, 1]          # a small face of another big face
    with pytest.raises(ValueError):
        O.Oracle(bad, 1, None)
