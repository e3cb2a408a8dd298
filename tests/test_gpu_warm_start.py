"""Locating each particle from its continued reference coordinates (guess bit
1: the previous stage's xi moved by J^-1 dx, J from that stage's last Newton
iteration; after a crossing or reflection the paper's guess instead).  Newton
converges to the same root from any guess in its basin, so the trajectories
equal the paper-guess run and the oracle (which uses the paper's guess) to
the Newton tolerance, with fewer iterations."""
import numpy as np
import pytest

import oracle as O
from paper_2211_05458_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_05458_amd.lib import FlexiPart
    return FlexiPart


def _run(w, v, steps, dt, guess, precision=0, U=None, deposit=False):
    FlexiPart = _gpu()
    g = FlexiPart(w.mesh, w.N, w.n_particles)
    g.set_fluid_state(w.U if U is None else U)
    g.push(w.x, v, w.d, w.elem_hint)
    g.reset_stats()
    for _ in range(steps):
        g.step(dt, 1, rk=1, drag=1, guess=guess, precision=precision)
        if deposit:
            g.deposit(kind=0)
    return g.read(), g.stats()


@pytest.mark.parametrize("N,seed", [(5, 61), (7, 62)])
def test_warm_start_equals_paper_guess_and_oracle(N, seed):
    """Curved box with walls, 10x velocities (many crossings and
    reflections), 12 steps of three stages; the sources in between locate
    the final positions from the continued coordinates as well."""
    w = W.curved_box(cells=5, N=N, n_particles=3000, n_steps=1, seed=seed)
    v = w.v * 10.0
    dt = 2e-3
    r0, s0 = _run(w, v, 12, dt, guess=0, deposit=True)
    r2, s2 = _run(w, v, 12, dt, guess=2, deposit=True)
    it0 = s0["newton_iters"] / s0["newton_calls"]
    it2 = s2["newton_iters"] / s2["newton_calls"]
    print("Newton iterations per solve: paper guess %.3f, continued %.3f; crossings %d, wall hits %d"
          % (it0, it2, s2["crossings"], s2["wall_hits"]))
    assert s2["crossings"] > 1000 and s2["wall_hits"] > 20 and s2["lost"] == 0
    np.testing.assert_array_equal(r2["elem"], r0["elem"])
    np.testing.assert_array_equal(r2["status"], r0["status"])
    np.testing.assert_array_equal(r2["hits"], r0["hits"])
    assert np.abs(r2["x"] - r0["x"]).max() <= 1e-12
    assert s2["newton_iters"] < 0.85 * s0["newton_iters"]
    o = O.Oracle(w.mesh, w.N, w.U)
    o.push(w.x, v, w.d, w.elem_hint)
    o.step(dt, 12, rk=1, drag=1)
    ro = o.read()
    np.testing.assert_array_equal(r2["elem"], ro["elem"])
    np.testing.assert_array_equal(r2["hits"], ro["hits"])
    assert np.abs(r2["x"] - ro["x"]).max() <= 1e-10


def test_warm_start_mixed_form_and_learned_bits():
    """Mixed form with the continued coordinates: same bits as the mixed form
    with the paper's guess (the FP32 parts do not see the guess); guess = 3
    (continued coordinates, then the learned guess on flagged elements) on the
    annular passage with an all-zero network (guess: the element centre): the
    result still equals the paper-guess run."""
    import torch
    w = W.curved_box(cells=5, N=5, n_particles=3000, n_steps=1, seed=63)
    U32 = torch.from_numpy(w.U.astype(np.float32))
    v = w.v * 10.0
    r0, _ = _run(w, v, 8, 2e-3, guess=0, precision=1, U=U32)
    r2, s2 = _run(w, v, 8, 2e-3, guess=2, precision=1, U=U32)
    np.testing.assert_array_equal(r2["elem"], r0["elem"])
    np.testing.assert_array_equal(r2["hits"], r0["hits"])
    assert np.abs(r2["x"] - r0["x"]).max() <= 1e-12
    FlexiPart = _gpu()
    wa = W.config4(n_particles=3000, cells=(12, 6, 12), seed=64)
    g = FlexiPart(wa.mesh, wa.N, wa.n_particles)
    g.set_fluid_state(wa.U)
    g.push(wa.x, wa.v, wa.d, wa.elem_hint)
    wts = torch.zeros(FlexiPart.mlp_n_weights(), dtype=torch.float32, device="cuda")
    g.mlp_set_weights(wts, 0.05)
    g.step(wa.dt, 6, rk=1, drag=1, guess=3)
    ra = g.read()
    g0 = FlexiPart(wa.mesh, wa.N, wa.n_particles)
    g0.set_fluid_state(wa.U)
    g0.push(wa.x, wa.v, wa.d, wa.elem_hint)
    g0.step(wa.dt, 6, rk=1, drag=1, guess=0)
    rb = g0.read()
    np.testing.assert_array_equal(ra["elem"], rb["elem"])
    assert np.abs(ra["x"] - rb["x"]).max() <= 1e-12



def test_learned_guess_list_and_stage_sorts_on_the_annulus():
    """guess = 3 (continued coordinates; the learned guess, computed for the
    compacted list of particles without them, on flagged elements) in the
    mixed form on the annular passage: sorting before every stage gives the
    same bits as sorting once per step and as no sort (each particle's
    guesses and arithmetic do not depend on where it sits), and the learned
    guess takes part (the Newton iteration count differs from the run
    without it)."""
    import torch
    FlexiPart = _gpu()
    wt = W.config4(n_particles=20_000, cells=(12, 6, 12), seed=1044)
    gt = FlexiPart(wt.mesh, wt.N, wt.n_particles)
    gt.set_fluid_state(torch.from_numpy(wt.U))
    gt.push(wt.x, wt.v, wt.d, wt.elem_hint)
    feat, xi = gt.newton_pairs()
    weights, _ = gt.mlp_train(feat, xi, epochs=6, batch=512, lr=2e-3, seed=4)
    w = W.config4(n_particles=3000, cells=(12, 6, 12), seed=1045)
    U32 = torch.from_numpy(w.U.astype(np.float32))
    runs = {}
    for name, guess, se in (("step", 3, 1), ("stage", 3, -1), ("none", 3, 0), ("warm_only", 2, 1)):
        g = FlexiPart(w.mesh, w.N, w.n_particles)
        g.set_fluid_state(U32)
        g.push(w.x, w.v, w.d, w.elem_hint)
        g.mlp_set_weights(weights, 0.05)
        g.reset_stats()
        g.step(w.dt, 12, rk=1, drag=1, guess=guess, precision=1, sort_every=se)
        runs[name] = (g.read(), g.stats())
    for name in ("stage", "none"):
        for k in ("x", "v", "xi", "elem", "hits", "status"):
            np.testing.assert_array_equal(runs[name][0][k], runs["step"][0][k])
    st, s2 = runs["step"][1], runs["warm_only"][1]
    print("iterations per solve: continued + learned %.4f, continued only %.4f" %
          (st["newton_iters"] / st["newton_calls"], s2["newton_iters"] / s2["newton_calls"]))
    assert st["newton_iters"] != s2["newton_iters"]   # the learned guesses were used
    assert st["lost"] == 0 and s2["lost"] == 0
