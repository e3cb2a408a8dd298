"""Independent pins of the oracle's two-way source, learned-guess network,
Adam optimiser and curved-element flags.

Each test fixes the expected value from something the oracle does not compute
itself: node positions and volumes of an affine box in closed form (Gauss
nodes from numpy), a network whose output has a closed form, Adam's
bias-corrected moments under a constant or alternating gradient, and a single
element with a known bulge.  A plausible mistake in the oracle (a wrong kernel
exponent, a missing volume, a minimum-image slip, transposed weights, bias
correction frozen at the first step, a wrong deviation measure) fails one of
them.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2211_05458_amd import workloads as W

MU = 1.8e-5


# --------------------------------------------------------------------------
# shape-kernel source (Sec. 2.3, eq. theory:source; the kernel reading)
# --------------------------------------------------------------------------
def _affine_box_nodes(cells, N):
    """Physical DG node positions and quadrature volumes of the unit cube cut
    into cells^3 axis-aligned elements: x = lo + (g + 1) h / 2, V = w_i w_j w_k (h/2)^3."""
    g, w = np.polynomial.legendre.leggauss(N + 1)
    n = N + 1
    h = 1.0 / cells
    E = cells ** 3
    e = np.arange(E)
    lo = np.stack([e % cells, (e // cells) % cells, e // (cells * cells)], axis=1) * h
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()          # node q = i + n (j + n k)
    loc = np.stack([g[ii], g[jj], g[kk]], axis=1)
    xn = lo[:, None, :] + 0.5 * (loc[None] + 1.0) * h
    V = np.broadcast_to((w[ii] * w[jj] * w[kk]) * (0.5 * h) ** 3, (E, n ** 3))
    return xn, V


def _shape_source_closed_form(xn, V, xp, F, R, period):
    """S_k = -F K(r_k) / sum_j K(r_j) V_j, K(r) = (1 - (r/R)^2)^2 for r < R,
    r the minimum-image distance."""
    d = xn - xp
    for k in range(3):
        if period[k] > 0:
            d[..., k] -= period[k] * np.round(d[..., k] / period[k])
    r = np.sqrt((d ** 2).sum(-1))
    K = np.where(r < R, (1.0 - (r / R) ** 2) ** 2, 0.0)
    norm = (K * V).sum()
    return -F[None, :, None] * (K / norm)[:, None, :], K


def _one_particle(xp, v, d, u, cells=8, N=3):
    w = W.config1(n_particles=1, cells=cells)
    E = w.mesh.n_elem
    U = W.uniform_state(E, N, u)
    o = O.Oracle(w.mesh, N, U)
    c = np.floor(np.asarray(xp) * cells).astype(int)
    hint = np.array([c[0] + cells * (c[1] + cells * c[2])], np.int32)
    st, _ = o.push(np.array([xp]), np.array([v]), np.array([d]), hint)
    assert st[0] == O.ACTIVE
    return o


@pytest.mark.parametrize("xp", [(0.437, 0.512, 0.291),      # interior
                                (0.011, 0.503, 0.994)])     # next to two periodic faces
def test_shape_source_matches_closed_form_node_by_node(xp):
    cells, N = 8, 3
    h = 1.0 / cells
    R = 1.5 * h
    u = np.array([0.7, -0.2, 0.4])
    v = np.array([0.1, 0.25, -0.3])
    d = 1.0e-4
    o = _one_particle(xp, v, d, u, cells, N)
    S = o.deposit(kind=1, radius=R, period=(1.0, 1.0, 1.0), drag=0)
    # Stokes drag in a uniform state: F = 3 pi mu d (u - v), energy F . v
    Fm = 3.0 * math.pi * MU * d * (u - v)
    F = np.concatenate([Fm, [Fm @ v]])
    xn, V = _affine_box_nodes(cells, N)
    S_ref, K = _shape_source_closed_form(xn, V, np.asarray(xp), F, R, (1.0, 1.0, 1.0))
    scale = np.abs(S_ref).max()
    np.testing.assert_allclose(S, S_ref, rtol=0, atol=1e-11 * scale)
    # the support really wraps: nodes on the far side of the periodic faces
    hit = K > 0
    if xp[0] < R:
        assert (hit & (xn[..., 0] > 0.5)).any() and (hit & (xn[..., 0] < 0.5)).any()
    # conservation in the quadrature measure (a property of any normalisation)
    tot = (S * V[:, None, :]).sum(axis=(0, 2))
    np.testing.assert_allclose(tot, -F, rtol=1e-13, atol=1e-30)


def test_shape_source_first_moment_is_the_particle_position():
    """Far from walls the deposit is centred on the particle: the first moment
    of S V equals -F x_p up to the quadrature error of the kernel."""
    cells, N = 8, 3
    h = 1.0 / cells
    R = 1.5 * h
    xp = np.array([0.4321, 0.5678, 0.4876])
    u = np.array([0.3, 0.1, -0.2])
    v = np.zeros(3)
    o = _one_particle(xp, v, 1e-4, u, cells, N)
    S = o.deposit(kind=1, radius=R, period=(1.0, 1.0, 1.0), drag=0)
    xn, V = _affine_box_nodes(cells, N)
    m0 = (S[:, 0, :] * V).sum()
    m1 = np.array([(S[:, 0, :] * V * xn[..., k]).sum() for k in range(3)])
    np.testing.assert_allclose(m1 / m0, xp, rtol=0, atol=0.02 * h)


def test_shape_source_radius_cut_and_exponent():
    """A particle exactly at a node: K = 1 there; a node at r = R/2 carries
    (3/4)^2 of it; a node at r >= R carries nothing."""
    cells, N = 8, 3
    h = 1.0 / cells
    xn, V = _affine_box_nodes(cells, N)
    e, q = 100, 21
    xp = xn[e, q].copy()
    u = np.array([0.5, 0.0, 0.0])
    o = _one_particle(xp, np.zeros(3), 1e-4, u, cells, N)
    R = 1.5 * h
    S = o.deposit(kind=1, radius=R, period=(1.0, 1.0, 1.0), drag=0)
    dd = xn - xp
    dd -= np.round(dd)                       # minimum image, period 1 on every axis
    r = np.sqrt((dd ** 2).sum(-1))
    ratio = S[:, 0, :] / S[e, 0, q]
    inside = r < R
    np.testing.assert_allclose(ratio[inside], (1.0 - (r[inside] / R) ** 2) ** 2, rtol=1e-12, atol=1e-14)
    assert np.all(S[:, 0, :][~inside] == 0.0)


# --------------------------------------------------------------------------
# learned-guess network: forward pass with a closed-form output
# --------------------------------------------------------------------------
H, NI, NO = O.MLP_H, O.MLP_NIN, O.MLP_NOUT


def _split(w):
    sizes = [H * NI, H, H * H, H, H * H, H, NO * H, NO]
    out, o = [], 0
    for s in sizes:
        out.append(w[o:o + s])
        o += s
    return out


def test_mlp_forward_constant_network():
    """W1 = W2 = W3 = 0: the output is W4 tanh(tanh... (b)) + b4, independent of the input."""
    rng = np.random.default_rng(3)
    w = np.zeros(O.mlp_n_weights())
    W1, b1, W2, b2, W3, b3, W4, b4 = _split(w)
    b1[:] = rng.normal(size=H)
    b2[:] = rng.normal(size=H)
    b3[:] = rng.normal(size=H)
    W4[:] = rng.normal(size=NO * H)
    b4[:] = rng.normal(size=NO)
    x = rng.normal(size=(5, NI))
    out = O.mlp_forward(w, x)
    ref = W4.reshape(NO, H) @ np.tanh(b3) + b4
    np.testing.assert_allclose(out, np.broadcast_to(ref, out.shape), rtol=0, atol=1e-14)


def test_mlp_forward_single_path_network():
    """One nonzero weight per layer: out_2 = e tanh(c3 tanh(c2 tanh(c1 x_5 + b)) ) + b4_2;
    a transposed weight matrix or a shifted layer offset breaks the path."""
    w = np.zeros(O.mlp_n_weights())
    W1, b1, W2, b2, W3, b3, W4, b4 = _split(w)
    a, b, c2, c3, e4, bo = 0.8, 0.1, -1.3, 0.9, 2.5, -0.25
    W1.reshape(H, NI)[3, 5] = a
    b1[3] = b
    W2.reshape(H, H)[7, 3] = c2
    W3.reshape(H, H)[1, 7] = c3
    W4.reshape(NO, H)[2, 1] = e4
    b4[2] = bo
    x = np.zeros((3, NI))
    x[:, 5] = [0.3, -1.1, 2.0]
    x[:, 6] = 5.0            # must not matter
    out = O.mlp_forward(w, x)
    ref2 = e4 * np.tanh(c3 * np.tanh(c2 * np.tanh(a * x[:, 5] + b))) + bo
    np.testing.assert_allclose(out[:, 2], ref2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(out[:, :2], 0.0, atol=0)
    # the loss of the same network (the forward pass inside the gradient code)
    target = np.zeros((3, NO))
    loss, _ = O.mlp_loss_grad(w, x, target)
    np.testing.assert_allclose(loss, (ref2 ** 2).sum() / (3 * NO), rtol=1e-13)


# --------------------------------------------------------------------------
# Adam (Kingma & Ba 2015): bias correction at every step
# --------------------------------------------------------------------------
def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step moves w by lr g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    n = 50
    g = rng.normal(size=n) * 10.0 ** rng.uniform(-4, 2, size=n)
    w0 = rng.normal(size=n)
    w = w0.copy(); m = np.zeros(n); v = np.zeros(n)
    lr, eps = 1e-3, 1e-8
    for t in range(1, 6):
        O.adam(w, m, v, g, t, lr, eps=eps)
        np.testing.assert_allclose(w, w0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)


def test_adam_alternating_gradient_second_step():
    """g then -g with eps = 0: m_hat_2 = -g/19 and v_hat_2 = g^2, so the second
    step moves w back by lr/19 sign(g)."""
    rng = np.random.default_rng(6)
    n = 20
    g = rng.normal(size=n)
    w0 = rng.normal(size=n)
    w = w0.copy(); m = np.zeros(n); v = np.zeros(n)
    lr = 1e-2
    O.adam(w, m, v, g, 1, lr, eps=0.0)
    O.adam(w, m, v, -g, 2, lr, eps=0.0)
    np.testing.assert_allclose(w, w0 - lr * np.sign(g) + lr / 19.0 * np.sign(g), rtol=0, atol=1e-15)


def test_adam_is_scale_invariant():
    """With eps = 0 every Adam step is invariant to scaling all gradients by c > 0."""
    rng = np.random.default_rng(7)
    n = 30
    gs = rng.normal(size=(4, n))
    w0 = rng.normal(size=n)
    res = []
    for c in (1.0, 1e-3, 7.5e4):
        w = w0.copy(); m = np.zeros(n); v = np.zeros(n)
        for t in range(4):
            O.adam(w, m, v, c * gs[t], t + 1, 3e-3, eps=0.0)
        res.append(w)
    np.testing.assert_allclose(res[1], res[0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(res[2], res[0], rtol=0, atol=1e-14)


# --------------------------------------------------------------------------
# curved-element flags (the learned guess's element selection)
# --------------------------------------------------------------------------
def _bulged_element(n_geo, amp):
    """Cube [0,1]^3 whose geometry nodes are pushed along z by amp (1-xi1^2)(1-xi2^2)(1-xi3^2)."""
    def fn(xi):
        x = 0.5 * (xi + 1.0)
        b = (1 - xi[:, 0] ** 2) * (1 - xi[:, 1] ** 2) * (1 - xi[:, 2] ** 2)
        x = x.copy()
        x[:, 2] += amp * b
        return x
    return W.single_element(n_geo, fn)


@pytest.mark.parametrize("n_geo", [2, 4, 6])
def test_curved_flags_affine_zero_and_bulge_threshold(n_geo):
    # the longest corner edge of the unit cube is 1, the bulge peaks at the centre node
    thresh = 0.05
    for amp, expect in [(0.0, 0), (0.049, 0), (0.051, 1), (0.3, 1)]:
        mesh = _bulged_element(n_geo, amp)
        o = O.Oracle(mesh, 1, W.uniform_state(1, 1, (0.0, 0.0, 0.0)))
        assert int(o.curved_flags(thresh)[0]) == expect, (n_geo, amp)
    # an affine (sheared) element is never flagged
    A = np.array([[1.0, 0.3, 0.1], [0.0, 0.8, 0.2], [0.1, 0.0, 1.2]])
    mesh = W.single_element(n_geo, lambda xi: xi @ A.T)
    o = O.Oracle(mesh, 1, W.uniform_state(1, 1, (0.0, 0.0, 0.0)))
    assert int(o.curved_flags(1e-9)[0]) == 0


# --------------------------------------------------------------------------
# seeded draws of a training run (SplitMix64, Steele, Lea and Flood 2014)
# --------------------------------------------------------------------------
def test_training_draws_follow_the_published_generator():
    """The first outputs of SplitMix64 seeded with 1234567 are the published
    test values 6457827717110365317, 3203168211198807973, 9817491932198370423;
    the first weights are the Xavier-uniform values they give, biases are zero,
    and every epoch order is a permutation."""
    published = [6457827717110365317, 3203168211198807973, 9817491932198370423]
    w0, orders = O.mlp_draws(1234567, 1000, 3)
    a = math.sqrt(6.0 / (H + NI))
    ref = [a * (2.0 * ((z >> 11) * 2.0 ** -53) - 1.0) for z in published]
    np.testing.assert_allclose(w0[:3], ref, rtol=0, atol=1e-16)
    W1, b1, W2, b2, W3, b3, W4, b4 = _split(w0)
    assert not b1.any() and not b2.any() and not b3.any() and not b4.any()
    assert np.abs(W2).max() <= math.sqrt(6.0 / 128) and np.abs(W4).max() <= math.sqrt(6.0 / 67)
    for ep in range(3):
        assert sorted(orders[ep].tolist()) == list(range(1000))
    assert (orders[0] != orders[1]).any()
