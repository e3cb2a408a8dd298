"""Pins of the oracle's extra terms of the equation of motion (eq. theory:maxey):
buoyancy, the undisturbed-flow stress m_f Du/Dt, added mass and Saffman lift
(Sec. 2.2), and the velocity gradient they need.

Each is checked against something the mathematics or the physics fixes: exact
gradients of polynomial fields on a sheared affine element, the closed-form
fall of a particle under buoyancy and added mass, a neutrally buoyant particle
riding a solid-body rotation, Saffman's classical lift in its own notation and
direction, and the continuity of Mei's lift correction.
"""
import math

import numpy as np

import oracle as O
from paper_2211_05458_amd import workloads as W

MU, RHO_F = W.MU, W.RHO_F


# ---------------------------------------------------------------------------
# velocity gradient
# ---------------------------------------------------------------------------
def _monomials(deg):
    return [(a, b, c) for a in range(deg + 1) for b in range(deg + 1) for c in range(deg + 1) if a + b + c <= deg]


def _poly(coef, pw, x):
    return sum(cf * x[0] ** a * x[1] ** b * x[2] ** c for cf, (a, b, c) in zip(coef, pw))


def _poly_grad(coef, pw, x):
    g = np.zeros(3)
    for cf, (a, b, c) in zip(coef, pw):
        if a:
            g[0] += cf * a * x[0] ** (a - 1) * x[1] ** b * x[2] ** c
        if b:
            g[1] += cf * b * x[0] ** a * x[1] ** (b - 1) * x[2] ** c
        if c:
            g[2] += cf * c * x[0] ** a * x[1] ** b * x[2] ** (c - 1)
    return g


def test_velocity_gradient_exact_on_sheared_affine_element():
    """Density and momentum cubic in x on an affine, sheared element with N = 3:
    the interpolant reproduces them, so u = m/rho and du_i/dx_j from the oracle
    equal the analytic values (a transposed J^-1 or a dropped -u grad(rho)
    term fails)."""
    A = np.array([[0.6, 0.25, -0.1], [0.05, 0.45, 0.2], [-0.15, 0.1, 0.55]])
    b = np.array([0.3, -0.2, 0.1])
    mesh = W.single_element(1, lambda xi: xi @ A.T + b)
    N = 3
    g, _ = np.polynomial.legendre.leggauss(N + 1)
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")       # node order i + n (j + n k)
    xi_nodes = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    xn = xi_nodes @ A.T + b
    rng = np.random.default_rng(71)
    pw = _monomials(3)
    c_rho = rng.uniform(-0.05, 0.05, len(pw)); c_rho[0] = 1.2
    c_m = [rng.uniform(-1, 1, len(pw)) for _ in range(3)]
    U = np.zeros((1, 5, (N + 1) ** 3))
    for q in range(len(xn)):
        U[0, 0, q] = _poly(c_rho, pw, xn[q])
        for i in range(3):
            U[0, 1 + i, q] = _poly(c_m[i], pw, xn[q])
        U[0, 4, q] = 2.5e5
    o = O.Oracle(mesh, N, U)
    for _ in range(20):
        xi = rng.uniform(-1, 1, 3)
        x = A @ xi + b
        rho, grho = _poly(c_rho, pw, x), _poly_grad(c_rho, pw, x)
        m = np.array([_poly(c, pw, x) for c in c_m])
        gm = np.array([_poly_grad(c, pw, x) for c in c_m])
        u = m / rho
        G = (gm - np.outer(u, grho)) / rho
        prim, Go = o.fluid_grad(0, xi)
        np.testing.assert_allclose(prim[1:4], u, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(Go, G, rtol=1e-11, atol=1e-12 * np.abs(G).max())


# ---------------------------------------------------------------------------
# buoyancy and added mass: closed-form fall in a quiescent fluid
# ---------------------------------------------------------------------------
def test_buoyancy_and_added_mass_closed_form():
    """No drag, quiescent fluid, gravity g: (m_p + m_f/2) dv/dt = g (m_p - m_f),
    so v = g t (1 - r) / (1 + r/2) with r = rho_f / rho_p; without the added
    mass v = g t (1 - r).  A bubble (r = 2) rises.  The 3-stage RK integrates
    the quadratic path exactly."""
    w = W.config1(n_particles=20)
    U = W.uniform_state(w.mesh.n_elem, w.N, np.zeros(3))
    gvec = np.array([0.0, 0.0, -9.81])
    dt, K = 1e-3, 50
    t = dt * K
    for r, forces, factor in ((0.5, O.F_BUOYANCY | O.F_ADDED_MASS, 0.5 / 1.25),
                              (2.0, O.F_BUOYANCY | O.F_ADDED_MASS, -1.0 / 2.0),
                              (0.5, O.F_BUOYANCY, 0.5),
                              (0.5, 0, 1.0)):
        o = O.Oracle(w.mesh, w.N, U, rho_p=RHO_F / r)
        x0 = np.random.default_rng(5).uniform(0.2, 0.8, (20, 3))
        o.push(x0, np.zeros((20, 3)), np.full(20, 1e-4), None)
        o.step(dt, K, rk=1, drag=2, gravity=gvec, forces=forces)
        res = o.read()
        np.testing.assert_allclose(res["v"], np.tile(gvec * t * factor, (20, 1)), rtol=0, atol=1e-13)
        dx = res["x"] - (x0 + 0.5 * gvec * t * t * factor)
        dx -= np.round(dx)                       # unit periods
        assert np.abs(dx).max() < 1e-13


# ---------------------------------------------------------------------------
# undisturbed-flow stress and added mass: neutrally buoyant tracer
# ---------------------------------------------------------------------------
def _rotation_box(omega, c):
    def node_map(I1, I2, I3, M):
        out = np.empty(np.broadcast_shapes(I1.shape, I2.shape, I3.shape) + (3,))
        out[..., 0] = I1 / M[0]
        out[..., 1] = I2 / M[1]
        out[..., 2] = I3 / M[2]
        return out
    X, ne, nf, bc, sh, _ = W.structured_mesh((2, 2, 2), 1, node_map, (False, False, False), wall_bc=W.BC_OPEN)
    mesh = W.Mesh(1, X, ne, nf, bc, sh, h=0.5, cells=(2, 2, 2))
    N = 2
    g, _ = np.polynomial.legendre.leggauss(N + 1)
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    U = np.zeros((8, 5, (N + 1) ** 3))
    for e in range(8):
        i1, i2, i3 = e % 2, (e // 2) % 2, e // 4
        x = np.stack([(i1 + 0.5 * (ii.ravel() + 1.0)) / 2, (i2 + 0.5 * (jj.ravel() + 1.0)) / 2,
                      (i3 + 0.5 * (kk.ravel() + 1.0)) / 2], axis=1)
        u = np.stack([-omega * (x[:, 1] - c[1]), omega * (x[:, 0] - c[0]), np.zeros(len(x))], axis=1)
        U[e, 0] = RHO_F
        U[e, 1:4] = (RHO_F * u).T
        U[e, 4] = W.P0 / 0.4 + 0.5 * RHO_F * (u * u).sum(1)
    return mesh, N, U


def test_neutrally_buoyant_particle_rides_solid_body_rotation():
    """u = Omega e_z x (x - c), r = 1, no drag: with the stress term (alone or
    with added mass) dv/dt = Du/Dt = (u . grad) u, the centripetal
    acceleration, so a particle released with the fluid velocity stays on its
    circle; without the terms it leaves it along the tangent."""
    omega, c = 1.0, np.array([0.5, 0.5, 0.5])
    mesh, N, U = _rotation_box(omega, c)
    rng = np.random.default_rng(9)
    n = 12
    rad = rng.uniform(0.1, 0.3, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    z = rng.uniform(0.2, 0.8, n)
    x0 = np.stack([c[0] + rad * np.cos(ph), c[1] + rad * np.sin(ph), z], axis=1)
    v0 = np.stack([-omega * (x0[:, 1] - c[1]), omega * (x0[:, 0] - c[0]), np.zeros(n)], axis=1)
    dt, K = 1e-3, 500
    ang = omega * dt * K
    R = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    exact = (x0 - c) @ R.T + c
    errs = {}
    for forces in (O.F_STRESS, O.F_STRESS | O.F_ADDED_MASS, 0):
        o = O.Oracle(mesh, N, U, rho_p=RHO_F)
        o.push(x0, v0, np.full(n, 1e-4), None)
        o.step(dt, K, rk=1, drag=2, forces=forces)
        res = o.read()
        assert np.all(res["status"] == O.ACTIVE)
        errs[forces] = np.abs(res["x"] - exact).max()
    assert errs[O.F_STRESS] < 1e-8 and errs[O.F_STRESS | O.F_ADDED_MASS] < 1e-8
    assert errs[0] > 1e-2


# ---------------------------------------------------------------------------
# Saffman lift
# ---------------------------------------------------------------------------
def _lift(o, prim, G, v, d):
    a, F = o.particle_accel(2, O.F_SAFFMAN, prim, G, v, d)
    return a, F


def test_saffman_lift_direction_and_classical_magnitude():
    """Simple shear u = (kappa y, 0, 0): a particle lagging the fluid is lifted
    towards the faster fluid (+y), a leading one away from it (Saffman 1965).
    At Re_p -> 0 the magnitude is Saffman's L = 6.46 mu a^2 V sqrt(kappa / nu)
    (a = d/2, nu = mu/rho), here in the paper's diameter form."""
    w = W.config1(n_particles=1)
    rho_p = 2500.0
    o = O.Oracle(w.mesh, w.N, W.uniform_state(w.mesh.n_elem, w.N, np.zeros(3)), rho_p=rho_p)
    kappa, y = 1000.0, 0.03
    G = np.array([[0.0, kappa, 0.0], [0, 0, 0], [0, 0, 0]])
    u = np.array([kappa * y, 0.0, 0.0])
    prim = np.array([RHO_F, u[0], u[1], u[2], W.P0])
    d, V = 1e-6, 2e-3                         # theta = d kappa / (2 V) = 0.25, Re_p = 1.3e-4
    a_lag, F_lag = _lift(o, prim, G, u - [V, 0, 0], d)
    a_lead, _ = _lift(o, prim, G, u + [V, 0, 0], d)
    assert a_lag[1] > 0 and a_lead[1] < 0
    assert abs(a_lag[0]) == 0 and abs(a_lag[2]) == 0
    mp = rho_p * math.pi * d ** 3 / 6
    L = 6.46 * MU * (d / 2) ** 2 * V * math.sqrt(kappa / (MU / RHO_F))
    assert abs(mp * a_lag[1] / L - 1.0) < 1e-4
    # the source force is the lift itself (no drag, no other term)
    np.testing.assert_allclose(F_lag, mp * a_lag, rtol=1e-14)


def test_saffman_lift_is_normal_to_vorticity_and_slip():
    w = W.config1(n_particles=1)
    o = O.Oracle(w.mesh, w.N, W.uniform_state(w.mesh.n_elem, w.N, np.zeros(3)))
    rng = np.random.default_rng(12)
    for _ in range(20):
        G = rng.normal(size=(3, 3)) * 50
        u = rng.normal(size=3)
        v = u + rng.normal(size=3) * 0.05
        prim = np.array([RHO_F, *u, W.P0])
        a, _ = _lift(o, prim, G, v, 5e-5)
        om = np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
        s = np.linalg.norm(a)
        assert s > 0
        assert abs(a @ om) <= 1e-12 * s * np.linalg.norm(om)
        assert abs(a @ (u - v)) <= 1e-12 * s * np.linalg.norm(u - v)


def test_mei_correction_is_continuous_at_re_40():
    """The Re_p <= 40 branch, read as (1 - 0.3314 sqrt(th)) exp(-Re/10)
    + 0.3314 sqrt(th), meets 0.0524 sqrt(th Re) at Re = 40 up to the
    exp(-4) term; the other bracketing jumps by a factor of about ten."""
    w = W.config1(n_particles=1)
    o = O.Oracle(w.mesh, w.N, W.uniform_state(w.mesh.n_elem, w.N, np.zeros(3)))
    kappa, th = 1000.0, 0.1
    G = np.array([[0.0, kappa, 0.0], [0, 0, 0], [0, 0, 0]])
    prim = np.array([RHO_F, 0.0, 0.0, 0.0, W.P0])
    vals = []
    for Re in (40.0 * (1 - 1e-9), 40.0 * (1 + 1e-9)):
        d = math.sqrt(2 * th * MU * Re / (RHO_F * kappa))
        V = d * kappa / (2 * th)
        a, _ = _lift(o, prim, G, np.array([-V, 0.0, 0.0]), d)
        # divide out everything but C_S: a ~ C_S d^2 sqrt(rho mu / kappa) kappa V / m_p
        mp = 2500.0 * math.pi * d ** 3 / 6
        vals.append(a[1] * mp / (1.615 * d * d * math.sqrt(RHO_F * MU / kappa) * kappa * V))
    below, above = vals
    assert above > 0 and 1.0 < below / above < 1.2


# ---------------------------------------------------------------------------
# two-way source with the extra terms
# ---------------------------------------------------------------------------
def test_source_with_extra_forces_conserves_the_fluid_force():
    """Nearest-DOF and shape-kernel sources with all terms: sum S V equals minus
    the summed fluid force of the equation of motion (drag, stress, added mass
    with dv/dt from the same equation, lift), and the energy source minus F.v."""
    w = W.curved_box(cells=4, N=3, n_particles=300, n_steps=1, seed=61)
    o = O.Oracle(w.mesh, w.N, w.U)
    o.push(w.x, w.v + 0.3, w.d * 3, w.elem_hint)
    forces = O.F_BUOYANCY | O.F_STRESS | O.F_ADDED_MASS | O.F_SAFFMAN
    gvec = np.array([0.0, -9.81, 0.0])
    r = o.read()
    Ftot = np.zeros(4)
    for p in range(len(w.x)):
        prim, G = o.fluid_grad(r["elem"][p], r["xi"][p])
        _, F = o.particle_accel(1, forces, prim, G, r["v"][p], w.d[p] * 3, gvec)
        Ftot[:3] += F
        Ftot[3] += F @ r["v"][p]
    n3 = (w.N + 1) ** 3
    V = np.array([[o.volume(e, q) for q in range(n3)] for e in range(w.mesh.n_elem)])
    for kind, R in ((0, 0.0), (1, 1.5 / 4)):
        S = o.deposit(kind=kind, radius=R, period=np.array([1.0, 0.0, 1.0]) if kind else None,
                      drag=1, forces=forces, gravity=gvec)
        tot = np.einsum("ecq,eq->c", S, V)
        np.testing.assert_allclose(tot, -Ftot, rtol=1e-10, atol=1e-14)
    S0 = o.deposit(kind=0, drag=1)
    assert np.abs(np.einsum("ecq,eq->c", S0, V)[:3] + Ftot[:3]).max() > 1e-6 * np.abs(Ftot[:3]).max()
