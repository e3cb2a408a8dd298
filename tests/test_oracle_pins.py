"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine, a closed form derived in the test, brute force, or an invariant.  A
plausible mistake in the oracle (dropped term, wrong sign or index, transposed
operand) fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.special import comb

import oracle as O
from paper_2211_05458_amd import workloads as W


# --------------------------------------------------------------------------
# 1-D bases (Sec. 3.1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 12])
def test_gauss_nodes_match_numpy(n):
    x, w = O.gauss_nodes(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=1e-15, rtol=0)
    np.testing.assert_allclose(w, wr, atol=1e-14, rtol=0)


def test_gauss_two_point_closed_form():
    x, w = O.gauss_nodes(2)
    np.testing.assert_allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-16)
    np.testing.assert_allclose(w, [1.0, 1.0], atol=1e-15)


def test_lobatto_closed_forms():
    x, w = O.lobatto_nodes(3)
    np.testing.assert_allclose(x, [-1, 0, 1], atol=1e-16)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = O.lobatto_nodes(4)
    s = 1 / math.sqrt(5)
    np.testing.assert_allclose(x, [-1, -s, s, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("n", [2, 4, 6, 8])
def test_lagrange_delta_partition_and_derivative(n):
    nodes, _ = np.polynomial.legendre.leggauss(n)
    for j, xj in enumerate(nodes):
        l, _ = O.lagrange(nodes, xj)
        np.testing.assert_allclose(l, np.eye(n)[j], atol=1e-13)
    rng = np.random.default_rng(0)
    coef = rng.normal(size=n)          # polynomial of degree n-1
    for xi in rng.uniform(-1, 1, 5):
        l, dl = O.lagrange(nodes, xi)
        assert abs(l.sum() - 1.0) < 1e-13
        assert abs(dl.sum()) < 1e-11
        vals = np.polynomial.polynomial.polyval(nodes, coef)
        der = np.polynomial.polynomial.polyval(xi, np.polynomial.polynomial.polyder(coef))
        assert abs(l @ vals - np.polynomial.polynomial.polyval(xi, coef)) < 1e-12
        assert abs(dl @ vals - der) < 1e-10


# --------------------------------------------------------------------------
# Runge-Kutta coefficients (Sec. 3.1): Butcher form and order conditions
# --------------------------------------------------------------------------
def _butcher_from_2n(A, B):
    """Stage values y_j = y0 + sum_m a_jm F_m for the 2N-storage recursion."""
    s = len(A)
    k = np.zeros(s)        # coefficients of the register in terms of F_0..F_{s-1}
    y = np.zeros(s)
    a = np.zeros((s, s))   # a[i] = coefficients of the stage value used by stage i
    for i in range(s):
        a[i] = y
        k = A[i] * k
        k[i] += 1.0
        y = y + B[i] * k
    return a, y


@pytest.mark.parametrize("scheme,order", [(0, 4), (1, 3)])
def test_rk_order_conditions(scheme, order):
    A, B, c = O.rk_coeffs(scheme)
    assert A[0] == 0.0
    a, b = _butcher_from_2n(A, B)
    cc = a.sum(axis=1)
    np.testing.assert_allclose(cc, c, atol=1e-15)
    cond = {1: [(b.sum(), 1.0)],
            2: [(b @ cc, 0.5)],
            3: [(b @ cc ** 2, 1 / 3), (b @ a @ cc, 1 / 6)],
            4: [(b @ cc ** 3, 0.25), (b @ (cc * (a @ cc)), 1 / 8), (b @ a @ cc ** 2, 1 / 12),
                (b @ a @ a @ cc, 1 / 24)]}
    for p in range(1, order + 1):
        for val, ref in cond[p]:
            assert abs(val - ref) < 1e-14, (p, val, ref)
    # the scheme is not of higher order (order conditions of the next order fail)
    if order == 3:
        assert abs(b @ cc ** 3 - 0.25) > 1e-3 or abs(b @ a @ a @ cc - 1 / 24) > 1e-3


def _stab_poly(A, B):
    a, b = _butcher_from_2n(A, B)
    s = len(A)
    # R(z) = 1 + z b^T (I - z a)^{-1} 1 = sum_k z^k b^T a^{k-1} 1
    coef = [1.0]
    v = np.ones(s)
    for _ in range(s):
        coef.append(b @ v)
        v = a @ v
    return np.array(coef)


def test_rk_stability_polynomials():
    """Explicit s-stage methods of order p have R(z) = exp(z) up to z^p."""
    for scheme, p in [(0, 4), (1, 3)]:
        A, B, _ = O.rk_coeffs(scheme)
        R = _stab_poly(A, B)
        for k in range(p + 1):
            assert abs(R[k] - 1.0 / math.factorial(k)) < 1e-14
    # the paper's 2.75 tau_p for a fourth-order RK is the real-axis bound of the
    # classical RK4 polynomial (textbook value 2.7853)
    r4 = np.array([1, 1, 1 / 2, 1 / 6, 1 / 24])
    xs = np.linspace(0.01, 3.0, 30000)
    ok = np.abs(np.polynomial.polynomial.polyval(-xs, r4)) <= 1.0
    assert abs(xs[ok].max() - 2.7853) < 1e-3


# --------------------------------------------------------------------------
# geometry: map, Newton (Sec. 3.2.1)
# --------------------------------------------------------------------------
def _poly_map(xi):
    """A degree-2 polynomial map of the reference cube (exactly representable with Ng >= 2)."""
    x, y, z = xi[..., 0], xi[..., 1], xi[..., 2]
    out = np.empty(xi.shape)
    out[..., 0] = 1.0 + 0.5 * x + 0.05 * y * y + 0.02 * x * z
    out[..., 1] = -0.3 + 0.45 * y + 0.04 * x * x - 0.03 * z
    out[..., 2] = 0.2 + 0.55 * z + 0.03 * x * y + 0.02 * y
    return out


def _dummy_state(E, N):
    return W.uniform_state(E, N, np.zeros(3))


def test_map_reproduces_polynomial_geometry():
    for ng in (2, 4):
        mesh = W.single_element(ng, _poly_map)
        o = O.Oracle(mesh, 2, _dummy_state(1, 2))
        rng = np.random.default_rng(1)
        for xi in rng.uniform(-1, 1, (20, 3)):
            x, J = o.map(0, xi)
            np.testing.assert_allclose(x, _poly_map(xi[None])[0], atol=1e-14)
            h = 1e-6
            for d in range(3):
                e = np.zeros(3); e[d] = h
                fd = (_poly_map((xi + e)[None])[0] - _poly_map((xi - e)[None])[0]) / (2 * h)
                np.testing.assert_allclose(J[:, d], fd, atol=1e-9)


def test_newton_affine_closed_form():
    Amat = np.array([[0.5, 0.1, 0.02], [-0.05, 0.4, 0.1], [0.03, 0.02, 0.6]])
    bvec = np.array([1.0, 2.0, -1.0])
    mesh = W.single_element(1, lambda xi: xi @ Amat.T + bvec)
    o = O.Oracle(mesh, 3, _dummy_state(1, 3))
    rng = np.random.default_rng(2)
    for xi_true in rng.uniform(-1, 1, (20, 3)):
        x = Amat @ xi_true + bvec
        ok, xi, it = o.newton(0, x, np.zeros(3))
        assert ok and it == 2
        np.testing.assert_allclose(xi, np.linalg.solve(Amat, x - bvec), atol=1e-14)


def test_newton_curved_quadratic_convergence():
    mesh = W.single_element(4, _poly_map)
    o = O.Oracle(mesh, 2, _dummy_state(1, 2))
    rng = np.random.default_rng(3)
    for xi_true in rng.uniform(-1, 1, (30, 3)):
        x = _poly_map(xi_true[None])[0]
        ok, xi, it = o.newton(0, x, o.guess(0, x))
        assert ok and it <= 6
        np.testing.assert_allclose(xi, xi_true, atol=1e-12)
    # the guess is the nearest geometry node (approach 2 of Sec. 3.2.1)
    x = _poly_map(np.array([[0.49, -0.51, 0.99]]))[0]
    np.testing.assert_allclose(o.guess(0, x), [0.5, -0.5, 1.0])


def test_guess_nearest_dg_node_for_straight_elements():
    mesh = W.single_element(1, lambda xi: 0.5 * (xi + 1.0))    # unit cube
    o = O.Oracle(mesh, 3, _dummy_state(1, 3))
    g, _ = np.polynomial.legendre.leggauss(4)
    x = 0.5 * (np.array([g[1], g[3], g[0]]) + 1.0) + 1e-3
    np.testing.assert_allclose(o.guess(0, x), [g[1], g[3], g[0]])
    # third approach: exact for a parallelepiped
    xi_true = np.array([0.3, -0.7, 0.1])
    np.testing.assert_allclose(o.guess_faces(0, 0.5 * (xi_true + 1.0)), xi_true, atol=1e-14)


# --------------------------------------------------------------------------
# interpolation (eq. part_interpolation)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 3, 5])
def test_interpolation_reproduces_tensor_polynomials(N):
    n = N + 1
    g, _ = np.polynomial.legendre.leggauss(n)
    mesh = W.single_element(1, lambda xi: xi)
    rng = np.random.default_rng(4)
    exps = [(rng.integers(0, n), rng.integers(0, n), rng.integers(0, n)) for _ in range(5)]
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    U = np.zeros((1, 5, n ** 3))
    for var, (a, b, c) in enumerate(exps):
        U[0, var] = (ii ** a * jj ** b * kk ** c).ravel()
    o = O.Oracle(mesh, N, U)
    for xi in rng.uniform(-1, 1, (10, 3)):
        out = o.interp(0, xi)
        ref = [xi[0] ** a * xi[1] ** b * xi[2] ** c for (a, b, c) in exps]
        np.testing.assert_allclose(out, ref, atol=1e-13)


def test_interpolation_config1_cubic_field_exact():
    w = W.config1(n_particles=50)
    o = O.Oracle(w.mesh, w.N, w.U)
    for p in range(50):
        e, xi = o.locate(w.x[p], int(w.elem_hint[p]))
        assert e == w.elem_hint[p]
        Uc = o.interp(e, xi)
        np.testing.assert_allclose(Uc[1:4] / Uc[0], w.velocity(w.x[p:p + 1])[0], atol=1e-12)


# --------------------------------------------------------------------------
# drag (Sec. 2.2.1)
# --------------------------------------------------------------------------
def test_drag_factor_values():
    mesh = W.single_element(1, lambda xi: xi)
    o = O.Oracle(mesh, 1, _dummy_state(1, 1))
    mu, rho_p, d = 1.8e-5, 2500.0, 1e-4
    tau = rho_p * d * d / (18 * mu)
    rho = 1.2
    for Re, fref in [(1e-14, 1.0), (1.0, 1.15), (800 - 1e-9, 1 + 0.15 * 800 ** 0.687)]:
        slip = Re * mu / (rho * d)
        prim = np.array([rho, slip, 0.0, 0.0, 1e5])
        a, fD = o.drag_accel(1, prim, np.zeros(3), d)
        assert abs(fD - fref) < 1e-8 * fref
        np.testing.assert_allclose(a, [fD * slip / tau, 0, 0], rtol=1e-12)
    assert abs(1 + 0.15 * 800 ** 0.687 - 15.8086) < 1e-4
    a, fD = o.drag_accel(0, np.array([rho, 3.0, -1.0, 2.0, 1e5]), np.array([1.0, 1.0, 1.0]), d)
    assert fD == 1.0
    np.testing.assert_allclose(a, np.array([2.0, -2.0, 1.0]) / tau, rtol=1e-14)


# --------------------------------------------------------------------------
# time integration: Stokes particle in uniform flow, and the paper's V1 case
# --------------------------------------------------------------------------
def _periodic_cube(cells, N, u):
    w = W.config1(n_particles=1, cells=cells)
    return w.mesh, W.uniform_state(w.mesh.n_elem, N, u)


def test_stokes_relaxation_uniform_flow_order():
    u = np.array([0.3, -0.2, 0.1])
    mesh, U = _periodic_cube(4, 1, u)
    mu, rho_p = 1.8e-5, 2500.0
    tau = 0.05
    d = math.sqrt(tau * 18 * mu / rho_p)
    x0 = np.array([0.41, 0.52, 0.63])
    T = 0.2
    for scheme, order in [(0, 4), (1, 3)]:
        errs = []
        dts = [0.02, 0.01, 0.005, 0.0025]
        for dt in dts:
            o = O.Oracle(mesh, 1, U)
            o.push(x0[None], np.zeros((1, 3)), np.array([d]))
            o.step(dt, int(round(T / dt)), rk=scheme, drag=0)
            r = o.read()
            xe = x0 + u * T - tau * u * (1 - math.exp(-T / tau))
            ve = u * (1 - math.exp(-T / tau))
            dx = (r["x"][0] - xe + 0.5) % 1.0 - 0.5
            errs.append(max(np.abs(dx).max(), np.abs(r["v"][0] - ve).max()))
            assert r["status"][0] == O.ACTIVE
        slopes = np.diff(np.log(errs)) / np.diff(np.log(dts))
        assert abs(slopes[-1] - order) < 0.15, (scheme, errs, slopes)


def v1_exact(t, tau, g=-9.81, y0=2.0):
    """Closed-form V1 trajectory (drag in x only, gravity in y) with the t^3/3 term."""
    E = math.exp(-t / tau)
    x1 = t - tau * (1 - E) + g / (2 * y0) * (t ** 3 / 3 - t * t * tau + 2 * tau * tau * t + 2 * tau ** 3 * (E - 1))
    v1 = 1 - E + g / (2 * y0) * (t * t - 2 * t * tau + 2 * tau * tau - 2 * tau * tau * E)
    return x1, v1, 0.5 * g * t * t + y0, g * t


def test_v1_closed_form_is_exact_solution():
    # the closed form satisfies tau v1' + v1 = u1(y(t)) = y(t)/y0 and x1' = v1
    for tau in (0.2, 2.0, 20.0):
        for t in (0.1, 0.25, 0.4):
            h = 1e-5
            x1p, v1p, _, _ = v1_exact(t + h, tau)
            x1m, v1m, _, _ = v1_exact(t - h, tau)
            x1, v1, y, _ = v1_exact(t, tau)
            assert abs((x1p - x1m) / (2 * h) - v1) < 1e-6
            assert abs(tau * (v1p - v1m) / (2 * h) + v1 - y / 2.0) < 1e-6


def _v1_mesh():
    def node_map(I1, I2, I3, M):
        out = np.empty(np.broadcast_shapes(I1.shape, I2.shape, I3.shape) + (3,))
        out[..., 0] = 2.0 * I1 / M[0]
        out[..., 1] = 2.0 * I2 / M[1]
        out[..., 2] = 2.0 * I3 / M[2]
        return out
    X, ne, nf, bc, sh, _ = W.structured_mesh((2, 2, 2), 1, node_map, (False, False, False),
                                             wall_bc=W.BC_OPEN)
    return W.Mesh(1, X, ne, nf, bc, sh, h=1.0, cells=(2, 2, 2))


def test_v1_fourth_order_time_integration():
    """Sec. 5.1: linear shear u = [y/y0, 0, 0], rho = p = 1, drag in x only, gravity in y."""
    mesh = _v1_mesh()
    N = 2
    g, _ = np.polynomial.legendre.leggauss(N + 1)
    U = np.zeros((8, 5, (N + 1) ** 3))
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    for e in range(8):
        iy = (e // 2) % 2
        y = iy + 0.5 * (jj.ravel() + 1.0)             # h = 1
        U[e, 0] = 1.0
        U[e, 1] = y / 2.0
        U[e, 4] = 1.0 / 0.4 + 0.5 * (y / 2.0) ** 2
    mu, rho_p = 1.8e-5, 2500.0
    for St in (0.1, 1.0, 10.0):
        tau = 2.0 * St
        d = math.sqrt(tau * 18 * mu / rho_p)
        errs = []
        dts = [0.0125 * 2 ** k for k in range(5)]
        for dt in dts:
            o = O.Oracle(mesh, N, U, mu=mu, rho_p=rho_p)
            st, nbad = o.push(np.array([[0.0, 2.0, 0.5]]), np.zeros((1, 3)), np.array([d]))
            assert nbad == 0
            o.step(dt, int(round(0.4 / dt)), rk=0, drag=0, gravity=(0.0, -9.81, 0.0),
                   drag_mask=(1.0, 0.0, 0.0))
            r = o.read()
            assert r["status"][0] == O.ACTIVE
            x1, _, y, _ = v1_exact(0.4, tau)
            errs.append(abs(r["x"][0, 0] - x1))
            assert abs(r["x"][0, 1] - y) < 1e-12
        errs = np.array(errs)
        slopes = np.diff(np.log(errs)) / np.diff(np.log(dts))
        # fourth order wherever the error is above the rounding floor of the
        # closed form (~1e-12 at tau = 20)
        use = (errs[:-1] > 1e-10) & (errs[1:] > 1e-10)
        assert use.sum() >= 2
        assert np.all(np.abs(slopes[use] - 4.0) < 0.5), (St, errs, slopes)
        assert abs(slopes[use][0] - 4.0) < 0.1, (St, errs, slopes)


# --------------------------------------------------------------------------
# faces and intersections (Sec. 3.2.4)
# --------------------------------------------------------------------------
def _bernstein_patch(cp, ng, u, v):
    deg = ng - 1
    s, t = 0.5 * (u + 1), 0.5 * (v + 1)
    Bu = np.array([comb(deg, m) * s ** m * (1 - s) ** (deg - m) for m in range(ng)])
    Bv = np.array([comb(deg, m) * t ** m * (1 - t) ** (deg - m) for m in range(ng)])
    P = cp.reshape(ng, ng, 3)     # [n][m]
    return np.einsum("nmc,m,n->c", P, Bu, Bv)


def test_bezier_faces_equal_geometry():
    ng = 5
    mesh = W.single_element(4, _poly_map)
    o = O.Oracle(mesh, 2, _dummy_state(1, 2))
    rng = np.random.default_rng(5)
    for f in range(6):
        cp, typ = o.face(0, f)
        assert typ == O.FACE_CURVED
        d, a, b = f // 2, (1 if f // 2 == 0 else 0), (1 if f // 2 == 2 else 2)
        for u, v in rng.uniform(-1, 1, (10, 2)):
            xi = np.zeros(3)
            xi[d] = -1.0 if f % 2 == 0 else 1.0
            xi[a] = u; xi[b] = v
            np.testing.assert_allclose(_bernstein_patch(cp, ng, u, v), _poly_map(xi[None])[0], atol=1e-14)


def test_face_classification():
    cube = W.single_element(1, lambda xi: xi)
    o = O.Oracle(cube, 1, _dummy_state(1, 1))
    assert all(o.face(0, f)[1] == O.FACE_PLANAR for f in range(6))

    def twisted(xi):
        out = xi.copy()
        out[..., 0] += 0.2 * xi[..., 1] * xi[..., 2]    # faces x = +-1 become hyperbolic paraboloids
        return out
    o2 = O.Oracle(W.single_element(1, twisted), 1, _dummy_state(1, 1))
    assert o2.face(0, 0)[1] == O.FACE_BILINEAR and o2.face(0, 1)[1] == O.FACE_BILINEAR
    o3 = O.Oracle(W.single_element(2, _poly_map), 1, _dummy_state(1, 1))
    assert o3.face(0, 0)[1] == O.FACE_CURVED


def test_planar_intersection_closed_form():
    cube = W.single_element(1, lambda xi: xi)
    o = O.Oracle(cube, 1, _dummy_state(1, 1))
    x0 = np.array([0.1, 0.2, -0.3])
    t = np.array([0.8, 0.1, 0.2]); t /= np.linalg.norm(t)
    al, uv = o.face_intersect(0, 1, x0, t)         # face x = +1
    assert len(al) == 1
    a = (1.0 - x0[0]) / t[0]
    assert abs(al[0] - a) < 1e-15
    np.testing.assert_allclose(uv[0], [x0[1] + a * t[1], x0[2] + a * t[2]], atol=1e-15)


def _brute_roots(surface, x0, t, grid=300):
    """Roots of surface(u, v) = x0 + alpha t by dense grid search + Newton polish (3x3)."""
    us = np.linspace(-1.3, 1.3, grid)
    U_, V_ = np.meshgrid(us, us, indexing="ij")
    P = surface(U_, V_)                                     # (g, g, 3)
    r = P - x0
    perp = r - (r @ t)[..., None] * t
    dist = np.linalg.norm(perp, axis=-1)
    roots = []
    cand = np.argwhere(dist < 0.05)
    order = np.argsort(dist[cand[:, 0], cand[:, 1]])
    for idx in cand[order]:
        u, v = us[idx[0]], us[idx[1]]
        al = (surface(np.array(u), np.array(v)) - x0) @ t
        z = np.array([u, v, al])
        for _ in range(30):
            h = 1e-7
            F = surface(np.array(z[0]), np.array(z[1])) - x0 - z[2] * t
            Ju = (surface(np.array(z[0] + h), np.array(z[1])) - surface(np.array(z[0] - h), np.array(z[1]))) / (2 * h)
            Jv = (surface(np.array(z[0]), np.array(z[1] + h)) - surface(np.array(z[0]), np.array(z[1] - h))) / (2 * h)
            Jm = np.stack([Ju, Jv, -t], axis=1)
            try:
                dz = np.linalg.solve(Jm, -F)
            except np.linalg.LinAlgError:
                break
            z = z + dz
            if np.abs(dz).max() < 1e-15:
                break
        F = surface(np.array(z[0]), np.array(z[1])) - x0 - z[2] * t
        if np.abs(F).max() < 1e-12 and abs(z[0]) <= 1 and abs(z[1]) <= 1:
            if not any(np.abs(z - q).max() < 1e-8 for q in roots):
                roots.append(z)
    return roots


def test_bilinear_intersection_brute_force():
    C00 = np.array([0.0, 0.0, 0.0]); CN0 = np.array([1.0, 0.1, 0.2])
    C0N = np.array([-0.1, 1.0, 0.1]); CNN = np.array([1.1, 0.9, -0.4])

    def surf(u, v):
        s, t = 0.5 * (np.asarray(u) + 1), 0.5 * (np.asarray(v) + 1)
        return ((1 - s) * (1 - t))[..., None] * C00 + (s * (1 - t))[..., None] * CN0 + \
            ((1 - s) * t)[..., None] * C0N + (s * t)[..., None] * CNN

    def node_fn(xi):
        out = np.empty(xi.shape)
        # element whose face 4 (xi3 = -1) is the bilinear patch; faces param (xi1, xi2)
        base = surf(xi[..., 0], xi[..., 1])
        out[:] = base
        out[..., 2] += 0.5 * (xi[..., 2] + 1.0) + 0.0
        return out
    o = O.Oracle(W.single_element(1, node_fn), 1, _dummy_state(1, 1))
    assert o.face(0, 4)[1] == O.FACE_BILINEAR
    rng = np.random.default_rng(6)
    n_two = 0
    for _ in range(40):
        x0 = np.array([rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(0.5, 1.0)])
        t = rng.normal(size=3); t[2] = -abs(t[2]) - 0.2; t /= np.linalg.norm(t)
        al, uv = o.face_intersect(0, 4, x0, t)
        got = [np.array([u, v, a]) for a, (u, v) in zip(al, uv) if abs(u) <= 1 and abs(v) <= 1]
        ref = _brute_roots(surf, x0, t)
        assert len(got) == len(ref)
        for r in ref:
            assert min(np.abs(r - g).max() for g in got) < 1e-10
        n_two += len(ref) == 2
    # grazing rays through the saddle: two roots
    x0 = np.array([0.5, 0.5, 0.1]); t = np.array([1.0, 0.05, 0.0]); t /= np.linalg.norm(t)
    al, uv = o.face_intersect(0, 4, x0, t)
    ref = _brute_roots(surf, x0, t)
    got = [np.array([u, v, a]) for a, (u, v) in zip(al, uv) if abs(u) <= 1 and abs(v) <= 1]
    assert len(got) == len(ref)


def test_curved_bezier_clipping_brute_force():
    """Random lines against a strongly curved degree-4 face; all roots found."""
    amp = 0.15

    def face_map(u, v):
        u = np.asarray(u, dtype=float); v = np.asarray(v, dtype=float)
        out = np.empty(np.broadcast(u, v).shape + (3,))
        out[..., 0] = u + 0.1 * v * v
        out[..., 1] = v - 0.05 * u * u * v
        out[..., 2] = amp * (u ** 4 - 0.5 * v ** 3 + u * v) + 0.2 * u * u
        return out
    ng = 5
    r = np.linspace(-1, 1, ng)
    V_, U_ = np.meshgrid(r, r, indexing="ij")
    nodes = face_map(U_, V_).reshape(-1, 3)     # [n][m] with m (u) fastest
    # Lagrange -> Bernstein by solving the interpolation system in numpy
    deg = ng - 1
    M = np.array([[comb(deg, b) * (0.5 * (s + 1)) ** b * (1 - 0.5 * (s + 1)) ** (deg - b) for b in range(ng)] for s in r])
    Minv = np.linalg.inv(M)
    cp = np.einsum("am,bn,nmc->bac", Minv, Minv, nodes.reshape(ng, ng, 3)).reshape(-1, 3)
    rng = np.random.default_rng(7)
    total = 0
    for trial in range(60):
        t = rng.normal(size=3)
        if trial % 3 == 0:
            t[2] = -abs(t[2]) - 0.3
        else:
            t[2] = -0.2 * abs(t[2])             # shallow rays: more double roots
        t /= np.linalg.norm(t)
        if trial % 4 == 3:                      # random line, often a miss
            x0 = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), rng.uniform(0.6, 1.2)])
        else:                                   # line through a random point of the face
            x0 = face_map(*rng.uniform(-0.95, 0.95, 2)) - rng.uniform(0.2, 1.0) * t
        al, uv = O.bezier_intersect(cp, x0, t)
        got = [np.array([u, v, a]) for a, (u, v) in zip(al, uv) if abs(u) <= 1 + 1e-12 and abs(v) <= 1 + 1e-12]
        ref = _brute_roots(face_map, x0, t, grid=240)
        assert len(got) == len(ref), (trial, got, ref)
        for rr in ref:
            assert min(np.abs(rr - g).max() for g in got) < 1e-9
        total += len(ref)
    assert total > 20


# --------------------------------------------------------------------------
# tracking: ballistic billiard (closed form with exact wall-hit counts)
# --------------------------------------------------------------------------
def _fold(X):
    m = np.floor(X)
    r = X - m
    return np.where(m % 2 == 0, r, 1.0 - r), np.abs(m).astype(int)


def _box(cells, periodic, n_geo=1, amp=0.0):
    def node_map(I1, I2, I3, M):
        out = np.empty(np.broadcast_shapes(I1.shape, I2.shape, I3.shape) + (3,))
        out[..., 0] = I1 / M[0]
        out[..., 1] = I2 / M[1]
        out[..., 2] = I3 / M[2]
        return out
    X, ne, nf, bc, sh, _ = W.structured_mesh((cells,) * 3, n_geo, node_map, periodic, periods=np.eye(3))
    return W.Mesh(n_geo, X, ne, nf, bc, sh, h=1.0 / cells, cells=(cells,) * 3)


@pytest.mark.parametrize("rk", [0, 1])
def test_billiard_reflective_box(rk):
    mesh = _box(4, (False, False, False))
    U = W.uniform_state(mesh.n_elem, 1, np.zeros(3))
    rng = np.random.default_rng(8)
    n = 200
    x0 = rng.uniform(0.02, 0.98, (n, 3))
    v0 = rng.uniform(-3, 3, (n, 3))
    o = O.Oracle(mesh, 1, U)
    st, nbad = o.push(x0, v0, np.full(n, 1e-4))
    assert nbad == 0
    dt, ns = 0.01, 50
    o.step(dt, ns, rk=rk, drag=2)
    r = o.read()
    T = dt * ns
    xf, hits = _fold(x0 + v0 * T)
    assert np.all(r["status"] == O.ACTIVE)
    np.testing.assert_allclose(r["x"], xf, atol=1e-12)
    np.testing.assert_array_equal(r["hits"], hits.sum(axis=1))
    # speed is preserved by the specular reflections
    np.testing.assert_allclose(np.linalg.norm(r["v"], axis=1), np.linalg.norm(v0, axis=1), rtol=1e-14)
    # final element is the one containing the folded position
    cells = np.minimum((xf * 4).astype(int), 3)
    np.testing.assert_array_equal(r["elem"], cells[:, 0] + 4 * (cells[:, 1] + 4 * cells[:, 2]))


def test_billiard_periodic_box():
    mesh = _box(8, (True, True, True))
    U = W.uniform_state(mesh.n_elem, 1, np.zeros(3))
    rng = np.random.default_rng(9)
    n = 200
    x0 = rng.uniform(0.01, 0.99, (n, 3))
    v0 = rng.uniform(-3, 3, (n, 3))
    o = O.Oracle(mesh, 1, U)
    o.push(x0, v0, np.full(n, 1e-4))
    o.step(0.01, 40, rk=1, drag=2)
    r = o.read()
    xf = np.mod(x0 + v0 * 0.4, 1.0)
    d = (r["x"] - xf + 0.5) % 1.0 - 0.5
    assert np.abs(d).max() < 1e-12
    assert np.all(r["hits"] == 0)
    assert np.all(r["status"] == O.ACTIVE)


def test_billiard_curved_wall_speed_and_inside():
    """Curved (sine) mesh, reflective curved walls: every particle stays inside
    and keeps its speed; walls are hit."""
    w = W.curved_box(cells=4, N=2, n_particles=300, n_steps=1, seed=11)
    o = O.Oracle(w.mesh, w.N, w.U)
    rng = np.random.default_rng(12)
    v0 = rng.uniform(-2, 2, (300, 3))
    o.push(w.x, v0, w.d, w.elem_hint)
    o.step(0.01, 30, rk=1, drag=2)
    r = o.read()
    assert np.all(r["status"] == O.ACTIVE)
    assert r["hits"].sum() > 50
    np.testing.assert_allclose(np.linalg.norm(r["v"], axis=1), np.linalg.norm(v0, axis=1), rtol=1e-13)
    assert np.all(np.abs(r["xi"]) <= 1 + 1e-10)


# --------------------------------------------------------------------------
# deposition (Sec. 2.3)
# --------------------------------------------------------------------------
def test_volumes_sum_to_element_volume():
    Amat = np.array([[0.5, 0.1, 0.0], [0.0, 0.4, 0.1], [0.05, 0.0, 0.6]])
    o = O.Oracle(W.single_element(1, lambda xi: xi @ Amat.T), 3, _dummy_state(1, 3))
    vols = np.array([o.volume(0, q) for q in range(64)])
    assert abs(vols.sum() - 8 * np.linalg.det(Amat)) < 1e-14
    o2 = O.Oracle(W.single_element(4, _poly_map), 3, _dummy_state(1, 3))
    vols = np.array([o2.volume(0, q) for q in range(64)])
    # the Jacobian determinant of _poly_map is a polynomial of degree <= 5 per axis: exact at n=4
    g, wg = np.polynomial.legendre.leggauss(6)
    ref = 0.0
    for i in range(6):
        for j in range(6):
            for k in range(6):
                xi = np.array([g[i], g[j], g[k]])
                _, J = o2.map(0, xi)
                ref += wg[i] * wg[j] * wg[k] * np.linalg.det(J)
    assert abs(vols.sum() - ref) < 1e-12


def test_deposit_conservation_and_single_node():
    w = W.curved_box(cells=4, N=3, n_particles=400, n_steps=1, seed=13)
    o = O.Oracle(w.mesh, w.N, w.U)
    v = w.v + 0.3
    o.push(w.x, v, w.d, w.elem_hint)
    n3 = (w.N + 1) ** 3
    V = np.array([[o.volume(e, q) for q in range(n3)] for e in range(w.mesh.n_elem)])
    # reference force from the oracle components
    Ftot = np.zeros(4)
    for p in range(400):
        e, xi = o.locate(w.x[p], int(w.elem_hint[p]))
        Uc = o.interp(e, xi)
        prim = np.array([Uc[0], Uc[1] / Uc[0], Uc[2] / Uc[0], Uc[3] / Uc[0], 0.0])
        a, fD = o.drag_accel(1, prim, v[p], w.d[p])
        F = 3 * math.pi * 1.8e-5 * w.d[p] * fD * (prim[1:4] - v[p])
        Ftot[:3] += F
        Ftot[3] += F @ v[p]
    for kind, R in [(0, 0.0), (1, 1.5 / 4)]:
        S = o.deposit(kind=kind, radius=R, period=np.array([1.0, 0.0, 1.0]))
        tot = np.einsum("ecq,eq->c", S, V)
        np.testing.assert_allclose(tot, -Ftot, rtol=1e-12)
    # a single particle at a DG node deposits only there
    e0 = 5
    q0 = 1 + 4 * (2 + 4 * 3)
    xn = o.dg_node_pos(e0, q0)
    o.push(xn[None], np.zeros((1, 3)), np.array([1e-4]), np.array([e0]))
    S = o.deposit(kind=0)
    nz = np.argwhere(np.abs(S).sum(axis=1) > 0)
    assert nz.tolist() == [[e0, q0]]
    _, xi = o.locate(xn, e0)
    Uc = o.interp(e0, xi)
    u = Uc[1:4] / Uc[0]
    a, fD = o.drag_accel(1, np.array([Uc[0], *u, 0.0]), np.zeros(3), 1e-4)
    F = 3 * math.pi * 1.8e-5 * 1e-4 * fD * u
    np.testing.assert_allclose(S[e0, :3, q0], -F / V[e0, q0], rtol=1e-12)


# --------------------------------------------------------------------------
# learned guess: backprop against central differences
# --------------------------------------------------------------------------
def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(14)
    nw = O.mlp_n_weights()
    assert nw == 64 * 84 + 64 + 2 * (64 * 64 + 64) + 3 * 64 + 3
    w = rng.normal(scale=0.2, size=nw)
    inp = rng.normal(size=(16, 84))
    tgt = rng.uniform(-1, 1, size=(16, 3))
    loss, g = O.mlp_loss_grad(w, inp, tgt)
    out = O.mlp_forward(w, inp)
    assert abs(loss - np.mean((out - tgt) ** 2)) < 1e-14
    idx = rng.choice(nw, 60, replace=False)
    idx = np.concatenate([idx, [0, 64 * 84, nw - 1, nw - 4]])
    h = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        fd = (O.mlp_loss_grad(wp, inp, tgt)[0] - O.mlp_loss_grad(wm, inp, tgt)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_adam_matches_definition():
    rng = np.random.default_rng(15)
    w = rng.normal(size=10); m = np.zeros(10); v = np.zeros(10)
    w0 = w.copy()
    g1 = rng.normal(size=10)
    O.adam(w, m, v, g1, 1, 1e-2)
    # first Adam step moves every weight by lr * sign(g) (bias-corrected m/sqrt(v) = g/|g|)
    np.testing.assert_allclose(w, w0 - 1e-2 * g1 / (np.abs(g1) + 1e-8), rtol=1e-12)


def test_mlp_features_carry_corners_curvature_and_point():
    """Corners, the deviation from the trilinear corner map (exact for a
    polynomial map) and the point, scaled by the mean corner-edge length."""
    mesh = W.single_element(4, _poly_map)
    o = O.Oracle(mesh, 2, _dummy_state(1, 2))
    x = np.array([1.1, -0.2, 0.3])
    f = o.mlp_features(0, x)
    c = np.array([[i, j, k] for k in (-1, 1) for j in (-1, 1) for i in (-1, 1)], dtype=float)
    cor = _poly_map(c)
    ctr = cor.mean(axis=0)
    edges = [np.linalg.norm(cor[a] - cor[a ^ (1 << b)]) for a in range(8) for b in range(3) if a ^ (1 << b) > a]
    h = np.mean(edges)
    np.testing.assert_allclose(f[:24], ((cor - ctr) / h).ravel(), atol=1e-14)
    np.testing.assert_allclose(f[81:], (x - ctr) / h, atol=1e-14)
    pts = [np.array([i - 1.0, j - 1.0, k - 1.0]) for k in range(3) for j in range(3) for i in range(3)
           if 1 in (i, j, k)]
    for r, xi in enumerate(pts):
        w8 = np.array([0.125 * (1 + ci[0] * xi[0]) * (1 + ci[1] * xi[1]) * (1 + ci[2] * xi[2]) for ci in c])
        dev = _poly_map(xi[None])[0] - w8 @ cor
        np.testing.assert_allclose(f[24 + 3 * r: 27 + 3 * r], dev / h, atol=1e-13)
    # an affine element has no curvature features
    o2 = O.Oracle(W.single_element(4, lambda xi: xi @ np.diag([0.5, 0.4, 0.6]).T), 2, _dummy_state(1, 2))
    assert np.abs(o2.mlp_features(0, x)[24:81]).max() < 1e-14


def test_grazing_face_crossings_stay_tracked():
    """Straight (drag-free) paths crossing curved internal faces at incidence
    angles 1e-7..1e-1: every particle ends in the element that contains its
    final position (an independent Newton check) and at the straight-line
    position (modulo the periodic directions).  Exercises the entry-face
    threshold after a hand-off and the neighbour recovery of crossings that
    the clipping misses."""
    from grazing_paths import grazing_paths
    w = W.curved_box(cells=4, N=3, n_particles=1, n_steps=1, seed=13)
    o = O.Oracle(w.mesh, w.N, w.U)
    rng = np.random.default_rng(14)
    L, dt = 0.05, 1e-3
    x0, d, h = grazing_paths(o, w.mesh, 1500, rng, L)
    st, nbad = o.push(x0, d * (L / dt), np.full(len(x0), 1e-5), h)
    ok = st == O.ACTIVE
    o.step(dt, 1, rk=1, drag=2)
    r = o.read()
    assert np.all(r["status"][ok] == O.ACTIVE)
    s = o.stats()
    assert s["lost"] == 0 and s["recovered"] > 0 and s["crossings"] > 1000
    for p in np.nonzero(ok)[0]:
        conv, xi, _ = o.newton(r["elem"][p], r["x"][p], o.guess(r["elem"][p], r["x"][p]))
        assert conv and np.abs(xi).max() <= 1 + 1e-10
    free = ok & (r["hits"] == 0)
    dx = r["x"][free] - (x0[free] + d[free] * L)
    dx[:, [0, 2]] -= np.round(dx[:, [0, 2]])            # periods 1 in x and z
    assert np.abs(dx).max() < 1e-12


def test_reference_space_localisation_equals_physical_tracking():
    """Internal faces do not change a path, so localising the segments that
    cannot reach a boundary face (instead of tracing them) must give the same
    elements, positions, velocities and wall hits, bit for bit."""
    w = W.curved_box(cells=8, N=3, n_particles=6000, n_steps=1, seed=31)
    out = []
    for tracking in (0, 1):
        o = O.Oracle(w.mesh, w.N, w.U)
        o.push(w.x, w.v * 20.0, w.d, w.elem_hint)
        o.step(2e-3, 12, rk=1, drag=1, tracking=tracking)
        out.append((o.read(), o.stats()))
    (a, sa), (b, sb) = out
    for k in ("status", "elem", "hits", "x", "v"):
        np.testing.assert_array_equal(a[k], b[k])
    assert sa["wall_hits"] > 100 and sb["crossings"] < 0.8 * sa["crossings"] and sb["recovered"] > 1000


def _annulus_localisation_case():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "annulus_localisation_case.json")
    with open(path) as f:
        c = json.load(f)
    return (np.array([c["x"]]), np.array([c["v"]]), np.array([c["d"]]),
            np.array([c["elem_hint"]], np.int32))


def test_reference_space_localises_where_newton_diverges():
    """Strongly curved annular passage (N_geo = 6), one particle of its seeded
    workload (fixture written by tests/golden/make_annulus_localisation_case.py):
    its step crosses two internal faces without coming near a wall, so under
    reference-space localisation no segment is traced.  Newton on the map of
    the element it started in diverges at the end point (from every guess),
    so the location step must fall back to the background-mesh candidates
    (Sec. 3.2.3); the result equals physical tracking bit for bit."""
    w = W.config4(n_particles=1)
    x, v, d, h = _annulus_localisation_case()
    o = O.Oracle(w.mesh, w.N, w.U)
    out = []
    for tracking in (0, 1):
        o.reset_stats()
        st, _ = o.push(x, v, d, h)
        assert st[0] == O.ACTIVE
        o.step(w.dt, 1, rk=w.rk, drag=w.drag, tracking=tracking)
        out.append((o.read(), o.stats()))
    (a, sa), (b, sb) = out
    for k in ("status", "elem", "hits", "x", "v"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["status"][0] == O.ACTIVE and a["elem"][0] != h[0] and sa["crossings"] >= 2
    assert sb["crossings"] == 0 and sb["recovered"] >= 1 and sb["lost"] == 0
    # the premise: the start element's map cannot be inverted at the end point
    xe = a["x"][0]
    assert not o.newton(int(h[0]), xe, o.guess(int(h[0]), xe))[0]
    assert not o.newton(int(h[0]), xe, o.guess_faces(int(h[0]), xe))[0]
    conv, xi, _ = o.newton(int(a["elem"][0]), xe, o.guess(int(a["elem"][0]), xe))
    assert conv and np.abs(xi).max() <= 1.0


def test_boundary_distance_is_a_lower_bound():
    """Brute force: points of each element against dense samples of every wall
    and periodic face; no point is closer to such a face than the element's
    bound, and interior elements get a positive bound."""
    w = W.curved_box(cells=6, N=2, n_particles=1, n_steps=1, seed=32)
    o = O.Oracle(w.mesh, w.N, w.U)
    mesh = w.mesh
    E = mesh.n_elem
    g = np.linspace(-1, 1, 9)
    U, V = np.meshgrid(g, g, indexing="ij")
    pts_face = []
    for e in range(E):
        for f in range(6):
            if mesh.bc[e, f] == 0:
                continue
            ax = f // 2
            free = [a for a in range(3) if a != ax]
            for u, v in zip(U.ravel(), V.ravel()):
                xi = np.zeros(3)
                xi[ax] = 1.0 if f % 2 else -1.0
                xi[free[0]], xi[free[1]] = u, v
                pts_face.append(o.map(e, xi)[0])
    pts_face = np.array(pts_face)
    rng = np.random.default_rng(33)
    d = np.array([o.boundary_distance(e) for e in range(E)])
    assert (d > 0).sum() >= 4 * 4 * 2          # elements two layers from walls and periodic faces
    for e in range(E):
        if d[e] == 0.0:
            continue
        xs = np.array([o.map(e, rng.uniform(-1, 1, 3))[0] for _ in range(20)])
        dist = np.sqrt(((xs[:, None, :] - pts_face[None, :, :]) ** 2).sum(-1)).min()
        assert dist >= d[e]


def test_face_sign_gives_outward_normals():
    """The exit-direction rule uses n_out = s_f (dp/du x dp/dv) with face
    parameters the two other reference axes in increasing order and
    s = (-1, 1, 1, -1, -1, 1).  Checked with finite differences of the element
    map (not the face code): at face centres and random face points of curved
    elements, n_out points away from the element's interior."""
    s = [-1.0, 1.0, 1.0, -1.0, -1.0, 1.0]
    w = W.curved_box(cells=3, N=2, n_particles=1, n_steps=1, seed=34)
    o = O.Oracle(w.mesh, w.N, w.U)
    rng = np.random.default_rng(35)
    hstep = 1e-6
    for e in range(w.mesh.n_elem):
        for f in range(6):
            ax = f // 2
            a, b = [k for k in range(3) if k != ax]
            for uv in [(0.0, 0.0)] + [tuple(rng.uniform(-0.9, 0.9, 2)) for _ in range(2)]:
                xi = np.zeros(3)
                xi[ax] = 1.0 if f % 2 else -1.0
                xi[a], xi[b] = uv
                def at(d, k):
                    z = xi.copy(); z[k] += d
                    return o.map(e, z)[0]
                pu = (at(hstep, a) - at(-hstep, a)) / (2 * hstep)
                pv = (at(hstep, b) - at(-hstep, b)) / (2 * hstep)
                n = s[f] * np.cross(pu, pv)
                inward = o.map(e, xi * np.where(np.arange(3) == ax, 0.9, 1.0))[0] - o.map(e, xi)[0]
                assert np.dot(n, inward) < 0
