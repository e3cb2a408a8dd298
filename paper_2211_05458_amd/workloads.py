"""Seeded synthetic workloads: meshes, fluid states and particles.

This module only *describes* inputs.  It contains none of the particle method's
arithmetic (no Lagrange mapping, no Newton, no interpolation, no tracking): meshes
are produced by evaluating an analytic map on an integer node lattice, fluid
states by evaluating an analytic velocity field at the analytic image of the DG
node positions, and particles by drawing a logical cell and a point inside it.
Both the CPU oracle and the HIP library consume exactly these arrays.

Array conventions shared by every consumer
------------------------------------------
* ``X``      float64 ``[E][(Ng+1)^3][3]``; node index ``i + n*(j + n*k)`` with
  ``i`` along xi^1 (fastest).  Geometry nodes are equidistant on [-1, 1].
* ``nbr_elem``/``nbr_face`` int32 ``[E][6]``; local faces are
  0: xi^1=-1, 1: xi^1=+1, 2: xi^2=-1, 3: xi^2=+1, 4: xi^3=-1, 5: xi^3=+1.
* ``bc`` int8 ``[E][6]``: 0 internal, 1 open, 2 reflective, 3 periodic.
* ``shift`` float64 ``[E][6][3]``: translation applied to a particle that
  crosses a periodic face.
* ``U`` float64 ``[E][5][(N+1)^3]``: conservative variables
  (rho, rho u1, rho u2, rho u3, rho e) at the Legendre-Gauss nodes.
* particles: ``x``, ``v`` float64 ``[Np][3]``, ``d`` float64 ``[Np]``,
  ``elem_hint`` int32 ``[Np]``.

Physical constants (fluid at rest conditions, particle material): air-like gas
with constant viscosity, glass-like particles.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

KAPPA = 1.4
MU = 1.8e-5
RHO_F = 1.2
P0 = 1.0e5
RHO_P = 2500.0

BC_INTERNAL, BC_OPEN, BC_REFLECT, BC_PERIODIC, BC_MORTAR = 0, 1, 2, 3, 4

VERBOSE = False   # report generation progress on stderr (large workloads)


def _progress(what, done, total):
    if VERBOSE:
        import sys
        print("[workloads] %s %d/%d" % (what, done, total), file=sys.stderr, flush=True)


@dataclasses.dataclass
class Mesh:
    n_geo: int
    X: np.ndarray          # [E][(ng)^3][3] f64
    nbr_elem: np.ndarray   # [E][6] i32
    nbr_face: np.ndarray   # [E][6] i32
    bc: np.ndarray         # [E][6] i8
    shift: np.ndarray      # [E][6][3] f64
    h: float               # nominal element width
    cells: tuple = ()      # logical lattice size (n1, n2, n3) when structured
    mortar: np.ndarray = None  # [n_mortar][4][2] i32: (small element, its face) per big mortar face, -1 unused

    @property
    def n_elem(self) -> int:
        return int(self.X.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    N: int                 # DG degree
    U: np.ndarray          # [E][5][(N+1)^3] f64
    x: np.ndarray          # [Np][3]
    v: np.ndarray          # [Np][3]
    d: np.ndarray          # [Np]
    elem_hint: np.ndarray  # [Np] i32
    dt: float
    n_steps: int
    rk: int                # 0 = 5-stage 4th order low storage, 1 = 3-stage 3rd order
    drag: int              # 0 = Stokes, 1 = Schiller-Naumann
    mu: float = MU
    kappa: float = KAPPA
    rho_p: float = RHO_P
    velocity: Optional[Callable] = None   # analytic field u(x) (N, 3) -> (N, 3), for tests

    @property
    def n_particles(self) -> int:
        return int(self.x.shape[0])


# ----------------------------------------------------------------------------
# integer-lattice trigonometry: sin(2*pi*num/den) with the argument reduced in
# integers, so that periodic images of a lattice node are bitwise equal.
# ----------------------------------------------------------------------------
def sin2pi(num, den):
    num = np.asarray(num, dtype=np.int64)
    r = np.mod(num, den).astype(np.float64) / float(den)
    return np.sin(2.0 * np.pi * r)


def structured_mesh(cells, n_geo, node_map, periodic, wall_bc=BC_REFLECT, periods=None):
    """Hex mesh on a logical lattice.

    ``node_map(I1, I2, I3, M)`` receives integer lattice indices (broadcastable
    int64 arrays) with ``M = (n1*Ng, n2*Ng, n3*Ng)`` and returns the physical
    coordinates ``(..., 3)``.  Element e = i1 + n1*(i2 + n2*i3) takes the
    lattice block starting at (i1*Ng, i2*Ng, i3*Ng); shared faces are therefore
    bitwise identical.  ``periods[a]`` is the physical translation of a
    periodic axis a (3-vector).
    """
    n1, n2, n3 = cells
    ng = n_geo + 1
    M = (n1 * n_geo, n2 * n_geo, n3 * n_geo)
    I1 = np.arange(M[0] + 1, dtype=np.int64)[None, None, :]
    I2 = np.arange(M[1] + 1, dtype=np.int64)[None, :, None]
    I3 = np.arange(M[2] + 1, dtype=np.int64)[:, None, None]
    L = node_map(I1, I2, I3, M)            # [M3+1][M2+1][M1+1][3]
    loc = np.arange(ng, dtype=np.int64)
    e1 = np.arange(n1, dtype=np.int64)
    e2 = np.arange(n2, dtype=np.int64)
    e3 = np.arange(n3, dtype=np.int64)
    # (n3, n2, n1, k, j, i)
    A1 = (e1[None, None, :, None, None, None] * n_geo + loc[None, None, None, None, None, :])
    A2 = (e2[None, :, None, None, None, None] * n_geo + loc[None, None, None, None, :, None])
    A3 = (e3[:, None, None, None, None, None] * n_geo + loc[None, None, None, :, None, None])
    X = L[A3, A2, A1]                       # (n3, n2, n1, ng, ng, ng, 3)
    E = n1 * n2 * n3
    X = np.ascontiguousarray(X.reshape(E, ng ** 3, 3))

    idx = np.arange(E, dtype=np.int64)
    i1 = idx % n1
    i2 = (idx // n1) % n2
    i3 = idx // (n1 * n2)
    nbr_elem = np.full((E, 6), -1, dtype=np.int32)
    nbr_face = np.full((E, 6), -1, dtype=np.int32)
    bc = np.zeros((E, 6), dtype=np.int8)
    shift = np.zeros((E, 6, 3), dtype=np.float64)
    cnt = (n1, n2, n3)
    coords = [i1, i2, i3]
    strides = (1, n1, n1 * n2)
    for a in range(3):
        for side in (0, 1):
            f = 2 * a + side
            step = -1 if side == 0 else 1
            c = coords[a] + step
            inside = (c >= 0) & (c < cnt[a])
            nb = idx + step * strides[a]
            nbr_elem[inside, f] = nb[inside]
            nbr_face[inside, f] = 2 * a + (1 - side)
            bc[inside, f] = BC_INTERNAL
            out = ~inside
            if periodic[a]:
                wrapped = idx + (c % cnt[a] - coords[a]) * strides[a]
                nbr_elem[out, f] = wrapped[out]
                nbr_face[out, f] = 2 * a + (1 - side)
                bc[out, f] = BC_PERIODIC
                P = np.asarray(periods[a], dtype=np.float64)
                shift[out, f, :] = -P if side == 1 else P
            else:
                bc[out, f] = wall_bc
    return X, nbr_elem, nbr_face, bc, shift, L


# ----------------------------------------------------------------------------
# velocity fields
# ----------------------------------------------------------------------------
def cubic_field(rng):
    """Each component a cubic of total degree <= 3 in (x, y, z); 20 coefficients ~U(-1,1)."""
    exps = [(a, b, c) for a in range(4) for b in range(4) for c in range(4) if a + b + c <= 3]
    coef = rng.uniform(-1.0, 1.0, size=(3, len(exps)))

    def u(x):
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape[:-1] + (3,))
        for m, (a, b, c) in enumerate(exps):
            mono = x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c
            for comp in range(3):
                out[..., comp] += coef[comp, m] * mono
        return out
    return u


def fourier_field(rng, n_modes=16, kmax=4, urms=1.0):
    """Divergence-free random Fourier field with amplitude decay |k|^(-5/3)."""
    ks = np.array([(a, b, c) for a in range(-kmax, kmax + 1) for b in range(-kmax, kmax + 1)
                   for c in range(-kmax, kmax + 1) if max(abs(a), abs(b), abs(c)) >= 1], dtype=np.float64)
    pick = rng.choice(len(ks), size=n_modes, replace=False)
    k = ks[pick]
    rnd = rng.normal(size=(n_modes, 3))
    sig = np.cross(k, rnd)
    sig /= np.linalg.norm(sig, axis=1, keepdims=True)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    amp = np.linalg.norm(k, axis=1) ** (-5.0 / 3.0)
    U0 = urms / np.sqrt(0.5 * np.sum(amp ** 2))

    def u(x):
        x = np.asarray(x, dtype=np.float64)
        arg = 2.0 * np.pi * (x @ k.T) + phase             # (..., m)
        return U0 * (np.cos(arg) * amp) @ sig
    return u


def conservative(u, rho=RHO_F, p=P0, kappa=KAPPA):
    """(rho, rho u, rho e) from a velocity array (..., 3) at uniform rho and p."""
    rhoe = p / (kappa - 1.0) + 0.5 * rho * np.sum(u * u, axis=-1)
    out = np.empty(u.shape[:-1] + (5,))
    out[..., 0] = rho
    out[..., 1:4] = rho * u
    out[..., 4] = rhoe
    return out


def gauss_nodes(n_pts):
    """Legendre-Gauss nodes on [-1, 1] (numpy's routine; used only to place samples)."""
    x, _ = np.polynomial.legendre.leggauss(n_pts)
    return x


def _dg_state(cells, N, logical_to_phys, field):
    """Sample the analytic field at the analytic image of each element's Gauss nodes."""
    n1, n2, n3 = cells
    n = N + 1
    g = gauss_nodes(n)
    E = n1 * n2 * n3
    idx = np.arange(E)
    c = np.stack([idx % n1, (idx // n1) % n2, idx // (n1 * n2)], axis=1).astype(np.float64)
    ii, jj, kk = np.meshgrid(g, g, g, indexing="ij")  # ii along xi1
    # node order i + n(j + n k): build (k, j, i)
    loc = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                    kk.transpose(2, 1, 0).ravel()], axis=1)          # (n^3, 3)
    cnt = np.array([n1, n2, n3], dtype=np.float64)
    U = np.empty((E, 5, n ** 3))
    chunk = max(1, 500_000 // (n ** 3))
    report = max(chunk, (E // 10) // chunk * chunk)

    def fill(s):
        if s % report == 0:
            _progress("fluid state", s, E)
        cs = c[s:s + chunk]
        sl = (cs[:, None, :] + 0.5 * (loc[None, :, :] + 1.0)) / cnt   # logical coords
        xp = logical_to_phys(sl)
        cv = conservative(field(xp))                                     # (e, n^3, 5)
        U[s:s + chunk] = cv.transpose(0, 2, 1)
    _chunked(fill, range(0, E, chunk))
    return U


def _chunked(fn, starts):
    """Run fn over independent chunks on a thread pool (numpy releases the GIL
    in its array operations; every chunk writes its own slice)."""
    import concurrent.futures as cf
    import os
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fn, starts))


def _particles(rng, cells, n_particles, logical_to_phys, field):
    n1, n2, n3 = cells
    E = n1 * n2 * n3
    e = rng.integers(0, E, size=n_particles)
    xi = rng.uniform(-1.0, 1.0, size=(n_particles, 3))
    d = rng.lognormal(mean=-9.2, sigma=0.3, size=n_particles)
    c = np.stack([e % n1, (e // n1) % n2, e // (n1 * n2)], axis=1).astype(np.float64)
    sl = (c + 0.5 * (xi + 1.0)) / np.array([n1, n2, n3], dtype=np.float64)
    x = np.empty_like(sl)
    v = np.empty_like(sl)
    chunk = 500_000

    def fill(s):
        x[s:s + chunk] = logical_to_phys(sl[s:s + chunk])
        v[s:s + chunk] = field(x[s:s + chunk])
    _chunked(fill, range(0, n_particles, chunk))
    return x, v, d, e.astype(np.int32)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def config1(n_particles=10_000, cells=8, n_steps=100, seed=1001):
    """Unit cube, cells^3 straight hexes, Ng=1, all faces periodic, N=3 cubic field, Stokes, 5-stage RK."""
    rng = np.random.default_rng(seed)
    n_geo = 1

    def node_map(I1, I2, I3, M):
        out = np.empty(np.broadcast_shapes(I1.shape, I2.shape, I3.shape) + (3,))
        out[..., 0] = I1 / M[0]
        out[..., 1] = I2 / M[1]
        out[..., 2] = I3 / M[2]
        return out
    cc = (cells, cells, cells)
    X, ne, nf, bc, sh, _ = structured_mesh(cc, n_geo, node_map, (True, True, True),
                                           periods=np.eye(3))
    mesh = Mesh(n_geo, X, ne, nf, bc, sh, h=1.0 / cells, cells=cc)
    field = cubic_field(rng)
    U = _dg_state(cc, 3, lambda s: s, field)
    x, v, d, e = _particles(rng, cc, n_particles, lambda s: s, field)
    return Workload("config1_cube%d_N3_Ng1_periodic" % cells, mesh, 3, U, x, v, d, e,
                    dt=1e-3, n_steps=n_steps, rk=0, drag=0, velocity=field)


def sine_map_logical(s, amp=0.05):
    """Phi(s) = s + amp*(sin2pi s2 sin2pi s3, sin2pi s3 sin2pi s1, sin2pi s1 sin2pi s2)."""
    S = np.sin(2.0 * np.pi * s)
    out = s.copy()
    out[..., 0] += amp * S[..., 1] * S[..., 2]
    out[..., 1] += amp * S[..., 2] * S[..., 0]
    out[..., 2] += amp * S[..., 0] * S[..., 1]
    return out


def sine_mesh(cells, n_geo=4, amp=0.05, wall_bc=BC_REFLECT):
    def node_map(I1, I2, I3, M):
        shp = np.broadcast_shapes(I1.shape, I2.shape, I3.shape)
        s1 = np.broadcast_to(I1 / M[0], shp)
        s2 = np.broadcast_to(I2 / M[1], shp)
        s3 = np.broadcast_to(I3 / M[2], shp)
        S1 = np.broadcast_to(sin2pi(I1, M[0]), shp)
        S2 = np.broadcast_to(sin2pi(I2, M[1]), shp)
        S3 = np.broadcast_to(sin2pi(I3, M[2]), shp)
        out = np.empty(shp + (3,))
        out[..., 0] = s1 + amp * (S2 * S3)
        out[..., 1] = s2 + amp * (S3 * S1)
        out[..., 2] = s3 + amp * (S1 * S2)
        return out
    cc = (cells, cells, cells)
    X, ne, nf, bc, sh, _ = structured_mesh(cc, n_geo, node_map, (True, False, True),
                                           periods=np.eye(3), wall_bc=wall_bc)
    return Mesh(n_geo, X, ne, nf, bc, sh, h=1.0 / cells, cells=cc)


def curved_box(cells=32, N=5, n_particles=1_000_000, n_steps=500, seed=1002, name="config2",
               n_geo=4, wall_bc=BC_REFLECT):
    """Sine-mapped periodic (x, z) box with curved walls (reflective, or open
    with wall_bc=BC_OPEN) at logical y=0/1."""
    rng = np.random.default_rng(seed)
    mesh = sine_mesh(cells, n_geo, wall_bc=wall_bc)
    cc = mesh.cells
    field = fourier_field(rng)
    U = _dg_state(cc, N, sine_map_logical, field)
    x, v, d, e = _particles(rng, cc, n_particles, sine_map_logical, field)
    return Workload("%s_sine%d_N%d_Ng%d" % (name, cells, N, n_geo), mesh, N, U, x, v, d, e,
                    dt=1e-3, n_steps=n_steps, rk=1, drag=1, velocity=field)


def peaked_box(displace=0.08, cells=3, N=3, n_geo=4):
    """The sine box of curved_box with the centre geometry node of the central
    element moved by -displace * h along x: the element stays valid (det J > 0)
    but its map is compressed at the centre of its face xi_1 = +1, where
    |grad xi_1| peaks far above its value at any point of a lattice that skips
    xi = 0 (the face stays shared with the neighbour, which is untouched).
    Returns the workload (no particles) and the element index."""
    assert cells % 2 == 1 and n_geo % 2 == 0
    mesh = sine_mesh(cells, n_geo)
    c = cells // 2
    e = c + cells * (c + cells * c)
    ng = n_geo + 1
    m = n_geo // 2
    X = mesh.X.copy()
    X[e, (m * ng + m) * ng + m, 0] -= displace * mesh.h
    mesh = Mesh(mesh.n_geo, X, mesh.nbr_elem, mesh.nbr_face, mesh.bc, mesh.shift, mesh.h, mesh.cells)
    U = uniform_state(mesh.n_elem, N, (0.0, 0.0, 0.0))
    z = np.zeros((0, 3))
    return Workload("peaked_box%d_N%d_Ng%d" % (cells, N, n_geo), mesh, N, U, z, z, np.zeros(0),
                    np.zeros(0, np.int32), dt=1e-3, n_steps=1, rk=1, drag=2, velocity=None), e


def config2(n_particles=1_000_000, cells=32, n_steps=500):
    return curved_box(cells, 5, n_particles, n_steps, seed=1002, name="config2")


def config3(n_particles=10_000_000, cells=64, n_steps=200):
    return curved_box(cells, 7, n_particles, n_steps, seed=1003, name="config3")


def config5(n_particles=20_000_000, cells=96, n_steps=100):
    return curved_box(cells, 5, n_particles, n_steps, seed=1005, name="config5")


# annular sector passage -----------------------------------------------------
ANN_RH, ANN_RT, ANN_THETA, ANN_L = 1.0, 1.25, 2.0 * np.pi / 30.0, 0.5


def annulus_logical(sl):
    """Element logical coordinates (s, eta, q) -> physical (x, y, z)."""
    s, eta, q = sl[..., 0], sl[..., 1], sl[..., 2]
    r = ANN_RH + (ANN_RT - ANN_RH) * (eta + 0.04 * np.sin(np.pi * eta) * np.sin(24 * np.pi * s)
                                      * np.sin(24 * np.pi * q))
    th = ANN_THETA * (q - 0.5 + 0.02 * np.sin(24 * np.pi * s) * np.sin(np.pi * eta)) \
        + 0.15 * np.sin(2 * np.pi * s)
    out = np.empty(sl.shape)
    out[..., 0] = r * np.cos(th)
    out[..., 1] = r * np.sin(th)
    out[..., 2] = ANN_L * s
    return out


def annulus_mesh(cells=(48, 24, 48), n_geo=6):
    """Axial (xi1 = s) periodic, span (xi2 = eta) and pitch (xi3 = q) walls reflective."""
    def node_map(I1, I2, I3, M):
        shp = np.broadcast_shapes(I1.shape, I2.shape, I3.shape)
        s = np.broadcast_to(I1 / M[0], shp)
        eta = np.broadcast_to(I2 / M[1], shp)
        q = np.broadcast_to(I3 / M[2], shp)
        s24 = np.broadcast_to(sin2pi(12 * I1, M[0]), shp)      # sin(24 pi s)
        s2 = np.broadcast_to(sin2pi(I1, M[0]), shp)            # sin(2 pi s)
        q24 = np.broadcast_to(sin2pi(12 * I3, M[2]), shp)      # sin(24 pi q)
        pe = np.broadcast_to(sin2pi(I2, 2 * M[1]), shp)        # sin(pi eta)
        r = ANN_RH + (ANN_RT - ANN_RH) * (eta + 0.04 * pe * s24 * q24)
        th = ANN_THETA * (q - 0.5 + 0.02 * s24 * pe) + 0.15 * s2
        out = np.empty(shp + (3,))
        out[..., 0] = r * np.cos(th)
        out[..., 1] = r * np.sin(th)
        out[..., 2] = ANN_L * s
        return out
    periods = np.array([[0.0, 0.0, ANN_L], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    X, ne, nf, bc, sh, _ = structured_mesh(cells, n_geo, node_map, (True, False, False),
                                           periods=periods)
    h = ANN_L / cells[0]
    return Mesh(n_geo, X, ne, nf, bc, sh, h=h, cells=tuple(cells))


def config4(n_particles=10_000_000, cells=(48, 24, 48), n_steps=100, seed=1004):
    rng = np.random.default_rng(seed)
    mesh = annulus_mesh(cells, 6)
    field = fourier_field(rng)
    U = _dg_state(mesh.cells, 5, annulus_logical, field)
    x, v, d, e = _particles(rng, mesh.cells, n_particles, annulus_logical, field)
    return Workload("config4_annulus%dx%dx%d_N5_Ng6" % tuple(cells), mesh, 5, U, x, v, d, e,
                    dt=1e-3, n_steps=n_steps, rk=1, drag=1, velocity=field)


# ----------------------------------------------------------------------------
# non-conforming mesh (mortar faces)
# ----------------------------------------------------------------------------
def _mortar_map(n_geo, amp):
    if n_geo == 1:
        # trilinear: twisted (bilinear) faces
        def phi(s):
            x, y, z = s[..., 0], s[..., 1], s[..., 2]
            return np.stack([x + amp * y * z, y + amp * x * z, z + amp * x * y], axis=-1)
    else:
        # quadratic: curved faces, reproduced exactly by any geometry degree >= 2
        def phi(s):
            x, y, z = s[..., 0], s[..., 1], s[..., 2]
            return np.stack([x + amp * ((y - 0.5) ** 2 + z * (1.0 - z)), y + amp * x * (2.0 - x) * 0.5,
                             z + amp * x * y], axis=-1)
    return phi


def mortar_box(n_geo=4, N=3, refine=(2, 2), n_particles=2000, seed=51, amp=0.05, vscale=1.0, cells=(2, 2, 2)):
    """Box [0,2]x[0,1]x[0,1] (logical) with walls all round: a coarse block
    (x < 1) of cx x cy x cz elements and a fine block (x > 1) of
    cx x (ry cy) x (rz cz) elements.  Each coarse face on x = 1 is a big mortar
    face matched by ry*rz small faces (refine (2, 2): 4:1, (2, 1): 2:1), listed
    z-major.  Elements: coarse i + cx (j + cy k), then fine.  The map is
    trilinear (n_geo = 1) or quadratic (n_geo >= 2), so every element
    represents it exactly and the small faces tile the big ones exactly."""
    rng = np.random.default_rng(seed)
    ry, rz = refine
    cx, cy, cz = cells
    fx, fy, fz = cx, ry * cy, rz * cz
    nc, nf_ = cx * cy * cz, fx * fy * fz
    E = nc + nf_

    def block(n1, n2, n3, x0, dx):
        idx = np.arange(n1 * n2 * n3)
        i, j, k = idx % n1, (idx // n1) % n2, idx // (n1 * n2)
        lo = np.stack([x0 + i * dx[0], j * dx[1], k * dx[2]], axis=1)
        return lo, lo + np.asarray(dx), (i, j, k)

    loc, hic, (ic, jc, kc) = block(cx, cy, cz, 0.0, (1.0 / cx, 1.0 / cy, 1.0 / cz))
    lof, hif, (i_f, j_f, k_f) = block(fx, fy, fz, 1.0, (1.0 / fx, 1.0 / fy, 1.0 / fz))
    lo = np.concatenate([loc, lof])
    hi = np.concatenate([hic, hif])
    phi = _mortar_map(n_geo, amp)
    ng = n_geo + 1
    r = np.linspace(-1.0, 1.0, ng)
    kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
    xi = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    X = np.ascontiguousarray(phi(lo[:, None, :] + 0.5 * (xi[None] + 1.0) * (hi - lo)[:, None, :]))
    nbr_elem = np.full((E, 6), -1, np.int32)
    nbr_face = np.full((E, 6), -1, np.int32)
    bc = np.full((E, 6), BC_REFLECT, np.int8)
    shift = np.zeros((E, 6, 3))
    # structured neighbours inside each block
    for off, (n1, n2, n3), (i, j, k) in ((0, (cx, cy, cz), (ic, jc, kc)), (nc, (fx, fy, fz), (i_f, j_f, k_f))):
        idx = np.arange(n1 * n2 * n3)
        cnt, coords, strides = (n1, n2, n3), (i, j, k), (1, n1, n1 * n2)
        for a in range(3):
            for side in (0, 1):
                f = 2 * a + side
                step = -1 if side == 0 else 1
                inside = (coords[a] + step >= 0) & (coords[a] + step < cnt[a])
                nbr_elem[off + idx[inside], f] = off + idx[inside] + step * strides[a]
                nbr_face[off + idx[inside], f] = 2 * a + (1 - side)
                bc[off + idx[inside], f] = BC_INTERNAL
    # the interface x = 1: coarse +x faces are big mortar faces
    big = np.nonzero(ic == cx - 1)[0]
    mortar = np.full((len(big), 4, 2), -1, np.int32)
    for m, e in enumerate(big):
        q = 0
        for dz in range(rz):
            for dy in range(ry):
                s = nc + 0 + fx * ((ry * jc[e] + dy) + fy * (rz * kc[e] + dz))
                mortar[m, q] = (s, 0)
                nbr_elem[s, 0], nbr_face[s, 0], bc[s, 0] = e, 1, BC_INTERNAL
                q += 1
        nbr_elem[e, 1], nbr_face[e, 1], bc[e, 1] = m, -1, BC_MORTAR
    mesh = Mesh(n_geo, X, nbr_elem, nbr_face, bc, shift, h=1.0 / (2 * max(cx, cy, cz)), mortar=mortar)
    field = fourier_field(rng)
    n = N + 1
    g = gauss_nodes(n)
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    xq = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    U = np.empty((E, 5, n ** 3))
    for s0 in range(0, E, 4096):
        sl = slice(s0, min(E, s0 + 4096))
        xd = phi(lo[sl, None, :] + 0.5 * (xq[None] + 1.0) * (hi - lo)[sl, None, :])
        U[sl] = conservative(field(xd.reshape(-1, 3)) * vscale).reshape(-1, n ** 3, 5).transpose(0, 2, 1)
    e = rng.integers(0, E, size=n_particles)
    xs = rng.uniform(-1.0, 1.0, size=(n_particles, 3))
    d = rng.lognormal(mean=-9.2, sigma=0.3, size=n_particles)
    x = phi(lo[e] + 0.5 * (xs + 1.0) * (hi - lo)[e])
    v = field(x) * vscale
    return Workload("mortar_box_ng%d_N%d_%dx%d_%dx%dx%d" % (n_geo, N, ry, rz, cx, cy, cz), mesh, N, U, x, v, d,
                    e.astype(np.int32), dt=1e-3, n_steps=1, rk=1, drag=1, velocity=field)


# ----------------------------------------------------------------------------
# tiny meshes for component tests
# ----------------------------------------------------------------------------
def single_element(n_geo, node_fn):
    """One element whose equidistant geometry nodes are node_fn(xi (..., 3)) -> (..., 3); all faces open."""
    ng = n_geo + 1
    r = np.linspace(-1.0, 1.0, ng)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    xi = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    X = np.ascontiguousarray(node_fn(xi)[None, :, :])
    ne = np.full((1, 6), -1, np.int32)
    nf = np.full((1, 6), -1, np.int32)
    bc = np.full((1, 6), BC_OPEN, np.int8)
    sh = np.zeros((1, 6, 3))
    return Mesh(n_geo, X, ne, nf, bc, sh, h=2.0)


def uniform_state(E, N, u, rho=RHO_F, p=P0):
    n3 = (N + 1) ** 3
    cv = conservative(np.asarray(u, dtype=np.float64)[None, :], rho, p)[0]
    U = np.empty((E, 5, n3))
    U[:, :, :] = cv[None, :, None]
    return U


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
