"""FP64 CPU oracle (ctypes binding over liboracle.so, built from oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports or links
it, and it shares no code with the product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

ACTIVE, OPEN_EXIT, LOST_NEWTON, LOST_TRACK, MAX_CROSS, REJECTED = range(6)
FACE_PLANAR, FACE_BILINEAR, FACE_CURVED = range(3)
MLP_NIN, MLP_H, MLP_NOUT = 84, 64, 3


def build(force=True):
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]
    subprocess.check_call(cmd)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


P = C.c_void_p
I = C.c_int
I64 = C.c_int64
D = C.c_double


def _declare(L):
    L.or_create.restype = P
    L.or_create.argtypes = [I, I, P, P, P, P, P, I, I]
    L.or_destroy.argtypes = [P]
    L.or_num_threads.restype = I
    L.or_set_num_threads.argtypes = [I]
    L.or_set_fluid.argtypes = [P, P, D, D, D]
    L.or_gauss_nodes.argtypes = [I, P, P]
    L.or_lobatto_nodes.argtypes = [I, P, P]
    L.or_lagrange.argtypes = [I, P, D, P, P]
    L.or_rk_coeffs.argtypes = [I, P, P, P, P]
    L.or_map.argtypes = [P, I, P, P, P]
    L.or_newton.restype = I
    L.or_newton.argtypes = [P, I, P, P, P, P]
    L.or_guess.argtypes = [P, I, P, P]
    L.or_guess_faces.argtypes = [P, I, P, P]
    L.or_interp.argtypes = [P, I, P, P]
    L.or_drag_accel.argtypes = [P, I, P, P, D, P, P, P]
    L.or_face_info.restype = I
    L.or_face_info.argtypes = [P, I, I, P, P]
    L.or_face_intersect.restype = I
    L.or_face_intersect.argtypes = [P, I, I, P, P, P, P, I]
    L.or_bezier_intersect.restype = I
    L.or_bezier_intersect.argtypes = [I, P, P, P, P, P, I]
    L.or_volume.restype = D
    L.or_volume.argtypes = [P, I, I]
    L.or_dg_node_pos.argtypes = [P, I, I, P]
    L.or_locate.restype = I
    L.or_locate.argtypes = [P, P, I, P]
    L.or_boundary_distance.restype = C.c_double
    L.or_boundary_distance.argtypes = [P, I]
    L.or_push.restype = I
    L.or_push.argtypes = [P, I64, P, P, P, P, P]
    L.or_default_opts.argtypes = [P]
    L.or_step.restype = I
    L.or_step.argtypes = [P, D, I, P]
    L.or_read.argtypes = [P, P, P, P, P, P, P]
    L.or_stats.argtypes = [P, P]
    L.or_reset_stats.argtypes = [P]
    L.or_deposit.restype = I
    L.or_deposit.argtypes = [P, P, I, D, P, I, I, P]
    L.or_fluid_grad.argtypes = [P, I, P, P, P]
    L.or_set_mortar.argtypes = [P, I, P]
    L.or_set_mortar.restype = I
    L.or_particle_accel.argtypes = [P, I, I, P, P, P, D, P, P, P]
    L.or_mlp_n_weights.restype = I64
    L.or_mlp_features.argtypes = [P, I, P, P]
    L.or_mlp_forward.argtypes = [P, I64, P, P]
    L.or_mlp_loss_grad.restype = D
    L.or_mlp_loss_grad.argtypes = [P, I64, P, P, P]
    L.or_adam.argtypes = [P, P, P, P, I64, I64, D, D, D, D]
    L.or_mlp_train.restype = D
    L.or_mlp_train.argtypes = [P, P, P, P, P, P, P, I64, I, D, P]
    L.or_set_mlp.argtypes = [P, P, P]
    L.or_curved_flags.argtypes = [P, D, P]
    L.or_mlp_draws.argtypes = [C.c_uint64, I64, I, P, P]


class StepOpts(C.Structure):
    _fields_ = [("rk", C.c_int32), ("drag", C.c_int32), ("max_newton_it", C.c_int32),
                ("max_crossings", C.c_int32), ("use_mlp", C.c_int32), ("tracking", C.c_int32),
                ("gravity", C.c_double * 3), ("drag_mask", C.c_double * 3), ("forces", C.c_int32)]


# extra terms of the equation of motion (bit flags of StepOpts.forces)
F_BUOYANCY, F_STRESS, F_ADDED_MASS, F_SAFFMAN = 1, 2, 4, 8


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# stateless helpers
# ---------------------------------------------------------------------------
def gauss_nodes(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().or_gauss_nodes(n, _p(x), _p(w))
    return x, w


def lobatto_nodes(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().or_lobatto_nodes(n, _p(x), _p(w))
    return x, w


def lagrange(nodes, xi):
    nodes = _f64(nodes)
    n = len(nodes)
    l = np.zeros(n); dl = np.zeros(n)
    lib().or_lagrange(n, _p(nodes), float(xi), _p(l), _p(dl))
    return l, dl


def rk_coeffs(scheme):
    s = C.c_int(0)
    A = np.zeros(5); B = np.zeros(5); c = np.zeros(5)
    lib().or_rk_coeffs(scheme, C.byref(s), _p(A), _p(B), _p(c))
    return A[:s.value].copy(), B[:s.value].copy(), c[:s.value].copy()


def bezier_intersect(cp, x0, t, max_roots=16):
    cp = _f64(cp)
    ng = int(round(np.sqrt(cp.size // 3)))
    al = np.zeros(max_roots); uv = np.zeros(2 * max_roots)
    n = lib().or_bezier_intersect(ng, _p(cp), _p(_f64(x0)), _p(_f64(t)), _p(al), _p(uv), max_roots)
    return al[:n].copy(), uv[:2 * n].reshape(n, 2).copy()


def mlp_n_weights():
    return int(lib().or_mlp_n_weights())


def mlp_forward(w, inp):
    w = _f64(w); inp = _f64(inp)
    out = np.zeros((inp.shape[0], MLP_NOUT))
    lib().or_mlp_forward(_p(w), inp.shape[0], _p(inp), _p(out))
    return out


def mlp_loss_grad(w, inp, target):
    w = _f64(w); inp = _f64(inp); target = _f64(target)
    g = np.zeros(mlp_n_weights())
    loss = lib().or_mlp_loss_grad(_p(w), inp.shape[0], _p(inp), _p(target), _p(g))
    return loss, g


def adam(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    lib().or_adam(_p(w), _p(m), _p(v), _p(_f64(g)), w.size, int(t), lr, b1, b2, eps)


def mlp_train_epoch(w, m, v, t, inp, target, order, batch, lr):
    """One epoch of minibatch Adam; w, m, v updated in place; returns (mean loss, t, losses)."""
    tt = C.c_int64(int(t))
    order = np.ascontiguousarray(order, dtype=np.int32)
    nb = len(order) // batch
    hist = np.zeros(max(nb, 1))
    mean = lib().or_mlp_train(_p(w), _p(m), _p(v), C.byref(tt), _p(_f64(inp)), _p(_f64(target)),
                              _p(order), len(order), batch, lr, _p(hist))
    return mean, tt.value, hist[:nb]


def mlp_draws(seed, n, epochs):
    """Initial weights and per-epoch row orders of a seeded training run."""
    w0 = np.zeros(mlp_n_weights())
    orders = np.zeros((max(epochs, 1), n), np.int32)
    lib().or_mlp_draws(int(seed), int(n), int(epochs), _p(w0), _p(orders))
    return w0, orders[:epochs]


def num_threads():
    return int(lib().or_num_threads())


def set_num_threads(n):
    lib().or_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# stateful oracle
# ---------------------------------------------------------------------------
class Oracle:
    def __init__(self, mesh, N, U=None, mu=1.8e-5, kappa=1.4, rho_p=2500.0, dg_nodes=0):
        L = lib()
        self._keep = [_f64(mesh.X), np.ascontiguousarray(mesh.nbr_elem, np.int32),
                      np.ascontiguousarray(mesh.nbr_face, np.int32),
                      np.ascontiguousarray(mesh.bc, np.int8), _f64(mesh.shift)]
        self.E = mesh.n_elem
        self.n_geo = mesh.n_geo
        self.N = N
        self.ctx = L.or_create(self.E, mesh.n_geo, *[_p(a) for a in self._keep], N, dg_nodes)
        if not self.ctx:
            raise ValueError("oracle: invalid mesh")
        mortar = getattr(mesh, "mortar", None)
        if mortar is not None and len(mortar):
            tab = np.ascontiguousarray(mortar, np.int32)
            self._keep.append(tab)
            if L.or_set_mortar(self.ctx, int(tab.shape[0]), _p(tab)) != 0:
                raise ValueError("oracle: inconsistent mortar table")
        self.U = None
        if U is not None:
            self.set_fluid(U, mu, kappa, rho_p)
        self.np = 0

    def close(self):
        if self.ctx:
            lib().or_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fluid(self, U, mu=1.8e-5, kappa=1.4, rho_p=2500.0):
        self.U = _f64(U)
        lib().or_set_fluid(self.ctx, _p(self.U), mu, kappa, rho_p)

    # components
    def map(self, e, xi):
        x = np.zeros(3); J = np.zeros(9)
        lib().or_map(self.ctx, int(e), _p(_f64(xi)), _p(x), _p(J))
        return x, J.reshape(3, 3)

    def newton(self, e, x, xi0):
        xi = np.zeros(3); it = C.c_int(0)
        ok = lib().or_newton(self.ctx, int(e), _p(_f64(x)), _p(_f64(xi0)), _p(xi), C.byref(it))
        return bool(ok), xi, it.value

    def guess(self, e, x):
        g = np.zeros(3)
        lib().or_guess(self.ctx, int(e), _p(_f64(x)), _p(g))
        return g

    def guess_faces(self, e, x):
        g = np.zeros(3)
        lib().or_guess_faces(self.ctx, int(e), _p(_f64(x)), _p(g))
        return g

    def interp(self, e, xi):
        out = np.zeros(5)
        lib().or_interp(self.ctx, int(e), _p(_f64(xi)), _p(out))
        return out

    def drag_accel(self, drag, prim, v, d, g=None):
        a = np.zeros(3); fD = np.zeros(1)
        lib().or_drag_accel(self.ctx, drag, _p(_f64(prim)), _p(_f64(v)), float(d),
                            _p(_f64(g)) if g is not None else None, _p(a), _p(fD))
        return a, fD[0]

    def fluid_grad(self, e, xi):
        """Primitive state (5) and velocity gradient G[i][j] = du_i/dx_j at xi."""
        prim = np.zeros(5); G = np.zeros(9)
        lib().or_fluid_grad(self.ctx, int(e), _p(_f64(xi)), _p(prim), _p(G))
        return prim, G.reshape(3, 3)

    def particle_accel(self, drag, forces, prim, G, v, d, g=None):
        """dv/dt and the fluid force of the two-way source (equation of motion)."""
        a = np.zeros(3); F = np.zeros(3)
        lib().or_particle_accel(self.ctx, int(drag), int(forces), _p(_f64(prim)), _p(_f64(G).ravel()),
                                _p(_f64(v)), float(d), _p(_f64(g)) if g is not None else None, _p(a), _p(F))
        return a, F

    def face(self, e, f):
        ng = self.n_geo + 1
        cp = np.zeros(ng * ng * 3); t = C.c_int(0)
        lib().or_face_info(self.ctx, int(e), int(f), _p(cp), C.byref(t))
        return cp.reshape(ng * ng, 3), t.value

    def face_intersect(self, e, f, x0, t, max_roots=16):
        al = np.zeros(max_roots); uv = np.zeros(2 * max_roots)
        n = lib().or_face_intersect(self.ctx, int(e), int(f), _p(_f64(x0)), _p(_f64(t)), _p(al),
                                    _p(uv), max_roots)
        return al[:n].copy(), uv[:2 * n].reshape(n, 2).copy()

    def volume(self, e, node):
        return lib().or_volume(self.ctx, int(e), int(node))

    def dg_node_pos(self, e, node):
        x = np.zeros(3)
        lib().or_dg_node_pos(self.ctx, int(e), int(node), _p(x))
        return x

    def boundary_distance(self, e):
        return lib().or_boundary_distance(self.ctx, int(e))

    def locate(self, x, hint=-1):
        xi = np.zeros(3)
        e = lib().or_locate(self.ctx, _p(_f64(x)), int(hint), _p(xi))
        return e, xi

    # particles
    def push(self, x, v, d, elem_hint=None):
        x = _f64(x); v = _f64(v); d = _f64(d)
        n = x.shape[0]
        st = np.zeros(n, np.int32)
        h = np.ascontiguousarray(elem_hint, np.int32) if elem_hint is not None else None
        nbad = lib().or_push(self.ctx, n, _p(x), _p(v), _p(d), _p(h), _p(st))
        self.np = n
        return st, nbad

    def step(self, dt, n_steps=1, rk=0, drag=1, max_newton_it=50, max_crossings=64,
             gravity=(0, 0, 0), drag_mask=(1, 1, 1), use_mlp=False, tracking=0, forces=0):
        o = StepOpts()
        o.forces = int(forces)
        o.rk = rk; o.drag = drag; o.max_newton_it = max_newton_it; o.max_crossings = max_crossings
        o.use_mlp = int(bool(use_mlp))
        o.tracking = int(tracking)
        for k in range(3):
            o.gravity[k] = gravity[k]
            o.drag_mask[k] = drag_mask[k]
        return lib().or_step(self.ctx, float(dt), int(n_steps), C.byref(o))

    def read(self):
        n = self.np
        out = dict(x=np.zeros((n, 3)), v=np.zeros((n, 3)), elem=np.zeros(n, np.int32),
                   xi=np.zeros((n, 3)), hits=np.zeros(n, np.int32), status=np.zeros(n, np.int8))
        lib().or_read(self.ctx, _p(out["x"]), _p(out["v"]), _p(out["elem"]), _p(out["xi"]),
                      _p(out["hits"]), _p(out["status"]))
        return out

    def stats(self):
        s = np.zeros(7, np.int64)
        lib().or_stats(self.ctx, _p(s))
        return dict(newton_iters=int(s[0]), newton_calls=int(s[1]), crossings=int(s[2]),
                    wall_hits=int(s[3]), lost=int(s[4]), fallbacks=int(s[5]), recovered=int(s[6]))

    def reset_stats(self):
        lib().or_reset_stats(self.ctx)

    def deposit(self, kind=0, radius=0.0, period=None, drag=1, S=None, forces=0, gravity=None):
        n3 = (self.N + 1) ** 3
        if S is None:
            S = np.zeros((self.E, 4, n3))
        per = _f64(period) if period is not None else None
        g = _f64(gravity) if gravity is not None else None
        lib().or_deposit(self.ctx, _p(S), int(kind), float(radius), _p(per), int(drag), int(forces), _p(g))
        return S

    # learned guess
    def mlp_features(self, e, x):
        f = np.zeros(MLP_NIN)
        lib().or_mlp_features(self.ctx, int(e), _p(_f64(x)), _p(f))
        return f

    def curved_flags(self, thresh=0.05):
        fl = np.zeros(self.E, np.uint8)
        lib().or_curved_flags(self.ctx, float(thresh), _p(fl))
        return fl

    def set_mlp(self, w, flags):
        if w is None:
            lib().or_set_mlp(self.ctx, None, None)
            return
        self._mlp_keep = (_f64(w), np.ascontiguousarray(flags, np.uint8))
        lib().or_set_mlp(self.ctx, _p(self._mlp_keep[0]), _p(self._mlp_keep[1]))
