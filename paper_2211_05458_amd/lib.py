"""Python binding of libflexipart.so (argument marshalling only).

Every step of the particle method runs in the HIP kernels of the library;
PyTorch provides device memory (workspace, fluid state, sources, MLP tensors)
and the stream.  There is no CPU fallback: if the library is missing the
binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflexipart.so")

FP_OK, FP_EINVAL, FP_EMESH, FP_EDEVICE, FP_ESTATE, FP_WDT = 0, -1, -2, -3, -4, 1
ACTIVE, OPEN_EXIT, LOST_NEWTON, LOST_TRACK, MAX_CROSS, REJECTED = range(6)
F32, F64 = 0, 1

EXPORTS = ["fp_create", "fp_destroy", "fp_last_error", "fp_init_mesh", "fp_workspace_size",
           "fp_bind_workspace", "fp_set_fluid_state", "fp_push_particles", "fp_step",
           "fp_deposit_source", "fp_read_particles", "fp_get_stats", "fp_reset_stats",
           "fp_mlp_n_weights", "fp_mlp_features", "fp_newton_pairs", "fp_mlp_forward",
           "fp_mlp_loss_grad", "fp_mlp_train_epoch", "fp_mlp_set_weights", "fp_mlp_num_flagged",
           "fp_set_timing", "fp_get_timing", "fp_node_volumes", "fp_bind_particles",
           "fp_particle_block_layout", "fp_mlp_train", "fp_mlp_loss_grad_static", "fp_bind_deposit_list",
           "fp_deposit_list_bytes"]
TIMING_CLASSES = ("sort", "stage_elem", "finalize", "deposit_nearest", "deposit_shape", "stage_lane", "track",
                  "deposit_norm", "deposit_gather", "learned_guess")


class FPError(RuntimeError):
    pass


class MeshDesc(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("n_geo", C.c_int32), ("X", C.c_void_p),
                ("nbr_elem", C.c_void_p), ("nbr_face", C.c_void_p), ("bc", C.c_void_p),
                ("periodic_shift", C.c_void_p), ("n_dg", C.c_int32), ("dg_nodes", C.c_int32),
                ("n_mortar", C.c_int32), ("mortar", C.c_void_p)]


class FluidParams(C.Structure):
    _fields_ = [("mu", C.c_double), ("kappa", C.c_double), ("rho_p", C.c_double)]


class StepOpts(C.Structure):
    _fields_ = [("rk", C.c_int32), ("drag", C.c_int32), ("precision", C.c_int32), ("guess", C.c_int32),
                ("sort_every", C.c_int32), ("max_newton_it", C.c_int32), ("max_crossings", C.c_int32),
                ("tracking", C.c_int32), ("forces", C.c_int32), ("gravity", C.c_double * 3)]


# extra terms of the equation of motion (fp_step_opts.forces bits)
F_BUOYANCY, F_STRESS, F_ADDED_MASS, F_SAFFMAN = 1, 2, 4, 8


_lib = None


def load():
    """Load the built library (never builds; call paper_2211_05458_amd.build.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FPError("libflexipart.so is not built (run: python -m paper_2211_05458_amd.build)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.fp_create.argtypes = [C.POINTER(P), P]
    L.fp_destroy.argtypes = [P]
    L.fp_destroy.restype = None
    L.fp_last_error.argtypes = [P]
    L.fp_last_error.restype = C.c_char_p
    L.fp_init_mesh.argtypes = [P, C.POINTER(MeshDesc)]
    L.fp_workspace_size.argtypes = [P, I64, C.POINTER(C.c_size_t)]
    L.fp_bind_workspace.argtypes = [P, P, C.c_size_t]
    L.fp_set_fluid_state.argtypes = [P, P, C.c_int, C.POINTER(FluidParams)]
    L.fp_push_particles.argtypes = [P, I64, P, P, P, P, P]
    L.fp_step.argtypes = [P, D, I32, C.POINTER(StepOpts)]
    L.fp_deposit_source.argtypes = [P, P, C.c_int, I32, D, P, I32, I32, P]
    L.fp_read_particles.argtypes = [P, C.POINTER(I64), P, P, P, P, P, P]
    L.fp_get_stats.argtypes = [P, P]
    L.fp_reset_stats.argtypes = [P]
    L.fp_mlp_n_weights.argtypes = []
    L.fp_mlp_n_weights.restype = I64
    L.fp_mlp_features.argtypes = [P, I64, P, P, P]
    L.fp_newton_pairs.argtypes = [P, C.POINTER(I64), P, P, P, I64]
    L.fp_mlp_forward.argtypes = [P, P, I64, P, P]
    L.fp_mlp_loss_grad.argtypes = [P, P, I64, P, P, P, P]
    L.fp_mlp_train_epoch.argtypes = [P, P, P, P, C.POINTER(I64), P, P, P, I64, I32, C.c_float, P]
    L.fp_mlp_set_weights.argtypes = [P, P, D]
    L.fp_mlp_num_flagged.argtypes = [P, C.POINTER(I64)]
    L.fp_set_timing.argtypes = [P, I32]
    L.fp_node_volumes.argtypes = [P, P]
    L.fp_get_timing.argtypes = [P, P]
    L.fp_particle_block_layout.argtypes = [I64, C.c_int, P, C.POINTER(C.c_size_t)]
    L.fp_bind_particles.argtypes = [P, I64, C.c_int, P]
    L.fp_mlp_train.argtypes = [P, P, P, I64, I32, I32, C.c_float, C.c_uint64, P, P]
    L.fp_mlp_loss_grad_static.argtypes = [P, P, I64, P, P, P, P]
    L.fp_bind_deposit_list.argtypes = [P, P, C.c_size_t]
    L.fp_deposit_list_bytes.argtypes = [P, I32, C.POINTER(C.c_size_t)]
    for name in EXPORTS:       # every documented entry point must resolve
        getattr(L, name)
    _lib = L
    return L


MLP_IN = 84
MLP_SHAPES = [(64, MLP_IN), (64,), (64, 64), (64,), (64, 64), (64,), (3, 64), (3,)]


def xavier_init(rng):
    """Xavier-uniform weights and zero biases of the 84-64-64-64-3 network, flat (FP64)."""
    parts = []
    for shp in MLP_SHAPES:
        if len(shp) == 2:
            a = np.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-a, a, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())     # torch tensor


class FlexiPart:
    """One mesh + particle set on one GPU (a context of the C library)."""

    def __init__(self, mesh, N, max_particles, dg_nodes=0, device="cuda"):
        import torch
        self.torch = torch
        self.L = load()
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        self._check(self.L.fp_create(C.byref(self.ctx), C.c_void_p(self.stream.cuda_stream)), "fp_create")
        self.E = mesh.n_elem
        self.N = N
        self.n3 = (N + 1) ** 3
        keep = [np.ascontiguousarray(mesh.X, np.float64), np.ascontiguousarray(mesh.nbr_elem, np.int32),
                np.ascontiguousarray(mesh.nbr_face, np.int32), np.ascontiguousarray(mesh.bc, np.int8),
                np.ascontiguousarray(mesh.shift, np.float64)]
        mortar = getattr(mesh, "mortar", None)
        mortar = np.ascontiguousarray(mortar if mortar is not None else np.zeros((0, 4, 2)), np.int32)
        keep.append(mortar)
        desc = MeshDesc(self.E, mesh.n_geo, *[_ptr(a) for a in keep[:5]], N, dg_nodes, int(mortar.shape[0]),
                        _ptr(mortar) if mortar.shape[0] else None)
        self._check(self.L.fp_init_mesh(self.ctx, C.byref(desc)), "fp_init_mesh")
        sz = C.c_size_t(0)
        self._check(self.L.fp_workspace_size(self.ctx, int(max_particles), C.byref(sz)), "fp_workspace_size")
        self.ws = torch.empty(sz.value + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self._check(self.L.fp_bind_workspace(self.ctx, C.c_void_p(base + off), sz.value), "fp_bind_workspace")
        self.U = None
        self.np = 0
        self.mlp_w = None

    def _check(self, rc, what):
        if rc < 0:
            msg = self.L.fp_last_error(self.ctx).decode() if self.ctx else ""
            raise FPError("%s failed (%d): %s" % (what, rc, msg))
        return rc

    def close(self):
        if self.ctx:
            self.L.fp_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fluid_state(self, U, mu=1.8e-5, kappa=1.4, rho_p=2500.0):
        t = self.torch
        if not isinstance(U, t.Tensor):
            U = t.from_numpy(np.ascontiguousarray(U))
        U = U.to(self.device).contiguous()
        assert U.shape == (self.E, 5, self.n3), U.shape
        self.U = U
        prm = FluidParams(mu, kappa, rho_p)
        dt = F64 if U.dtype == t.float64 else F32
        self._check(self.L.fp_set_fluid_state(self.ctx, _ptr(U), dt, C.byref(prm)), "fp_set_fluid_state")

    def push(self, x, v, d, elem_hint=None, n=None):
        """Host arrays x, v, d; or x = v = d = None with a bound particle block
        whose first n entries of x, v and d are already filled."""
        if x is None:
            xp = vp = dp = None
        else:
            x = np.ascontiguousarray(x, np.float64)
            v = np.ascontiguousarray(v, np.float64)
            d = np.ascontiguousarray(d, np.float64)
            n = x.shape[0]
            xp, vp, dp = _ptr(x), _ptr(v), _ptr(d)
        h = np.ascontiguousarray(elem_hint, np.int32) if elem_hint is not None else None
        st = np.zeros(n, np.int32)
        rc = self._check(self.L.fp_push_particles(self.ctx, n, xp, vp, dp, _ptr(h), _ptr(st)), "fp_push_particles")
        self.np = n
        return st, rc

    @staticmethod
    def particle_block_layout(capacity):
        """(byte offsets of the 10 arrays, block bytes) of a caller-owned particle block."""
        off = np.zeros(10, np.int64)
        nb = C.c_size_t(0)
        rc = load().fp_particle_block_layout(int(capacity), F64, _ptr(off), C.byref(nb))
        if rc != 0:
            raise FPError("fp_particle_block_layout failed (%d)" % rc)
        return off, nb.value

    def bind_particles(self, block, capacity):
        """Bind a caller-owned device block (uint8 tensor of the documented layout),
        or None to return to the workspace's own particle buffer."""
        self.block = block
        self._check(self.L.fp_bind_particles(self.ctx, int(capacity), F64, _ptr(block)), "fp_bind_particles")
        self.np = 0

    def bind_deposit_list(self, cap):
        """Allocate (torch) and bind the FP32 source's per-target reuse list with
        cap rows per element; cap = 0 unbinds."""
        if cap <= 0:
            self.dep_list = None
            return self._check(self.L.fp_bind_deposit_list(self.ctx, None, 0), "fp_bind_deposit_list")
        nb = C.c_size_t(0)
        self._check(self.L.fp_deposit_list_bytes(self.ctx, int(cap), C.byref(nb)), "fp_deposit_list_bytes")
        self.dep_list = self.torch.empty(nb.value + 256, dtype=self.torch.uint8, device=self.device)
        base = self.dep_list.data_ptr()
        off = (-base) % 256
        return self._check(self.L.fp_bind_deposit_list(self.ctx, C.c_void_p(base + off), nb.value),
                           "fp_bind_deposit_list")

    def step(self, dt, n_steps=1, rk=1, drag=1, precision=0, guess=0, sort_every=1, max_newton_it=50,
             max_crossings=64, gravity=(0.0, 0.0, 0.0), tracking=0, forces=0):
        o = StepOpts(rk, drag, precision, guess, sort_every, max_newton_it, max_crossings, int(tracking),
                     int(forces), (C.c_double * 3)(*gravity))
        return self._check(self.L.fp_step(self.ctx, float(dt), int(n_steps), C.byref(o)), "fp_step")

    def deposit(self, S=None, kind=0, radius=0.0, period=None, drag=1, dtype=None, forces=0, gravity=None):
        t = self.torch
        if S is None:
            S = t.zeros((self.E, 4, self.n3), dtype=dtype or t.float64, device=self.device)
        per = np.ascontiguousarray(period, np.float64) if period is not None else None
        g = np.ascontiguousarray(gravity, np.float64) if gravity is not None else None
        dt = F64 if S.dtype == t.float64 else F32
        self._check(self.L.fp_deposit_source(self.ctx, _ptr(S), dt, int(kind), float(radius), _ptr(per), int(drag),
                                             int(forces), _ptr(g)), "fp_deposit_source")
        return S

    def node_volumes(self):
        V = self.torch.empty((self.E, self.n3), dtype=self.torch.float64, device=self.device)
        self._check(self.L.fp_node_volumes(self.ctx, _ptr(V)), "fp_node_volumes")
        return V

    def read(self):
        n = self.np
        out = dict(x=np.zeros((n, 3)), v=np.zeros((n, 3)), elem=np.zeros(n, np.int32), xi=np.zeros((n, 3)),
                   hits=np.zeros(n, np.int32), status=np.zeros(n, np.int8))
        nn = C.c_int64(0)
        self._check(self.L.fp_read_particles(self.ctx, C.byref(nn), _ptr(out["x"]), _ptr(out["v"]),
                                             _ptr(out["elem"]), _ptr(out["xi"]), _ptr(out["hits"]),
                                             _ptr(out["status"])), "fp_read_particles")
        return out

    def stats(self):
        s = np.zeros(11, np.int64)
        self._check(self.L.fp_get_stats(self.ctx, _ptr(s)), "fp_get_stats")
        return dict(newton_iters=int(s[0]), newton_calls=int(s[1]), crossings=int(s[2]), wall_hits=int(s[3]),
                    lost=int(s[4]), fallbacks=int(s[5]), sorts=int(s[6]), stragglers=int(s[7]),
                    track_queue=int(s[8]), recovered=int(s[9]), deposit_pairs=int(s[10]))

    def set_timing(self, enable=True, count_pairs=False):
        """HIP-event timing of the step and source kernels; count_pairs also
        counts the shape-kernel pairs within the radius (stats deposit_pairs)."""
        flags = (1 if enable else 0) | (2 if count_pairs else 0)
        self._check(self.L.fp_set_timing(self.ctx, flags), "fp_set_timing")

    def timing(self):
        """{class: (launches, total ms)} since the last call (synchronises)."""
        out = np.zeros(2 * len(TIMING_CLASSES))
        self._check(self.L.fp_get_timing(self.ctx, _ptr(out)), "fp_get_timing")
        return {k: (int(out[2 * i]), float(out[2 * i + 1])) for i, k in enumerate(TIMING_CLASSES)}

    def reset_stats(self):
        self._check(self.L.fp_reset_stats(self.ctx), "fp_reset_stats")

    # ---- learned guess ----------------------------------------------------
    @staticmethod
    def mlp_n_weights():
        return int(load().fp_mlp_n_weights())

    def mlp_features(self, elem, x):
        t = self.torch
        elem = t.as_tensor(np.ascontiguousarray(elem, np.int32), device=self.device)
        x = t.as_tensor(np.ascontiguousarray(x, np.float64), device=self.device)
        feat = t.empty((elem.shape[0], MLP_IN), dtype=t.float32, device=self.device)
        self._check(self.L.fp_mlp_features(self.ctx, elem.shape[0], _ptr(elem), _ptr(x), _ptr(feat)),
                    "fp_mlp_features")
        return feat

    def newton_pairs(self, with_ids=False):
        t = self.torch
        feat = t.empty((max(self.np, 1), MLP_IN), dtype=t.float32, device=self.device)
        xi = t.empty((max(self.np, 1), 3), dtype=t.float32, device=self.device)
        ids = t.empty(max(self.np, 1), dtype=t.int32, device=self.device)
        n = C.c_int64(0)
        self._check(self.L.fp_newton_pairs(self.ctx, C.byref(n), _ptr(feat), _ptr(xi), _ptr(ids), feat.shape[0]),
                    "fp_newton_pairs")
        if with_ids:
            return feat[:n.value], xi[:n.value], ids[:n.value]
        return feat[:n.value], xi[:n.value]

    def mlp_forward(self, w, inp):
        out = self.torch.empty((inp.shape[0], 3), dtype=self.torch.float32, device=self.device)
        self._check(self.L.fp_mlp_forward(self.ctx, _ptr(w), inp.shape[0], _ptr(inp), _ptr(out)), "fp_mlp_forward")
        return out

    def mlp_loss_grad(self, w, inp, target):
        t = self.torch
        g = t.empty(w.shape[0], dtype=t.float32, device=self.device)
        loss = t.empty(1, dtype=t.float32, device=self.device)
        self._check(self.L.fp_mlp_loss_grad(self.ctx, _ptr(w), inp.shape[0], _ptr(inp), _ptr(target), _ptr(g),
                                            _ptr(loss)), "fp_mlp_loss_grad")
        return loss, g

    def mlp_train_epoch(self, w, m, v, t_step, inp, target, order, batch, lr):
        t = self.torch
        n = order.shape[0]
        losses = t.zeros(max(n // batch, 1), dtype=t.float32, device=self.device)
        tt = C.c_int64(int(t_step))
        self._check(self.L.fp_mlp_train_epoch(self.ctx, _ptr(w), _ptr(m), _ptr(v), C.byref(tt), _ptr(inp),
                                              _ptr(target), _ptr(order), n, int(batch), float(lr), _ptr(losses)),
                    "fp_mlp_train_epoch")
        return tt.value, losses[:n // batch]

    def mlp_train(self, feat, target, epochs=20, batch=4096, lr=1e-3, seed=4):
        """Train from scratch with fp_mlp_train (initial weights and row orders
        drawn by the library from `seed`); returns (weights, mean loss per epoch)."""
        t = self.torch
        w = t.empty(self.mlp_n_weights(), dtype=t.float32, device=self.device)
        hist = np.zeros(max(int(epochs), 1), np.float32)
        self._check(self.L.fp_mlp_train(self.ctx, _ptr(feat), _ptr(target), int(feat.shape[0]), int(epochs),
                                        int(batch), float(lr), int(seed), _ptr(w), _ptr(hist)), "fp_mlp_train")
        return w, [float(v) for v in hist[:epochs]]

    def mlp_set_weights(self, w, thresh=0.05):
        self.mlp_w = w
        self._check(self.L.fp_mlp_set_weights(self.ctx, _ptr(w), float(thresh)), "fp_mlp_set_weights")
        n = C.c_int64(0)
        self.L.fp_mlp_num_flagged(self.ctx, C.byref(n))
        return n.value
