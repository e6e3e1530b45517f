"""Python binding of libgd.so (include/gd.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
(host pointers) or torch CUDA/HIP tensors (device pointers, with
GD_F_DEVICE_PTRS) into the plain pointers and sizes of the C ABI, and turns
negative return codes into ``GDError``.  Loading fails loudly when the
library has not been built (``python -m paper_1807_00699_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgd.so")

# enums / flags (mirror include/gd.h)
GD_OK = 0
GD_E_INVALID_ARG, GD_E_NOT_SYMMETRIC, GD_E_NONFINITE, GD_E_OOM = -1, -2, -3, -4
GD_E_DEVICE, GD_E_STATE, GD_E_DIVERGED, GD_E_UNSUPPORTED = -5, -6, -7, -8
GD_ISING, GD_XY, GD_ISING_COMPLEX, GD_POTTS = 0, 1, 2, 3
GD_EULER, GD_RK4 = 0, 1
GD_PREC_FP32, GD_PREC_BF16, GD_PREC_FP16 = 0, 1, 2
GD_SPINS_I8, GD_SPINS_ANGLE_F32, GD_SPINS_STATE_I32 = 0, 1, 2
GD_VARIANT_GD, GD_VARIANT_MOD = 0, 1
GD_F_DEVICE_PTRS, GD_F_ASYNC, GD_F_PROFILE = 0x1, 0x2, 0x4

# exported symbols of include/gd.h
EXPORTS = (
    "gd_default_params", "gd_create", "gd_destroy", "gd_set_init", "gd_run", "gd_energy",
    "gd_energy_device", "gd_spins", "gd_get_state", "gd_set_state", "gd_stats",
    "gd_coupling_scale", "gd_error_string", "gd_last_error", "gd_create_batch", "gd_set_targets",
    "gd_ttt", "gd_features", "gd_mlp_create", "gd_mlp_destroy", "gd_mlp_set_params",
    "gd_mlp_get_params", "gd_mlp_forward", "gd_mlp_train_step", "gd_propose", "gd_mod_couplings",
    "gd_spins_noalloc", "gd_trajectory_status", "gd_best_trace",
)
GD_NFEAT = 20
GD_MLP_NPARAM = 5634


class gd_params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("integrator", C.c_int32), ("precision", C.c_int32),
        ("flags", C.c_uint32), ("dt", C.c_double), ("eps", C.c_double), ("rho_th", C.c_double),
        ("gamma_c", C.c_double), ("gamma0", C.c_double), ("j_scale", C.c_double),
        ("init_amp", C.c_double), ("seed", C.c_uint64), ("check_interval", C.c_int32),
        ("has_target", C.c_int32), ("target_energy", C.c_double), ("stream", C.c_void_p),
        ("noise_D", C.c_double), ("noise_seed", C.c_uint64), ("q", C.c_int32),
        ("variant", C.c_int32), ("h_q", C.c_double), ("eps_hat", C.c_double),
    ]


class gd_run_stats(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("batch", C.c_int32), ("steps_done", C.c_int64),
        ("spin_updates", C.c_int64), ("run_seconds", C.c_double), ("kernel_ms", C.c_double),
        ("kernel_launches", C.c_int64), ("diverged", C.c_int32), ("target_reached", C.c_int32),
        ("ttt_seconds", C.c_double), ("ttt_steps", C.c_int64), ("best_energy", C.c_double),
        ("best_index", C.c_int32), ("kernel_config", C.c_int32),
    ]


class gd_instance(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("J", C.c_void_p), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
        ("val", C.c_void_p), ("g", C.c_void_p),
    ]


class GDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libgd.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_1807_00699_amd.build`")
    # torch ships its own HIP runtime with the same SONAME as ROCm's.  Loading
    # torch first makes libgd.so bind to that copy, so the process has one HIP
    # runtime and torch tensors / streams are valid handles for the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.gd_default_params.argtypes = [C.POINTER(gd_params)]
    lib.gd_default_params.restype = None
    lib.gd_create.argtypes = [C.POINTER(vp), i32, vp, vp, i32, C.POINTER(gd_params)]
    lib.gd_destroy.argtypes = [vp]
    lib.gd_destroy.restype = None
    lib.gd_set_init.argtypes = [vp, i32, vp, vp, vp]
    lib.gd_run.argtypes = [vp, i32, i64]
    lib.gd_energy.argtypes = [vp, vp, vp]
    lib.gd_energy_device.argtypes = [vp, vp, vp]
    lib.gd_spins.argtypes = [vp, vp, i32]
    lib.gd_spins_noalloc.argtypes = [vp, vp, i32]
    lib.gd_get_state.argtypes = [vp, vp, vp, vp]
    lib.gd_set_state.argtypes = [vp, i32, vp, vp, i64]
    lib.gd_stats.argtypes = [vp, C.POINTER(gd_run_stats)]
    lib.gd_trajectory_status.argtypes = [vp, vp, i64]
    lib.gd_best_trace.argtypes = [vp, vp, vp, i32, C.POINTER(C.c_int32)]
    lib.gd_coupling_scale.argtypes = [vp, C.POINTER(C.c_double)]
    lib.gd_create_batch.argtypes = [C.POINTER(vp), i32, vp, i32, C.POINTER(gd_params)]
    lib.gd_set_targets.argtypes = [vp, vp]
    lib.gd_ttt.argtypes = [vp, vp, vp, vp]
    lib.gd_features.argtypes = [vp, i32, vp, vp, vp]
    lib.gd_mlp_create.argtypes = [C.POINTER(vp), vp, C.c_uint64, C.c_uint32]
    lib.gd_mlp_destroy.argtypes = [vp]
    lib.gd_mlp_destroy.restype = None
    lib.gd_mlp_set_params.argtypes = [vp, vp]
    lib.gd_mlp_get_params.argtypes = [vp, vp]
    lib.gd_mlp_forward.argtypes = [vp, i32, vp, vp, i32]
    lib.gd_mlp_train_step.argtypes = [vp, i32, vp, vp, i32, vp, C.c_float, C.POINTER(C.c_double), vp]
    lib.gd_propose.argtypes = [vp, vp, i32, i32, C.c_double, C.c_double, C.c_uint64]
    lib.gd_error_string.argtypes = [C.c_int]
    lib.gd_error_string.restype = C.c_char_p
    lib.gd_last_error.argtypes = []
    lib.gd_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("gd_default_params", "gd_destroy", "gd_error_string", "gd_last_error",
                        "gd_mlp_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc, what):
    if rc != GD_OK:
        msg = load().gd_last_error().decode(errors="replace")
        raise GDError(rc, f"{what}: {msg}")


def _ptr(a, dtype=np.float32, device=False):
    """Pointer of a numpy array (host) or torch tensor (device); None -> NULL."""
    if a is None:
        return None, None
    if device:
        return C.c_void_p(a.data_ptr()), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(C.c_void_p), arr


def default_params(**kw) -> gd_params:
    p = gd_params()
    load().gd_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------- C-named calls

def gd_create(J, g=None, model=GD_ISING, params: gd_params | None = None):
    """Returns an opaque handle (c_void_p).  J: [n][n] float32 (numpy, or a
    device tensor when params.flags has GD_F_DEVICE_PTRS)."""
    lib = load()
    dev = bool(params is not None and params.flags & GD_F_DEVICE_PTRS)
    n = int(J.shape[0])
    if tuple(J.shape) != (n, n):
        raise ValueError("J must be square")
    pj, _kj = _ptr(J, device=dev)
    pg, _kg = _ptr(g, device=dev)
    h = C.c_void_p()
    _check(lib.gd_create(C.byref(h), n, pj, pg, int(model),
                         C.byref(params) if params is not None else None), "gd_create")
    return h


def gd_destroy(h):
    load().gd_destroy(h)


def gd_set_init(h, batch, psi0=None, gamma0=None, eps=None, device=False):
    p0, _a = _ptr(psi0, device=device)
    pg, _b = _ptr(gamma0, device=device)
    pe, _c = _ptr(eps, device=device)
    _check(load().gd_set_init(h, int(batch), p0, pg, pe), "gd_set_init")


def gd_run(h, batch, steps):
    rc = load().gd_run(h, int(batch), int(steps))
    _check(rc, "gd_run")


def gd_energy(h, batch, device_path=False):
    """Energies [batch] (float64) and argmin."""
    E = np.empty(int(batch), np.float64)
    best = C.c_int32()
    fn = load().gd_energy_device if device_path else load().gd_energy
    _check(fn(h, E.ctypes.data_as(C.c_void_p), C.byref(best)), "gd_energy")
    return E, int(best.value)


def gd_spins(h, batch, n, fmt=GD_SPINS_I8):
    dtype = {GD_SPINS_I8: np.int8, GD_SPINS_STATE_I32: np.int32}.get(fmt, np.float32)
    out = np.empty((int(batch), int(n)), dtype)
    _check(load().gd_spins(h, out.ctypes.data_as(C.c_void_p), int(fmt)), "gd_spins")
    return out


def gd_spins_noalloc(h, batch, n, fmt=GD_SPINS_I8):
    dtype = {GD_SPINS_I8: np.int8, GD_SPINS_STATE_I32: np.int32}.get(fmt, np.float32)
    out = np.empty((int(batch), int(n)), dtype)
    _check(load().gd_spins_noalloc(h, out.ctypes.data_as(C.c_void_p), int(fmt)), "gd_spins_noalloc")
    return out


def gd_get_state(h, batch, n, complex_mode):
    psi = np.empty((batch, n, 2) if complex_mode else (batch, n), np.float32)
    gam = np.empty((batch, n), np.float32)
    step = C.c_int64()
    _check(load().gd_get_state(h, psi.ctypes.data_as(C.c_void_p), gam.ctypes.data_as(C.c_void_p),
                               C.byref(step)), "gd_get_state")
    return psi, gam, int(step.value)


def gd_set_state(h, batch, psi, gamma, step=0):
    pp, _a = _ptr(psi)
    pg, _b = _ptr(gamma)
    _check(load().gd_set_state(h, int(batch), pp, pg, int(step)), "gd_set_state")


def gd_stats(h) -> gd_run_stats:
    st = gd_run_stats()
    st.struct_size = C.sizeof(gd_run_stats)
    _check(load().gd_stats(h, C.byref(st)), "gd_stats")
    return st


def gd_trajectory_status(h, count):
    """int32 [count]: 1 for each trajectory that became non-finite"""
    out = np.empty(count, np.int32)
    _check(load().gd_trajectory_status(h, out.ctypes.data_as(C.c_void_p), int(count)),
           "gd_trajectory_status")
    return out


def gd_best_trace(h):
    """(steps int64 [m], best-so-far energy float64 [m]) of the device checks"""
    n = C.c_int32()
    _check(load().gd_best_trace(h, None, None, 0, C.byref(n)), "gd_best_trace")
    steps = np.empty(n.value, np.int64)
    best = np.empty(n.value, np.float64)
    _check(load().gd_best_trace(h, steps.ctypes.data_as(C.c_void_p), best.ctypes.data_as(C.c_void_p),
                                n.value, C.byref(n)), "gd_best_trace")
    return steps, best


def gd_coupling_scale(h) -> float:
    v = C.c_double()
    _check(load().gd_coupling_scale(h, C.byref(v)), "gd_coupling_scale")
    return float(v.value)


class Solver:
    """Owning wrapper of one gd_solver handle (host arrays)."""

    def __init__(self, J, g=None, model=GD_ISING, **params):
        self.n = int(J.shape[0])
        self.model = model
        self.params = default_params(**params)
        self.h = gd_create(np.asarray(J, np.float32), None if g is None else np.asarray(g, np.float32),
                           model, self.params)
        self.batch = 0

    def close(self):
        if self.h is not None:
            gd_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_init(self, batch, psi0=None, gamma0=None, eps=None):
        gd_set_init(self.h, batch, psi0, gamma0, eps)
        self.batch = int(batch)

    def run(self, steps, batch=None):
        gd_run(self.h, self.batch if batch is None else batch, steps)
        if batch is not None:
            self.batch = int(batch)

    def state(self):
        return gd_get_state(self.h, self.batch, self.n, self.model != GD_ISING)

    def set_state(self, psi, gamma, step=0):
        psi = np.asarray(psi, np.float32)
        gd_set_state(self.h, psi.shape[0], psi, gamma, step)
        self.batch = psi.shape[0]

    def energy(self, device_path=False):
        return gd_energy(self.h, self.batch, device_path)

    def spins(self, fmt=None):
        if fmt is None:
            fmt = {GD_ISING: GD_SPINS_I8, GD_ISING_COMPLEX: GD_SPINS_I8,
                   GD_POTTS: GD_SPINS_STATE_I32}.get(self.model, GD_SPINS_ANGLE_F32)
        return gd_spins(self.h, self.batch, self.n, fmt)

    def stats(self):
        return gd_stats(self.h)

    def trajectory_status(self):
        """1 for each trajectory that became non-finite, else 0"""
        return gd_trajectory_status(self.h, gd_stats(self.h).batch)

    def best_trace(self):
        """steps and best-so-far energy of each device check since set_init"""
        return gd_best_trace(self.h)

    def mod_couplings(self, traj):
        """GD-mod: K [n][n] of trajectory `traj`."""
        K = np.empty((self.n, self.n), np.float32)
        _check(load().gd_mod_couplings(self.h, int(traj), K.ctypes.data_as(C.c_void_p)),
               "gd_mod_couplings")
        return K

    @property
    def scale(self):
        return gd_coupling_scale(self.h)


def gd_create_batch(instances, model=GD_ISING, params: gd_params | None = None):
    """instances: list of dicts with 'n' and either 'J' (dense [n][n]) or CSR
    'row_ptr', 'col', 'val', optional 'g' (host numpy).  Returns (handle, keep)
    where keep holds the marshalled arrays alive for the call."""
    lib = load()
    arr = (gd_instance * len(instances))()
    keep = []
    for k, inst in enumerate(instances):
        a = arr[k]
        a.n = int(inst["n"])
        for name, dt in (("J", np.float32), ("row_ptr", np.int32), ("col", np.int32),
                         ("val", np.float32), ("g", np.float32)):
            v = inst.get(name)
            if v is not None:
                v = np.ascontiguousarray(v, dtype=dt)
                keep.append(v)
                setattr(a, name, v.ctypes.data_as(C.c_void_p))
    h = C.c_void_p()
    _check(lib.gd_create_batch(C.byref(h), len(instances), C.cast(arr, C.c_void_p), int(model),
                               C.byref(params) if params is not None else None), "gd_create_batch")
    return h


def gd_set_targets(h, targets):
    t = None if targets is None else np.ascontiguousarray(targets, np.float64)
    _check(load().gd_set_targets(h, None if t is None else t.ctypes.data_as(C.c_void_p)), "gd_set_targets")


def gd_ttt(h, count):
    sec = np.empty(count, np.float64)
    st = np.empty(count, np.int64)
    be = np.empty(count, np.float64)
    _check(load().gd_ttt(h, sec.ctypes.data_as(C.c_void_p), st.ctypes.data_as(C.c_void_p),
                         be.ctypes.data_as(C.c_void_p)), "gd_ttt")
    return sec, st, be


class BatchSolver:
    """Owning wrapper of a gd_create_batch handle (host arrays, Ising, Euler)."""

    def __init__(self, instances, **params):
        self.ns = [int(i["n"]) for i in instances]
        self.K = len(instances)
        self.total = int(sum(self.ns))
        self.params = default_params(**params)
        self.h = gd_create_batch(instances, GD_ISING, self.params)
        self.R = 0

    def close(self):
        if self.h is not None:
            gd_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_init(self, R, psi0=None, gamma0=None, eps=None):
        gd_set_init(self.h, R, psi0, gamma0, eps)
        self.R = int(R)

    def run(self, steps, R=None):
        gd_run(self.h, self.R if R is None else R, steps)
        if R is not None:
            self.R = int(R)

    def state(self):
        psi = np.empty(self.total * self.R, np.float32)
        gam = np.empty(self.total * self.R, np.float32)
        step = C.c_int64()
        _check(load().gd_get_state(self.h, psi.ctypes.data_as(C.c_void_p),
                                   gam.ctypes.data_as(C.c_void_p), C.byref(step)), "gd_get_state")
        return psi, gam, int(step.value)

    def set_state(self, psi, gamma, R, step=0):
        gd_set_state(self.h, R, np.ravel(psi), np.ravel(gamma), step)
        self.R = int(R)

    def trajectory_status(self):
        """[instances][R]: 1 for each trajectory that became non-finite"""
        return gd_trajectory_status(self.h, len(self.ns) * self.R).reshape(len(self.ns), self.R)

    def split(self, flat):
        """concatenated [sum_k R n_k] -> list of [R][n_k]"""
        out, off = [], 0
        for n in self.ns:
            out.append(np.asarray(flat[off:off + self.R * n]).reshape(self.R, n))
            off += self.R * n
        return out

    def energy(self):
        E = np.empty(self.K * self.R, np.float64)
        best = np.empty(self.K, np.int32)
        _check(load().gd_energy(self.h, E.ctypes.data_as(C.c_void_p), best.ctypes.data_as(C.c_void_p)),
               "gd_energy")
        return E.reshape(self.K, self.R), best

    def spins(self):
        out = np.empty(self.total * self.R, np.int8)
        _check(load().gd_spins(self.h, out.ctypes.data_as(C.c_void_p), GD_SPINS_I8), "gd_spins")
        return out

    def set_targets(self, targets):
        gd_set_targets(self.h, targets)

    def ttt(self):
        return gd_ttt(self.h, self.K)

    def stats(self):
        return gd_stats(self.h)


def gd_features(h, total, K, iters=30):
    """features [total][GD_NFEAT], lambda [K][8], Ritz vectors [total][8]"""
    f = np.empty((total, GD_NFEAT), np.float32)
    lam = np.empty((K, 8), np.float32)
    vec = np.empty((total, 8), np.float32)
    _check(load().gd_features(h, int(iters), f.ctypes.data_as(C.c_void_p), lam.ctypes.data_as(C.c_void_p),
                              vec.ctypes.data_as(C.c_void_p)), "gd_features")
    return f, lam, vec


class MLP:
    """Owning wrapper of a gd_mlp handle.  device=False: numpy arrays;
    device=True (GD_F_DEVICE_PTRS): X, labels and outputs are contiguous
    float32 device tensors, seg stays a host array, params stay host arrays."""

    def __init__(self, params=None, seed=0, device=False):
        lib = load()
        self.h = C.c_void_p()
        self.device = bool(device)
        pp, _keep = _ptr(params, device=self.device)
        _check(lib.gd_mlp_create(C.byref(self.h), pp, int(seed), GD_F_DEVICE_PTRS if self.device else 0),
               "gd_mlp_create")

    def close(self):
        if self.h is not None:
            load().gd_mlp_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self):
        if self.device:
            raise GDError(GD_E_INVALID_ARG, "params of a device-pointer MLP: use a host MLP")
        p = np.empty(GD_MLP_NPARAM, np.float32)
        _check(load().gd_mlp_get_params(self.h, p.ctypes.data_as(C.c_void_p)), "gd_mlp_get_params")
        return p

    @params.setter
    def params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        _check(load().gd_mlp_set_params(self.h, p.ctypes.data_as(C.c_void_p)), "gd_mlp_set_params")

    def forward_device(self, X, out, fp16=False):
        """X [M][GD_NFEAT], out [M][2]: contiguous float32 device tensors."""
        _check(load().gd_mlp_forward(self.h, int(X.shape[0]), C.c_void_p(X.data_ptr()),
                                     C.c_void_p(out.data_ptr()), int(bool(fp16))), "gd_mlp_forward")

    def train_step_device(self, X, labels, seg, lr):
        """X, labels: contiguous float32 device tensors; seg: host int32."""
        seg = np.ascontiguousarray(seg, np.int32)
        loss = C.c_double()
        _check(load().gd_mlp_train_step(self.h, int(X.shape[0]), C.c_void_p(X.data_ptr()),
                                        C.c_void_p(labels.data_ptr()), len(seg) - 1,
                                        seg.ctypes.data_as(C.c_void_p), float(lr), C.byref(loss), None),
               "gd_mlp_train_step")
        return float(loss.value)

    def forward(self, X, fp16=False):
        X = np.ascontiguousarray(X, np.float32)
        out = np.empty((X.shape[0], 2), np.float32)
        _check(load().gd_mlp_forward(self.h, X.shape[0], X.ctypes.data_as(C.c_void_p),
                                     out.ctypes.data_as(C.c_void_p), int(bool(fp16))), "gd_mlp_forward")
        return out

    def train_step(self, X, labels, seg, lr, want_grad=False):
        X = np.ascontiguousarray(X, np.float32)
        lab = np.ascontiguousarray(labels, np.float32)
        seg = np.ascontiguousarray(seg, np.int32)
        loss = C.c_double()
        g = np.empty(GD_MLP_NPARAM, np.float32) if want_grad else None
        _check(load().gd_mlp_train_step(self.h, X.shape[0], X.ctypes.data_as(C.c_void_p),
                                        lab.ctypes.data_as(C.c_void_p), len(seg) - 1,
                                        seg.ctypes.data_as(C.c_void_p), float(lr), C.byref(loss),
                                        None if g is None else g.ctypes.data_as(C.c_void_p)),
               "gd_mlp_train_step")
        return (float(loss.value), g) if want_grad else float(loss.value)


def gd_propose(h, mlp, R, feat_iters=30, alpha=0.5, beta=0.0, seed=0):
    _check(load().gd_propose(h, mlp.h, int(R), int(feat_iters), float(alpha), float(beta), int(seed)),
           "gd_propose")
