"""Python binding of libpfnks.so (C ABI in include/pfnks.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.
PyTorch provides the device workspace (one uint8 tensor per problem) and the stream.
The library must be built first (``python -m paper_2209_08001_amd.build``); loading
fails loudly if it is missing -- there is no CPU fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfnks.so")

PFNKS_OK = 0
PFNKS_EINVAL = -1
PFNKS_EDOMAIN = -2
PFNKS_ENOSPACE = -3
PFNKS_ENOCONV = -4
PFNKS_EDEVICE = -5

PC_RAS = 0
PC_RAS_SPECTRAL = 1
PC_NONE = 2
PC_SPECTRAL = 3
PC_AS = 4     # classical additive Schwarz (extended solutions summed)
PC_RRAS = 5   # right-RAS (right-hand side restricted to the owned nodes, solutions summed)

FP64 = 0   # every vector and kernel in double
MIXED = 1  # float Krylov basis, preconditioner and tile solve; double residual, J v, update

EXPORTED = [
    "pfnks_workspace_bytes", "pfnks_create_problem", "pfnks_step", "pfnks_energy", "pfnks_mass",
    "pfnks_get_state", "pfnks_set_state", "pfnks_destroy", "pfnks_strerror", "pfnks_last_error",
    "pfnks_debug_residual", "pfnks_debug_jv", "pfnks_debug_pc", "pfnks_debug_counters",
    "pfnks_debug_profile", "pfnks_debug_kernel_time", "pfnks_batch_step", "pfnks_residual_static",
    "pfnks_group_workspace_bytes", "pfnks_group_create", "pfnks_group_step", "pfnks_group_get_state",
    "pfnks_group_counters", "pfnks_group_destroy", "pfnks_group_set_instance",
]

MAX_GROUP = 32  # instances of one lockstep group

KERNEL_KINDS = ["residual", "linearise", "jv", "ras", "spectral", "multidot", "update"]


class pfnks_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double)]


class pfnks_model(ctypes.Structure):
    _fields_ = [
        ("theta", ctypes.c_double), ("w_c", ctypes.c_double), ("e0", ctypes.c_double),
        ("L", ctypes.c_double * 4), ("U1", ctypes.c_double), ("U4", ctypes.c_double),
        ("gamma_c", ctypes.c_double), ("gamma_eta", ctypes.c_double), ("kappa", ctypes.c_double),
        ("L_eta", ctypes.c_double), ("eps0", ctypes.c_double), ("C11", ctypes.c_double),
        ("C12", ctypes.c_double), ("C44", ctypes.c_double), ("Lscale", ctypes.c_double),
        ("S", ctypes.c_int),
    ]


class pfnks_solver(ctypes.Structure):
    _fields_ = [
        ("newton_rtol", ctypes.c_double), ("newton_atol_rms", ctypes.c_double),
        ("newton_maxit", ctypes.c_int), ("gmres_rtol", ctypes.c_double),
        ("gmres_atol_rms", ctypes.c_double), ("gmres_restart", ctypes.c_int),
        ("gmres_maxit", ctypes.c_int), ("tile", ctypes.c_int * 3), ("overlap", ctypes.c_int),
        ("sweeps", ctypes.c_int), ("sor_omega", ctypes.c_double), ("pc", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("ls_alpha", ctypes.c_double), ("ls_max_halvings", ctypes.c_int),
        ("newton_stol", ctypes.c_double), ("pc_refresh", ctypes.c_int),
    ]


class pfnks_step_stats(ctypes.Structure):
    _fields_ = [
        ("newton_its", ctypes.c_int), ("gmres_its", ctypes.c_int), ("ls_backtracks", ctypes.c_int),
        ("status", ctypes.c_int), ("res0", ctypes.c_double), ("res_final", ctypes.c_double),
        ("dx_rms", ctypes.c_double), ("energy", ctypes.c_double),
        ("energy_parts", ctypes.c_double * 3), ("mass", ctypes.c_double),
        ("update_rel", ctypes.c_double),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "energy_parts"}
        d["energy_parts"] = tuple(self.energy_parts)
        return d


_lib = None


def load():
    """Load libpfnks.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run python -m paper_2209_08001_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.pfnks_workspace_bytes.argtypes = [ctypes.POINTER(pfnks_grid), ctypes.POINTER(pfnks_model),
                                          ctypes.POINTER(pfnks_solver), ctypes.POINTER(ctypes.c_size_t)]
    lib.pfnks_create_problem.argtypes = [ctypes.POINTER(pfnks_grid), ctypes.POINTER(pfnks_model),
                                         ctypes.POINTER(pfnks_solver), dp, dp, P, ctypes.c_size_t, P,
                                         ctypes.POINTER(P)]
    lib.pfnks_step.argtypes = [P, ctypes.c_double, ctypes.POINTER(pfnks_step_stats)]
    lib.pfnks_energy.argtypes = [P, dp, dp]
    lib.pfnks_mass.argtypes = [P, dp]
    lib.pfnks_get_state.argtypes = [P, dp, dp]
    lib.pfnks_set_state.argtypes = [P, dp, ctypes.c_double]
    lib.pfnks_destroy.argtypes = [P]
    lib.pfnks_strerror.argtypes = [ctypes.c_int]
    lib.pfnks_strerror.restype = ctypes.c_char_p
    lib.pfnks_last_error.argtypes = []
    lib.pfnks_last_error.restype = ctypes.c_char_p
    lib.pfnks_debug_residual.argtypes = [P, dp, ctypes.c_double, dp]
    lib.pfnks_debug_jv.argtypes = [P, dp, ctypes.c_double, dp, dp]
    lib.pfnks_debug_pc.argtypes = [P, dp, ctypes.c_double, dp, dp]
    lib.pfnks_debug_counters.argtypes = [P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    lib.pfnks_debug_profile.argtypes = [P, ctypes.c_int]
    lib.pfnks_debug_kernel_time.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong), dp, dp]
    lib.pfnks_batch_step.argtypes = [ctypes.POINTER(P), ctypes.c_int, dp, ctypes.c_int,
                                     ctypes.POINTER(pfnks_step_stats), ctypes.POINTER(ctypes.c_int)]
    lib.pfnks_residual_static.argtypes = [ctypes.POINTER(pfnks_grid), ctypes.POINTER(pfnks_model), ctypes.c_double,
                                          ctypes.c_double, P, P, P, dp, dp, P]
    lib.pfnks_group_workspace_bytes.argtypes = [ctypes.POINTER(pfnks_grid), ctypes.POINTER(pfnks_model),
                                                ctypes.POINTER(pfnks_solver), ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_size_t)]
    lib.pfnks_group_create.argtypes = [ctypes.POINTER(pfnks_grid), ctypes.POINTER(pfnks_model),
                                       ctypes.POINTER(pfnks_solver), ctypes.c_int, dp, dp, P, ctypes.c_size_t, P,
                                       ctypes.POINTER(P)]
    lib.pfnks_group_step.argtypes = [P, dp, ctypes.POINTER(pfnks_step_stats), ctypes.POINTER(ctypes.c_int)]
    lib.pfnks_group_get_state.argtypes = [P, ctypes.c_int, dp, dp]
    lib.pfnks_group_set_instance.argtypes = [P, ctypes.c_int, dp, dp]
    lib.pfnks_group_counters.argtypes = [P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    lib.pfnks_group_destroy.argtypes = [P]
    for name in EXPORTED:
        if name not in ("pfnks_strerror", "pfnks_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class PfnksError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = lib.pfnks_strerror(status).decode()
        if status == PFNKS_EDEVICE:
            msg += ": " + lib.pfnks_last_error().decode()
        super().__init__(f"{where}: {msg} ({status})")
        self.status = status


def _check(status, where):
    if status != PFNKS_OK:
        raise PfnksError(status, where)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_grid(n, h):
    g = pfnks_grid()
    g.dim = len(n)
    g.n[0], g.n[1] = n[0], n[1]
    g.n[2] = n[2] if len(n) == 3 else 1
    g.h = h
    return g


def make_model(d):
    m = pfnks_model()
    for k in ("theta", "w_c", "e0", "U1", "U4", "gamma_c", "gamma_eta", "kappa", "L_eta", "eps0",
              "C11", "C12", "C44", "Lscale"):
        setattr(m, k, float(d[k]))
    for i in range(4):
        m.L[i] = float(d["L"][i])
    m.S = int(d["S"])
    return m


def make_solver(d, dim):
    s = pfnks_solver()
    s.newton_rtol = d["newton_rtol"]
    s.newton_atol_rms = d["newton_atol_rms"]
    s.newton_maxit = d["newton_maxit"]
    s.gmres_rtol = d["gmres_rtol"]
    s.gmres_atol_rms = d["gmres_atol_rms"]
    s.gmres_restart = d["gmres_restart"]
    s.gmres_maxit = d["gmres_maxit"]
    t = d["tile"]
    s.tile[0], s.tile[1], s.tile[2] = t[0], t[1], (t[2] if dim == 3 else 1)
    s.overlap = d["overlap"]
    s.sweeps = d.get("sweeps", 6)
    s.sor_omega = float(d.get("sor_omega", 1.0))
    s.pc = d.get("pc", PC_RAS_SPECTRAL)
    s.precision = d.get("precision", FP64)
    s.ls_alpha = d["ls_alpha"]
    s.ls_max_halvings = d["ls_max_halvings"]
    s.newton_stol = d.get("newton_stol", 0.0)
    s.pc_refresh = int(d.get("pc_refresh", 0))
    return s


def workspace_bytes(n, h, model, solver):
    lib = load()
    g = make_grid(n, h)
    m = make_model(model)
    s = make_solver(solver, len(n))
    out = ctypes.c_size_t(0)
    _check(lib.pfnks_workspace_bytes(ctypes.byref(g), ctypes.byref(m), ctypes.byref(s), ctypes.byref(out)),
           "pfnks_workspace_bytes")
    return out.value


def residual_static(n, h, model, cbar0, dt, X, Xn, F, stream=None, sync=True):
    """pfnks_residual_static on device tensors X, Xn (read) and F (written), each 4 + d
    contiguous float64 planes on the current device: F = F(X; Xn, dt) with the library's own
    scratch (no allocation).  Returns (||F||, out-of-domain count) when sync, else None."""
    lib = load()
    for a in (X, Xn, F):
        if not (a.is_cuda and a.is_contiguous() and str(a.dtype) == "torch.float64"):
            raise ValueError("X, Xn, F must be contiguous float64 device tensors")
        if a.numel() != (4 + len(n)) * int(np.prod(n)):
            raise ValueError("X, Xn, F must hold 4 + dim planes of the grid")
    g = make_grid(n, h)
    m = make_model(model)
    nrm = ctypes.c_double(0.0)
    bad = ctypes.c_double(0.0)
    sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib.pfnks_residual_static(ctypes.byref(g), ctypes.byref(m), float(cbar0), float(dt),
                                     ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Xn.data_ptr()),
                                     ctypes.c_void_p(F.data_ptr()), ctypes.byref(nrm) if sync else None,
                                     ctypes.byref(bad) if sync else None, sp), "pfnks_residual_static")
    return (nrm.value, bad.value) if sync else None


def batch_step(problems, dts, threads=0):
    """One step of every problem (pfnks_batch_step): returns (statuses, stats dicts).
    Raises on errors other than ENOCONV; an ENOCONV problem is left unchanged."""
    lib = load()
    k = len(problems)
    hs = (ctypes.c_void_p * k)(*[p._h.value for p in problems])
    d = (ctypes.c_double * k)(*[float(x) for x in dts])
    st = (pfnks_step_stats * k)()
    status = (ctypes.c_int * k)()
    rc = lib.pfnks_batch_step(hs, ctypes.c_int(k), d, ctypes.c_int(threads), st, status)
    for s_ in status:
        if s_ not in (PFNKS_OK, PFNKS_ENOCONV):
            _check(s_, "pfnks_batch_step")
    if rc not in (PFNKS_OK, PFNKS_ENOCONV):
        _check(rc, "pfnks_batch_step")
    return list(status), [x.as_dict() for x in st]


class Problem:
    """One phase-field problem resident on the GPU (same names as the C ABI)."""

    def __init__(self, n, h, model, solver, c0, eta0, device="cuda:0", stream=None):
        import torch

        lib = load()
        self.n = tuple(n)
        self.dim = len(n)
        self.nf = 4 + self.dim
        self.N = int(np.prod(n))
        self._g = make_grid(n, h)
        self._m = make_model(model)
        self._s = make_solver(solver, self.dim)
        nbytes = ctypes.c_size_t(0)
        _check(lib.pfnks_workspace_bytes(ctypes.byref(self._g), ctypes.byref(self._m), ctypes.byref(self._s),
                                         ctypes.byref(nbytes)), "pfnks_workspace_bytes")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._stream = stream if stream is not None else torch.cuda.current_stream(device)
        c0 = np.ascontiguousarray(c0, dtype=np.float64).ravel()
        eta0 = np.ascontiguousarray(eta0, dtype=np.float64).ravel()
        if c0.size != self.N or eta0.size != 3 * self.N:
            raise ValueError("c0 / eta0 sizes do not match the grid")
        h_ = ctypes.c_void_p()
        torch.cuda.synchronize(device)
        _check(lib.pfnks_create_problem(ctypes.byref(self._g), ctypes.byref(self._m), ctypes.byref(self._s),
                                        _dp(c0), _dp(eta0), ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes.value),
                                        ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h_)),
               "pfnks_create_problem")
        self._h = h_

    def step(self, dt):
        """One NSOA-1 step; raises PfnksError (status ENOCONV leaves the state unchanged)."""
        st = pfnks_step_stats()
        _check(load().pfnks_step(self._h, ctypes.c_double(dt), ctypes.byref(st)), "pfnks_step")
        return st.as_dict()

    def try_step(self, dt):
        """Like step() but returns (status, stats) instead of raising on ENOCONV."""
        st = pfnks_step_stats()
        status = load().pfnks_step(self._h, ctypes.c_double(dt), ctypes.byref(st))
        if status not in (PFNKS_OK, PFNKS_ENOCONV):
            _check(status, "pfnks_step")
        return status, st.as_dict()

    def energy(self):
        tot = ctypes.c_double()
        parts = (ctypes.c_double * 3)()
        _check(load().pfnks_energy(self._h, ctypes.byref(tot), parts), "pfnks_energy")
        return tot.value, tuple(parts)

    def mass(self):
        m = ctypes.c_double()
        _check(load().pfnks_mass(self._h, ctypes.byref(m)), "pfnks_mass")
        return m.value

    def get_state(self):
        X = np.empty((self.nf,) + tuple(reversed(self.n)))
        t = ctypes.c_double()
        _check(load().pfnks_get_state(self._h, _dp(X), ctypes.byref(t)), "pfnks_get_state")
        return X, t.value

    def set_state(self, X, t):
        X = np.ascontiguousarray(X, dtype=np.float64)
        _check(load().pfnks_set_state(self._h, _dp(X), ctypes.c_double(t)), "pfnks_set_state")

    def debug_residual(self, X, dt):
        X = np.ascontiguousarray(X, dtype=np.float64)
        F = np.empty_like(X)
        _check(load().pfnks_debug_residual(self._h, _dp(X), ctypes.c_double(dt), _dp(F)), "pfnks_debug_residual")
        return F

    def debug_jv(self, X, dt, v):
        X = np.ascontiguousarray(X, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        w = np.empty_like(X)
        _check(load().pfnks_debug_jv(self._h, _dp(X), ctypes.c_double(dt), _dp(v), _dp(w)), "pfnks_debug_jv")
        return w

    def debug_pc(self, X, dt, r):
        X = np.ascontiguousarray(X, dtype=np.float64)
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(X)
        _check(load().pfnks_debug_pc(self._h, _dp(X), ctypes.c_double(dt), _dp(r), _dp(z)), "pfnks_debug_pc")
        return z

    def counters(self):
        a = ctypes.c_longlong()
        b = ctypes.c_longlong()
        _check(load().pfnks_debug_counters(self._h, ctypes.byref(a), ctypes.byref(b)), "pfnks_debug_counters")
        return a.value, b.value

    def profile(self, kinds):
        """Live kernel timing (HIP events on the problem's stream) for the given kernel kinds
        (names, True for all, False/None for none); clears the totals."""
        if kinds is True:
            mask = (1 << len(KERNEL_KINDS)) - 1
        elif not kinds:
            mask = 0
        else:
            mask = 0
            for k in ([kinds] if isinstance(kinds, str) else kinds):
                mask |= 1 << KERNEL_KINDS.index(k)
        _check(load().pfnks_debug_profile(self._h, mask), "pfnks_debug_profile")

    def kernel_time(self, kind):
        """(launches, total ms, total algorithmic bytes) of one kernel kind since profile(True)."""
        k = KERNEL_KINDS.index(kind) if isinstance(kind, str) else int(kind)
        a = ctypes.c_longlong()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(load().pfnks_debug_kernel_time(self._h, k, ctypes.byref(a), ctypes.byref(ms), ctypes.byref(by)),
               "pfnks_debug_kernel_time")
        return a.value, ms.value, by.value

    def kernel_table(self):
        out = {}
        for k in KERNEL_KINDS:
            n, ms, by = self.kernel_time(k)
            if n:
                out[k] = {"launches": n, "total_ms": ms, "avg_us": 1e3 * ms / n,
                          "GB_s": by / (ms * 1e-3) / 1e9 if ms > 0 else None}
        return out

    def roofline(self, peak_gbs):
        """Roofline entry of the kernel kind with the largest total time: algorithmic bytes per
        launch over its average launch duration, against the HBM peak."""
        best = None
        for k in KERNEL_KINDS:
            n, ms, by = self.kernel_time(k)
            if n and (best is None or ms > best[2]):
                best = (k, n, ms, by)
        if best is None:
            return None
        k, n, ms, by = best
        achieved = by / (ms * 1e-3) / 1e9
        return {"kernel": k, "bound": "hbm", "achieved": achieved, "peak": peak_gbs, "unit": "GB/s",
                "frac": achieved / peak_gbs, "traffic": None, "launches": n,
                "avg_launch_us": 1e3 * ms / n, "bytes_per_launch": by / n}

    def close(self):
        if getattr(self, "_h", None):
            load().pfnks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """A lockstep group of problems of one grid shape (same names as the C ABI): every kernel of
    a step is launched once for all instances still working in that phase."""

    def __init__(self, n, h, model, solver, c0s, eta0s, device="cuda:0", stream=None):
        import torch

        lib = load()
        self.n = tuple(n)
        self.dim = len(n)
        self.nf = 4 + self.dim
        self.N = int(np.prod(n))
        self.count = len(c0s)
        if self.count != len(eta0s) or not 1 <= self.count <= MAX_GROUP:
            raise ValueError(f"a group holds 1..{MAX_GROUP} instances with one c0 and eta0 each")
        self._g = make_grid(n, h)
        self._m = make_model(model)
        self._s = make_solver(solver, self.dim)
        nbytes = ctypes.c_size_t(0)
        _check(lib.pfnks_group_workspace_bytes(ctypes.byref(self._g), ctypes.byref(self._m), ctypes.byref(self._s),
                                               ctypes.c_int(self.count), ctypes.byref(nbytes)),
               "pfnks_group_workspace_bytes")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self._stream = stream if stream is not None else torch.cuda.current_stream(device)
        c0 = np.ascontiguousarray(np.stack([np.asarray(c, dtype=np.float64).ravel() for c in c0s]))
        eta0 = np.ascontiguousarray(np.stack([np.asarray(e, dtype=np.float64).ravel() for e in eta0s]))
        if c0.shape[1] != self.N or eta0.shape[1] != 3 * self.N:
            raise ValueError("c0 / eta0 sizes do not match the grid")
        h_ = ctypes.c_void_p()
        torch.cuda.synchronize(device)
        _check(lib.pfnks_group_create(ctypes.byref(self._g), ctypes.byref(self._m), ctypes.byref(self._s),
                                      ctypes.c_int(self.count), _dp(c0), _dp(eta0), ctypes.c_void_p(aligned),
                                      ctypes.c_size_t(nbytes.value), ctypes.c_void_p(self._stream.cuda_stream),
                                      ctypes.byref(h_)), "pfnks_group_create")
        self._h = h_

    def step(self, dts):
        """One step of every instance; returns (statuses, stats dicts).  Raises only on errors
        other than an instance's ENOCONV (which leaves that instance unchanged)."""
        dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dts, dtype=np.float64), (self.count,)))
        st = (pfnks_step_stats * self.count)()
        status = (ctypes.c_int * self.count)()
        rc = load().pfnks_group_step(self._h, _dp(dts), st, status)
        if rc not in (PFNKS_OK, PFNKS_ENOCONV):
            _check(rc, "pfnks_group_step")
        return list(status), [s.as_dict() for s in st]

    def set_instance(self, i, c0, eta0):
        """A new initial state for instance i (a freed slot taking a new problem)."""
        c0 = np.ascontiguousarray(c0, dtype=np.float64).ravel()
        eta0 = np.ascontiguousarray(eta0, dtype=np.float64).ravel()
        if c0.size != self.N or eta0.size != 3 * self.N:
            raise ValueError("c0 / eta0 sizes do not match the grid")
        _check(load().pfnks_group_set_instance(self._h, ctypes.c_int(i), _dp(c0), _dp(eta0)),
               "pfnks_group_set_instance")

    def get_state(self, i):
        X = np.empty((self.nf,) + tuple(reversed(self.n)))
        t = ctypes.c_double()
        _check(load().pfnks_group_get_state(self._h, ctypes.c_int(i), _dp(X), ctypes.byref(t)),
               "pfnks_group_get_state")
        return X, t.value

    def counters(self):
        a = ctypes.c_longlong()
        b = ctypes.c_longlong()
        _check(load().pfnks_group_counters(self._h, ctypes.byref(a), ctypes.byref(b)), "pfnks_group_counters")
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            load().pfnks_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
