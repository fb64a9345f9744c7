"""Thin ctypes binding of libbbwadg.so (argument marshalling only).

Every step of the right-hand side and the time step runs in the HIP kernels of the
library; this module only converts arguments. Device buffers are torch tensors on the
current CUDA (HIP) device and work is queued on torch's current stream. If the library
is not built, loading fails loudly: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# BBWADG_LIB selects another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("BBWADG_LIB") or os.path.join(_PKG, "libbbwadg.so")

OK, EINVAL, EMESH, EC2, ENOMEM, EHIP = 0, -1, -2, -3, -4, -5
F64, F32 = 0, 1
BC_P0, BC_RIGID = 0, 1
DEVICE, HOST_ONLY = 0, 1

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = (
    "bbwadg_create", "bbwadg_destroy", "bbwadg_last_error", "bbwadg_sizes",
    "bbwadg_element_vertices", "bbwadg_geometry", "bbwadg_projection_npoints",
    "bbwadg_projection_points", "bbwadg_project_samples", "bbwadg_project_c2",
    "bbwadg_set_c2", "bbwadg_get_c2", "bbwadg_rhs", "bbwadg_step", "bbwadg_suggest_dt",
    "bbwadg_l2norm2", "bbwadg_l2norm2_noalloc", "bbwadg_l2error2", "bbwadg_energy", "bbwadg_project_fn", "bbwadg_coef_index",
    "bbwadg_dense_npoints", "bbwadg_dense_points", "bbwadg_dense_set_c2", "bbwadg_dense_update",
    "bbwadg_rhs_dense", "bbwadg_set_source", "bbwadg_set_receivers", "bbwadg_receiver_elements",
    "bbwadg_misfit_gradient", "bbwadg_adjoint_apply", "bbwadg_elastic_set_media", "bbwadg_elastic_update",
    "bbwadg_elastic_rhs", "bbwadg_elastic_step",
    "bbwadg_wadg_update", "bbwadg_set_c2_policy", "bbwadg_c2_positivity", "bbwadg_bernstein_positivity",
    "bbwadg_sur_create", "bbwadg_sur_destroy", "bbwadg_sur_num_params", "bbwadg_sur_layout",
    "bbwadg_sur_get_params", "bbwadg_sur_set_params", "bbwadg_sur_forward", "bbwadg_sur_loss_grad",
    "bbwadg_sur_train_step", "bbwadg_sur_input_grad",
    "bbwadg_projection_coefficients", "bbwadg_version",
)


class BBWADGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bbwadg error {code}: {msg}")
        self.code = code


class _Mesh(C.Structure):
    _fields_ = [("num_vertices", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("num_elements", C.c_int64), ("etov", C.POINTER(C.c_int32)), ("bc", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("N", C.c_int32), ("M", C.c_int32), ("dtype", C.c_int32), ("mode", C.c_int32),
                ("tau_p", C.c_double), ("tau_u", C.c_double)]


C2_CALLBACK = C.CFUNCTYPE(C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbbwadg.so (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    # torch ships its own HIP runtime; load it first so that this library binds to the same
    # one (both share the runtime's soname) and device pointers and streams agree.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pd, pi32, pi64 = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    sig = {
        "bbwadg_create": (C.c_int, [C.POINTER(_Mesh), C.POINTER(_Opts), C.POINTER(vp)]),
        "bbwadg_destroy": (C.c_int, [vp]),
        "bbwadg_last_error": (C.c_char_p, []),
        "bbwadg_sizes": (C.c_int, [vp, pi32, pi32, pi32, pi64]),
        "bbwadg_element_vertices": (C.c_int, [vp, pi32]),
        "bbwadg_geometry": (C.c_int, [vp, pd, pd, pd, pd, pi32]),
        "bbwadg_projection_npoints": (C.c_int, [vp, i32, pi64]),
        "bbwadg_projection_points": (C.c_int, [vp, i32, i64, i64, pd]),
        "bbwadg_project_samples": (C.c_int, [vp, i32, i64, i64, pd, pd]),
        "bbwadg_project_c2": (C.c_int, [vp, C2_CALLBACK, vp, vp, vp]),
        "bbwadg_set_c2": (C.c_int, [vp, pd]),
        "bbwadg_get_c2": (C.c_int, [vp, pd]),
        "bbwadg_rhs": (C.c_int, [vp, vp, vp, dbl, vp]),
        "bbwadg_step": (C.c_int, [vp, vp, vp, dbl, dbl, i32, vp]),
        "bbwadg_suggest_dt": (C.c_int, [vp, dbl, pd]),
        "bbwadg_l2norm2": (C.c_int, [vp, vp, pd, vp]),
        "bbwadg_l2norm2_noalloc": (C.c_int, [vp, vp, vp, vp]),
        "bbwadg_l2error2": (C.c_int, [vp, vp, i64, i64, vp, pd, vp]),
        "bbwadg_energy": (C.c_int, [vp, vp, i64, i64, pd, vp]),
        "bbwadg_project_fn": (C.c_int, [vp, C2_CALLBACK, vp, i32, vp, vp]),
        "bbwadg_coef_index": (C.c_int32, [i32, i32, i32]),
        "bbwadg_dense_npoints": (C.c_int, [vp, pi64]),
        "bbwadg_dense_points": (C.c_int, [vp, i64, i64, pd]),
        "bbwadg_dense_set_c2": (C.c_int, [vp, vp, vp]),
        "bbwadg_dense_update": (C.c_int, [vp, vp, vp, vp]),
        "bbwadg_rhs_dense": (C.c_int, [vp, vp, vp, dbl, vp]),
        "bbwadg_set_source": (C.c_int, [vp, vp, dbl, dbl, dbl]),
        "bbwadg_set_receivers": (C.c_int, [vp, i32, pd]),
        "bbwadg_receiver_elements": (C.c_int, [vp, C.POINTER(C.c_int32)]),
        "bbwadg_misfit_gradient": (C.c_int, [vp, vp, dbl, dbl, i32, vp, i32, vp, pd, vp, vp]),
        "bbwadg_adjoint_apply": (C.c_int, [vp, vp, vp, vp]),
        "bbwadg_elastic_set_media": (C.c_int, [vp, pd, pd, pd]),
        "bbwadg_elastic_update": (C.c_int, [vp, vp, vp, vp]),
        "bbwadg_elastic_rhs": (C.c_int, [vp, vp, vp, i32, dbl, dbl, i32, vp]),
        "bbwadg_elastic_step": (C.c_int, [vp, vp, vp, dbl, i32, i32, dbl, dbl, vp]),
        "bbwadg_wadg_update": (C.c_int, [vp, vp, vp, vp]),
        "bbwadg_set_c2_policy": (C.c_int, [vp, i32]),
        "bbwadg_c2_positivity": (C.c_int, [vp, pi64, pi64]),
        "bbwadg_bernstein_positivity": (C.c_int, [i32, i64, pd, pi64, pi64, pi64]),
        "bbwadg_sur_create": (C.c_int, [i32, i32, i32, C.c_uint64, C.POINTER(vp)]),
        "bbwadg_sur_destroy": (C.c_int, [vp]),
        "bbwadg_sur_num_params": (C.c_int64, [vp]),
        "bbwadg_sur_layout": (C.c_int, [vp, i32, C.POINTER(C.c_int32)]),
        "bbwadg_sur_get_params": (C.c_int, [vp, vp]),
        "bbwadg_sur_set_params": (C.c_int, [vp, vp]),
        "bbwadg_sur_forward": (C.c_int, [vp, vp, i32, vp, vp]),
        "bbwadg_sur_loss_grad": (C.c_int, [vp, vp, vp, i32, pd, vp, vp]),
        "bbwadg_sur_train_step": (C.c_int, [vp, vp, vp, i32, C.c_float, pd, vp]),
        "bbwadg_sur_input_grad": (C.c_int, [vp, vp, vp, i32, pd, vp, vp]),
        "bbwadg_projection_coefficients": (C.c_int, [i32, i32, pd]),
        "bbwadg_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise BBWADGError(rc, _lib.bbwadg_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def dimp(n: int) -> int:
    return (n + 1) * (n + 2) * (n + 3) // 6


def coef_index(a1: int, a2: int, a3: int) -> int:
    """Position of the coefficient of multi-index (n - a1 - a2 - a3, a1, a2, a3)."""
    lib = load_library()
    i = lib.bbwadg_coef_index(a1, a2, a3)
    if i < 0:
        _check(i)
    return i


def projection_coefficients(N: int, M: int) -> np.ndarray:
    """c_j of the telescoped projection (M >= 0) or of the inverse mass matrix (M = -1)."""
    lib = load_library()
    out = np.zeros(N + 1)
    _check(lib.bbwadg_projection_coefficients(N, M, _dptr(out)))
    return out


def bernstein_positivity(degree: int, coef) -> tuple:
    """(not positive, undecided, first such set or -1) over sets of degree-`degree` Bernstein
    coefficients [n, dimp(degree)] (bbwadg_bernstein_positivity)."""
    lib = load_library()
    c = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1, dimp(degree))
    a, b, f = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib.bbwadg_bernstein_positivity(int(degree), c.shape[0], _dptr(c), C.byref(a), C.byref(b), C.byref(f)))
    return a.value, b.value, f.value


class Solver:
    """BBWADG acoustic solver on an affine tetrahedral mesh (one context of the library)."""

    def __init__(self, xyz, etov, N: int, M: int, dtype: str = "f64", tau_p: float = 1.0,
                 tau_u: float = 1.0, bc: str = "p0", host_only: bool = False):
        self._lib = load_library()
        self._ctx = C.c_void_p()
        if not host_only:
            # torch owns the device buffers and streams: initialise its runtime first
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("a HIP device is needed (use host_only=True for setup-only contexts)")
            torch.cuda.current_device()
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self._etov = np.ascontiguousarray(etov, dtype=np.int32)
        if self._xyz.ndim != 2 or self._xyz.shape[1] != 3 or self._etov.ndim != 2 or self._etov.shape[1] != 4:
            raise ValueError("xyz must be [Nv, 3] and etov [K, 4]")
        mesh = _Mesh(self._xyz.shape[0], _dptr(self._xyz), self._etov.shape[0],
                     self._etov.ctypes.data_as(C.POINTER(C.c_int32)),
                     {"p0": BC_P0, "rigid": BC_RIGID}[bc])
        if dtype not in ("f64", "f32"):
            raise ValueError("dtype must be 'f64' or 'f32'")
        opts = _Opts(N, M, F64 if dtype == "f64" else F32, HOST_ONLY if host_only else DEVICE,
                     float(tau_p), float(tau_u))
        _check(self._lib.bbwadg_create(C.byref(mesh), C.byref(opts), C.byref(self._ctx)))
        self.N, self.M, self.dtype, self.bc = N, M, dtype, bc
        self.host_only = host_only
        np_, nfp, mp, K = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        _check(self._lib.bbwadg_sizes(self._ctx, C.byref(np_), C.byref(nfp), C.byref(mp), C.byref(K)))
        self.Np, self.Nfp, self.Mp, self.K = np_.value, nfp.value, mp.value, K.value

    # ---------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.bbwadg_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ----------------------------------------------------------------- queries
    def element_vertices(self) -> np.ndarray:
        out = np.empty((self.K, 4), dtype=np.int32)
        _check(self._lib.bbwadg_element_vertices(self._ctx, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def geometry(self) -> dict:
        K = self.K
        J, G = np.empty(K), np.empty((K, 3, 3))
        nrm, fs = np.empty((K, 4, 3)), np.empty((K, 4))
        nbr = np.empty((K, 4), dtype=np.int32)
        _check(self._lib.bbwadg_geometry(self._ctx, _dptr(J), _dptr(G), _dptr(nrm), _dptr(fs),
                                         nbr.ctypes.data_as(C.POINTER(C.c_int32))))
        return {"J": J, "G": G, "normal": nrm, "Fscale": fs, "nbr": nbr}

    # ------------------------------------------------------------- projections
    def projection_npoints(self, degree: int) -> int:
        n = C.c_int64()
        _check(self._lib.bbwadg_projection_npoints(self._ctx, degree, C.byref(n)))
        return n.value

    def projection_points(self, degree: int, k0: int = 0, k1: int | None = None) -> np.ndarray:
        k1 = self.K if k1 is None else k1
        nq = self.projection_npoints(degree)
        out = np.empty((k1 - k0, nq, 3))
        _check(self._lib.bbwadg_projection_points(self._ctx, degree, k0, k1, _dptr(out)))
        return out

    def project_samples(self, degree: int, samples, k0: int = 0, k1: int | None = None) -> np.ndarray:
        k1 = self.K if k1 is None else k1
        s = np.ascontiguousarray(samples, dtype=np.float64)
        nq = self.projection_npoints(degree)
        if s.shape != (k1 - k0, nq):
            raise ValueError(f"samples must be [{k1 - k0}, {nq}]")
        out = np.empty((k1 - k0, dimp(degree)))
        _check(self._lib.bbwadg_project_samples(self._ctx, degree, k0, k1, _dptr(s), _dptr(out)))
        return out

    def project_function(self, fn, degree: int, chunk: int = 8192) -> np.ndarray:
        """Per-element L^2 projection of a vectorised f(x, y, z) onto degree `degree`
        (host FP64); returns Bernstein coefficients [K, dimp(degree)]."""
        out = np.empty((self.K, dimp(degree)))
        for k0 in range(0, self.K, chunk):
            k1 = min(self.K, k0 + chunk)
            X = self.projection_points(degree, k0, k1)
            vals = np.asarray(fn(X[..., 0], X[..., 1], X[..., 2]), dtype=np.float64)
            out[k0:k1] = self.project_samples(degree, np.broadcast_to(vals, X.shape[:2]), k0, k1)
        return out

    def project_c2(self, fn) -> np.ndarray:
        """c^2_M: per-element projection of c^2 onto P^M, stored in the context."""
        coef = self.project_function(fn, self.M)
        self.set_c2(coef)
        return coef

    def project_c2_callback(self, fn_scalar, c2_out=None):
        """The C-callback entry point (fn_scalar(x, y, z) -> float); optional device copy."""
        cb = C2_CALLBACK(lambda x, y, z, u: float(fn_scalar(x, y, z)))
        ptr = None if c2_out is None else C.c_void_p(c2_out.data_ptr())
        stream = None if c2_out is None else self._stream()
        _check(self._lib.bbwadg_project_c2(self._ctx, cb, None, ptr, stream))

    def project_fn_callback(self, fn_scalar, field: int, q_out):
        """The C-callback projection of one state field (fn_scalar(x, y, z) -> float) into
        field `field` of the device state q_out."""
        self._check_state(q_out, "q_out")
        cb = C2_CALLBACK(lambda x, y, z, u: float(fn_scalar(x, y, z)))
        _check(self._lib.bbwadg_project_fn(self._ctx, cb, None, int(field), C.c_void_p(q_out.data_ptr()),
                                           self._stream()))
        return q_out

    def set_c2(self, coef):
        c = np.ascontiguousarray(coef, dtype=np.float64)
        if c.shape != (self.K, self.Mp):
            raise ValueError(f"c2 coefficients must be [{self.K}, {self.Mp}]")
        _check(self._lib.bbwadg_set_c2(self._ctx, _dptr(c)))

    def set_c2_policy(self, accept_nonpositive: bool):
        """Accept a c^2_M (or elastic medium) that is not positive everywhere (True), or reject
        it with EC2 (False, the default)."""
        _check(self._lib.bbwadg_set_c2_policy(self._ctx, 1 if accept_nonpositive else 0))

    def c2_positivity(self) -> tuple:
        """(elements where the stored c^2_M takes a value <= 0, elements left undecided)."""
        a, b = C.c_int64(), C.c_int64()
        _check(self._lib.bbwadg_c2_positivity(self._ctx, C.byref(a), C.byref(b)))
        return a.value, b.value

    def get_c2(self) -> np.ndarray:
        out = np.empty((self.K, self.Mp))
        _check(self._lib.bbwadg_get_c2(self._ctx, _dptr(out)))
        return out

    def initial_state(self, fns) -> np.ndarray:
        """Host FP64 Bernstein coefficients [4, K, Np] of four functions (p, u, v, w)."""
        return np.stack([self.project_function(f, self.N) for f in fns])

    def set_source(self, g=None, amp: float = 1.0, omega: float = 0.0, phase: float = 0.0):
        """Pressure source f = amp sin(omega t + phase) g(x): g is a vectorised function (projected
        onto P^N here) or Bernstein coefficients [K, Np]; None removes the source."""
        if g is None:
            _check(self._lib.bbwadg_set_source(self._ctx, None, 0.0, 0.0, 0.0))
            return None
        coef = self.project_function(g, self.N) if callable(g) else np.ascontiguousarray(g, dtype=np.float64)
        if coef.shape != (self.K, self.Np):
            raise ValueError(f"source coefficients must be [{self.K}, {self.Np}]")
        _check(self._lib.bbwadg_set_source(self._ctx, C.c_void_p(coef.ctypes.data), float(amp), float(omega),
                                           float(phase)))
        return coef

    # ------------------------------------------------------------ receivers, misfit, gradient
    def set_receivers(self, pts):
        """Receivers at physical points [nrec, 3] (pressure sampled after every step)."""
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        _check(self._lib.bbwadg_set_receivers(self._ctx, len(pts), _dptr(pts)))
        self.nrec = len(pts)

    def receiver_elements(self) -> np.ndarray:
        out = np.empty(getattr(self, "nrec", 0), dtype=np.int32)
        _check(self._lib.bbwadg_receiver_elements(self._ctx, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def misfit_gradient(self, q0, dt: float, nsteps: int, data=None, checkpoint_every: int = 50, t0: float = 0.0,
                        gradient: bool = True):
        """Misfit J = 1/2 sum (p(x_r, t_n) - data[n, r])^2 of nsteps LSRK4 steps from q0, the
        traces [nsteps, nrec] (device FP64) and, with ``gradient``, dJ/dc [K, Mp] (device FP64)."""
        import torch
        self._check_state(q0, "q0")
        nrec = getattr(self, "nrec", 0)
        traces = torch.empty((nsteps, nrec), dtype=torch.float64, device="cuda")
        dptr = None
        if data is not None:
            data = torch.as_tensor(data, dtype=torch.float64, device="cuda").contiguous()
            if tuple(data.shape) != (nsteps, nrec):
                raise ValueError(f"data must be [{nsteps}, {nrec}]")
            dptr = C.c_void_p(data.data_ptr())
        grad = torch.empty((self.K, self.Mp), dtype=torch.float64, device="cuda") if gradient else None
        J = C.c_double()
        _check(self._lib.bbwadg_misfit_gradient(self._ctx, C.c_void_p(q0.data_ptr()), float(t0), float(dt), int(nsteps),
                                                dptr, int(checkpoint_every), C.c_void_p(traces.data_ptr()),
                                                C.byref(J), C.c_void_p(grad.data_ptr()) if gradient else None,
                                                self._stream()))
        return J.value, grad, traces

    def adjoint_apply(self, z, out=None):
        """out = B(W z): the transposed operator in the mass-weighted, velocity-reflected variables."""
        self._check_state(z, "z")
        if out is None:
            out = self.empty_state()
        self._check_state(out, "out")
        _check(self._lib.bbwadg_adjoint_apply(self._ctx, C.c_void_p(z.data_ptr()), C.c_void_p(out.data_ptr()),
                                              self._stream()))
        return out

    def wadg_update(self, r, out=None):
        """out = Pi_N(c^2_M r) for one field r [K, Np] (device, context dtype)."""
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        for t, name in ((r, "r"), (out, "out")):
            if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != want or
                                  tuple(t.shape) != (self.K, self.Np) or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous device {want} tensor of shape ({self.K}, {self.Np})")
        if out is None:
            out = torch.empty_like(r)
        _check(self._lib.bbwadg_wadg_update(self._ctx, C.c_void_p(r.data_ptr()), C.c_void_p(out.data_ptr()),
                                            self._stream()))
        return out

    # ------------------------------------------------------------------ elastic update
    def elastic_set_media(self, rho_inv, lam, mu):
        """Isotropic media as degree-M Bernstein coefficients [K, Mp] (or vectorised functions,
        projected onto P^M here) of 1/rho, lambda and mu."""
        arrs = []
        for f in (rho_inv, lam, mu):
            a = self.project_function(f, self.M) if callable(f) else np.ascontiguousarray(f, dtype=np.float64)
            if a.shape != (self.K, self.Mp):
                raise ValueError(f"media coefficients must be [{self.K}, {self.Mp}]")
            arrs.append(a)
        _check(self._lib.bbwadg_elastic_set_media(self._ctx, *[_dptr(a) for a in arrs]))
        return arrs

    def elastic_update(self, r, out=None):
        """Weight-adjusted update of the 9 elastic fields r [9, K, Np] (device)."""
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        for t, name in ((r, "r"), (out, "out")):
            if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != want or
                                  tuple(t.shape) != (9, self.K, self.Np) or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous device {want} tensor of shape (9, {self.K}, {self.Np})")
        if out is None:
            out = torch.empty_like(r)
        _check(self._lib.bbwadg_elastic_update(self._ctx, C.c_void_p(r.data_ptr()), C.c_void_p(out.data_ptr()),
                                               self._stream()))
        return out

    def elastic_rhs(self, q, out=None, wall: str = "free", tau_v: float = 1.0, tau_s: float = 1.0,
                    weighted: bool = True):
        """Elastic DG right-hand side of q [9, K, Np] (device); weighted=True applies the
        weight-adjusted update of the media set by elastic_set_media."""
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        for t, name in ((q, "q"), (out, "out")):
            if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != want or
                                  tuple(t.shape) != (9, self.K, self.Np) or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous device {want} tensor of shape (9, {self.K}, {self.Np})")
        if wall not in ("free", "rigid"):
            raise ValueError("wall must be 'free' or 'rigid'")
        if out is None:
            out = torch.empty_like(q)
        _check(self._lib.bbwadg_elastic_rhs(self._ctx, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()),
                                            0 if wall == "free" else 1, float(tau_v), float(tau_s),
                                            1 if weighted else 0, self._stream()))
        return out

    def elastic_step(self, q, res, dt: float, nsteps: int, wall: str = "free", tau_v: float = 1.0,
                     tau_s: float = 1.0):
        """Advance the elastic state q [9, K, Np] (device, in place) by nsteps low-storage RK4
        steps; res is the 2N-storage register (zero for a fresh run)."""
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        for t, name in ((q, "q"), (res, "res")):
            if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != want or
                    tuple(t.shape) != (9, self.K, self.Np) or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous device {want} tensor of shape (9, {self.K}, {self.Np})")
        if wall not in ("free", "rigid"):
            raise ValueError("wall must be 'free' or 'rigid'")
        _check(self._lib.bbwadg_elastic_step(self._ctx, C.c_void_p(q.data_ptr()), C.c_void_p(res.data_ptr()),
                                             float(dt), int(nsteps), 0 if wall == "free" else 1, float(tau_v),
                                             float(tau_s), self._stream()))
        return q, res

    def suggest_dt(self, cfl: float) -> float:
        dt = C.c_double()
        _check(self._lib.bbwadg_suggest_dt(self._ctx, float(cfl), C.byref(dt)))
        return dt.value

    # ---------------------------------------------------------------- hot path
    def _stream(self):
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _check_state(self, t, name):
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if t.dtype != want or tuple(t.shape) != (4, self.K, self.Np) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {want} tensor of shape (4, {self.K}, {self.Np})")

    def empty_state(self):
        import torch
        return torch.zeros((4, self.K, self.Np), dtype=torch.float64 if self.dtype == "f64" else torch.float32,
                           device="cuda")

    def to_device(self, arr):
        import torch
        return torch.as_tensor(np.ascontiguousarray(arr), device="cuda").to(
            torch.float64 if self.dtype == "f64" else torch.float32).contiguous()

    def rhs(self, q, out=None, t: float = 0.0):
        self._check_state(q, "q")
        if out is None:
            out = self.empty_state()
        self._check_state(out, "out")
        _check(self._lib.bbwadg_rhs(self._ctx, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()),
                                    float(t), self._stream()))
        return out

    def step(self, q, res, dt: float, nsteps: int = 1, t0: float = 0.0):
        self._check_state(q, "q")
        self._check_state(res, "res")
        _check(self._lib.bbwadg_step(self._ctx, C.c_void_p(q.data_ptr()), C.c_void_p(res.data_ptr()),
                                     float(t0), float(dt), int(nsteps), self._stream()))
        return q

    def l2norm2(self, q) -> np.ndarray:
        self._check_state(q, "q")
        out = np.zeros(4)
        _check(self._lib.bbwadg_l2norm2(self._ctx, C.c_void_p(q.data_ptr()), _dptr(out), self._stream()))
        return out

    def l2norm2_noalloc(self, q, out=None):
        """bbwadg_l2norm2_noalloc: the squared norms into a device double[4] tensor, with no
        allocation and no synchronisation in the library (out is allocated here if None)."""
        import torch
        self._check_state(q, "q")
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=q.device)
        if out.dtype != torch.float64 or out.numel() < 4 or not out.is_contiguous() or out.device != q.device:
            raise ValueError("out must be a contiguous float64 device tensor of 4 values")
        _check(self._lib.bbwadg_l2norm2_noalloc(self._ctx, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()),
                                                self._stream()))
        return out

    def l2error2(self, q, fns, k0: int = 0, k1: int | None = None, chunk: int = 16384) -> np.ndarray:
        """Per-field squared L^2 error of q against four vectorised functions f(x, y, z),
        over elements [k0, k1); the reference values are sampled on the host at the
        library's rule points and handed over in pieces of `chunk` elements."""
        import torch
        self._check_state(q, "q")
        k1 = self.K if k1 is None else k1
        total = np.zeros(4)
        out = np.zeros(4)
        for a in range(k0, k1, chunk):
            b = min(k1, a + chunk)
            X = self.projection_points(self.N, a, b)
            ex = np.stack([np.broadcast_to(np.asarray(f(X[..., 0], X[..., 1], X[..., 2]), dtype=np.float64),
                                           X.shape[:2]) for f in fns])
            d = torch.as_tensor(np.ascontiguousarray(ex), device="cuda")
            _check(self._lib.bbwadg_l2error2(self._ctx, C.c_void_p(q.data_ptr()), a, b, C.c_void_p(d.data_ptr()),
                                             _dptr(out), self._stream()))
            total += out
        return total

    def l2error2_samples(self, q, exact, k0: int = 0, k1: int | None = None) -> np.ndarray:
        """As l2error2, with the reference values already on the device: FP64 [4, k1-k0, nq]."""
        import torch
        self._check_state(q, "q")
        k1 = self.K if k1 is None else k1
        nq = self.projection_npoints(self.N)
        if (not isinstance(exact, torch.Tensor) or not exact.is_cuda or exact.dtype != torch.float64
                or tuple(exact.shape) != (4, k1 - k0, nq) or not exact.is_contiguous()):
            raise ValueError(f"exact must be a contiguous float64 device tensor of shape (4, {k1 - k0}, {nq})")
        out = np.zeros(4)
        _check(self._lib.bbwadg_l2error2(self._ctx, C.c_void_p(q.data_ptr()), k0, k1, C.c_void_p(exact.data_ptr()),
                                         _dptr(out), self._stream()))
        return out

    def energy(self, q, k0: int = 0, k1: int | None = None) -> np.ndarray:
        """Acoustic energy terms [p^2/c^2, u^2, v^2, w^2] (each with the factor 1/2) over
        elements [k0, k1); the energy is their sum."""
        self._check_state(q, "q")
        k1 = self.K if k1 is None else k1
        out = np.zeros(4)
        _check(self._lib.bbwadg_energy(self._ctx, C.c_void_p(q.data_ptr()), k0, k1, _dptr(out), self._stream()))
        return out

    # ------------------------------------------------- dense quadrature WADG (baseline)
    def dense_npoints(self) -> int:
        n = C.c_int64()
        _check(self._lib.bbwadg_dense_npoints(self._ctx, C.byref(n)))
        return n.value

    def dense_points(self, k0: int = 0, k1: int | None = None) -> np.ndarray:
        k1 = self.K if k1 is None else k1
        out = np.empty((k1 - k0, self.dense_npoints(), 3))
        _check(self._lib.bbwadg_dense_points(self._ctx, k0, k1, _dptr(out)))
        return out

    def dense_set_c2(self, fn=None, chunk: int = 8192):
        """c^2 at the dense points: None evaluates the stored c^2_M; a vectorised fn(x, y, z)
        gives the quadrature WADG of the true wavespeed."""
        if fn is None:
            _check(self._lib.bbwadg_dense_set_c2(self._ctx, None, self._stream()))
            return
        nq = self.dense_npoints()
        vals = np.empty((self.K, nq))
        for a in range(0, self.K, chunk):
            b = min(self.K, a + chunk)
            X = self.dense_points(a, b)
            vals[a:b] = np.broadcast_to(np.asarray(fn(X[..., 0], X[..., 1], X[..., 2]), dtype=np.float64), X.shape[:2])
        _check(self._lib.bbwadg_dense_set_c2(self._ctx, C.c_void_p(vals.ctypes.data), self._stream()))

    def dense_update(self, r, out=None):
        """out[k] = P_q diag(c^2) V_q r[k] for device arrays of shape (K, Np) of the context dtype."""
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        if out is None:
            out = torch.empty_like(r)
        for t, name in ((r, "r"), (out, "out")):
            if not (t.is_cuda and t.dtype == want and tuple(t.shape) == (self.K, self.Np) and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous {want} device tensor of shape ({self.K}, {self.Np})")
        _check(self._lib.bbwadg_dense_update(self._ctx, C.c_void_p(r.data_ptr()), C.c_void_p(out.data_ptr()),
                                             self._stream()))
        return out

    def rhs_dense(self, q, out=None, t: float = 0.0):
        self._check_state(q, "q")
        if out is None:
            out = self.empty_state()
        self._check_state(out, "out")
        _check(self._lib.bbwadg_rhs_dense(self._ctx, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()),
                                          float(t), self._stream()))
        return out
