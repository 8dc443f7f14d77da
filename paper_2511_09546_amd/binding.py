"""ctypes binding of libipeps.so (argument marshalling only).

Mirrors include/ipeps.h: the same entry points, host numpy arrays in C order,
status codes turned into exceptions (``IpepsError``), warnings returned.
Every computation runs in the library; when the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libipeps.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, ENOMEM, EHIP, ECG_BREAKDOWN, ESTATE, ENOTIMPL = -1, -2, -3, -4, -5, -6
ESCRATCH = -7
# size of the fixed scratch array of precond_apply_dev_noalloc (per GPU)
NOALLOC_SCRATCH_BYTES = 192 << 20
FP64, FP32, BF16, BF16X1 = 0, 1, 2, 3
GRAD_FULL, GRAD_K, GRAD_FP = 0, 1, 2

# every function declared in include/ipeps.h (checked by the CPU tests)
API_FUNCTIONS = [
    "ipeps_default_opts", "ctm_init", "ctm_set_state", "ctm_converge",
    "ipeps_energy_grad", "precond_apply", "ipeps_corner_spectra",
    "ipeps_get_env", "ipeps_set_env", "ipeps_env_size", "ctm_free",
    "ipeps_get_env_dev", "ipeps_set_env_dev", "bp_converge",
    "ipeps_bp_messages", "precond_apply_bp", "precond_apply_bp_dev",
    "ipeps_strerror", "ipeps_version", "ipeps_profile_enable",
    "ipeps_profile_read", "ctm_set_state_dev", "ipeps_energy_grad_dev",
    "precond_apply_dev", "ipeps_footprint_bytes", "ipeps_release_cache",
    "precond_apply_dev_noalloc", "precond_noalloc_bytes",
    "ipeps_lbfgs_default_params", "ipeps_lbfgs_create", "ipeps_lbfgs_step",
    "ipeps_lbfgs_free", "ipeps_get_state", "precond_apply_gmres",
    "precond_apply_gmres_dev", "log_norm_grad", "metric_full_apply",
    "metric_full_apply_dev", "precond_apply_full", "precond_apply_full_dev",
    "c4v_block_size", "c4v_converge", "c4v_energy_grad",
    "c4v_energy_grad_dev", "c4v_get_env", "c4v_set_env",
]
PROF_GEMM, PROF_JACOBI, PROF_PERMUTE, PROF_GEMM32, PROF_GEMM16 = 0, 1, 2, 3, 4
PROF_NET = 5  # GEMMs of the network contractions (subset of 0, 3, 4)
PROF_WIDE = 6  # the 128 x 144-tile FP32 GEMM (chi^2 D^8 products; subset of 3)
DEBUG_FUNCTIONS = ["ipeps_debug_gemm", "ipeps_debug_sym_eig",
                   "ipeps_debug_svd_ts", "ipeps_debug_stats",
                   "ipeps_debug_gemm_prec", "ipeps_debug_gemm_time",
                   "ipeps_debug_permute", "ipeps_debug_set_fault",
                   "ipeps_debug_einsum", "ipeps_debug_memcheck"]


class IpepsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")


class Term(ctypes.Structure):
    _fields_ = [("kind", c_int), ("site", c_int), ("dx", c_int),
                ("dy", c_int), ("coef", c_double), ("mat", POINTER(c_double))]


class Opts(ctypes.Structure):
    _fields_ = [("prec", c_int), ("svd_cutoff", c_double), ("grad_K", c_int),
                ("svd_oversample", c_int), ("svd_max_iter", c_int),
                ("svd_tol", c_double), ("grad_mode", c_int),
                ("adj_tol", c_double), ("grad_checkpoint", c_int),
                ("adj_cg_tol", c_double), ("ladder", c_int)]


_lib = None
_DP = POINTER(c_double)
_IP = POINTER(c_int)


def load():
    """Load libipeps.so (once).  Raises ImportError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run __graft_entry__.build() "
            "(or python -m paper_2511_09546_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.ipeps_default_opts.argtypes = [POINTER(Opts)]
    lib.ipeps_default_opts.restype = None
    lib.ctm_init.argtypes = [POINTER(c_void_p), c_int, c_int, c_int, c_int,
                             c_int, _DP, POINTER(Opts), c_void_p]
    lib.ctm_set_state.argtypes = [c_void_p, _DP]
    lib.ctm_converge.argtypes = [c_void_p, c_double, c_int, _IP, _DP]
    lib.ipeps_energy_grad.argtypes = [c_void_p, c_int, POINTER(Term), _DP,
                                      _DP]
    lib.precond_apply.argtypes = [c_void_p, _DP, c_double, c_double, c_int,
                                  _DP, _IP, _DP]
    lib.ipeps_corner_spectra.argtypes = [c_void_p, _DP]
    lib.ipeps_get_env.argtypes = [c_void_p, _DP]
    lib.ipeps_set_env.argtypes = [c_void_p, _DP]
    lib.ipeps_get_env_dev.argtypes = [c_void_p, c_void_p]
    lib.ipeps_get_env_dev.restype = c_int
    lib.bp_converge.argtypes = [c_void_p, c_double, c_int, _IP, _DP]
    lib.bp_converge.restype = c_int
    lib.ipeps_bp_messages.argtypes = [c_void_p, _DP]
    lib.ipeps_bp_messages.restype = c_int
    lib.precond_apply_bp.argtypes = [c_void_p, _DP, c_double, _DP]
    lib.precond_apply_bp.restype = c_int
    lib.precond_apply_bp_dev.argtypes = [c_void_p, c_void_p, c_double,
                                         c_void_p]
    lib.precond_apply_bp_dev.restype = c_int
    lib.ipeps_set_env_dev.argtypes = [c_void_p, c_void_p]
    lib.precond_apply_gmres.argtypes = [c_void_p, _DP, c_double, c_int,
                                        c_double, _DP, _IP, _DP]
    lib.precond_apply_gmres_dev.argtypes = [c_void_p, c_void_p, c_double,
                                            c_int, c_double, c_void_p, _IP,
                                            _DP]
    lib.log_norm_grad.argtypes = [c_void_p, _DP, _DP, _DP]
    lib.metric_full_apply.argtypes = [c_void_p, _DP, c_double, _DP]
    lib.metric_full_apply_dev.argtypes = [c_void_p, c_void_p, c_double,
                                          c_void_p]
    lib.precond_apply_full.argtypes = [c_void_p, _DP, c_double, c_int,
                                       c_double, c_double, _DP, _IP, _DP]
    lib.precond_apply_full_dev.argtypes = [c_void_p, c_void_p, c_double,
                                           c_int, c_double, c_double,
                                           c_void_p, _IP, _DP]
    lib.c4v_block_size.argtypes = [c_int]
    lib.c4v_converge.argtypes = [c_void_p, c_double, c_int, _IP, _DP]
    lib.c4v_energy_grad.argtypes = [c_void_p, c_int, POINTER(Term), _DP,
                                    _DP]
    lib.c4v_energy_grad_dev.argtypes = [c_void_p, c_int, POINTER(Term), _DP,
                                        c_void_p]
    lib.c4v_get_env.argtypes = [c_void_p, _DP, _DP, _DP, _IP]
    lib.c4v_set_env.argtypes = [c_void_p, _DP, _DP, _DP]
    for name in ("c4v_block_size", "c4v_converge", "c4v_energy_grad",
                 "c4v_energy_grad_dev", "c4v_get_env", "c4v_set_env"):
        getattr(lib, name).restype = c_int
    for name in ("precond_apply_gmres", "precond_apply_gmres_dev",
                 "log_norm_grad", "metric_full_apply",
                 "metric_full_apply_dev", "precond_apply_full",
                 "precond_apply_full_dev"):
        getattr(lib, name).restype = c_int
    lib.ipeps_set_env_dev.restype = c_int
    lib.ipeps_env_size.argtypes = [c_int, c_int, c_int, c_int]
    lib.ipeps_env_size.restype = c_size_t
    lib.ipeps_footprint_bytes.argtypes = [c_int, c_int, c_int, c_int, c_int,
                                          c_void_p]
    lib.ipeps_footprint_bytes.restype = c_size_t
    lib.ipeps_release_cache.argtypes = [c_size_t, POINTER(c_size_t)]
    lib.ipeps_release_cache.restype = c_int
    lib.ctm_free.argtypes = [c_void_p]
    lib.ctm_free.restype = None
    lib.ipeps_strerror.argtypes = [c_int]
    lib.ipeps_strerror.restype = ctypes.c_char_p
    lib.ipeps_version.restype = ctypes.c_char_p
    lib.ctm_set_state_dev.argtypes = [c_void_p, c_void_p]
    lib.ipeps_energy_grad_dev.argtypes = [c_void_p, c_int, POINTER(Term),
                                          _DP, c_void_p]
    lib.precond_apply_dev.argtypes = [c_void_p, c_void_p, c_double,
                                      c_double, c_int, c_void_p, _IP, _DP]
    lib.precond_apply_dev_noalloc.argtypes = [c_void_p, c_void_p, c_double,
                                              c_double, c_int, c_void_p, _IP,
                                              _DP]
    lib.precond_apply_dev_noalloc.restype = c_int
    lib.precond_noalloc_bytes.argtypes = [c_int, c_int, c_int, c_int, c_int]
    lib.precond_noalloc_bytes.restype = c_size_t
    lib.ipeps_profile_enable.argtypes = [c_void_p, c_int]
    lib.ipeps_profile_read.argtypes = [c_void_p, c_int,
                                       POINTER(ctypes.c_long), _DP, _DP, _DP]
    lib.ipeps_debug_gemm.argtypes = [c_int, c_int, c_int, c_int, c_int,
                                     c_double, _DP, _DP, c_double, _DP]
    lib.ipeps_debug_gemm_prec.argtypes = [c_int, c_int, c_int, c_int, c_int,
                                          c_int, c_double, _DP, _DP,
                                          c_double, _DP]
    lib.ipeps_debug_gemm_time.argtypes = [c_int, c_int, c_int, c_int, c_int,
                                          c_int, c_int, c_int, _DP]
    lib.ipeps_debug_sym_eig.argtypes = [c_int, c_int, _DP, _DP, _DP]
    lib.ipeps_debug_permute.argtypes = [c_int, POINTER(ctypes.c_long),
                                        _IP, c_double, _DP, c_double, _DP]
    lib.ipeps_debug_einsum.argtypes = [
        ctypes.c_char_p, c_int, c_int, c_int, c_int, POINTER(ctypes.c_long),
        _DP, c_int, POINTER(ctypes.c_long), _DP, c_double, c_double, _DP,
        _IP]
    lib.ipeps_debug_stats.argtypes = [c_void_p, _DP]
    lib.ipeps_debug_set_fault.argtypes = [c_void_p, c_int, c_double]
    lib.ipeps_debug_memcheck.argtypes = [c_void_p, POINTER(ctypes.c_long)]
    lib.ipeps_debug_svd_ts.argtypes = [c_int, c_int, c_int, _DP, _DP, _DP,
                                       _DP]
    for name in ("ctm_init", "ctm_set_state", "ctm_converge",
                 "ipeps_energy_grad", "precond_apply", "ipeps_corner_spectra",
                 "ipeps_get_env", "ipeps_set_env", "ipeps_debug_gemm",
                 "ipeps_profile_enable", "ipeps_profile_read",
                 "ctm_set_state_dev", "ipeps_energy_grad_dev",
                 "precond_apply_dev",
                 "ipeps_debug_sym_eig", "ipeps_debug_svd_ts",
                 "ipeps_debug_stats", "ipeps_debug_gemm_prec",
                 "ipeps_debug_gemm_time", "ipeps_debug_permute",
                 "ipeps_debug_set_fault", "ipeps_debug_einsum",
                 "ipeps_debug_memcheck"):
        getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().ipeps_strerror(status).decode()


def c4v_block_size(chi: int) -> int:
    """Columns of the C4v subspace-iteration block for this chi."""
    return load().c4v_block_size(chi)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def default_opts() -> Opts:
    o = Opts()
    load().ipeps_default_opts(ctypes.byref(o))
    return o


def noalloc_bytes(Lx, Ly, d, D, chi) -> int:
    """Scratch bytes of precond_apply_dev_noalloc (precond_noalloc_bytes)."""
    return int(load().precond_noalloc_bytes(Lx, Ly, d, D, chi))


def footprint_bytes(Lx, Ly, d, D, chi, opts=None) -> int:
    """Peak device bytes of one context (ipeps_footprint_bytes)."""
    return int(load().ipeps_footprint_bytes(
        Lx, Ly, d, D, chi, ctypes.byref(opts) if opts is not None else None))


def release_cache(keep_bytes: int = 0) -> int:
    """Returns the device memory of destroyed contexts cached in this
    process to HIP down to keep_bytes (ipeps_release_cache); returns the
    bytes still cached."""
    left = c_size_t(0)
    st = load().ipeps_release_cache(int(keep_bytes), ctypes.byref(left))
    if st != OK:
        raise IpepsError(st, "ipeps_release_cache")
    return int(left.value)


def make_terms(terms):
    """(kind, site, dx, dy, coef, mat) tuples -> (ctypes array, keepalive)."""
    mats = [_f64(t[5]) for t in terms]
    arr = (Term * max(1, len(terms)))()
    for i, (t, m) in enumerate(zip(terms, mats)):
        arr[i] = Term(int(t[0]), int(t[1]), int(t[2]), int(t[3]),
                      float(t[4]), _dp(m))
    return arr, mats


class Context:
    """One iPEPS state with its environment on the device."""

    def __init__(self, A, chi: int, opts: Opts | None = None, stream=None):
        lib = load()
        A = _f64(A)
        if A.ndim != 7:
            raise ValueError("A must be [Ly, Lx, d, D, D, D, D]")
        self.Ly, self.Lx, self.d, self.D = A.shape[:4]
        self.chi = chi
        self.shape = A.shape
        h = c_void_p()
        st = lib.ctm_init(ctypes.byref(h), self.Lx, self.Ly, self.d, self.D,
                          chi, _dp(A), ctypes.byref(opts) if opts else None,
                          c_void_p(stream) if stream else None)
        if st != OK:
            raise IpepsError(st, "ctm_init")
        self._h = h
        self.last_status = OK

    def close(self):
        if getattr(self, "_h", None):
            load().ctm_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_state(self, A):
        A = _f64(A)
        if A.shape != self.shape:
            raise ValueError("shape mismatch")
        st = load().ctm_set_state(self._h, _dp(A))
        if st != OK:
            raise IpepsError(st, "ctm_set_state")

    def converge(self, tol: float, max_iter: int):
        """Returns (n_iter, delta, converged)."""
        n = c_int(0)
        dl = c_double(0.0)
        st = load().ctm_converge(self._h, tol, max_iter, ctypes.byref(n),
                                 ctypes.byref(dl))
        if st < 0:
            raise IpepsError(st, "ctm_converge")
        self.last_status = st
        return n.value, dl.value, st == OK

    def energy_grad(self, terms, grad: bool = True):
        arr, keep = make_terms(terms)
        e = c_double(0.0)
        g = np.zeros(self.shape) if grad else None
        st = load().ipeps_energy_grad(self._h, len(terms), arr,
                                      ctypes.byref(e),
                                      _dp(g) if grad else None)
        del keep
        if st < 0:
            raise IpepsError(st, "ipeps_energy_grad")
        self.last_status = st  # NOT_CONVERGED: a solver hit its limit
        return e.value, g

    def precond(self, g, delta: float, cg_tol: float, cg_maxiter: int):
        """Returns (x, n_iter, rel_resid, breakdown)."""
        g = _f64(g)
        x = np.zeros(self.shape)
        n = c_int(0)
        rr = c_double(0.0)
        st = load().precond_apply(self._h, _dp(g), delta, cg_tol, cg_maxiter,
                                  _dp(x), ctypes.byref(n), ctypes.byref(rr))
        if st < 0 and st != ECG_BREAKDOWN:
            raise IpepsError(st, "precond_apply")
        return x, n.value, rr.value, st == ECG_BREAKDOWN

    # ---- device-pointer twins: arguments are device addresses (int) of
    # FP64 buffers in the layout of A (e.g. torch_tensor.data_ptr())
    def set_state_dev(self, d_A: int):
        st = load().ctm_set_state_dev(self._h, c_void_p(d_A))
        if st != OK:
            raise IpepsError(st, "ctm_set_state_dev")

    def energy_grad_dev(self, terms, d_grad: int) -> float:
        arr, keep = make_terms(terms)
        e = c_double(0.0)
        st = load().ipeps_energy_grad_dev(self._h, len(terms), arr,
                                          ctypes.byref(e), c_void_p(d_grad))
        del keep
        if st < 0:
            raise IpepsError(st, "ipeps_energy_grad_dev")
        self.last_status = st
        return e.value

    def precond_dev(self, d_g: int, d_x: int, delta: float, cg_tol: float,
                    cg_maxiter: int):
        """Returns (n_iter, rel_resid, breakdown)."""
        n = c_int(0)
        rr = c_double(0.0)
        st = load().precond_apply_dev(self._h, c_void_p(d_g), delta, cg_tol,
                                      cg_maxiter, c_void_p(d_x),
                                      ctypes.byref(n), ctypes.byref(rr))
        if st < 0 and st != ECG_BREAKDOWN:
            raise IpepsError(st, "precond_apply_dev")
        return n.value, rr.value, st == ECG_BREAKDOWN

    def precond_dev_noalloc(self, d_g: int, d_x: int, delta: float,
                            cg_tol: float, cg_maxiter: int):
        """precond_apply_dev_noalloc: (n_iter, rel_resid, breakdown)."""
        n = c_int(0)
        rr = c_double(0.0)
        st = load().precond_apply_dev_noalloc(
            self._h, c_void_p(d_g), delta, cg_tol, cg_maxiter, c_void_p(d_x),
            ctypes.byref(n), ctypes.byref(rr))
        if st < 0 and st != ECG_BREAKDOWN:
            raise IpepsError(st, "precond_apply_dev_noalloc")
        return n.value, rr.value, st == ECG_BREAKDOWN

    def spectra(self) -> np.ndarray:
        out = np.zeros((4, self.Lx * self.Ly, self.chi))
        st = load().ipeps_corner_spectra(self._h, _dp(out))
        if st != OK:
            raise IpepsError(st, "ipeps_corner_spectra")
        return out

    def env_size(self) -> int:
        return int(load().ipeps_env_size(self.Lx, self.Ly, self.D, self.chi))

    def get_env(self):
        """(C[4][n][chi][chi], T[4][n][chi][D^2][chi])"""
        buf = np.zeros(self.env_size())
        st = load().ipeps_get_env(self._h, _dp(buf))
        if st != OK:
            raise IpepsError(st, "ipeps_get_env")
        n, chi, D2 = self.Lx * self.Ly, self.chi, self.D * self.D
        nc = 4 * n * chi * chi
        return (buf[:nc].reshape(4, n, chi, chi),
                buf[nc:].reshape(4, n, chi, D2, chi))

    def profile(self, on: bool):
        st = load().ipeps_profile_enable(self._h, int(on))
        if st != OK:
            raise IpepsError(st, "ipeps_profile_enable")

    def profile_read(self, family: int):
        """(launches, seconds, flop, bytes) of one kernel family."""
        n = ctypes.c_long(0)
        sec, fl, by = c_double(0), c_double(0), c_double(0)
        st = load().ipeps_profile_read(self._h, family, ctypes.byref(n),
                                       ctypes.byref(sec), ctypes.byref(fl),
                                       ctypes.byref(by))
        if st != OK:
            raise IpepsError(st, "ipeps_profile_read")
        return n.value, sec.value, fl.value, by.value

    def memcheck(self) -> int:
        """Damaged guard bands of a context created with IPEPS_MEMCHECK set
        (ipeps_debug_memcheck; -1 without the check)."""
        n = ctypes.c_long(0)
        st = load().ipeps_debug_memcheck(self._h, ctypes.byref(n))
        if st != OK:
            raise IpepsError(st, "ipeps_debug_memcheck")
        return n.value

    def stats(self) -> dict:
        out = np.zeros(12)
        st = load().ipeps_debug_stats(self._h, _dp(out))
        if st != OK:
            raise IpepsError(st, "ipeps_debug_stats")
        return dict(svd_iters=int(out[0]), svd_calls=int(out[1]),
                    svd_worst_residual=float(out[2]), cg_iters=int(out[3]),
                    cg_solves=int(out[4]), pool_bytes=int(out[5]),
                    peak_live_bytes=int(out[6]), grad_K_used=int(out[7]),
                    svd_unconverged=int(out[8]), cg_unconverged=int(out[9]),
                    work_prec=int(out[10]), cg_true_residual=float(out[11]))

    def set_fault(self, kind: int, value: float = 0.0):
        """Failure injection (ipeps_debug_set_fault): 0 clear, 1 memory
        budget in bytes, 2 CG breakdown before iteration `value`."""
        st = load().ipeps_debug_set_fault(self._h, int(kind), float(value))
        if st != OK:
            raise IpepsError(st, "ipeps_debug_set_fault")

    def set_env(self, C, T):
        buf = np.concatenate([_f64(C).ravel(), _f64(T).ravel()])
        if buf.size != self.env_size():
            raise ValueError("environment size mismatch")
        st = load().ipeps_set_env(self._h, _dp(buf))
        if st != OK:
            raise IpepsError(st, "ipeps_set_env")

    # ---- belief-propagation (chi = 1) preconditioner
    def bp_converge(self, tol: float = 1e-12, max_iter: int = 500):
        """Returns (updates, last change, converged)."""
        n = c_int(0)
        ch = c_double(0.0)
        st = load().bp_converge(self._h, tol, max_iter, ctypes.byref(n),
                                ctypes.byref(ch))
        if st < 0:
            raise IpepsError(st, "bp_converge")
        return n.value, ch.value, st == OK

    def bp_messages(self) -> np.ndarray:
        """[Lx*Ly][4][D][D]: messages into the left, up, right, down legs."""
        out = np.zeros((self.Lx * self.Ly, 4, self.D, self.D))
        st = load().ipeps_bp_messages(self._h, _dp(out))
        if st != OK:
            raise IpepsError(st, "ipeps_bp_messages")
        return out

    def precond_bp(self, g, delta: float) -> np.ndarray:
        g = _f64(g)
        x = np.zeros(self.shape)
        st = load().precond_apply_bp(self._h, _dp(g), delta, _dp(x))
        if st != OK:
            raise IpepsError(st, "precond_apply_bp")
        return x

    # ---- C4v ansatz and QR-CTMRG (1x1 cells)
    def c4v_converge(self, tol: float, max_iter: int):
        """QR-CTMRG of the projected state: (n_iter, delta, converged)."""
        n = c_int(0)
        dl = c_double(0.0)
        st = load().c4v_converge(self._h, tol, max_iter, ctypes.byref(n),
                                 ctypes.byref(dl))
        if st < 0:
            raise IpepsError(st, "c4v_converge")
        return n.value, dl.value, st == OK

    def c4v_energy_grad(self, terms, grad: bool = True):
        arr, keep = make_terms(terms)
        e = c_double(0.0)
        g = np.zeros(self.shape) if grad else None
        st = load().c4v_energy_grad(self._h, len(terms), arr,
                                    ctypes.byref(e),
                                    _dp(g) if grad else None)
        del keep
        if st != OK:
            raise IpepsError(st, "c4v_energy_grad")
        return e.value, g

    def c4v_energy_grad_dev(self, terms, d_grad: int) -> float:
        arr, keep = make_terms(terms)
        e = c_double(0.0)
        st = load().c4v_energy_grad_dev(self._h, len(terms), arr,
                                        ctypes.byref(e), c_void_p(d_grad))
        del keep
        if st != OK:
            raise IpepsError(st, "c4v_energy_grad_dev")
        return e.value

    def c4v_get_env(self):
        """(C [chi][chi], T [chi][D^2][chi], V [chi D^2][b], bond)."""
        chi, D2 = self.chi, self.D * self.D
        b = c4v_block_size(chi)
        C = np.zeros((chi, chi))
        T = np.zeros((chi, D2, chi))
        V = np.zeros((chi * D2, b))
        bond = c_int(0)
        st = load().c4v_get_env(self._h, _dp(C), _dp(T), _dp(V),
                                ctypes.byref(bond))
        if st != OK:
            raise IpepsError(st, "c4v_get_env")
        return C, T, V, bond.value

    def c4v_set_env(self, C, T, V=None):
        chi, D2 = self.chi, self.D * self.D
        C = _f64(C).reshape(chi, chi)
        T = _f64(T).reshape(chi, D2, chi)
        if V is not None:
            V = _f64(V).reshape(chi * D2, c4v_block_size(chi))
        st = load().c4v_set_env(self._h, _dp(C), _dp(T),
                                _dp(V) if V is not None else None)
        if st != OK:
            raise IpepsError(st, "c4v_set_env")

    # ---- GMRES solves and the full metric (1x1 cells)
    def precond_gmres(self, g, delta: float, m: int = 30, tol: float = 0.0):
        """(N_local + delta)^-1 g by one GMRES cycle: (x, n_used, resid)."""
        g = _f64(g).reshape(self.shape)
        x = np.zeros(self.shape)
        n = c_int(0)
        rr = c_double(0.0)
        st = load().precond_apply_gmres(self._h, _dp(g), delta, m, tol,
                                        _dp(x), ctypes.byref(n),
                                        ctypes.byref(rr))
        if st != OK:
            raise IpepsError(st, "precond_apply_gmres")
        return x, n.value, rr.value

    def precond_gmres_dev(self, d_g: int, d_x: int, delta: float,
                          m: int = 30, tol: float = 0.0):
        n = c_int(0)
        rr = c_double(0.0)
        st = load().precond_apply_gmres_dev(self._h, c_void_p(d_g), delta, m,
                                            tol, c_void_p(d_x),
                                            ctypes.byref(n), ctypes.byref(rr))
        if st != OK:
            raise IpepsError(st, "precond_apply_gmres_dev")
        return n.value, rr.value

    def log_norm_grad(self, A_ket=None, grad: bool = True):
        """(F, dF/dA_bra) of the per-site log-norm at (A_ket, A)."""
        F = c_double(0.0)
        ak = (_f64(A_ket).reshape(self.shape) if A_ket is not None
              else None)
        g = np.zeros(self.shape) if grad else None
        st = load().log_norm_grad(self._h, _dp(ak) if ak is not None else None,
                                  ctypes.byref(F), _dp(g) if grad else None)
        if st != OK:
            raise IpepsError(st, "log_norm_grad")
        return F.value, g

    def metric_full(self, B, rel_step: float = 0.0) -> np.ndarray:
        B = _f64(B).reshape(self.shape)
        y = np.zeros(self.shape)
        st = load().metric_full_apply(self._h, _dp(B), rel_step, _dp(y))
        if st != OK:
            raise IpepsError(st, "metric_full_apply")
        return y

    def metric_full_dev(self, d_B: int, d_NB: int, rel_step: float = 0.0):
        st = load().metric_full_apply_dev(self._h, c_void_p(d_B), rel_step,
                                          c_void_p(d_NB))
        if st != OK:
            raise IpepsError(st, "metric_full_apply_dev")

    def precond_full(self, g, delta: float, m: int = 30, tol: float = 0.0,
                     rel_step: float = 0.0):
        """(N + delta)^-1 g, N the full metric: (x, n_used, resid)."""
        g = _f64(g).reshape(self.shape)
        x = np.zeros(self.shape)
        n = c_int(0)
        rr = c_double(0.0)
        st = load().precond_apply_full(self._h, _dp(g), delta, m, tol,
                                       rel_step, _dp(x), ctypes.byref(n),
                                       ctypes.byref(rr))
        if st != OK:
            raise IpepsError(st, "precond_apply_full")
        return x, n.value, rr.value

    def precond_full_dev(self, d_g: int, d_x: int, delta: float, m: int = 30,
                         tol: float = 0.0, rel_step: float = 0.0):
        n = c_int(0)
        rr = c_double(0.0)
        st = load().precond_apply_full_dev(self._h, c_void_p(d_g), delta, m,
                                           tol, rel_step, c_void_p(d_x),
                                           ctypes.byref(n), ctypes.byref(rr))
        if st != OK:
            raise IpepsError(st, "precond_apply_full_dev")
        return n.value, rr.value

    def precond_bp_dev(self, d_g: int, d_x: int, delta: float):
        st = load().precond_apply_bp_dev(self._h, c_void_p(d_g), delta,
                                         c_void_p(d_x))
        if st != OK:
            raise IpepsError(st, "precond_apply_bp_dev")

    def get_env_dev(self, d_out: int):
        """Environment into a device buffer of env_size() doubles."""
        st = load().ipeps_get_env_dev(self._h, c_void_p(d_out))
        if st != OK:
            raise IpepsError(st, "ipeps_get_env_dev")

    def set_env_dev(self, d_in: int):
        """Environment from a device buffer of env_size() doubles."""
        st = load().ipeps_set_env_dev(self._h, c_void_p(d_in))
        if st != OK:
            raise IpepsError(st, "ipeps_set_env_dev")


# ------------------------------------------------------------- test hooks
def debug_gemm(A, B, C, tA=False, tB=False, alpha=1.0, beta=0.0):
    A, B, C = _f64(A), _f64(B), _f64(C).copy()
    M, K = (A.shape[1], A.shape[0]) if tA else A.shape
    N = B.shape[0] if tB else B.shape[1]
    st = load().ipeps_debug_gemm(int(tA), int(tB), M, N, K, alpha, _dp(A),
                                 _dp(B), beta, _dp(C))
    if st != OK:
        raise IpepsError(st, "ipeps_debug_gemm")
    return C


def debug_gemm_prec(prec, A, B, C, tA=False, tB=False, alpha=1.0,
                    beta=0.0):
    A, B, C = _f64(A), _f64(B), _f64(C).copy()
    M, K = (A.shape[1], A.shape[0]) if tA else A.shape
    N = B.shape[0] if tB else B.shape[1]
    st = load().ipeps_debug_gemm_prec(int(prec), int(tA), int(tB), M, N, K,
                                      alpha, _dp(A), _dp(B), beta, _dp(C))
    if st != OK:
        raise IpepsError(st, "ipeps_debug_gemm_prec")
    return C


def debug_gemm_time(prec, tA, tB, M, N, K, batch=1, reps=20):
    """Average device microseconds of one GEMM call."""
    us = ctypes.c_double(0.0)
    st = load().ipeps_debug_gemm_time(int(prec), int(tA), int(tB), M, N, K,
                                      batch, reps, ctypes.byref(us))
    if st != OK:
        raise IpepsError(st, "ipeps_debug_gemm_time")
    return us.value


def debug_sym_eig(G):
    G = _f64(G)
    batch, b = G.shape[0], G.shape[1]
    V = np.zeros_like(G)
    lam = np.zeros((batch, b))
    st = load().ipeps_debug_sym_eig(b, batch, _dp(G), _dp(V), _dp(lam))
    if st != OK:
        raise IpepsError(st, "ipeps_debug_sym_eig")
    return lam, V


def debug_permute(X, perm, alpha=1.0, beta=0.0, out=None):
    """alpha X.transpose(perm) + beta out by the library's permute kernels."""
    X = _f64(X)
    r = X.ndim
    perm = [int(p) for p in perm]
    oshape = tuple(X.shape[p] for p in perm)
    out = np.zeros(oshape) if out is None else _f64(out).copy()
    sh = (ctypes.c_long * r)(*X.shape)
    pm = np.ascontiguousarray(perm, dtype=np.int32)
    st = load().ipeps_debug_permute(r, sh, pm.ctypes.data_as(_IP), alpha,
                                    _dp(X), beta, _dp(out))
    if st != OK:
        raise IpepsError(st, "ipeps_debug_permute")
    return out


def debug_einsum(spec, A, B, out, prec=0, mode=0, alpha=1.0, beta=0.0):
    """alpha einsum(spec, A[i], B[i]) + beta out[i] for the items i of the
    leading axis of A, B, out, by the library's contraction planner (one
    batched launch).  Returns (result, number of launches whose GEMM wrote
    the permuted output from its epilogue)."""
    A, B = _f64(A), _f64(B)
    out = _f64(out).copy()
    n = A.shape[0]
    sa = (ctypes.c_long * (A.ndim - 1))(*A.shape[1:])
    sb = (ctypes.c_long * (B.ndim - 1))(*B.shape[1:])
    sc = c_int(0)
    st = load().ipeps_debug_einsum(spec.encode(), prec, mode, n, A.ndim - 1,
                                   sa, _dp(A), B.ndim - 1, sb, _dp(B), alpha,
                                   beta, _dp(out), ctypes.byref(sc))
    if st != OK:
        raise IpepsError(st, "ipeps_debug_einsum")
    return out, sc.value


def debug_svd_ts(W):
    W = _f64(W)
    batch, n, b = W.shape
    U = np.zeros_like(W)
    s = np.zeros((batch, b))
    J = np.zeros((batch, b, b))
    st = load().ipeps_debug_svd_ts(n, b, batch, _dp(W), _dp(U), _dp(s),
                                   _dp(J))
    if st != OK:
        raise IpepsError(st, "ipeps_debug_svd_ts")
    return U, s, J


# ------------------------------------------------------------ optimiser
class LbfgsParams(ctypes.Structure):
    _fields_ = [("m", c_int), ("precondition", c_int), ("delta_mode", c_int),
                ("delta0", c_double), ("delta_min", c_double),
                ("delta_max", c_double), ("ctm_tol", c_double),
                ("ctm_max_iter", c_int), ("cg_tol", c_double),
                ("cg_maxiter", c_int), ("max_evals", c_int),
                ("psi0", c_double), ("hz_delta", c_double),
                ("hz_sigma", c_double), ("hz_eps", c_double),
                ("hz_theta", c_double), ("hz_gamma", c_double),
                ("hz_rho", c_double), ("gmres_m", c_int),
                ("fd_step", c_double)]


# ipeps_lbfgs_params.precondition
PRECOND_NONE, PRECOND_LOCAL, PRECOND_BP = 0, 1, 2
PRECOND_LOCAL_GMRES, PRECOND_FULL_GMRES = 3, 4


class LbfgsInfo(ctypes.Structure):
    _fields_ = [("e", c_double), ("alpha", c_double), ("n_evals", c_int),
                ("ls_ok", c_int), ("gnorm", c_double), ("delta", c_double),
                ("ctm_iters", c_int)]


STATIONARY = 2


def _load_lbfgs(lib):
    if getattr(lib, "_lbfgs_ready", False):
        return lib
    lib.ipeps_lbfgs_default_params.argtypes = [POINTER(LbfgsParams)]
    lib.ipeps_lbfgs_default_params.restype = None
    lib.ipeps_lbfgs_create.argtypes = [c_void_p, c_int, POINTER(Term),
                                       POINTER(LbfgsParams),
                                       POINTER(c_void_p), _DP]
    lib.ipeps_lbfgs_create.restype = c_int
    lib.ipeps_lbfgs_step.argtypes = [c_void_p, POINTER(LbfgsInfo)]
    lib.ipeps_lbfgs_step.restype = c_int
    lib.ipeps_lbfgs_free.argtypes = [c_void_p]
    lib.ipeps_lbfgs_free.restype = None
    lib.ipeps_get_state.argtypes = [c_void_p, _DP]
    lib.ipeps_get_state.restype = c_int
    lib._lbfgs_ready = True
    return lib


def lbfgs_default_params() -> LbfgsParams:
    p = LbfgsParams()
    _load_lbfgs(load()).ipeps_lbfgs_default_params(ctypes.byref(p))
    return p


def get_state(ctx: "Context") -> np.ndarray:
    A = np.zeros(ctx.shape)
    st = _load_lbfgs(load()).ipeps_get_state(ctx._h, _dp(A))
    if st != OK:
        raise IpepsError(st, "ipeps_get_state")
    return A


class Lbfgs:
    """Preconditioned L-BFGS on a context's state (ipeps_lbfgs_*)."""

    def __init__(self, ctx: "Context", terms, params: LbfgsParams = None):
        lib = _load_lbfgs(load())
        self._arr, self._keep = make_terms(terms)
        self.ctx = ctx
        h = c_void_p()
        e0 = c_double(0.0)
        st = lib.ipeps_lbfgs_create(ctx._h, len(terms), self._arr,
                                    ctypes.byref(params) if params else None,
                                    ctypes.byref(h), ctypes.byref(e0))
        if st < 0:
            raise IpepsError(st, "ipeps_lbfgs_create")
        self._h = h
        self.e0 = e0.value
        self.last_status = st

    def step(self) -> dict:
        info = LbfgsInfo()
        st = load().ipeps_lbfgs_step(self._h, ctypes.byref(info))
        if st < 0:
            raise IpepsError(st, "ipeps_lbfgs_step")
        self.last_status = st
        return dict(e=info.e, alpha=info.alpha, n_evals=info.n_evals,
                    ls_ok=bool(info.ls_ok), gnorm=info.gnorm,
                    delta=info.delta, ctm_iters=info.ctm_iters, status=st)

    def close(self):
        if getattr(self, "_h", None):
            load().ipeps_lbfgs_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
