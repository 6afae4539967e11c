"""ctypes binding of libsynchem (include/synchem.h).  Argument marshalling only: torch tensors
supply device memory and the current HIP stream; every step of the EM iteration runs in the HIP
library.  There is no fallback: without the built library every entry point raises."""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynchem.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "synchem.h")

EM_OK, EM_EINVAL, EM_ENOMEM, EM_EDEVICE, EM_ESTATE, EM_ENONFINITE, EM_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "EM_OK", -1: "EM_EINVAL", -2: "EM_ENOMEM", -3: "EM_EDEVICE",
                -4: "EM_ESTATE", -5: "EM_ENONFINITE", -6: "EM_EUNSUPPORTED"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16": 3, "bf16": 4}
EM_FLAG_KEEP_LSE, EM_FLAG_TIMING, EM_FLAG_GENERAL_PASS, EM_FLAG_WIDE_PASS = 1, 2, 4, 8
EM_FLAG_STAGED_PASS = 32
EM_FLAG_FACTORED = 16
EM_STATS_FIELDS = 6
STATS_COLUMNS = ("t", "loglik", "objective", "delta_a2", "stop_metric", "entropy_rho")


class EmParams(C.Structure):
    _fields_ = [("n_obs", C.c_int64), ("K", C.c_int32), ("Q", C.c_int32), ("L", C.c_int32),
                ("window_lo", C.c_int32), ("window_count", C.c_int32),
                ("sigma2", C.c_double), ("gamma", C.c_double),
                ("update_rho", C.c_int32), ("precision", C.c_int32), ("flags", C.c_uint64),
                ("gamma_a_inv", C.POINTER(C.c_double)), ("a0", C.POINTER(C.c_double)),
                ("angles", C.POINTER(C.c_double))]


class EmInfo(C.Structure):
    _fields_ = [("rows_per_tile", C.c_int32), ("grid", C.c_int32), ("threads", C.c_int32),
                ("window_padded", C.c_int32), ("bytes_per_row", C.c_int64),
                ("lds_bytes", C.c_int64), ("kernel", C.c_char * 64)]


class SynchemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def load() -> C.CDLL:
    """Load libsynchem.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2105_07372_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, vp, i32, i64, dbl = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "em_init": (i32, [P(vp), P(EmParams), vp, P(dbl), vp]),
        "em_step": (i32, [vp, i32, dbl, P(i32), P(dbl)]),
        "em_loglik": (i32, [vp, P(dbl)]),
        "em_posterior": (i32, [vp, i64, i64, vp, vp, vp]),
        "em_get_state": (i32, [vp, P(dbl), P(dbl), P(i64)]),
        "em_set_state": (i32, [vp, P(dbl), P(dbl), i64]),
        "em_loglik_fwd": (i32, [vp, vp, dbl, vp, P(dbl)]),
        "em_loglik_bwd": (i32, [vp, dbl, vp, P(dbl), vp]),
        "em_get_stats": (i32, [vp, P(dbl), i32, P(i32)]),
        "em_learn_prior": (i32, [vp, i64, i32, i32, i32, P(dbl), P(i64), P(i64), vp]),
        "em_relative_rotations": (i32, [vp, i64, i32, i32, i32, vp, vp, vp, vp]),
        "em_ppm": (i32, [vp, i64, i32, i32, vp, vp]),
        "em_nearest": (i32, [vp, i64, i32, i32, i64, vp, vp, vp]),
        "em_sync_match": (i32, [vp, i64, i32, i32, i32, i64, i32, vp, vp, vp]),
        "em_align": (i32, [vp, i64, i32, i32, vp, vp, vp]),
        "em_aligned_mean": (i32, [vp, i64, i32, i32, vp, vp, vp]),
        "em_aligned_mean_noalloc": (i32, [vp, i64, i32, i32, vp, vp, vp]),
        "em_error_bins": (i32, [vp, vp, i64, i32, i32, vp, vp]),
        "em_set_stream": (i32, [vp, vp]),
        "em_pass_time": (i32, [vp, P(dbl), P(i64), i32]),
        "em_get_info": (i32, [vp, P(EmInfo)]),
        "em_destroy": (None, [vp]),
        "em_last_error": (C.c_char_p, [vp]),
        "em_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def header_symbols() -> list[str]:
    """Function names declared in include/synchem.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:em_status|void|const char \*)\s*(em_\w+)\s*\(", text,
                                 flags=re.M)))


def _check(st: int, ctx=None):
    if st != EM_OK:
        msg = load().em_last_error(ctx)
        raise SynchemError(st, msg.decode() if msg else "")


def _dptr(arr) -> C.POINTER(C.c_double):
    return arr.ctypes.data_as(C.POINTER(C.c_double))


def _stream_handle(stream=None) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class EM:
    """One EM problem resident on the GPU (a thin owner of an em_ctx)."""

    def __init__(self, obs, *, K: int, Q: int, L: int, sigma2: float,
                 window: Optional[tuple[int, int]] = None, prior=None, gamma: float = 0.0,
                 update_rho: bool = True, precision: str = "fp32", gamma_a_inv=None, a0=None,
                 keep_lse: bool = False, timing: bool = False, general_pass: bool = False,
                 wide_pass: bool = False, factored: bool = False, angles=None,
                 staged_pass: bool = False, stream=None):
        import torch
        lib = load()
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        want = torch.complex128 if precision == "fp64" else torch.complex64
        if not (isinstance(obs, torch.Tensor) and obs.is_cuda and obs.dtype == want
                and obs.dim() == 2 and obs.is_contiguous() and obs.shape[1] == K * Q):
            raise ValueError(f"obs must be a contiguous CUDA {want} tensor of shape (N, {K * Q})")
        if angles is not None:
            angles = np.ascontiguousarray(angles, dtype=np.float64).ravel()
            if window is not None and tuple(window) != (0, len(angles)):
                raise ValueError("with angles, window must be None or (0, len(angles))")
            window = (0, len(angles))
        lo, W = (0, L) if window is None else window
        self.K, self.Q, self.D, self.L, self.lo, self.W = K, Q, K * Q, L, lo, W
        self.N = int(obs.shape[0])
        self.precision = precision
        self._stream = _stream_handle(stream)
        p = EmParams()
        p.n_obs, p.K, p.Q, p.L, p.window_lo, p.window_count = self.N, K, Q, L, lo, W
        p.sigma2, p.gamma = float(sigma2), float(gamma)
        p.update_rho, p.precision = int(bool(update_rho)), PRECISIONS[precision]
        p.flags = ((EM_FLAG_KEEP_LSE if keep_lse else 0) | (EM_FLAG_TIMING if timing else 0)
                   | (EM_FLAG_GENERAL_PASS if general_pass else 0)
                   | (EM_FLAG_WIDE_PASS if wide_pass else 0)
                   | (EM_FLAG_FACTORED if factored else 0)
                   | (EM_FLAG_STAGED_PASS if staged_pass else 0))
        keep = []
        if gamma_a_inv is not None:
            g = np.ascontiguousarray(gamma_a_inv, dtype=np.float64)
            keep.append(g)
            p.gamma_a_inv = _dptr(g)
        if a0 is not None:
            a = np.ascontiguousarray(np.asarray(a0, dtype=np.complex128)).view(np.float64)
            keep.append(a)
            p.a0 = _dptr(a)
        if angles is not None:
            keep.append(angles)
            p.angles = _dptr(angles)
        pr = None
        if prior is not None:
            pr = np.ascontiguousarray(prior, dtype=np.float64)
        self.sigma2 = float(sigma2)
        ctx = C.c_void_p()
        st = lib.em_init(C.byref(ctx), C.byref(p), C.c_void_p(obs.data_ptr()),
                         _dptr(pr) if pr is not None else None, C.c_void_p(self._stream))
        _check(st, None)
        self._ctx = ctx
        self._keep_lse = bool(keep_lse)
        # bumped whenever the library's adjoint checkpoint stops matching the last loglik_fwd
        # (a new forward, an EM step that stores its own LSE, a state reset): MarginalLogLik's
        # backward then runs its forward again
        self._fwd_gen = 0

    # -- lifecycle
    def close(self):
        if getattr(self, "_ctx", None):
            load().em_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self):
        if not self._ctx:
            raise RuntimeError("EM context is closed")
        return self._ctx

    def set_stream(self, stream=None):
        self._stream = _stream_handle(stream)
        _check(load().em_set_stream(self._c(), C.c_void_p(self._stream)), self._ctx)

    # -- EM
    def step(self, n: int = 1, tol: float = 0.0, sync: bool = True):
        """Run up to n iterations; returns (iterations done, log-likelihood of the last
        iteration's starting state) when sync, else (None, None) without waiting."""
        done, ll = C.c_int32(0), C.c_double(0.0)
        if self._keep_lse and n > 0:
            self._fwd_gen += 1
        if sync:
            _check(load().em_step(self._c(), int(n), float(tol), C.byref(done), C.byref(ll)),
                   self._ctx)
            return done.value, ll.value
        _check(load().em_step(self._c(), int(n), float(tol), None, None), self._ctx)
        return None, None

    def loglik(self) -> float:
        ll = C.c_double(0.0)
        _check(load().em_loglik(self._c(), C.byref(ll)), self._ctx)
        return ll.value

    def posterior(self, row0: int = 0, nrows: Optional[int] = None, weights: bool = True):
        """(w [nrows, W] float32 or None, argmax int32, margin float32) as CUDA tensors."""
        import torch
        nrows = self.N - row0 if nrows is None else nrows
        dev = torch.device("cuda", torch.cuda.current_device())
        w = torch.empty((nrows, self.W), dtype=torch.float32, device=dev) if weights else None
        am = torch.empty(nrows, dtype=torch.int32, device=dev)
        mg = torch.empty(nrows, dtype=torch.float32, device=dev)
        _check(load().em_posterior(self._c(), int(row0), int(nrows),
                                   C.c_void_p(w.data_ptr()) if w is not None else None,
                                   C.c_void_p(am.data_ptr()), C.c_void_p(mg.data_ptr())),
               self._ctx)
        return w, am, mg

    def state(self):
        a = np.zeros(2 * self.D)
        rho = np.zeros(self.W)
        t = C.c_int64(0)
        _check(load().em_get_state(self._c(), _dptr(a), _dptr(rho), C.byref(t)), self._ctx)
        return a.view(np.complex128).copy(), rho, t.value

    def set_state(self, a, rho=None, t: int = 0):
        av = np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)
        rv = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        self._fwd_gen += 1
        _check(load().em_set_state(self._c(), _dptr(av), _dptr(rv) if rv is not None else None,
                                   int(t)), self._ctx)

    def stats(self) -> np.ndarray:
        buf = np.zeros((1024, EM_STATS_FIELDS))
        n = C.c_int32(0)
        _check(load().em_get_stats(self._c(), _dptr(buf), 1024, C.byref(n)), self._ctx)
        return buf[:n.value].copy()

    def info(self) -> dict:
        inf = EmInfo()
        _check(load().em_get_info(self._c(), C.byref(inf)), self._ctx)
        return {"rows_per_tile": inf.rows_per_tile, "grid": inf.grid, "threads": inf.threads,
                "window_padded": inf.window_padded, "bytes_per_row": inf.bytes_per_row,
                "lds_bytes": inf.lds_bytes, "kernel": inf.kernel.decode()}

    def pass_time(self, reset: bool = False):
        ms, n = C.c_double(0.0), C.c_int64(0)
        _check(load().em_pass_time(self._c(), C.byref(ms), C.byref(n), int(bool(reset))),
               self._ctx)
        return ms.value, n.value

    # -- differentiable log-likelihood (used by MarginalLogLik)
    def loglik_fwd(self, a, sigma2: float, eta=None) -> float:
        import torch
        if not (a.is_cuda and a.dtype == torch.complex128 and a.is_contiguous()
                and a.numel() == self.D):
            raise ValueError("a must be a contiguous CUDA complex128 tensor of D entries")
        if eta is not None and not (eta.is_cuda and eta.dtype == torch.float64
                                    and eta.is_contiguous() and eta.numel() == self.W):
            raise ValueError("eta must be a contiguous CUDA float64 tensor of W entries")
        ll = C.c_double(0.0)
        _check(load().em_loglik_fwd(self._c(), C.c_void_p(a.data_ptr()), float(sigma2),
                                    C.c_void_p(eta.data_ptr()) if eta is not None else None,
                                    C.byref(ll)), self._ctx)
        self._fwd_gen += 1
        return ll.value

    def loglik_bwd(self, g: float, grad_a, grad_eta=None) -> float:
        gs = C.c_double(0.0)
        _check(load().em_loglik_bwd(self._c(), float(g), C.c_void_p(grad_a.data_ptr()),
                                    C.byref(gs),
                                    C.c_void_p(grad_eta.data_ptr()) if grad_eta is not None
                                    else None), self._ctx)
        return gs.value


def learn_prior(errors, L: int, lo: int, W: int, stream=None):
    """Histogram prior over the window from integer rotation errors on the GPU (int32 CUDA
    tensor).  Returns (rho_bar [W], counts [L] indexed by error mod L, draws inside the window)."""
    import torch
    if not (errors.is_cuda and errors.dtype == torch.int32 and errors.is_contiguous()):
        raise ValueError("errors must be a contiguous CUDA int32 tensor")
    rb = np.zeros(W)
    cnt = np.zeros(L, dtype=np.int64)
    nin = C.c_int64(0)
    st = load().em_learn_prior(C.c_void_p(errors.data_ptr()), int(errors.numel()), int(L),
                               int(lo), int(W), _dptr(rb),
                               cnt.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(nin),
                               C.c_void_p(_stream_handle(stream)))
    _check(st, None)
    return rb, cnt, nin.value


# ---- Synchronize and Match (the step before the EM path)

def _obs_c64(obs, K: int, Q: int):
    import torch
    if not (isinstance(obs, torch.Tensor) and obs.is_cuda and obs.dtype == torch.complex64
            and obs.dim() == 2 and obs.is_contiguous() and obs.shape[1] == K * Q):
        raise ValueError(f"obs must be a contiguous CUDA complex64 tensor of shape (N, {K * Q})")
    return C.c_void_p(obs.data_ptr())


def relative_rotations(obs, K: int, Q: int, L: int, P: Optional[int] = None, stream=None):
    """Relative rotations of all pairs of the first P rows of obs: (rel [P, P] int32, gap [P, P],
    dot [P, P]) as CUDA tensors (em_relative_rotations)."""
    import torch
    P = int(obs.shape[0]) if P is None else int(P)
    if not 2 <= P <= int(obs.shape[0]):
        raise ValueError("P must be in [2, number of rows of obs]")
    rel = torch.empty((P, P), dtype=torch.int32, device=obs.device)
    gap = torch.empty((P, P), dtype=torch.float32, device=obs.device)
    dot = torch.empty((P, P), dtype=torch.float32, device=obs.device)
    st = load().em_relative_rotations(_obs_c64(obs, K, Q), P, int(K), int(Q), int(L),
                                      C.c_void_p(rel.data_ptr()), C.c_void_p(gap.data_ptr()),
                                      C.c_void_p(dot.data_ptr()),
                                      C.c_void_p(_stream_handle(stream)))
    _check(st, None)
    return rel, gap, dot


def ppm(rel, L: int, iters: int, stream=None):
    """Projected power method on a [P, P] int32 CUDA tensor of relative rotations: theta [P]
    (float64 CUDA tensor, radians) (em_ppm)."""
    import torch
    if not (rel.is_cuda and rel.dtype == torch.int32 and rel.is_contiguous() and rel.dim() == 2
            and rel.shape[0] == rel.shape[1]):
        raise ValueError("rel must be a square contiguous CUDA int32 tensor")
    P = int(rel.shape[0])
    th = torch.empty(P, dtype=torch.float64, device=rel.device)
    st = load().em_ppm(C.c_void_p(rel.data_ptr()), P, int(L), int(iters),
                       C.c_void_p(th.data_ptr()), C.c_void_p(_stream_handle(stream)))
    _check(st, None)
    return th


def nearest(obs, K: int, Q: int, P: int, stream=None):
    """Nearest member of the first P rows for every row (itself excluded): (nn [N] int32, gap [N]
    float32) (em_nearest)."""
    import torch
    N = int(obs.shape[0])
    nn = torch.empty(N, dtype=torch.int32, device=obs.device)
    gap = torch.empty(N, dtype=torch.float32, device=obs.device)
    st = load().em_nearest(_obs_c64(obs, K, Q), N, int(K), int(Q), int(P),
                           C.c_void_p(nn.data_ptr()), C.c_void_p(gap.data_ptr()),
                           C.c_void_p(_stream_handle(stream)))
    _check(st, None)
    return nn, gap


def sync_match(obs, K: int, Q: int, L: int, P: int, iters: int = 50, stream=None):
    """Synchronize and Match: (theta [N] float64, nn [N] int32) CUDA tensors (em_sync_match)."""
    import torch
    N = int(obs.shape[0])
    th = torch.empty(N, dtype=torch.float64, device=obs.device)
    nn = torch.empty(N, dtype=torch.int32, device=obs.device)
    st = load().em_sync_match(_obs_c64(obs, K, Q), N, int(K), int(Q), int(L), int(P), int(iters),
                              C.c_void_p(th.data_ptr()), C.c_void_p(nn.data_ptr()),
                              C.c_void_p(_stream_handle(stream)))
    _check(st, None)
    return th, nn


def align(obs, K: int, Q: int, theta, stream=None):
    """Aligned observations v_i o exp(+i kbar theta_i) as a new complex64 CUDA tensor (em_align)."""
    import torch
    if not (theta.is_cuda and theta.dtype == torch.float64 and theta.is_contiguous()
            and theta.numel() == obs.shape[0]):
        raise ValueError("theta must be a contiguous CUDA float64 tensor with one entry per row")
    out = torch.empty_like(obs)
    st = load().em_align(_obs_c64(obs, K, Q), int(obs.shape[0]), int(K), int(Q),
                         C.c_void_p(theta.data_ptr()), C.c_void_p(out.data_ptr()),
                         C.c_void_p(_stream_handle(stream)))
    _check(st, None)
    return out


def aligned_mean(obs, K: int, Q: int, theta, stream=None, out=None, noalloc: bool = False):
    """(1/N) sum_i v_i o exp(+i kbar theta_i) as a complex128 CUDA tensor (em_aligned_mean).
    noalloc=True calls em_aligned_mean_noalloc (the library allocates nothing; the result is
    ready in stream order); out, if given, is a contiguous CUDA complex128 tensor of K*Q."""
    import torch
    if not (theta.is_cuda and theta.dtype == torch.float64 and theta.is_contiguous()
            and theta.numel() == obs.shape[0]):
        raise ValueError("theta must be a contiguous CUDA float64 tensor with one entry per row")
    if out is None:
        out = torch.empty(K * Q, dtype=torch.complex128, device=obs.device)
    elif not (out.is_cuda and out.dtype == torch.complex128 and out.is_contiguous()
              and out.numel() == K * Q):
        raise ValueError("out must be a contiguous CUDA complex128 tensor of K*Q entries")
    fn = load().em_aligned_mean_noalloc if noalloc else load().em_aligned_mean
    st = fn(_obs_c64(obs, K, Q), int(obs.shape[0]), int(K), int(Q),
            C.c_void_p(theta.data_ptr()), C.c_void_p(out.data_ptr()),
            C.c_void_p(_stream_handle(stream)))
    _check(st, None)
    return out


def error_bins(theta_hat, theta, L: int, lc: int, stream=None):
    """Binned centred errors floor((theta_hat - theta - 2 pi lc / L) L / 2 pi) mod L as an int32
    CUDA tensor (em_error_bins); feed them to learn_prior."""
    import torch
    for t in (theta_hat, theta):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("angles must be contiguous CUDA float64 tensors")
    if theta_hat.numel() != theta.numel():
        raise ValueError("theta_hat and theta must have the same length")
    bins = torch.empty(theta.numel(), dtype=torch.int32, device=theta.device)
    st = load().em_error_bins(C.c_void_p(theta_hat.data_ptr()), C.c_void_p(theta.data_ptr()),
                              int(theta.numel()), int(L), int(lc), C.c_void_p(bins.data_ptr()),
                              C.c_void_p(_stream_handle(stream)))
    _check(st, None)
    return bins


def global_rotation(x, abar, K: int, Q: int, L: int, stream=None) -> int:
    """The grid rotation l_c with R_{2 pi l_c / L} abar closest to x (the centring step of the
    algorithm that learns the rotation distribution): the relative rotation of the pair (x, abar)
    from em_relative_rotations (both complex CUDA vectors of length K*Q)."""
    import torch
    pair = torch.stack([x.to(torch.complex64), abar.to(torch.complex64)]).contiguous()
    rel, _, _ = relative_rotations(pair, K, Q, L, 2, stream=stream)
    return int(rel[0, 1].item())
