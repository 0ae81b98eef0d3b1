"""ctypes binding of the Block CUR C ABI (include/bcur.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device matrices are torch CUDA tensors (float32, row-major, 16-byte
aligned, leading dimension a multiple of 4); small host arrays are numpy.
Work is issued on torch's current stream.

The library must have been built (``python -m paper_1703_06065_amd.build``);
loading fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbcur.so")

OK, E_ARG, E_NONFINITE, E_NOMEM, E_HIP, E_RANKDEF, E_ADMIT, PENDING, E_STATE = range(9)
PREC_FP32, PREC_BF16 = 0, 1
FLAG_RANKDEF_C, FLAG_ILLCOND_C, FLAG_ZERO_SCORE, FLAG_RANKDEF_Y, FLAG_RANKDEF_R, FLAG_RANKDEF_W = 1, 2, 4, 8, 16, 32
FLAG_PINV_EIG = 64

# every symbol declared in include/bcur.h
SYMBOLS = [
    "bcur_create", "bcur_destroy", "bcur_synchronize", "bcur_status_str", "bcur_last_error",
    "bcur_workspace_bytes", "bcur_frob2", "bcur_range_finder", "bcur_block_scores", "bcur_sample_blocks",
    "bcur_gather_columns", "bcur_fit_columns", "bcur_decompose", "bcur_timing_enable", "bcur_timing_read",
    "bcur_sketch_pass", "bcur_release_workspace", "bcur_footprint", "bcur_server_create", "bcur_server_destroy",
    "bcur_server_submit", "bcur_server_poll", "bcur_server_wait", "bcur_server_stats", "bcur_decompose_alg1",
    "bcur_decompose_boost", "bcur_block_stable_rank", "bcur_incoherence", "bcur_decompose_alg1_boost",
    "bcur_test_matrix", "bcur_decompose_async", "bcur_wait", "bcur_decompose_noalloc",
]

STAGES = ["frob", "rf_AQ", "rf_AtZ", "rf_reduce", "rf_orth", "rf_rr", "scores", "sample", "gather", "fit_H",
          "fit_reduce", "fit_inv", "fit_U", "fit_E", "fit_F", "fit_dU", "rf_cast", "a1_rows", "a1_svdr", "a1_pinv",
          "a1_cu", "diag_alpha", "diag_mu"]


class BcurError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bcur status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("s", ctypes.c_int64), ("l", ctypes.c_int64), ("q", ctypes.c_int64),
                ("replace", ctypes.c_int32), ("precision", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("s_r", ctypes.c_int64), ("col_map", ctypes.POINTER(ctypes.c_int64)),
                ("row_map", ctypes.POINTER(ctypes.c_int64)), ("seed", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("idx", ctypes.POINTER(ctypes.c_int64)), ("weights", ctypes.POINTER(ctypes.c_double)),
                ("scores", ctypes.POINTER(ctypes.c_double)), ("ritz", ctypes.POINTER(ctypes.c_double)),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64), ("u_rows_cap", ctypes.c_int64),
                ("idx_r", ctypes.POINTER(ctypes.c_int64)), ("row_scores", ctypes.POINTER(ctypes.c_double)),
                ("c", ctypes.c_int64), ("r", ctypes.c_int64), ("frob2", ctypes.c_double), ("err", ctypes.c_double),
                ("rel_err", ctypes.c_double), ("min_margin", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("rr_sweeps", ctypes.c_uint32), ("kappa", ctypes.c_double), ("cond_c", ctypes.c_double)]


class Alg1Params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int64), ("kr", ctypes.c_int64), ("s", ctypes.c_int64), ("rank_k", ctypes.c_int64),
                ("replace", ctypes.c_int32), ("pinv_eig", ctypes.c_int32),
                ("col_map", ctypes.POINTER(ctypes.c_int64))]


class Alg1Result(ctypes.Structure):
    _fields_ = [("rows", ctypes.POINTER(ctypes.c_int64)), ("idx", ctypes.POINTER(ctypes.c_int64)),
                ("weights", ctypes.POINTER(ctypes.c_double)), ("scores", ctypes.POINTER(ctypes.c_double)),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
                ("u_rows_cap", ctypes.c_int64), ("c", ctypes.c_int64), ("rank_w", ctypes.c_int64),
                ("frob2", ctypes.c_double), ("err", ctypes.c_double), ("rel_err", ctypes.c_double),
                ("min_margin", ctypes.c_double), ("flags", ctypes.c_uint32), ("sweeps", ctypes.c_uint32)]


class Request(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("col_off", ctypes.POINTER(ctypes.c_int64)), ("G", ctypes.c_int64),
                ("row_off", ctypes.POINTER(ctypes.c_int64)), ("Gr", ctypes.c_int64), ("params", Params),
                ("omega", ctypes.c_void_p), ("draws", ctypes.POINTER(ctypes.c_uint64)), ("U", ctypes.c_void_p),
                ("ldu", ctypes.c_int64), ("u_rows_cap", ctypes.c_int64), ("stream", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("failed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("throughput", ctypes.c_double), ("hbm_held", ctypes.c_uint64),
                ("hbm_peak", ctypes.c_uint64), ("peak_running", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libbcur.so and declare the signatures of every exported call."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1703_06065_amd.build`")
    lib = ctypes.CDLL(path)
    i64, i32, u32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
    P = ctypes.POINTER
    sig = {
        "bcur_create": (i32, [P(vp), i32, vp, ctypes.c_size_t]),
        "bcur_test_matrix": (i32, [vp, i64, i64, ctypes.c_uint64, vp, i64]),
        "bcur_decompose_async": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(i64), i64, P(Params), vp,
                                       P(ctypes.c_uint64), P(Result)]),
        "bcur_wait": (i32, [vp]),
        "bcur_decompose_noalloc": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(i64), i64, P(Params), vp,
                                         P(ctypes.c_uint64), P(Result)]),
        "bcur_destroy": (i32, [vp]),
        "bcur_synchronize": (i32, [vp]),
        "bcur_status_str": (ctypes.c_char_p, [i32]),
        "bcur_last_error": (ctypes.c_char_p, [vp]),
        "bcur_workspace_bytes": (ctypes.c_size_t, [vp]),
        "bcur_frob2": (i32, [vp, vp, i64, i64, i64, P(dbl), P(i32)]),
        "bcur_range_finder": (i32, [vp, vp, i64, i64, i64, vp, i64, i64, i64, i32, vp, vp, P(dbl)]),
        "bcur_block_scores": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(dbl)]),
        "bcur_sample_blocks": (i32, [vp, P(dbl), i64, P(ctypes.c_uint64), i64, i32, P(i64), P(dbl), P(dbl)]),
        "bcur_gather_columns": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(i64), i64, vp, i64, P(i64)]),
        "bcur_fit_columns": (i32, [vp, vp, i64, i64, i64, vp, i64, i64, i32, vp, i64, P(dbl), P(u32)]),
        "bcur_sketch_pass": (i32, [vp, vp, i64, i64, i64, vp, i64, i64, i32, vp, i64]),
        "bcur_release_workspace": (i32, [vp]),
        "bcur_footprint": (i32, [i64, i64, P(i64), i64, P(i64), i64, P(Params), i32, P(ctypes.c_size_t)]),
        "bcur_server_create": (i32, [P(vp), i32, ctypes.c_size_t, i32]),
        "bcur_server_destroy": (i32, [vp]),
        "bcur_server_submit": (i32, [vp, P(Request), P(ctypes.c_uint64)]),
        "bcur_server_poll": (i32, [vp, ctypes.c_uint64, P(Result)]),
        "bcur_server_wait": (i32, [vp, ctypes.c_uint64, P(Result)]),
        "bcur_server_stats": (i32, [vp, P(Stats)]),
        "bcur_timing_enable": (i32, [vp, i32]),
        "bcur_timing_read": (i32, [vp, P(dbl), P(i64)]),
        "bcur_decompose": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(i64), i64, P(Params), vp,
                                 P(ctypes.c_uint64), P(Result)]),
        "bcur_block_stable_rank": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(i64), P(dbl), P(i32), P(dbl)]),
        "bcur_incoherence": (i32, [vp, vp, i64, i64, i64, P(dbl)]),
        "bcur_decompose_boost": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(Params), vp, i64, P(ctypes.c_uint64),
                                       P(Result), P(dbl), P(i64)]),
        "bcur_decompose_alg1_boost": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(Alg1Params), i64,
                                            P(ctypes.c_uint64), P(Alg1Result), P(dbl), P(i64)]),
        "bcur_decompose_alg1": (i32, [vp, vp, i64, i64, i64, P(i64), i64, P(Alg1Params), P(ctypes.c_uint64),
                                      P(Alg1Result)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def _check_dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major tensor")
    return t.data_ptr(), t.shape[0], t.shape[1], t.stride(0)


def to_device(a, device="cuda"):
    """Copy a 2-D host array to a float32 CUDA view with a padded leading dimension."""
    import torch
    a = np.asarray(a, dtype=np.float32)
    t = padded_empty(a.shape[0], a.shape[1], device)
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return t


def padded_empty(rows: int, cols: int, device="cuda"):
    """A rows x cols float32 CUDA view whose leading dimension is a multiple of 4."""
    import torch
    ld = (cols + 3) // 4 * 4
    return torch.empty((rows, ld), dtype=torch.float32, device=device)[:, :cols]


def _omega_arg(omega, m: int, n: int, k: int, l: Optional[int]):
    """(device pointer or None, l, seed) for a test-matrix argument that is a
    dense n x l CUDA tensor or an integer seed (the library then draws the
    Rademacher matrix of that seed; l defaults to min(k + 10, m, n, 128))."""
    if isinstance(omega, (int, np.integer)):
        if l is None:
            l = min(k + 10, m, n, 128)
        return None, int(l), int(omega) & ((1 << 64) - 1)
    po, on, lo, ldo = _check_dev(omega, "omega")
    if on != n or ldo != lo:
        raise ValueError("omega must be a dense n x l tensor")
    if l is not None and l != lo:
        raise ValueError("l does not match omega")
    return po, lo, 0


def _check_map(a, count, name):
    if a is None:
        return None
    a = _i64(a)
    if a.size != count:
        raise ValueError(f"{name} must have {count} entries")
    return a


class _DecomposeCall:
    """Arguments and result buffers of one bcur_decompose call (kept alive
    until its result is read)."""

    def __init__(self, A, offsets, k, s, omega, draws, q, replace, refine, precision, want_u, row_offsets, s_r,
                 U_out, col_map, row_map, l, seed):
        p, m, n, lda = _check_dev(A, "A")
        po, l, om_seed = _omega_arg(omega, m, n, k, l)
        self.keep = [A, omega, U_out]
        self.off = _i64(offsets)
        G = len(self.off) - 1
        rowv = row_offsets is not None and s_r > 0
        self.dr = np.ascontiguousarray(draws, dtype=np.uint64)
        if self.dr.size < s + (s_r if rowv else 0):
            raise ValueError("need s draws (s + s_r for the row-block variant)")
        prm = Params(k=k, s=s, l=l, q=q, replace=int(replace), precision=precision, refine=refine, reserved=0,
                     s_r=s_r, seed=om_seed if seed is None else int(seed))
        self.cmap = _check_map(col_map, n, "col_map")
        self.rmap = _check_map(row_map, m, "row_map")
        if self.cmap is not None:
            prm.col_map = _ptr(self.cmap, ctypes.c_int64)
        if self.rmap is not None:
            prm.row_map = _ptr(self.rmap, ctypes.c_int64)
        self.prm = prm
        self.idx = np.empty(s, dtype=np.int64)
        self.w = np.empty(s)
        self.sc = np.empty(G)
        self.ritz = np.empty(l)
        res = Result()
        res.idx = _ptr(self.idx, ctypes.c_int64)
        res.weights = _ptr(self.w, ctypes.c_double)
        res.scores = _ptr(self.sc, ctypes.c_double)
        res.ritz = _ptr(self.ritz, ctypes.c_double)
        self.U = None
        if want_u:
            cap = min(s * int(np.max(np.diff(self.off))), n)
            ucols = n
            if rowv:
                ucols = min(s_r * int(np.max(np.diff(_i64(row_offsets)))), m)
            self.U = U_out if U_out is not None else padded_empty(cap, ucols, A.device)
            res.U = self.U.data_ptr()
            res.ldu = self.U.stride(0)
            res.u_rows_cap = self.U.shape[0]
        roff_p, Gr = None, 0
        self.idx_r = self.rsc = None
        self.roff = None
        if row_offsets is not None:
            self.roff = _i64(row_offsets)
            Gr = len(self.roff) - 1
            roff_p = _ptr(self.roff, ctypes.c_int64)
            self.idx_r = np.empty(max(s_r, 1), dtype=np.int64)
            self.rsc = np.empty(Gr)
            res.idx_r = _ptr(self.idx_r, ctypes.c_int64)
            res.row_scores = _ptr(self.rsc, ctypes.c_double)
        self.res = res
        self.s_r = s_r
        self.args = (p, m, n, lda, _ptr(self.off, ctypes.c_int64), G, roff_p, Gr, ctypes.byref(prm), po,
                     _ptr(self.dr, ctypes.c_uint64), ctypes.byref(res))

    def result(self):
        res = self.res
        out = {"idx": self.idx, "weights": self.w, "scores": self.sc, "ritz": self.ritz, "c": res.c, "r": res.r,
               "frob2": res.frob2, "err": res.err, "rel_err": res.rel_err, "min_margin": res.min_margin,
               "flags": res.flags, "rr_sweeps": res.rr_sweeps, "kappa": res.kappa, "cond_c": res.cond_c}
        if self.U is not None:
            out["U"] = self.U[:res.c, :res.r] if res.r else self.U[:res.c]
        if self.idx_r is not None:
            out["idx_r"] = self.idx_r[:self.s_r]
            out["row_scores"] = self.rsc
        return out


class Context:
    """One library context bound to a device and to torch's current stream.

    scratch_budget: the most device workspace (bytes) the context may hold,
    0 for no limit."""

    def __init__(self, device: int = 0, stream=None, scratch_budget: int = 0):
        import torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        self._pending = None
        h = ctypes.c_void_p()
        st = self.lib.bcur_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream),
                                  ctypes.c_size_t(scratch_budget))
        if st != OK:
            raise BcurError(st, self.lib.bcur_status_str(st).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.bcur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != OK:
            raise BcurError(st, f"{self.lib.bcur_status_str(st).decode()}: {self.lib.bcur_last_error(self.h).decode()}")

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.bcur_workspace_bytes(self.h))

    # -- profiling ---------------------------------------------------------
    def timing_enable(self, on=True):
        """on: False (off), True (every stage), or an iterable of stage names."""
        if on is True:
            mask = -1
        elif not on:
            mask = 0
        else:
            mask = 0
            for name in on:
                mask |= 1 << STAGES.index(name)
        self._chk(self.lib.bcur_timing_enable(self.h, mask))

    def timing_read(self):
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), dtype=np.int64)
        self._chk(self.lib.bcur_timing_read(self.h, _ptr(ms, ctypes.c_double), _ptr(cnt, ctypes.c_int64)))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(STAGES)}

    # -- stages ------------------------------------------------------------
    def frob2(self, A):
        p, m, n, lda = _check_dev(A, "A")
        out = ctypes.c_double()
        fin = ctypes.c_int32()
        self._chk(self.lib.bcur_frob2(self.h, p, m, n, lda, ctypes.byref(out), ctypes.byref(fin)))
        return out.value, bool(fin.value)

    def range_finder(self, A, omega, k: int, q: int = 2, precision: int = PREC_FP32, want_u: bool = False):
        import torch
        p, m, n, lda = _check_dev(A, "A")
        po, on, l, ldo = _check_dev(omega, "omega")
        if on != n or ldo != l:
            raise ValueError("omega must be a dense n x l tensor")
        V = torch.empty((n, k), dtype=torch.float32, device=A.device)
        U = torch.empty((m, k), dtype=torch.float32, device=A.device) if want_u else None
        ritz = np.empty(l)
        self._chk(self.lib.bcur_range_finder(self.h, p, m, n, lda, po, l, k, q, precision, V.data_ptr(),
                                             U.data_ptr() if U is not None else None, _ptr(ritz, ctypes.c_double)))
        return V, U, ritz

    def sketch_pass(self, A, Q, precision: int = PREC_FP32):
        p, m, n, lda = _check_dev(A, "A")
        pq, qn, l, ldq = _check_dev(Q, "Q")
        if qn != n:
            raise ValueError("Q must have n rows")
        Y = padded_empty(n, l, A.device)
        self._chk(self.lib.bcur_sketch_pass(self.h, p, m, n, lda, pq, l, ldq, precision, Y.data_ptr(), Y.stride(0)))
        return Y

    def block_scores(self, V, offsets):
        p, n, k, ldv = _check_dev(V, "V")
        off = _i64(offsets)
        G = len(off) - 1
        out = np.empty(G)
        self._chk(self.lib.bcur_block_scores(self.h, p, n, k, ldv, _ptr(off, ctypes.c_int64), G,
                                             _ptr(out, ctypes.c_double)))
        return out

    def block_stable_rank(self, V, offsets, want_steps: bool = False, col_map=None):
        """(alpha, per-block ratios) of Def. 3 for the slices of V (n x k), and
        the squaring steps per block when want_steps."""
        p, n, k, ldv = _check_dev(V, "V")
        off = _i64(offsets)
        G = len(off) - 1
        ratios = np.empty(G)
        steps = np.empty(G, dtype=np.int32)
        alpha = ctypes.c_double()
        cmap = None if col_map is None else _i64(col_map)
        self._chk(self.lib.bcur_block_stable_rank(self.h, p, n, k, ldv, _ptr(off, ctypes.c_int64), G,
                                                  None if cmap is None else _ptr(cmap, ctypes.c_int64),
                                                  _ptr(ratios, ctypes.c_double), _ptr(steps, ctypes.c_int32),
                                                  ctypes.byref(alpha)))
        return (alpha.value, ratios, steps) if want_steps else (alpha.value, ratios)

    def incoherence(self, U):
        """mu of Def. 4 for U (m x k)."""
        p, m, k, ldu = _check_dev(U, "U")
        mu = ctypes.c_double()
        self._chk(self.lib.bcur_incoherence(self.h, p, m, k, ldu, ctypes.byref(mu)))
        return mu.value

    def sample_blocks(self, scores, draws, s: int, replace: bool = False):
        sc = np.ascontiguousarray(scores, dtype=np.float64)
        dr = np.ascontiguousarray(draws, dtype=np.uint64)
        if dr.size < s:
            raise ValueError("need s draws")
        idx = np.empty(s, dtype=np.int64)
        w = np.empty(s)
        mg = np.empty(s)
        self._chk(self.lib.bcur_sample_blocks(self.h, _ptr(sc, ctypes.c_double), len(sc),
                                              _ptr(dr, ctypes.c_uint64), s, int(replace), _ptr(idx, ctypes.c_int64),
                                              _ptr(w, ctypes.c_double), _ptr(mg, ctypes.c_double)))
        return idx, w, mg

    def gather_columns(self, A, offsets, idx):
        p, m, n, lda = _check_dev(A, "A")
        off = _i64(offsets)
        ix = _i64(idx)
        widths = np.diff(off)
        cap = int(sum(widths[j] for j in set(ix.tolist())))
        C = padded_empty(m, max(cap, 1), A.device)
        c = ctypes.c_int64()
        self._chk(self.lib.bcur_gather_columns(self.h, p, m, n, lda, _ptr(off, ctypes.c_int64), len(off) - 1,
                                               _ptr(ix, ctypes.c_int64), len(ix), C.data_ptr(), C.stride(0),
                                               ctypes.byref(c)))
        return C[:, :c.value]

    def fit_columns(self, A, C, refine: int = 1, U_out=None):
        """U = C^+ A (c x n) and err = ||A - C U||_F.  U_out: a c x n float32
        view to write (any row stride); only its c x n elements are written."""
        p, m, n, lda = _check_dev(A, "A")
        pc, mc, c, ldc = _check_dev(C, "C")
        if U_out is not None:
            _check_dev(U_out, "U_out")
            if tuple(U_out.shape) != (c, n):
                raise ValueError(f"U_out must be {c} x {n}")
        U = U_out if U_out is not None else padded_empty(c, n, A.device)
        err = ctypes.c_double()
        fl = ctypes.c_uint32()
        self._chk(self.lib.bcur_fit_columns(self.h, p, m, n, lda, pc, c, ldc, refine, U.data_ptr(), U.stride(0),
                                            ctypes.byref(err), ctypes.byref(fl)))
        return U, err.value, fl.value

    # -- the whole path ----------------------------------------------------
    def test_matrix(self, n: int, l: int, seed: int):
        """The n x l Rademacher test matrix the library draws from `seed`."""
        import torch
        om = torch.empty((n, l), dtype=torch.float32, device=f"cuda:{self.device}")
        self._chk(self.lib.bcur_test_matrix(self.h, n, l, int(seed) & ((1 << 64) - 1), om.data_ptr(), l))
        return om

    def footprint(self, m: int, n: int, offsets, k: int, s: int, l: int, q: int = 2,
                  precision: int = PREC_FP32, row_offsets=None, s_r: int = 0, library_holds_u: bool = False,
                  col_map=None, row_map=None) -> int:
        """bcur_footprint: device workspace bytes of one decomposition of these shapes."""
        off = _i64(offsets)
        prm = Params(k=k, s=s, l=l, q=q, precision=precision, s_r=s_r)
        cmap = _check_map(col_map, n, "col_map")
        rmap = _check_map(row_map, m, "row_map")
        if cmap is not None:
            prm.col_map = _ptr(cmap, ctypes.c_int64)
        if rmap is not None:
            prm.row_map = _ptr(rmap, ctypes.c_int64)
        roff = _i64(row_offsets) if row_offsets is not None else None
        out = ctypes.c_size_t()
        self._chk(self.lib.bcur_footprint(m, n, _ptr(off, ctypes.c_int64), len(off) - 1,
                                          None if roff is None else _ptr(roff, ctypes.c_int64),
                                          0 if roff is None else len(roff) - 1, ctypes.byref(prm),
                                          int(library_holds_u), ctypes.byref(out)))
        return int(out.value)

    def decompose(self, A, offsets, k: int, s: int, omega, draws, q: int = 2, replace: bool = False,
                  refine: int = 1, precision: int = PREC_FP32, want_u: bool = True, row_offsets=None,
                  s_r: int = 0, U_out=None, col_map=None, row_map=None, l: Optional[int] = None):
        """One decomposition.  omega: a dense n x l CUDA tensor, or an integer
        seed of the test matrix drawn on the device (sketch width `l`, by
        default min(k + 10, m, n, 128))."""
        call = _DecomposeCall(A, offsets, k, s, omega, draws, q, replace, refine, precision, want_u, row_offsets,
                              s_r, U_out, col_map, row_map, l, None)
        self._chk(self.lib.bcur_decompose(self.h, *call.args))
        return call.result()

    def decompose_async(self, A, offsets, k: int, s: int, omega, draws, q: int = 2, replace: bool = False,
                        refine: int = 1, precision: int = PREC_FP32, want_u: bool = True, row_offsets=None,
                        s_r: int = 0, U_out=None, col_map=None, row_map=None, l: Optional[int] = None):
        """bcur_decompose_async: returns at once; `wait()` returns the result."""
        if self._pending is not None:
            raise BcurError(E_STATE, "a decomposition is already in flight on this context")
        call = _DecomposeCall(A, offsets, k, s, omega, draws, q, replace, refine, precision, want_u, row_offsets,
                              s_r, U_out, col_map, row_map, l, None)
        self._chk(self.lib.bcur_decompose_async(self.h, *call.args))
        self._pending = call
        return call

    def decompose_noalloc(self, A, offsets, k: int, s: int, omega, draws, U_out, q: int = 2,
                          replace: bool = False, refine: int = 1, precision: int = PREC_FP32, row_offsets=None,
                          s_r: int = 0, l: Optional[int] = None):
        """bcur_decompose_noalloc: the library allocates nothing (its static
        scratch array and host staging serve); U_out is required."""
        if U_out is None:
            raise ValueError("U_out is required without allocation")
        call = _DecomposeCall(A, offsets, k, s, omega, draws, q, replace, refine, precision, True, row_offsets,
                              s_r, U_out, None, None, l, None)
        self._chk(self.lib.bcur_decompose_noalloc(self.h, *call.args))
        return call.result()

    def wait(self):
        """bcur_wait: the result of the decomposition in flight (None if none)."""
        call, self._pending = self._pending, None
        self._chk(self.lib.bcur_wait(self.h))
        return call.result() if call is not None else None

    def decompose_boost(self, A, offsets, k: int, s: int, omega, draws, t: int, q: int = 2, replace: bool = False,
                        refine: int = 1, precision: int = PREC_FP32, want_u: bool = True, U_out=None, col_map=None,
                        l: Optional[int] = None):
        """Boosting: t samplings (draws[i*s:(i+1)*s] for trial i) from one set of
        scores; returns the kept trial's result with every trial's err."""
        p, m, n, lda = _check_dev(A, "A")
        po, l, om_seed = _omega_arg(omega, m, n, k, l)
        off = _i64(offsets)
        G = len(off) - 1
        dr = np.ascontiguousarray(draws, dtype=np.uint64)
        if dr.size < t * s:
            raise ValueError("need t * s draws")
        prm = Params(k=k, s=s, l=l, q=q, replace=int(replace), precision=precision, refine=refine, reserved=0, s_r=0,
                     seed=om_seed)
        cmap = _check_map(col_map, n, "col_map")
        if cmap is not None:
            prm.col_map = _ptr(cmap, ctypes.c_int64)
        idx = np.empty(s, dtype=np.int64)
        w = np.empty(s)
        sc = np.empty(G)
        ritz = np.empty(l)
        errs = np.empty(t)
        best = ctypes.c_int64()
        res = Result()
        res.idx = _ptr(idx, ctypes.c_int64)
        res.weights = _ptr(w, ctypes.c_double)
        res.scores = _ptr(sc, ctypes.c_double)
        res.ritz = _ptr(ritz, ctypes.c_double)
        U = None
        if want_u:
            cap = min(s * int(np.max(np.diff(off))), n)
            U = U_out if U_out is not None else padded_empty(cap, n, A.device)
            res.U = U.data_ptr()
            res.ldu = U.stride(0)
            res.u_rows_cap = U.shape[0]
        self._chk(self.lib.bcur_decompose_boost(self.h, p, m, n, lda, _ptr(off, ctypes.c_int64), G, ctypes.byref(prm),
                                                po, t, _ptr(dr, ctypes.c_uint64), ctypes.byref(res),
                                                _ptr(errs, ctypes.c_double), ctypes.byref(best)))
        out = {"idx": idx, "weights": w, "scores": sc, "ritz": ritz, "c": res.c, "frob2": res.frob2, "err": res.err,
               "rel_err": res.rel_err, "min_margin": res.min_margin, "flags": res.flags, "rr_sweeps": res.rr_sweeps,
               "errs": errs, "best": best.value}
        if U is not None:
            out["U"] = U[:res.c]
        return out

    def decompose_alg1(self, A, offsets, r: int, s: int, draws, kr: Optional[int] = None, rank_k: int = 0,
                       replace: bool = False, want_u: bool = True, U_out=None, pinv_eig: bool = False,
                       trials: Optional[int] = None, col_map=None):
        """Algorithm 1 (uniform rows, U = W^+ or U_k = (W_k)^+).  draws: r row
        words then s column words (per trial when `trials` boosts over that many
        runs, keeping the smallest error).  U is the c x r core for the
        unscaled factors: A ~ A[:, cols] U A[rows, :]."""
        p, m, n, lda = _check_dev(A, "A")
        off = _i64(offsets)
        G = len(off) - 1
        kr = r if kr is None else kr
        dr = np.ascontiguousarray(draws, dtype=np.uint64)
        if dr.size < r + s:
            raise ValueError("need r + s draws")
        errs = best = None
        prm = Alg1Params(r=r, kr=kr, s=s, rank_k=rank_k, replace=int(replace), pinv_eig=int(pinv_eig))
        cmap = _check_map(col_map, n, "col_map")
        if cmap is not None:
            prm.col_map = _ptr(cmap, ctypes.c_int64)
        rows = np.empty(r, dtype=np.int64)
        idx = np.empty(s, dtype=np.int64)
        w = np.empty(s)
        sc = np.empty(G)
        res = Alg1Result()
        res.rows = _ptr(rows, ctypes.c_int64)
        res.idx = _ptr(idx, ctypes.c_int64)
        res.weights = _ptr(w, ctypes.c_double)
        res.scores = _ptr(sc, ctypes.c_double)
        U = None
        if want_u:
            cap = min(s * int(np.max(np.diff(off))), n)
            U = U_out if U_out is not None else padded_empty(cap, r, A.device)
            res.U = U.data_ptr()
            res.ldu = U.stride(0)
            res.u_rows_cap = U.shape[0]
        if trials is None:
            self._chk(self.lib.bcur_decompose_alg1(self.h, p, m, n, lda, _ptr(off, ctypes.c_int64), G,
                                                   ctypes.byref(prm), _ptr(dr, ctypes.c_uint64), ctypes.byref(res)))
        else:
            if dr.size < trials * (r + s):
                raise ValueError("need trials * (r + s) draws")
            errs = np.empty(trials)
            best = ctypes.c_int64()
            self._chk(self.lib.bcur_decompose_alg1_boost(self.h, p, m, n, lda, _ptr(off, ctypes.c_int64), G,
                                                         ctypes.byref(prm), trials, _ptr(dr, ctypes.c_uint64),
                                                         ctypes.byref(res), _ptr(errs, ctypes.c_double),
                                                         ctypes.byref(best)))
        out = {"rows": rows, "idx": idx, "weights": w, "scores": sc, "c": res.c, "rank_w": res.rank_w,
               "frob2": res.frob2, "err": res.err, "rel_err": res.rel_err, "min_margin": res.min_margin,
               "flags": res.flags, "sweeps": res.sweeps}
        if trials is not None:
            out["errs"] = errs
            out["best"] = best.value
        if U is not None:
            out["U"] = U[:res.c]
        return out


class Server:
    """Continuous-batching server (bcur_server_*): submit decompositions as
    they arrive, poll or wait for their results."""

    def __init__(self, device: int = 0, hbm_budget: int = 16 << 30, max_slots: int = 4):
        self.lib = load_library()
        h = ctypes.c_void_p()
        st = self.lib.bcur_server_create(ctypes.byref(h), device, hbm_budget, max_slots)
        if st != OK:
            raise BcurError(st, self.lib.bcur_status_str(st).decode())
        self.h = h
        self._live = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.bcur_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, A, offsets, k: int, s: int, omega, draws, q: int = 2, replace: bool = False,
               refine: int = 1, precision: int = PREC_FP32, row_offsets=None, s_r: int = 0, U_out=None,
               col_map=None, l: Optional[int] = None):
        """omega: a dense n x l CUDA tensor or an integer seed (as in Context.decompose)."""
        import torch
        p, m, n, lda = _check_dev(A, "A")
        po, l, om_seed = _omega_arg(omega, m, n, k, l)
        off = _i64(offsets)
        dr = np.ascontiguousarray(draws, dtype=np.uint64)
        if dr.size < s + (s_r if row_offsets is not None and s_r > 0 else 0):
            raise ValueError("need s draws (s + s_r for the row-block variant)")
        rq = Request()
        rq.A, rq.m, rq.n, rq.lda = p, m, n, lda
        rq.col_off, rq.G = _ptr(off, ctypes.c_int64), len(off) - 1
        roff = None
        if row_offsets is not None and s_r > 0:
            roff = _i64(row_offsets)
            rq.row_off, rq.Gr = _ptr(roff, ctypes.c_int64), len(roff) - 1
        rq.params = Params(k=k, s=s, l=l, q=q, replace=int(replace), precision=precision, refine=refine,
                           reserved=0, s_r=s_r if roff is not None else 0, seed=om_seed)
        cmap = _check_map(col_map, n, "col_map")   # copied by the server at submission
        if cmap is not None:
            rq.params.col_map = _ptr(cmap, ctypes.c_int64)
        rq.omega = po
        rq.draws = _ptr(dr, ctypes.c_uint64)
        if U_out is not None:
            rq.U, rq.ldu, rq.u_rows_cap = U_out.data_ptr(), U_out.stride(0), U_out.shape[0]
        rq.stream = torch.cuda.current_stream(A.device).cuda_stream
        t = ctypes.c_uint64()
        st = self.lib.bcur_server_submit(self.h, ctypes.byref(rq), ctypes.byref(t))
        if st != OK:
            raise BcurError(st, self.lib.bcur_status_str(st).decode())
        G = len(off) - 1
        Gr = len(roff) - 1 if roff is not None else 0
        # keep the request's tensors alive and the result arrays ready
        self._live[t.value] = (A, omega, U_out, np.empty(s, dtype=np.int64), np.empty(s), np.empty(G),
                               np.empty(l), np.empty(max(s_r, 1), dtype=np.int64), np.empty(max(Gr, 1)), s_r)
        return t.value

    def _collect(self, ticket, wait):
        A, om, U, idx, w, sc, rz, ir, rs, s_r = self._live[ticket]
        res = Result()
        res.idx = _ptr(idx, ctypes.c_int64)
        res.weights = _ptr(w, ctypes.c_double)
        res.scores = _ptr(sc, ctypes.c_double)
        res.ritz = _ptr(rz, ctypes.c_double)
        res.idx_r = _ptr(ir, ctypes.c_int64)
        res.row_scores = _ptr(rs, ctypes.c_double)
        fn = self.lib.bcur_server_wait if wait else self.lib.bcur_server_poll
        st = fn(self.h, ticket, ctypes.byref(res))
        if st == PENDING:
            return None
        del self._live[ticket]
        if st != OK:
            raise BcurError(st, self.lib.bcur_status_str(st).decode())
        out = {"idx": idx, "weights": w, "scores": sc, "ritz": rz, "c": res.c, "r": res.r, "frob2": res.frob2,
               "err": res.err, "rel_err": res.rel_err, "min_margin": res.min_margin, "flags": res.flags,
               "rr_sweeps": res.rr_sweeps, "kappa": res.kappa, "cond_c": res.cond_c}
        if U is not None:
            out["U"] = U[:res.c, :res.r] if res.r else U[:res.c]
        if s_r:
            out["idx_r"] = ir[:s_r]
            out["row_scores"] = rs
        return out

    def poll(self, ticket):
        return self._collect(ticket, False)

    def wait(self, ticket):
        return self._collect(ticket, True)

    def stats(self):
        st = Stats()
        r = self.lib.bcur_server_stats(self.h, ctypes.byref(st))
        if r != OK:
            raise BcurError(r, self.lib.bcur_status_str(r).decode())
        return {f: getattr(st, f) for f, _ in Stats._fields_}
