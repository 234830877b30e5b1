"""Python binding of libgevd.so (argument marshalling only).

Every step of the solve runs in the HIP kernels of libgevd.so; this module
passes torch tensors' device pointers and the current HIP stream through the
C interface declared in include/gevd.h, and turns nonzero return codes into
exceptions.  There is no CPU fallback: without the built library on a GPU
machine every call raises.

Matrices are column-major (Fortran order): a tensor M with M.stride(0) == 1
and M.stride(1) >= n.  ``colmajor(x)`` makes such a copy of any 2-D tensor.
Real problems are float64, complex problems complex128.
"""
from __future__ import annotations

import ctypes
import json
import os
import threading
import warnings

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libgevd.so")

GEVD_REAL, GEVD_COMPLEX = 0, 1
OPT_BAND, OPT_TIMING, OPT_LEAF, OPT_KSTATS, OPT_PRECISION, OPT_REFINE, OPT_PANEL, OPT_GEMM_TILE = 1, 2, 3, 4, 5, 6, 7, 8
OPT_STAGES = 9
PREC_FP64, PREC_FP32_REFINE = 0, 1
KFAMILIES = ("gemm", "panel", "chase", "backchase", "dc", "other", "small", "gemm32")
SMALL_MAX = 512
PHASES = ("cholesky", "invert", "multiply", "band", "tridiag", "solve", "back2", "back1", "mult")
E_NONFINITE, E_NOCONV, E_NOMEM, E_HIP, E_STATE, E_HANG, E_SCRATCH = -1001, -1002, -1003, -1004, -1005, -1006, -1007
E_RANK = -1008
W_ILLCOND = 1
ILLCOND_KAPPA = 1e12
NOALLOC_SCRATCH_BYTES, NOALLOC_MAX_COUNT = 64 << 20, 2048

_lib = None
_lock = threading.Lock()


class Problem(ctypes.Structure):
    """gevd_problem of include/gevd.h."""
    _fields_ = [("dtype", ctypes.c_int), ("n", ctypes.c_int), ("nev", ctypes.c_int),
                ("H", ctypes.c_void_p), ("ldh", ctypes.c_int), ("S", ctypes.c_void_p), ("lds", ctypes.c_int),
                ("eval", ctypes.c_void_p), ("C", ctypes.c_void_p), ("ldc", ctypes.c_int), ("flags", ctypes.c_int)]


PROBLEM_FACTORED = 1


class GevdError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s: %s (code %d)" % (where, strerror(code), code))


class NotPositiveDefinite(GevdError):
    pass


class IllConditionedOverlap(RuntimeWarning):
    """cond(S) is above what the Cholesky route resolves in FP64; the result
    is returned (see Solver.solve_reduced for the paper's alternative)."""


def load():
    """Load libgevd.so (built by paper_2502_02460_amd.build); raise if absent."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(SO_PATH):
            raise RuntimeError("libgevd.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(SO_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.gevd_create.argtypes = [ctypes.POINTER(P), I]
        L.gevd_destroy.argtypes = [P]
        L.gevd_set_stream.argtypes = [P, P]
        L.gevd_set_option.argtypes = [P, I, I]
        L.gevd_strerror.argtypes = [I]
        L.gevd_strerror.restype = ctypes.c_char_p
        L.gevd_workspace_bytes.argtypes = [I, I, I]
        L.gevd_workspace_bytes.restype = ctypes.c_size_t
        L.gevd_handle_workspace_bytes.argtypes = [P, I, I, I]
        L.gevd_handle_workspace_bytes.restype = ctypes.c_size_t
        L.gevd_get_warnings.argtypes = [P, ctypes.POINTER(D)]
        L.gevd_density.argtypes = [P, I, I, I, P, I, P, P, P, I, P, I]
        L.gevd_solve_reduced.argtypes = [P, I, I, I, D, P, I, P, I, P, P, I, ctypes.POINTER(I), P]
        L.gevd_solve.argtypes = [P, I, I, I, P, I, P, I, P, P, I]
        L.gevd_cholesky.argtypes = [P, I, I, P, I]
        L.gevd_set_overlap.argtypes = [P, I, I, P, I]
        L.gevd_solve_resident.argtypes = [P, I, P, I, P, P, I]
        L.gevd_invert_upper.argtypes = [P, I, I, P, I, P, I]
        L.gevd_reduce.argtypes = [P, I, I, P, I, P, I, P, I]
        L.gevd_eigh.argtypes = [P, I, I, I, P, I, P, P, I]
        L.gevd_backtransform.argtypes = [P, I, I, I, P, I, P, I, P, I]
        L.gevd_band.argtypes = [P, I, I, P, I, P, I]
        L.gevd_get_band.argtypes = [P, I, I]
        L.gevd_tridiagonalize.argtypes = [P, I, I, P, I, P, P]
        L.gevd_stedc.argtypes = [P, I, I, P, P, P, P, I]
        L.gevd_get_timings.argtypes = [P, ctypes.POINTER(D), I]
        L.gevd_get_kernel_stats.argtypes = [P, I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(D),
                                            ctypes.POINTER(D)]
        L.gevd_reset_kernel_stats.argtypes = [P]
        PP, IP = ctypes.POINTER(Problem), ctypes.POINTER(I)
        L.gevd_solve_batched.argtypes = [P, I, PP, IP]
        L.gevd_solve_batched_noalloc.argtypes = [P, I, PP, IP]
        L.gevd_batch_create.argtypes = [P, I, PP, ctypes.POINTER(P)]
        L.gevd_batch_run.argtypes = [P, IP]
        L.gevd_batch_run_async.argtypes = [P, P]
        L.gevd_batch_destroy.argtypes = [P]
        L.gevd_set_batch_shape.argtypes = [P, I, I, I, I]
        L.gevd_get_batch_shape.argtypes = [P, I, I, IP, IP]
        L.gevd_tune_batched.argtypes = [P, I, I, I, IP, IP]
        _lib = L
        return L


def strerror(code: int) -> str:
    return load().gevd_strerror(code).decode()


def _check(rc: int, where: str) -> int:
    if rc > 0:
        raise NotPositiveDefinite(rc, where)
    if rc != 0:
        raise GevdError(rc, where)
    return rc


def colmajor(x: torch.Tensor) -> torch.Tensor:
    """Column-major copy of a 2-D tensor (same logical values)."""
    return x.mT.contiguous().mT


def _ld(M: torch.Tensor, n_rows: int, name: str) -> int:
    if M.dim() != 2 or M.stride(0) != 1 or M.stride(1) < max(1, n_rows):
        raise ValueError("%s must be column-major (stride (1, ld >= %d)), got strides %s" %
                         (name, n_rows, tuple(M.stride())))
    if not M.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    return M.stride(1)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return GEVD_REAL
    if t.dtype == torch.complex128:
        return GEVD_COMPLEX
    raise TypeError("only float64 and complex128 are supported, got %s" % t.dtype)


def _empty_cm(rows: int, cols: int, dtype, device) -> torch.Tensor:
    return torch.empty((cols, rows), dtype=dtype, device=device).mT


class Solver:
    """A library handle bound to one device; keeps its workspace between
    calls.  Work goes to the current torch stream of that device."""

    def __init__(self, device=None, band: int = 0, leaf: int = 0, timing: bool = False, kstats: bool = False,
                 precision: str = "fp64", refine: int = 2, persistent_panel: bool = True, gemm_tile: int = -1,
                 stages: int = 2):
        """persistent_panel=False: one launch per full -> band panel column
        instead of one persistent launch per panel (for several solves
        sharing the device).  gemm_tile >= 0 forces one matrix-product tile
        (GEVD_OPT_GEMM_TILE).  stages=1 tridiagonalises in one stage
        (GEVD_OPT_STAGES)."""
        L = load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        h = ctypes.c_void_p()
        _check(L.gevd_create(ctypes.byref(h), self.device.index), "gevd_create")
        self._h = h
        if band:
            _check(L.gevd_set_option(h, OPT_BAND, band), "gevd_set_option")
        if leaf:
            _check(L.gevd_set_option(h, OPT_LEAF, leaf), "gevd_set_option")
        if timing:
            _check(L.gevd_set_option(h, OPT_TIMING, 1), "gevd_set_option")
        if kstats:
            _check(L.gevd_set_option(h, OPT_KSTATS, 1), "gevd_set_option")
        if not persistent_panel:
            _check(L.gevd_set_option(h, OPT_PANEL, 0), "gevd_set_option")
        if gemm_tile >= 0:
            _check(L.gevd_set_option(h, OPT_GEMM_TILE, gemm_tile), "gevd_set_option")
        if stages != 2:
            _check(L.gevd_set_option(h, OPT_STAGES, stages), "gevd_set_option")
        self.set_precision(precision, refine)

    def set_kstats(self, on: bool):
        """Enable or disable the per-family kernel accounting (HIP events
        around every launch)."""
        _check(load().gevd_set_option(self._h, OPT_KSTATS, 1 if on else 0), "gevd_set_option")

    def set_precision(self, precision: str = "fp64", refine: int = 2):
        """'fp64', or 'fp32+refine': full -> band and stage-1 back-transform
        products on the FP32 matrix cores, then `refine` FP64 refinement
        sweeps of the wanted pairs (see include/gevd.h)."""
        code = {"fp64": PREC_FP64, "fp32+refine": PREC_FP32_REFINE}[precision]
        _check(load().gevd_set_option(self._h, OPT_PRECISION, code), "gevd_set_option")
        _check(load().gevd_set_option(self._h, OPT_REFINE, int(refine)), "gevd_set_option")
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None):
            load().gevd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        load().gevd_set_stream(self._h, ctypes.c_void_p(s))

    # ------------------------------------------------------------------ steps
    def solve(self, H: torch.Tensor, S: torch.Tensor, nev: int, C: torch.Tensor | None = None,
              eval_out: torch.Tensor | None = None):
        """Generalized solve H c = eps S c.  H is clobbered; S's upper triangle
        receives U.  Returns (eval: all n ascending, C: n x nev)."""
        n = H.shape[0]
        t = _dtype_code(H)
        if S.dtype != H.dtype:
            raise TypeError("H and S must have the same dtype")
        ldh, lds = _ld(H, n, "H"), _ld(S, n, "S")
        if C is None:
            C = _empty_cm(n, nev, H.dtype, H.device)
        ldc = _ld(C, n, "C")
        w = eval_out if eval_out is not None else torch.empty(n, dtype=torch.float64, device=H.device)
        self._stream()
        _check(load().gevd_solve(self._h, t, n, nev, H.data_ptr(), ldh, S.data_ptr(), lds, w.data_ptr(),
                                 C.data_ptr(), ldc), "gevd_solve")
        self._warn()
        return w, C

    def warnings(self):
        """(GEVD_W_* bits, lower bound of cond(S)) of the last solve or
        set_overlap."""
        kap = ctypes.c_double()
        bits = load().gevd_get_warnings(self._h, ctypes.byref(kap))
        return bits, kap.value

    def _warn(self):
        bits, kap = self.warnings()
        if bits & W_ILLCOND:
            warnings.warn("cond(S) >= %.3g exceeds %.0e: the Cholesky route loses accuracy; "
                          "Solver.solve_reduced drops the overlap's near-null directions" % (kap, ILLCOND_KAPPA),
                          IllConditionedOverlap, stacklevel=3)

    def solve_reduced(self, H: torch.Tensor, S: torch.Tensor, nev: int, delta: float = 1e-5,
                      C: torch.Tensor | None = None):
        """The paper's route for an ill-conditioned overlap: omit the
        eigenvectors of S with sigma < delta and solve in the basis of the
        retained ones.  H is clobbered; S is not modified.  Returns (eval: the
        m eigenvalues ascending, C: n x nev, sigma: eigenvalues of S
        ascending, m)."""
        n = H.shape[0]
        t = _dtype_code(H)
        if S.dtype != H.dtype:
            raise TypeError("H and S must have the same dtype")
        ldh, lds = _ld(H, n, "H"), _ld(S, n, "S")
        if C is None:
            C = _empty_cm(n, nev, H.dtype, H.device)
        w = torch.empty(n, dtype=torch.float64, device=H.device)
        sigma = torch.empty(n, dtype=torch.float64, device=H.device)
        m = ctypes.c_int()
        self._stream()
        _check(load().gevd_solve_reduced(self._h, t, n, nev, float(delta), H.data_ptr(), ldh, S.data_ptr(), lds,
                                         w.data_ptr(), C.data_ptr(), _ld(C, n, "C"), ctypes.byref(m),
                                         sigma.data_ptr()), "gevd_solve_reduced")
        return w[: m.value], C, sigma, m.value

    def density(self, C: torch.Tensor, f: torch.Tensor, eval_: torch.Tensor | None = None,
                energy_weighted: bool = False):
        """Density matrix P_ij = sum_l f_l conj(c_li) c_lj from the eigenvector
        columns of C (n x k) and occupations f (k), and with energy_weighted
        also Q_ij = sum_l f_l eps_l conj(c_li) c_lj (eval_ holds eps).
        Returns P or (P, Q), column-major n x n."""
        n, k = C.shape
        f = f.to(device=C.device, dtype=torch.float64).contiguous()
        P = _empty_cm(n, n, C.dtype, C.device)
        Q = _empty_cm(n, n, C.dtype, C.device) if energy_weighted else None
        if energy_weighted:
            if eval_ is None:
                raise ValueError("energy_weighted needs the eigenvalues")
            eval_ = eval_[:k].to(device=C.device, dtype=torch.float64).contiguous()
        self._stream()
        _check(load().gevd_density(self._h, _dtype_code(C), n, k, C.data_ptr(), _ld(C, n, "C"), f.data_ptr(),
                                   eval_.data_ptr() if energy_weighted else None, P.data_ptr(), n,
                                   Q.data_ptr() if energy_weighted else None, n), "gevd_density")
        return (P, Q) if energy_weighted else P

    def workspace_bytes(self, dtype, n: int, nev: int) -> int:
        """Device workspace this handle holds for a (dtype, n, nev) solve
        under its current options."""
        return int(load().gevd_handle_workspace_bytes(self._h, _dt(dtype), n, nev))

    def set_overlap(self, S: torch.Tensor):
        """Factor S once and keep U^{-1} in the handle (S is not modified)."""
        n = S.shape[0]
        self._stream()
        _check(load().gevd_set_overlap(self._h, _dtype_code(S), n, S.data_ptr(), _ld(S, n, "S")), "gevd_set_overlap")
        self._warn()
        self.res_n, self.res_dtype = n, S.dtype

    def solve_resident(self, H: torch.Tensor, nev: int, C: torch.Tensor | None = None,
                       eval_out: torch.Tensor | None = None):
        """Solve with the overlap of the last set_overlap; H is clobbered."""
        n = H.shape[0]
        if C is None:
            C = _empty_cm(n, nev, H.dtype, H.device)
        w = eval_out if eval_out is not None else torch.empty(n, dtype=torch.float64, device=H.device)
        self._stream()
        _check(load().gevd_solve_resident(self._h, nev, H.data_ptr(), _ld(H, n, "H"), w.data_ptr(), C.data_ptr(),
                                          _ld(C, n, "C")), "gevd_solve_resident")
        return w, C

    def cholesky(self, S: torch.Tensor) -> torch.Tensor:
        n = S.shape[0]
        self._stream()
        _check(load().gevd_cholesky(self._h, _dtype_code(S), n, S.data_ptr(), _ld(S, n, "S")), "gevd_cholesky")
        return S

    def invert_upper(self, U: torch.Tensor) -> torch.Tensor:
        n = U.shape[0]
        Ui = _empty_cm(n, n, U.dtype, U.device)
        self._stream()
        _check(load().gevd_invert_upper(self._h, _dtype_code(U), n, U.data_ptr(), _ld(U, n, "U"), Ui.data_ptr(), n),
               "gevd_invert_upper")
        return Ui

    def reduce(self, H: torch.Tensor, Uinv: torch.Tensor) -> torch.Tensor:
        n = H.shape[0]
        A = _empty_cm(n, n, H.dtype, H.device)
        self._stream()
        _check(load().gevd_reduce(self._h, _dtype_code(H), n, H.data_ptr(), _ld(H, n, "H"), Uinv.data_ptr(),
                                  _ld(Uinv, n, "Uinv"), A.data_ptr(), n), "gevd_reduce")
        return A

    def eigh(self, A: torch.Tensor, nev: int):
        n = A.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=A.device)
        Z = _empty_cm(n, nev, A.dtype, A.device)
        self._stream()
        _check(load().gevd_eigh(self._h, _dtype_code(A), n, nev, A.data_ptr(), _ld(A, n, "A"), w.data_ptr(),
                                Z.data_ptr(), n), "gevd_eigh")
        return w, Z

    def backtransform(self, Uinv: torch.Tensor, Ct: torch.Tensor) -> torch.Tensor:
        n, nev = Ct.shape
        C = _empty_cm(n, nev, Ct.dtype, Ct.device)
        self._stream()
        _check(load().gevd_backtransform(self._h, _dtype_code(Ct), n, nev, Uinv.data_ptr(), _ld(Uinv, n, "Uinv"),
                                         Ct.data_ptr(), _ld(Ct, n, "Ct"), C.data_ptr(), n), "gevd_backtransform")
        return C

    def band_width(self, n: int, dtype=torch.float64) -> int:
        return load().gevd_get_band(self._h, GEVD_COMPLEX if dtype == torch.complex128 else GEVD_REAL, n)

    def band(self, A: torch.Tensor) -> torch.Tensor:
        """Lower band storage (b+1) x n of the first-stage band matrix."""
        n = A.shape[0]
        b = self.band_width(n, A.dtype)
        Bd = _empty_cm(b + 1, n, A.dtype, A.device)
        self._stream()
        _check(load().gevd_band(self._h, _dtype_code(A), n, A.data_ptr(), _ld(A, n, "A"), Bd.data_ptr(), b + 1),
               "gevd_band")
        return Bd

    def tridiagonalize(self, A: torch.Tensor):
        n = A.shape[0]
        d = torch.empty(n, dtype=torch.float64, device=A.device)
        e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=A.device)
        self._stream()
        _check(load().gevd_tridiagonalize(self._h, _dtype_code(A), n, A.data_ptr(), _ld(A, n, "A"), d.data_ptr(),
                                          e.data_ptr()), "gevd_tridiagonalize")
        return d, e[: n - 1]

    def stedc(self, d: torch.Tensor, e: torch.Tensor, nev: int):
        n = d.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=d.device)
        Z = _empty_cm(n, nev, torch.float64, d.device)
        ee = e if n > 1 else torch.zeros(1, dtype=torch.float64, device=d.device)
        self._stream()
        _check(load().gevd_stedc(self._h, n, nev, d.data_ptr(), ee.data_ptr(), w.data_ptr(), Z.data_ptr(), n),
               "gevd_stedc")
        return w, Z

    # --------------------------------------------------------- batched small
    def _problems(self, items, outs, factored=False):
        arr = (Problem * len(items))()
        keep = []
        for i, (H, S, nev) in enumerate(items):
            n = H.shape[0]
            if n > SMALL_MAX:
                raise ValueError("batched problems need n <= %d (got %d)" % (SMALL_MAX, n))
            if S.dtype != H.dtype:
                raise TypeError("H and S must have the same dtype")
            if outs is None:
                w = torch.empty(n, dtype=torch.float64, device=H.device)
                C = _empty_cm(n, nev, H.dtype, H.device)
            else:
                w, C = outs[i]
            keep.append((w, C))
            arr[i] = Problem(_dtype_code(H), n, nev, H.data_ptr(), _ld(H, n, "H"), S.data_ptr(), _ld(S, n, "S"),
                             w.data_ptr(), C.data_ptr(), _ld(C, n, "C"), PROBLEM_FACTORED if factored else 0)
        return arr, keep

    def solve_batched(self, items, outs=None, factored: bool = False):
        """Solve many small problems in fused persistent launches.

        items: sequence of (H, S, nev) with n <= 512 (H clobbered; S receives
        U in its upper and U^H in its strictly lower triangle).  outs: optional matching (eval, C)
        buffers.  factored: every S already holds its factor from an earlier
        batched solve (the Cholesky is skipped).  Returns (results, info):
        results[i] = (eval, C) and info[i] the problem's status (0, j > 0 not
        positive definite at minor j, or an E_* code); raises only for errors
        of the launch itself."""
        arr, keep = self._problems(items, outs, factored)
        info = (ctypes.c_int * len(items))()
        self._stream()
        _check(load().gevd_solve_batched(self._h, len(items), arr, info), "gevd_solve_batched")
        return keep, list(info)

    def solve_batched_noalloc(self, items, outs=None, factored: bool = False):
        """solve_batched through the entry point that allocates no device
        memory (fixed per-device scratch; at most NOALLOC_MAX_COUNT problems).
        Pass preallocated `outs` to keep the caller's side allocation-free."""
        arr, keep = self._problems(items, outs, factored)
        info = (ctypes.c_int * len(items))()
        self._stream()
        _check(load().gevd_solve_batched_noalloc(self._h, len(items), arr, info), "gevd_solve_batched_noalloc")
        return keep, list(info)

    def batch(self, items, outs=None, factored: bool = False) -> "Batch":
        """A reusable batch (descriptors uploaded, launches captured in a HIP
        graph) over fixed buffers; see Batch.run."""
        arr, keep = self._problems(items, outs, factored)
        b = ctypes.c_void_p()
        self._stream()
        _check(load().gevd_batch_create(self._h, len(items), arr, ctypes.byref(b)), "gevd_batch_create")
        return Batch(self, b, keep, list(items))

    def set_batch_shape(self, dtype, n: int, threads: int, wg_per_cu: int):
        _check(load().gevd_set_batch_shape(self._h, _dt(dtype), n, threads, wg_per_cu), "gevd_set_batch_shape")

    def batch_shape(self, dtype, n: int):
        t, w = ctypes.c_int(), ctypes.c_int()
        _check(load().gevd_get_batch_shape(self._h, _dt(dtype), n, ctypes.byref(t), ctypes.byref(w)),
               "gevd_get_batch_shape")
        return t.value, w.value

    def tune_batched(self, dtype, n: int, count: int = 512):
        """Run the launch-shape tuner for the bucket holding order n."""
        t, w = ctypes.c_int(), ctypes.c_int()
        self._stream()
        _check(load().gevd_tune_batched(self._h, _dt(dtype), n, count, ctypes.byref(t), ctypes.byref(w)),
               "gevd_tune_batched")
        return t.value, w.value

    def load_batch_shapes(self, path: str) -> int:
        """Apply tuned shapes saved by save_batch_shapes; returns how many."""
        if not os.path.exists(path):
            return 0
        with open(path) as f:
            table = json.load(f)
        k = 0
        for key, (t, w) in table.items():
            dt, n = key.split(":")
            self.set_batch_shape(torch.complex128 if dt == "z" else torch.float64, int(n), int(t), int(w))
            k += 1
        return k

    def save_batch_shapes(self, path: str, buckets=(64, 128, 256, 512)):
        table = {}
        for dt, tag in ((torch.float64, "d"), (torch.complex128, "z")):
            for n in buckets:
                table["%s:%d" % (tag, n)] = list(self.batch_shape(dt, n))
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)

    def kernel_stats(self) -> dict:
        """Per kernel family: launches, device ms (HIP events on the launch
        stream) and algorithmic flops, accumulated since the last reset."""
        out = {}
        for i, name in enumerate(KFAMILIES):
            n = ctypes.c_longlong()
            ms = ctypes.c_double()
            fl = ctypes.c_double()
            _check(load().gevd_get_kernel_stats(self._h, i, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)),
                   "gevd_get_kernel_stats")
            out[name] = {"launches": n.value, "ms": ms.value, "flops": fl.value}
        return out

    def reset_kernel_stats(self):
        _check(load().gevd_reset_kernel_stats(self._h), "gevd_reset_kernel_stats")

    def timings(self) -> dict:
        arr = (ctypes.c_double * len(PHASES))()
        _check(load().gevd_get_timings(self._h, arr, len(PHASES)), "gevd_get_timings")
        return dict(zip(PHASES, list(arr)))


class Batch:
    """A captured batch: run() replays it on the solver's current stream."""

    def __init__(self, solver: Solver, handle, results, items):
        self.solver = solver
        self._b = handle
        self.results = results  # [(eval, C)] in item order
        self.items = items      # keeps the input tensors alive

    def run(self, sync: bool = True):
        """Replay; with sync, wait and return the per-problem info list."""
        self.solver._stream()
        if sync:
            info = (ctypes.c_int * len(self.results))()
            _check(load().gevd_batch_run(self._b, info), "gevd_batch_run")
            return list(info)
        _check(load().gevd_batch_run(self._b, None), "gevd_batch_run")
        return None

    def run_async(self, info_dev: torch.Tensor):
        """Replay and copy the per-problem status into info_dev (int32 device
        tensor of one entry per problem) on the solver's current stream; no
        host synchronisation."""
        if info_dev.dtype != torch.int32 or not info_dev.is_cuda or not info_dev.is_contiguous():
            raise ValueError("info_dev must be a contiguous int32 device tensor")
        if info_dev.numel() < len(self.results):
            raise ValueError("info_dev holds %d entries, the batch has %d problems"
                             % (info_dev.numel(), len(self.results)))
        self.solver._stream()
        _check(load().gevd_batch_run_async(self._b, ctypes.c_void_p(info_dev.data_ptr())), "gevd_batch_run_async")

    def close(self):
        if getattr(self, "_b", None):
            load().gevd_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dt(dtype) -> int:
    if dtype in (torch.complex128, GEVD_COMPLEX, "z", "complex"):
        return GEVD_COMPLEX
    if dtype in (torch.float64, GEVD_REAL, "d", "real"):
        return GEVD_REAL
    raise TypeError("dtype must be float64 or complex128, got %r" % (dtype,))


def workspace_bytes(dtype, n: int, nev: int) -> int:
    return int(load().gevd_workspace_bytes(GEVD_COMPLEX if dtype == torch.complex128 else GEVD_REAL, n, nev))
