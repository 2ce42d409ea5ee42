"""Python binding of ``libhinqs.so``, the gfx950 selected-CI subspace solver.

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library (see ``include/hinqs.h``).  PyTorch supplies device
memory and the stream; the library is loaded from this directory and the
binding raises if it is missing -- there is no fallback path.

    solver = Hinqs()                               # cuda:0, current stream
    solver.set_integrals(h, eri, e_core)           # Sec. 2.2 Hamiltonian
    solver.set_determinants(alpha, beta, na, nb)   # sampled basis B
    S = solver.sigma(X)                            # S = H_B X
    E, c, stats = solver.lowest_eigenpair()        # Step 3 Davidson
    rdm1, rdm2 = solver.rdm12(c)
    E = HinqsEnergy.apply(h_t, eri_t, solver)      # differentiable in h, eri
"""
from __future__ import annotations

import ctypes
import os
import sys
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhinqs.so")

HINQS_OK = 0
HINQS_E = {
    -1: "INVALID_ARG", -2: "NOT_READY", -3: "ASYMMETRIC", -4: "BAD_OCCUPATION",
    -5: "DUPLICATE", -6: "UNSUPPORTED", -7: "NOT_CONVERGED", -8: "NONFINITE", -9: "OOM",
    -10: "HIP",
}
HINQS_FP64, HINQS_FP32 = 0, 1
SOLVE_FP64, SOLVE_MIXED = 0, 1
SORTED_ORDER = 1
AUTOTUNE = 2
NO_GRAPH = 4
LARGEST = 8
GROW_APPEND, GROW_REBUILD = 0, 1
EXC_1A, EXC_1B, EXC_2AA, EXC_2BB, EXC_2AB = 1, 2, 3, 4, 5

EXPORTED = ["hinqs_opts_default", "hinqs_create", "hinqs_destroy", "hinqs_last_error",
            "hinqs_set_integrals", "hinqs_set_determinants", "hinqs_sigma",
            "hinqs_lowest_eigenpair", "hinqs_rdm12", "hinqs_integral_grad", "hinqs_diag",
            "hinqs_connectivity", "hinqs_permutation", "hinqs_get_info",
            "hinqs_pair_descriptor", "hinqs_gram", "hinqs_set_determinants_device",
            "hinqs_autotune", "hinqs_batch_clear", "hinqs_batch_add", "hinqs_batch_info",
            "hinqs_batch_lowest_eigenpair", "hinqs_expand", "hinqs_pt2", "hinqs_top_k",
            "hinqs_teacher_weights", "hinqs_distinct_strings", "hinqs_update_determinants",
            "hinqs_grow_basis", "hinqs_get_determinants", "hinqs_product_closure",
            "hinqs_sigma_noalloc", "hinqs_pt2_members"]


class HinqsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{HINQS_E.get(code, code)}: {msg}")
        self.code = code
        self.name = HINQS_E.get(code, str(code))


class Opts(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("max_space", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("tol", ctypes.c_double), ("precision", ctypes.c_int),
                ("precond_floor", ctypes.c_double), ("mixed_switch", ctypes.c_double),
                ("flags", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("iterations_fp32", ctypes.c_int),
                ("sigma_blocks", ctypes.c_int), ("sigma_columns", ctypes.c_int),
                ("restarts", ctypes.c_int),
                ("residual", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_sigma", ctypes.c_double), ("nnz", ctypes.c_int64), ("second_passes", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("norb", ctypes.c_int), ("nalpha", ctypes.c_int), ("nbeta", ctypes.c_int),
                ("ndet", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("n_alpha_strings", ctypes.c_int32), ("n_beta_strings", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("ms_sort", ctypes.c_double),
                ("ms_connect", ctypes.c_double), ("ms_elements", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [("instances", ctypes.c_int), ("converged", ctypes.c_int), ("iterations", ctypes.c_int),
                ("graphs", ctypes.c_int), ("ms_total", ctypes.c_double), ("ms_setup", ctypes.c_double),
                ("ms_iterations", ctypes.c_double), ("max_residual", ctypes.c_double),
                ("ndet", ctypes.c_int64), ("nnz", ctypes.c_int64), ("sigma_team", ctypes.c_int),
                ("sigma_unroll", ctypes.c_int), ("sigma_occupancy", ctypes.c_int),
                ("sigma_elements", ctypes.c_double), ("chunk_rows", ctypes.c_int),
                ("rr_threads", ctypes.c_int), ("ms_tune", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_lock = threading.Lock()

# hinqs_alloc_fn / hinqs_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def load_library() -> ctypes.CDLL:
    """Load ``libhinqs.so``; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2606_26760_amd.build` (no fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        sig = {
            "hinqs_opts_default": (None, [P]),
            "hinqs_create": (i32, [P, i32, P, ALLOC_FN, FREE_FN, P]),
            "hinqs_destroy": (None, [P]),
            "hinqs_last_error": (ctypes.c_char_p, [P]),
            "hinqs_set_integrals": (i32, [P, i32, P, P, dbl]),
            "hinqs_set_determinants": (i32, [P, i64, P, P, i32, i32]),
            "hinqs_set_determinants_device": (i32, [P, i64, P, P, i32, i32]),
            "hinqs_sigma": (i32, [P, i32, P, P, i32, i32]),
            "hinqs_sigma_noalloc": (i32, [P, i32, P, P, i32, i32]),
            "hinqs_lowest_eigenpair": (i32, [P, P, P, P, P, P]),
            "hinqs_rdm12": (i32, [P, P, P, P, i32]),
            "hinqs_integral_grad": (i32, [P, P, dbl, P, P, i32]),
            "hinqs_diag": (i32, [P, P, i32]),
            "hinqs_connectivity": (i32, [P, P, P, P]),
            "hinqs_permutation": (i32, [P, P]),
            "hinqs_get_info": (i32, [P, P]),
            "hinqs_pair_descriptor": (ctypes.c_uint32, [ctypes.c_uint64] * 4),
            "hinqs_gram": (i32, [P, i64, P, i32, i32, P, i32, i32, P]),
            "hinqs_autotune": (i32, [P, i32, i32, P, P]),
            "hinqs_batch_clear": (i32, [P]),
            "hinqs_batch_add": (i32, [P, i32, P, P, dbl, i64, P, P, i32, i32, P]),
            "hinqs_batch_info": (i32, [P, P, P, P]),
            "hinqs_batch_lowest_eigenpair": (i32, [P, P, P, P, P, P, P]),
            "hinqs_expand": (i32, [P, P, i64, i64, P, P, P, P, i32]),
            "hinqs_pt2": (i32, [P, P, dbl, i64, P, P, P, P, P, i32]),
            "hinqs_pt2_members": (i32, [P, P, dbl, P, P, P, i32]),
            "hinqs_top_k": (i32, [P, i64, P, i64, i32, P]),
            "hinqs_teacher_weights": (i32, [P, P, P, P, P, i32]),
            "hinqs_distinct_strings": (i32, [P, P, P]),
            "hinqs_update_determinants": (i32, [P, i64, P, i64, P, P, P, P, i32, P]),
            "hinqs_grow_basis": (i32, [P, i32, i64, P, P, P, i64, P, i64, P, P, P, P, P]),
            "hinqs_get_determinants": (i32, [P, P, P]),
            "hinqs_product_closure": (i32, [P, i64, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def pair_descriptor(alpha_i: int, beta_i: int, alpha_j: int, beta_j: int) -> int:
    """Descriptor the coupling enumerator stores for x_i <- x_j (host-only helper)."""
    return int(load_library().hinqs_pair_descriptor(alpha_i, beta_i, alpha_j, beta_j))


def decode_descriptor(d):
    """(type, neg, h1, h2, p1, p2) arrays from descriptor values."""
    d = np.asarray(d, dtype=np.uint32)
    return (d & 7, (d >> 3) & 1, (d >> 4) & 31, (d >> 9) & 31, (d >> 14) & 31, (d >> 19) & 31)


def _torch():
    import torch
    return torch


def _host_f64(a) -> np.ndarray:
    t = _torch()
    if isinstance(a, t.Tensor):
        a = a.detach().to("cpu", t.float64).numpy()
    return np.ascontiguousarray(a, dtype=np.float64)


def _host_u64(a) -> np.ndarray:
    t = _torch()
    if isinstance(a, t.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a).astype(np.uint64))


class TorchAllocator:
    """Device memory from PyTorch's caching allocator, on the context's stream.

    ``alloc`` returns 0 when the pool cannot serve the request (the library
    then reports HINQS_E_OOM); ``free`` hands the block back to the pool, which
    reuses it in the stream's order without a device synchronisation.
    """

    def __init__(self, device: int, stream_handle: int):
        self.device = device
        self.stream_handle = stream_handle

    def alloc(self, nbytes: int) -> int:
        try:
            return int(_torch().cuda.caching_allocator_alloc(nbytes, self.device, self.stream_handle))
        except Exception:  # torch.OutOfMemoryError and the like: report NULL
            return 0

    def free(self, ptr: int) -> None:
        _torch().cuda.caching_allocator_delete(ptr)


class Hinqs:
    """One solver context on one device and stream.

    ``allocator``: ``"torch"`` (default) routes every device buffer of the
    library through PyTorch's caching allocator; ``"hip"`` leaves the library
    on hipMalloc/hipFree; any object with ``alloc(nbytes) -> int`` (0 when out
    of memory) and ``free(ptr)`` is used as given.
    """

    def __init__(self, device: int = 0, stream=None, allocator="torch"):
        torch = _torch()
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("Hinqs needs a ROCm GPU (gfx950); none is visible")
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._lib = lib
        if allocator == "torch":
            allocator = TorchAllocator(device, stream.cuda_stream)
        self.allocator = None if allocator == "hip" else allocator
        alloc_cb, free_cb = ALLOC_FN(), FREE_FN()  # NULL: hipMalloc / hipFree
        if self.allocator is not None:
            source = self.allocator

            def _alloc(nbytes, _stream, _user):
                try:
                    return source.alloc(int(nbytes)) or None
                except Exception:
                    return None

            def _free(ptr, _stream, _user):
                try:
                    source.free(int(ptr))
                except Exception:
                    pass

            alloc_cb, free_cb = ALLOC_FN(_alloc), FREE_FN(_free)
        # the callbacks must outlive every buffer of the context
        self._callbacks = (alloc_cb, free_cb)
        h = ctypes.c_void_p()
        rc = lib.hinqs_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream), alloc_cb,
                              free_cb, None)
        if rc != HINQS_OK:
            raise HinqsError(rc, "hinqs_create failed")
        self._h = h
        self.norb = self.na = self.nb = self.ndet = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hinqs_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the allocator callbacks can no longer run
        # Python; the process is ending and its device memory goes with it
        # (the function is bound at definition: module globals may be gone)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != HINQS_OK:
            msg = self._lib.hinqs_last_error(self._h)
            raise HinqsError(rc, msg.decode() if msg else "")

    @staticmethod
    def _ptr(t):
        return ctypes.c_void_p(t.data_ptr())

    def _dev(self, t, dtype):
        torch = _torch()
        if not (isinstance(t, torch.Tensor) and t.device == self.device and t.dtype == dtype
                and t.is_contiguous()):
            raise ValueError(f"expected a contiguous {dtype} tensor on {self.device}")
        return t

    # ---------------------------------------------------------------- inputs
    def set_integrals(self, h, eri, e_core: float = 0.0):
        h = _host_f64(h)
        eri = _host_f64(eri)
        norb = h.shape[0]
        if h.shape != (norb, norb) or eri.shape != (norb,) * 4:
            raise ValueError("h must be (n, n) and eri (n, n, n, n)")
        self._check(self._lib.hinqs_set_integrals(self._h, norb, h.ctypes.data_as(ctypes.c_void_p),
                                                  eri.ctypes.data_as(ctypes.c_void_p),
                                                  float(e_core)))
        self.norb = norb

    def set_determinants(self, alpha, beta, nalpha: int, nbeta: int):
        torch = _torch()
        if isinstance(alpha, torch.Tensor) and alpha.device.type == "cuda":
            # device-resident strings (int64 tensors holding the uint64 bit patterns)
            self._dev(alpha, torch.int64)
            self._dev(beta, torch.int64)
            if alpha.shape != beta.shape or alpha.dim() != 1:
                raise ValueError("alpha and beta must be 1-D and equally long")
            self._check(self._lib.hinqs_set_determinants_device(
                self._h, alpha.numel(), self._ptr(alpha), self._ptr(beta), nalpha, nbeta))
            self.na, self.nb, self.ndet = nalpha, nbeta, alpha.numel()
            return
        a = _host_u64(alpha)
        b = _host_u64(beta)
        if a.shape != b.shape or a.ndim != 1:
            raise ValueError("alpha and beta must be 1-D and equally long")
        self._check(self._lib.hinqs_set_determinants(self._h, len(a), a.ctypes.data_as(ctypes.c_void_p),
                                                     b.ctypes.data_as(ctypes.c_void_p), nalpha, nbeta))
        self.na, self.nb, self.ndet = nalpha, nbeta, len(a)

    # ------------------------------------------------------------- products
    def sigma(self, X, out=None, sorted_order: bool = False):
        torch = _torch()
        squeeze = X.dim() == 1
        if squeeze:
            X = X.unsqueeze(1)
        prec = HINQS_FP64 if X.dtype == torch.float64 else HINQS_FP32
        self._dev(X, X.dtype)
        if X.shape[0] != self.ndet:
            raise ValueError("X must have ndet rows")
        S = torch.empty_like(X) if out is None else self._dev(out, X.dtype)
        self._check(self._lib.hinqs_sigma(self._h, X.shape[1], self._ptr(X), self._ptr(S), prec,
                                          SORTED_ORDER if sorted_order else 0))
        return S.squeeze(1) if squeeze else S

    def sigma_noalloc(self, X, out, sorted_order: bool = False):
        """``sigma`` through hinqs_sigma_noalloc: the library allocates nothing
        (the caller provides ``out``); staging uses the static per-GPU array."""
        torch = _torch()
        squeeze = X.dim() == 1
        prec = HINQS_FP64 if X.dtype == torch.float64 else HINQS_FP32
        self._dev(X, X.dtype)
        self._dev(out, X.dtype)
        if X.shape != out.shape or X.shape[0] != self.ndet:
            raise ValueError("X and out must both be ndet x k")
        k = 1 if squeeze else X.shape[1]
        self._check(self._lib.hinqs_sigma_noalloc(self._h, k, self._ptr(X), self._ptr(out), prec,
                                                  SORTED_ORDER if sorted_order else 0))
        return out

    def lowest_eigenpair(self, guess=None, *, block=8, max_space=None, max_iter=200, tol=1e-8,
                         mixed=False, precond_floor=1e-8, mixed_switch=1e-5, sorted_order=False,
                         raise_on_not_converged=True, autotune=False):
        torch = _torch()
        o = Opts()
        self._lib.hinqs_opts_default(ctypes.byref(o))
        o.block = block
        o.max_space = max_space if max_space is not None else 6 * block
        o.max_iter = max_iter
        o.tol = tol
        o.precision = SOLVE_MIXED if mixed else SOLVE_FP64
        o.precond_floor = precond_floor
        o.mixed_switch = mixed_switch
        o.flags = (SORTED_ORDER if sorted_order else 0) | (AUTOTUNE if autotune else 0)
        c = torch.empty(self.ndet, dtype=torch.float64, device=self.device)
        e = ctypes.c_double(0.0)
        st = Stats()
        gp = None
        if guess is not None:
            gp = self._ptr(self._dev(guess, torch.float64))
        rc = self._lib.hinqs_lowest_eigenpair(self._h, ctypes.byref(o), gp, ctypes.byref(e),
                                              self._ptr(c), ctypes.byref(st))
        if rc == -7 and not raise_on_not_converged:
            return e.value, c, dict(st.as_dict(), converged=False)
        self._check(rc)
        return e.value, c, dict(st.as_dict(), converged=True)

    def rdm12(self, c, sorted_order=False):
        torch = _torch()
        self._dev(c, torch.float64)
        n = self.norb
        d1 = torch.empty((n, n), dtype=torch.float64, device=self.device)
        d2 = torch.empty((n, n, n, n), dtype=torch.float64, device=self.device)
        self._check(self._lib.hinqs_rdm12(self._h, self._ptr(c), self._ptr(d1), self._ptr(d2),
                                          SORTED_ORDER if sorted_order else 0))
        return d1, d2

    def integral_grad(self, c, scale=1.0, sorted_order=False):
        torch = _torch()
        self._dev(c, torch.float64)
        n = self.norb
        gh = torch.empty((n, n), dtype=torch.float64, device=self.device)
        ge = torch.empty((n, n, n, n), dtype=torch.float64, device=self.device)
        self._check(self._lib.hinqs_integral_grad(self._h, self._ptr(c), float(scale), self._ptr(gh),
                                                  self._ptr(ge), SORTED_ORDER if sorted_order else 0))
        return gh, ge

    # -------------------------------------------------------------- exports
    def diag(self, sorted_order=False):
        torch = _torch()
        d = torch.empty(self.ndet, dtype=torch.float64, device=self.device)
        self._check(self._lib.hinqs_diag(self._h, self._ptr(d), SORTED_ORDER if sorted_order else 0))
        return d

    def connectivity(self):
        """(rowptr, col, desc) in caller order, as device tensors."""
        torch = _torch()
        rowptr = torch.empty(self.ndet + 1, dtype=torch.int64, device=self.device)
        self._check(self._lib.hinqs_connectivity(self._h, self._ptr(rowptr), None, None))
        nnz = int(rowptr[-1].item())
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        desc = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        self._check(self._lib.hinqs_connectivity(self._h, self._ptr(rowptr), self._ptr(col),
                                                 self._ptr(desc)))
        return rowptr, col[:nnz], desc[:nnz]

    def permutation(self):
        torch = _torch()
        p = torch.empty(self.ndet, dtype=torch.int32, device=self.device)
        self._check(self._lib.hinqs_permutation(self._h, self._ptr(p)))
        return p

    def gram(self, A, B):
        """G = A^T B for device float64 tensors A (n x ma), B (n x nb) (row-major, contiguous)."""
        torch = _torch()
        self._dev(A, torch.float64)
        self._dev(B, torch.float64)
        n, ma = A.shape
        nb = B.shape[1]
        G = torch.empty((ma, nb), dtype=torch.float64, device=self.device)
        self._check(self._lib.hinqs_gram(self._h, n, self._ptr(A), ma, ma, self._ptr(B), nb, nb,
                                         self._ptr(G)))
        return G

    # ------------------------------------------------------ batched instances
    def batch_clear(self):
        self._check(self._lib.hinqs_batch_clear(self._h))

    def batch_add(self, h, eri, e_core, alpha, beta, nalpha: int, nbeta: int) -> int:
        """Add one independent instance (host inputs); returns its index."""
        h = _host_f64(h)
        eri = _host_f64(eri)
        norb = h.shape[0]
        if h.shape != (norb, norb) or eri.shape != (norb,) * 4:
            raise ValueError("h must be (n, n) and eri (n, n, n, n)")
        a = _host_u64(alpha)
        b = _host_u64(beta)
        if a.shape != b.shape or a.ndim != 1:
            raise ValueError("alpha and beta must be 1-D and equally long")
        idx = ctypes.c_int(-1)
        self._check(self._lib.hinqs_batch_add(
            self._h, norb, h.ctypes.data_as(ctypes.c_void_p), eri.ctypes.data_as(ctypes.c_void_p),
            float(e_core), len(a), a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p),
            nalpha, nbeta, ctypes.byref(idx)))
        return idx.value

    def batch_info(self):
        """(number of instances, coefficient offsets (n + 1), total couplings)."""
        n = ctypes.c_int(0)
        self._check(self._lib.hinqs_batch_info(self._h, ctypes.byref(n), None, None))
        off = np.zeros(n.value + 1, dtype=np.int64)
        nnz = ctypes.c_int64(0)
        self._check(self._lib.hinqs_batch_info(self._h, ctypes.byref(n), off.ctypes.data_as(ctypes.c_void_p),
                                               ctypes.byref(nnz)))
        return n.value, off, nnz.value

    def batch_lowest_eigenpair(self, *, block=8, max_space=None, max_iter=200, tol=1e-8, precond_floor=1e-8,
                               sorted_order=False, autotune=False, graph=True, raise_on_not_converged=True):
        """Lowest eigenpair of every batched instance.

        Returns (energies (n,), coefficient tensor (total determinants,) with instance i
        at offsets[i]:offsets[i+1], dict with offsets, status, iterations and stats)."""
        torch = _torch()
        n, off, _ = self.batch_info()
        o = Opts()
        self._lib.hinqs_opts_default(ctypes.byref(o))
        o.block = block
        o.max_space = max_space if max_space is not None else 6 * block
        o.max_iter = max_iter
        o.tol = tol
        o.precision = SOLVE_FP64
        o.precond_floor = precond_floor
        o.flags = ((SORTED_ORDER if sorted_order else 0) | (AUTOTUNE if autotune else 0)
                   | (0 if graph else NO_GRAPH))
        e = np.zeros(max(n, 1), dtype=np.float64)
        status = np.zeros(max(n, 1), dtype=np.int32)
        iters = np.zeros(max(n, 1), dtype=np.int32)
        c = torch.empty(int(off[-1]) if n else 1, dtype=torch.float64, device=self.device)
        st = BatchStats()
        rc = self._lib.hinqs_batch_lowest_eigenpair(
            self._h, ctypes.byref(o), e.ctypes.data_as(ctypes.c_void_p), self._ptr(c),
            status.ctypes.data_as(ctypes.c_void_p), iters.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st))
        if not (rc == -7 and not raise_on_not_converged):
            self._check(rc)
        return e[:n], c, {"offsets": off, "status": status[:n], "iterations": iters[:n],
                          "stats": st.as_dict(), "converged": rc == HINQS_OK}

    def autotune(self, k=8, precision=HINQS_FP64):
        """Tune the block-sigma launch shape for blocks of k vectors; returns
        ((team, unroll, workgroups per CU), tuned launch ms)."""
        shape = (ctypes.c_int * 3)()
        ms = ctypes.c_double(0.0)
        self._check(self._lib.hinqs_autotune(self._h, k, precision, shape, ctypes.byref(ms)))
        return tuple(shape), ms.value

    # ------------------------------------------------------------ selection
    def _dev_strings(self, x):
        """Determinant strings as a contiguous int64 device tensor (uint64 bit patterns)."""
        torch = _torch()
        if isinstance(x, torch.Tensor) and x.device.type == "cuda":
            return self._dev(x, torch.int64)
        return torch.from_numpy(_host_u64(x).view(np.int64)).to(self.device)

    def expand(self, c, ntop, sorted_order=False):
        """Classical expansion (Eq. 2) of the ntop largest-|c| determinants:
        (alpha, beta) of every coupled determinant outside B, ascending, as
        int64 device tensors, and the chosen indices (int32, largest |c| first)."""
        torch = _torch()
        self._dev(c, torch.float64)
        ntop = int(min(ntop, self.ndet))
        nv_a, nv_b = self.norb - self.na, self.norb - self.nb
        sa, sb = self.na * nv_a, self.nb * nv_b
        per = (sa + sb + self.na * (self.na - 1) // 2 * (nv_a * (nv_a - 1) // 2)
               + self.nb * (self.nb - 1) // 2 * (nv_b * (nv_b - 1) // 2) + sa * sb)
        cap = max(ntop * per, 1)
        out_a = torch.empty(cap, dtype=torch.int64, device=self.device)
        out_b = torch.empty(cap, dtype=torch.int64, device=self.device)
        top = torch.empty(max(ntop, 1), dtype=torch.int32, device=self.device)
        n = ctypes.c_int64(0)
        self._check(self._lib.hinqs_expand(self._h, self._ptr(c), ntop, cap, self._ptr(out_a),
                                           self._ptr(out_b), ctypes.byref(n), self._ptr(top),
                                           SORTED_ORDER if sorted_order else 0))
        n = n.value
        return out_a[:n].clone(), out_b[:n].clone(), top[:ntop]

    def pt2(self, c, e0, cand_alpha, cand_beta, sorted_order=False):
        """(numerator <x|H|Psi_0>, H_xx, score) of each candidate (Eq. 3) as
        float64 device tensors; candidates as device int64 tensors or host arrays."""
        torch = _torch()
        self._dev(c, torch.float64)
        ca, cb = self._dev_strings(cand_alpha), self._dev_strings(cand_beta)
        if ca.shape != cb.shape or ca.dim() != 1:
            raise ValueError("candidate alpha and beta must be 1-D and equally long")
        n = ca.numel()
        out = [torch.empty(max(n, 1), dtype=torch.float64, device=self.device) for _ in range(3)]
        self._check(self._lib.hinqs_pt2(self._h, self._ptr(c), float(e0), n, self._ptr(ca), self._ptr(cb),
                                        *[self._ptr(t) for t in out], SORTED_ORDER if sorted_order else 0))
        return tuple(t[:n] for t in out)

    def pt2_members(self, c, e0, sorted_order=False):
        """pt2() of every determinant of B (numerator = row of H_B c), from one sigma product."""
        torch = _torch()
        self._dev(c, torch.float64)
        out = [torch.empty(self.ndet, dtype=torch.float64, device=self.device) for _ in range(3)]
        self._check(self._lib.hinqs_pt2_members(self._h, self._ptr(c), float(e0), *[self._ptr(t) for t in out],
                                                SORTED_ORDER if sorted_order else 0))
        return tuple(out)

    def top_k(self, values, k, largest=False):
        """Indices (int32 device tensor) of the k smallest (largest) values, ties by lower index."""
        torch = _torch()
        self._dev(values, torch.float64)
        idx = torch.empty(max(int(k), 1), dtype=torch.int32, device=self.device)
        self._check(self._lib.hinqs_top_k(self._h, values.numel(), self._ptr(values), int(k),
                                          LARGEST if largest else 0, self._ptr(idx)))
        return idx[:k]

    def teacher_weights(self, c, sorted_order=False):
        """Spin-marginal teacher weights (Eqs. 5-6): (w over B, p_alpha, p_beta)
        as float64 device tensors; the marginals follow distinct_strings()."""
        torch = _torch()
        self._dev(c, torch.float64)
        inf = self.info()
        w = torch.empty(self.ndet, dtype=torch.float64, device=self.device)
        pa = torch.empty(inf["n_alpha_strings"], dtype=torch.float64, device=self.device)
        pb = torch.empty(inf["n_beta_strings"], dtype=torch.float64, device=self.device)
        self._check(self._lib.hinqs_teacher_weights(self._h, self._ptr(c), self._ptr(w), self._ptr(pa),
                                                    self._ptr(pb), SORTED_ORDER if sorted_order else 0))
        return w, pa, pb

    def distinct_strings(self):
        """Ascending distinct alpha and beta strings of B (int64 device tensors)."""
        torch = _torch()
        inf = self.info()
        a = torch.empty(inf["n_alpha_strings"], dtype=torch.int64, device=self.device)
        b = torch.empty(inf["n_beta_strings"], dtype=torch.int64, device=self.device)
        self._check(self._lib.hinqs_distinct_strings(self._h, self._ptr(a), self._ptr(b)))
        return a, b

    def update_determinants(self, add_alpha=None, add_beta=None, evict=None, coeffs=None, sorted_order=False):
        """Evict (int32 indices) and append (strings) determinants in place; returns
        (warm-start vector on the new set or None, update wall ms)."""
        torch = _torch()
        na_ = 0
        pa = pb = None
        if add_alpha is not None:
            ta, tb = self._dev_strings(add_alpha), self._dev_strings(add_beta)
            if ta.shape != tb.shape or ta.dim() != 1:
                raise ValueError("appended alpha and beta must be 1-D and equally long")
            na_ = ta.numel()
            pa, pb = self._ptr(ta), self._ptr(tb)
        ne = 0
        pe = None
        if evict is not None:
            te = evict if isinstance(evict, torch.Tensor) else torch.as_tensor(np.asarray(evict), dtype=torch.int32)
            te = te.to(device=self.device, dtype=torch.int32).contiguous()
            ne = te.numel()
            pe = self._ptr(te)
        c_new = None
        pc = pn = None
        if coeffs is not None:
            self._dev(coeffs, torch.float64)
            pc = self._ptr(coeffs)
            # sized for the largest possible new set; trimmed once the size is known
            c_new = torch.empty(self.ndet + na_, dtype=torch.float64, device=self.device)
            pn = self._ptr(c_new)
        ms = ctypes.c_double(0.0)
        self._check(self._lib.hinqs_update_determinants(self._h, ne, pe, na_, pa, pb, pc, pn,
                                                        SORTED_ORDER if sorted_order else 0, ctypes.byref(ms)))
        self.ndet = self.info()["ndet"]
        return (c_new[:self.ndet] if c_new is not None else None), ms.value

    def grow_basis(self, cand_alpha, cand_beta, cand_score, k, basis_score=None, b_max=0, coeffs=None,
                   rebuild=False):
        """Step-2 basis rules (append the k best candidates and cap at b_max, or
        rebuild from the k best of set + candidates).  Returns (warm start or
        None, scores of the new set or None, update ms)."""
        torch = _torch()
        ca, cb = self._dev_strings(cand_alpha), self._dev_strings(cand_beta)
        self._dev(cand_score, torch.float64)
        n = ca.numel()
        room = self.ndet + int(k)
        pc = pn = ps = pbs = None
        c_new = s_new = None
        if coeffs is not None:
            self._dev(coeffs, torch.float64)
            c_new = torch.empty(room, dtype=torch.float64, device=self.device)
            pc, pn = self._ptr(coeffs), self._ptr(c_new)
        if basis_score is not None:
            self._dev(basis_score, torch.float64)
            s_new = torch.empty(room, dtype=torch.float64, device=self.device)
            pbs, ps = self._ptr(basis_score), self._ptr(s_new)
        nn = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        self._check(self._lib.hinqs_grow_basis(
            self._h, GROW_REBUILD if rebuild else GROW_APPEND, n, self._ptr(ca), self._ptr(cb),
            self._ptr(cand_score), int(k), pbs, int(b_max), pc, pn, ps, ctypes.byref(nn), ctypes.byref(ms)))
        self.ndet = nn.value
        return (c_new[:self.ndet] if c_new is not None else None,
                s_new[:self.ndet] if s_new is not None else None, ms.value)

    def determinants(self):
        """(alpha, beta) of the current set in caller order (int64 device tensors)."""
        torch = _torch()
        a = torch.empty(self.ndet, dtype=torch.int64, device=self.device)
        b = torch.empty(self.ndet, dtype=torch.int64, device=self.device)
        self._check(self._lib.hinqs_get_determinants(self._h, self._ptr(a), self._ptr(b)))
        return a, b

    def product_closure(self):
        """(alpha, beta) int64 device tensors of the product-space determinants
        missing from the set, ascending."""
        torch = _torch()
        n = ctypes.c_int64(0)
        self._check(self._lib.hinqs_product_closure(self._h, 0, None, None, ctypes.byref(n)))
        a = torch.empty(max(n.value, 1), dtype=torch.int64, device=self.device)
        b = torch.empty(max(n.value, 1), dtype=torch.int64, device=self.device)
        self._check(self._lib.hinqs_product_closure(self._h, n.value, self._ptr(a), self._ptr(b),
                                                    ctypes.byref(n)))
        return a[:n.value], b[:n.value]

    def info(self):
        inf = Info()
        self._check(self._lib.hinqs_get_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()


def _make_energy_function():
    torch = _torch()

    class HinqsEnergy(torch.autograd.Function):
        """E_0(h, eri) on a fixed determinant set; backward returns the
        Hellmann-Feynman gradients (symmetrized 1- and 2-RDMs) from the
        library's adjoint kernel."""

        @staticmethod
        def forward(ctx, h, eri, solver, e_core=0.0, tol=1e-10, guess=None):
            solver.set_integrals(h, eri, e_core)
            e, c, st = solver.lowest_eigenpair(guess=guess, tol=tol)
            ctx.solver = solver
            ctx.save_for_backward(c)
            ctx.h_meta = (h.dtype, h.device)
            ctx.e_meta = (eri.dtype, eri.device)
            return torch.tensor(e, dtype=h.dtype, device=h.device)

        @staticmethod
        def backward(ctx, grad_out):
            (c,) = ctx.saved_tensors
            gh, ge = ctx.solver.integral_grad(c, float(grad_out))
            gh = gh.to(dtype=ctx.h_meta[0], device=ctx.h_meta[1])
            ge = ge.to(dtype=ctx.e_meta[0], device=ctx.e_meta[1])
            return gh, ge, None, None, None, None

    return HinqsEnergy


def __getattr__(name):
    if name == "HinqsEnergy":
        fn = _make_energy_function()
        globals()["HinqsEnergy"] = fn
        return fn
    raise AttributeError(name)
