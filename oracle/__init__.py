"""CPU oracle for the selected-CI hot path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
``paper_2606_26760_amd``; the two meet only in the seeded input generators of
``workloads``.

* ``oracle.c`` (plain C + OpenMP) applies creation/annihilation operators bit
  by bit to build rows of the projected Hamiltonian [H_B]_ij = <x_i|H|x_j>
  (paper Sec. 2.2, the Hamiltonian before Step 1, and Step 3), the sigma
  product H_B X, the excitation class and canonical sign of every coupled
  pair, and the one- and two-particle density matrices.
* The selection steps around Step 3 (Sec. 2.2, Steps 1' and 2): the classical
  expansion of Eq. 2 and the PT2 importance of Eq. 3, from the same operator
  application extended to determinants outside B.
* The lowest eigenpair (Step 3, "diagonalized with a Davidson eigensolver")
  is taken from LAPACK ``eigh`` on the dense matrix, or ARPACK ``eigsh`` on
  the sparse one for larger sets -- a library primitive standing in for the
  exact diagonalization within B that the paper asks of Step 3.

Every function here is pinned by ``tests/test_oracle_pins.py`` against closed
forms, textbook matrices, a Jordan-Wigner matrix construction, invariances and
density-matrix identities.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# excitation classes reported by rows(): see classify() in oracle.c
E_DIAG, E_1A, E_1B, E_2AA, E_2BB, E_2AB = 0, 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (-O2 -fopenmp)."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", src, "-o", _LIB_PATH + ".tmp",
           "-lm"]
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=True)
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            i64 = ctypes.c_int64
            lib.or_create.restype = P
            lib.or_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_double,
                                      i64, P, P, ctypes.POINTER(ctypes.c_int)]
            lib.or_destroy.argtypes = [P]
            lib.or_rows.restype = i64
            lib.or_rows.argtypes = [P, i64, P]
            lib.or_rows_export.argtypes = [P, P, P, P, P, P, P]
            lib.or_sigma_rows.restype = i64
            lib.or_sigma_rows.argtypes = [P, i64, P, ctypes.c_int, P, P]
            lib.or_rdm12.argtypes = [P, P, P, P]
            lib.or_rdm2_elements.argtypes = [P, P, i64, P, P]
            lib.or_num_threads.restype = ctypes.c_int
            lib.or_pt2.argtypes = [P, P, ctypes.c_double, i64, P, P, P, P, P, P]
            lib.or_expand.restype = i64
            lib.or_expand.argtypes = [P, P, i64, P, i64, P, P]
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


class Oracle:
    """Handle on one (integrals, determinant set) pair, caller order kept."""

    def __init__(self, norb, na, nb, h, eri, e_core, alpha, beta):
        lib = _load()
        self.norb, self.na, self.nb = int(norb), int(na), int(nb)
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.eri = np.ascontiguousarray(eri, dtype=np.float64)
        self.e_core = float(e_core)
        self.alpha = np.ascontiguousarray(alpha, dtype=np.uint64)
        self.beta = np.ascontiguousarray(beta, dtype=np.uint64)
        self.ndet = len(self.alpha)
        st = ctypes.c_int(0)
        self._h = lib.or_create(self.norb, self.na, self.nb, _ptr(self.h), _ptr(self.eri),
                                self.e_core, self.ndet, _ptr(self.alpha), _ptr(self.beta),
                                ctypes.byref(st))
        if not self._h:
            raise OracleError({1: "bad arguments", 2: "duplicate determinant",
                               3: "wrong electron count or stray bits"}.get(st.value, "error"))

    @classmethod
    def from_inputs(cls, ints, alpha, beta, na, nb):
        return cls(ints.norb, na, nb, ints.h, ints.eri, ints.e_core, alpha, beta)

    def __del__(self):
        if getattr(self, "_h", None):
            _load().or_destroy(self._h)
            self._h = None

    @staticmethod
    def num_threads() -> int:
        return int(_load().or_num_threads())

    # ------------------------------------------------------------ H_B rows
    def rows(self, rows=None):
        """Rows of H_B with their couplings.

        Returns dict(rowptr, col, val, etype, orb (n,4), sign); each row lists
        its diagonal first, then the coupled determinants in ascending index.
        """
        lib = _load()
        r = np.arange(self.ndet, dtype=np.int64) if rows is None else \
            np.ascontiguousarray(rows, dtype=np.int64)
        tot = lib.or_rows(self._h, len(r), _ptr(r))
        out = dict(rows=r,
                   rowptr=np.empty(len(r) + 1, np.int64),
                   col=np.empty(max(tot, 1), np.int64),
                   val=np.empty(max(tot, 1), np.float64),
                   etype=np.empty(max(tot, 1), np.int8),
                   orb=np.empty((max(tot, 1), 4), np.int8),
                   sign=np.empty(max(tot, 1), np.int8))
        lib.or_rows_export(self._h, _ptr(out["rowptr"]), _ptr(out["col"]), _ptr(out["val"]),
                           _ptr(out["etype"]), _ptr(out["orb"]), _ptr(out["sign"]))
        for key in ("col", "val", "etype", "orb", "sign"):
            out[key] = out[key][:tot]
        return out

    def sparse(self):
        """The whole H_B as a scipy CSR matrix (caller order)."""
        import scipy.sparse as sp
        o = self.rows()
        return sp.csr_matrix((o["val"], o["col"], o["rowptr"]), shape=(self.ndet, self.ndet))

    def dense(self):
        return self.sparse().toarray()

    def diag(self):
        o = self.rows()
        return o["val"][o["rowptr"][:-1]]

    # ------------------------------------------------------------- sigma
    def sigma_rows(self, X, rows=None, return_pairs=False):
        """S[r] = sum_j <x_rows[r]|H|x_j> X[j] by operator application (matrix-free).

        With return_pairs, also the number of stored (row, column) elements visited."""
        lib = _load()
        X = np.ascontiguousarray(X, dtype=np.float64)
        if X.ndim == 1:
            X = X[:, None]
        k = X.shape[1]
        r = np.arange(self.ndet, dtype=np.int64) if rows is None else \
            np.ascontiguousarray(rows, dtype=np.int64)
        S = np.empty((len(r), k), np.float64)
        pairs = lib.or_sigma_rows(self._h, len(r), _ptr(r), k, _ptr(X), _ptr(S))
        return (S, int(pairs)) if return_pairs else S

    # ---------------------------------------------------------- eigenpair
    def lowest_eigenpair(self, dense_max: int = 5000, tol: float = 1e-13):
        """Lowest eigenvalue and eigenvector of H_B (exact diagonalization in B).

        Sign gauge: the largest-|c| component is positive (ties: lowest index)."""
        if self.ndet <= dense_max:
            w, v = np.linalg.eigh(self.dense())
            e, c = float(w[0]), v[:, 0].copy()
        else:
            from scipy.sparse.linalg import eigsh
            H = self.sparse()
            w, v = eigsh(H, k=1, which="SA", tol=tol, ncv=40)
            e, c = float(w[0]), v[:, 0].copy()
        c /= np.linalg.norm(c)
        m = int(np.argmax(np.abs(c)))
        if c[m] < 0:
            c = -c
        return e, c

    def spectrum(self, nroots: int = 2):
        """Lowest ``nroots`` eigenvalues (dense for small sets, Lanczos otherwise)."""
        if self.ndet <= 5000:
            return np.linalg.eigvalsh(self.dense())[:nroots]
        from scipy.sparse.linalg import eigsh
        w = eigsh(self.sparse(), k=nroots, which="SA", tol=1e-13, ncv=max(40, 4 * nroots),
                  return_eigenvectors=False)
        return np.sort(w)

    # --------------------------------------------------------------- RDMs
    def rdm12(self, c):
        lib = _load()
        c = np.ascontiguousarray(c, dtype=np.float64)
        n = self.norb
        d1 = np.empty((n, n))
        d2 = np.empty((n, n, n, n))
        lib.or_rdm12(self._h, _ptr(c), _ptr(d1), _ptr(d2))
        return d1, d2

    def rdm2_elements(self, c, idx):
        lib = _load()
        c = np.ascontiguousarray(c, dtype=np.float64)
        idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 4)
        out = np.empty(len(idx))
        lib.or_rdm2_elements(self._h, _ptr(c), len(idx), _ptr(idx), _ptr(out))
        return out

    # ------------------------------------------------ selection (Eq. 2, Eq. 3)
    def pt2(self, c, e0, cand_alpha, cand_beta, with_scale=False):
        """(numerator <x|H|Psi_0>, H_xx, score) of each candidate determinant (Eq. 3);
        c in caller order.  with_scale adds sum_i |c_i <x_i|H|x>| per candidate."""
        c = np.ascontiguousarray(c, dtype=np.float64)
        ca = np.ascontiguousarray(cand_alpha, dtype=np.uint64)
        cb = np.ascontiguousarray(cand_beta, dtype=np.uint64)
        n = len(ca)
        num = np.zeros(n)
        hxx = np.zeros(n)
        score = np.zeros(n)
        absnum = np.zeros(n) if with_scale else None
        _load().or_pt2(self._h, _ptr(c), float(e0), n, _ptr(ca), _ptr(cb), _ptr(num), _ptr(hxx),
                       _ptr(score), _ptr(absnum) if with_scale else None)
        return (num, hxx, score, absnum) if with_scale else (num, hxx, score)

    def expand(self, c, ntop):
        """Classical expansion (Eq. 2): (alpha, beta) of every determinant outside B
        coupled to one of the ntop largest-|c| determinants, ascending (alpha, beta),
        and the caller indices of those ntop determinants."""
        lib = _load()
        c = np.ascontiguousarray(c, dtype=np.float64)
        ntop = int(min(ntop, self.ndet))
        top = np.zeros(max(ntop, 1), dtype=np.int32)
        z = np.zeros(1, dtype=np.uint64)
        n = lib.or_expand(self._h, _ptr(c), ntop, _ptr(top), 0, _ptr(z), _ptr(z))
        out_a = np.zeros(max(n, 1), dtype=np.uint64)
        out_b = np.zeros(max(n, 1), dtype=np.uint64)
        lib.or_expand(self._h, _ptr(c), ntop, _ptr(top), n, _ptr(out_a), _ptr(out_b))
        return out_a[:n], out_b[:n], top[:ntop]


def top_k(values, k, largest=False):
    """Indices of the k smallest (largest) values, ties by the lower index and
    -0.0 equal to +0.0: the ranking of Sec. 2.2 (cold start by H_xx, later
    iterations by the Eq. 3 score), written as a plain sort."""
    v = [float(x) + 0.0 for x in np.asarray(values, dtype=np.float64)]
    if any(x != x for x in v):
        raise OracleError("NaN in values")
    order = sorted(range(len(v)), key=lambda i: ((-v[i]) if largest else v[i], i))
    return np.array(order[:k], dtype=np.int64)


def teacher_weights(alpha, beta, c):
    """Spin-marginal teacher weights of Sec. 2.2 Step 4 (Eqs. 5-6), c in the
    order of (alpha, beta): p_alpha(s) sums c^2 over the determinants with
    alpha string s, p_beta likewise, and w(x) = p_alpha p_beta normalized over
    the set.  Returns (w, distinct alpha strings, p_alpha, distinct beta
    strings, p_beta), strings ascending."""
    a = np.asarray(alpha, dtype=np.uint64)
    b = np.asarray(beta, dtype=np.uint64)
    c2 = np.asarray(c, dtype=np.float64) ** 2
    ua, ia = np.unique(a, return_inverse=True)
    ub, ib = np.unique(b, return_inverse=True)
    pa = np.bincount(ia, weights=c2, minlength=len(ua))
    pb = np.bincount(ib, weights=c2, minlength=len(ub))
    w = pa[ia] * pb[ib]
    z = w.sum()
    if not z > 0:
        raise OracleError("the weights sum to zero")
    return w / z, ua, pa, ub, pb


def grow_basis(basis_score, cand_score, k, b_max=0, rebuild=False):
    """The basis-update rules of Sec. 2.2 Step 2, on indices: returns (kept
    basis indices in their order, chosen candidate indices in append order).
    Append (t >= 2): the k best candidates, best first; if the set then
    exceeds b_max (> 0), the lowest-scored of the set and of those k are
    dropped.  Rebuild (t = 1): the k best of set and candidates together.
    Ties by the lower index of [set; candidates] (via top_k)."""
    nb = len(basis_score) if basis_score is not None else 0
    if rebuild:
        comb = list(basis_score) + list(cand_score)
        chosen = [int(i) for i in top_k(comb, min(k, len(comb)), largest=True)]
        keep = set(i for i in chosen if i < nb)
        return [i for i in range(nb) if i in keep], [i - nb for i in chosen if i >= nb]
    kk = min(k, len(cand_score))
    apps = [int(i) for i in top_k(cand_score, kk, largest=True)] if kk else []
    kept = list(range(nb))
    if b_max and nb + kk > b_max:
        comb = list(basis_score) + [float(cand_score[t]) for t in apps]
        low = set(int(i) for i in top_k(comb, nb + kk - b_max))
        kept = [i for i in range(nb) if i not in low]
        apps = [t for j, t in enumerate(apps) if nb + j not in low]
    return kept, apps


def product_closure(alpha, beta):
    """The determinants of (distinct alpha strings) x (distinct beta strings)
    not in the set, ascending (alpha, beta): the product space the backends
    of Sec. 2.2 Step 3 diagonalize on, minus the set itself."""
    have = set(zip((int(x) for x in alpha), (int(y) for y in beta)))
    ua = sorted(set(int(x) for x in alpha))
    ub = sorted(set(int(y) for y in beta))
    out = [(x, y) for x in ua for y in ub if (x, y) not in have]
    return (np.array([p[0] for p in out], dtype=np.uint64), np.array([p[1] for p in out], dtype=np.uint64))
