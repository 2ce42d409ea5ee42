"""Pins for the CPU oracle: every check here is fixed by the paper or by the
mathematics, not by the oracle itself.

* Table 1 FCI dimensions (exact integers printed in the paper).
* A Jordan-Wigner Fock-space matrix built from Kronecker products (tests/jw.py)
  reproduces H_B element by element, signs included.
* Closed forms: one electron (spectrum of h), eri = 0 (sum of the lowest
  orbital energies), the textbook two-electron matrices (1 alpha 1 beta and
  2 alpha), the Hubbard dimer.
* Invariances: orbital rotations, Hermiticity, variational interlacing
  (Step 3 is an exact diagonalization within B, an upper bound).
* Density matrices: traces, partial trace, energy identity, Jordan-Wigner
  expectation values.
* Canonical excitation signs against Jordan-Wigner operator strings.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests import jw

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _ints(norb, seed, n_l=None, lo=-2.0, hi=-0.5):
    return W.gen_integrals(norb, n_l if n_l is not None else norb, lo, hi, seed)


def _rot_ints(ints, U):
    h = U.T @ ints.h @ U
    eri = np.einsum("pqrs,pa,qb,rc,sd->abcd", ints.eri, U, U, U, U, optimize=True)
    return W.Integrals(ints.norb, h, eri, ints.e_core)


# ----------------------------------------------------------------- Table 1
def test_table1_fci_dimensions():
    rows = []
    with open(os.path.join(GOLD, "table1_fci_dims.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, m, ne, dim, prec = line.split()
            rows.append((name, int(m), int(ne), float(dim), prec))
    assert len(rows) == 18
    for name, m, ne, dim, prec in rows:
        na = nb = ne // 2
        if math.comb(m, na) <= 100_000:
            n = len(W.fci_strings(m, na)) * len(W.fci_strings(m, nb))
        else:
            n = math.comb(m, na) * math.comb(m, nb)
        if prec == "exact":
            assert n == int(dim), name
        else:
            assert float(f"{n:.{int(prec)}g}") == dim, name


# ------------------------------------------------- Jordan-Wigner, element-wise
@pytest.mark.parametrize("norb,na,nb,seed", [(3, 2, 1, 11), (3, 1, 1, 12), (4, 2, 2, 13),
                                             (4, 3, 1, 14), (4, 2, 0, 15)])
def test_hamiltonian_matches_jordan_wigner(norb, na, nb, seed):
    ints = _ints(norb, seed)
    ints.e_core = 0.37
    alpha, beta = W.full_space(norb, na, nb)
    perm = np.random.default_rng(seed).permutation(len(alpha))
    alpha, beta = alpha[perm], beta[perm]
    o = oracle.Oracle.from_inputs(ints, alpha, beta, na, nb)
    H = o.dense()
    Hjw = jw.projected(ints.h, ints.eri, ints.e_core, alpha, beta)
    assert np.abs(H - Hjw).max() < 1e-13


def test_sampled_subset_matches_jordan_wigner():
    norb, na, nb = 4, 2, 2
    ints = _ints(norb, 21)
    alpha, beta = W.sample_determinants(norb, na, nb, 20, 0.5, 0.2, 22)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, na, nb)
    Hjw = jw.projected(ints.h, ints.eri, ints.e_core, alpha, beta)
    assert np.abs(o.dense() - Hjw).max() < 1e-13


# ---------------------------------------------------------------- closed forms
def test_one_electron_spectrum_is_eig_h():
    norb = 7
    ints = _ints(norb, 31)
    for na, nb in [(1, 0), (0, 1)]:
        alpha, beta = W.full_space(norb, na, nb)
        o = oracle.Oracle.from_inputs(ints, alpha, beta, na, nb)
        w = np.linalg.eigvalsh(o.dense())
        assert np.allclose(w, np.linalg.eigvalsh(ints.h), atol=1e-13)


def test_noninteracting_ground_state():
    """eri = 0 on the full space: E0 = E_core + lowest na + lowest nb eigenvalues of h."""
    norb, na, nb = 6, 3, 2
    ints = _ints(norb, 41)
    ints.eri[:] = 0.0
    ints.e_core = -1.25
    alpha, beta = W.full_space(norb, na, nb)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, na, nb)
    e, _ = o.lowest_eigenpair()
    eps = np.linalg.eigvalsh(ints.h)
    assert abs(e - (ints.e_core + eps[:na].sum() + eps[:nb].sum())) < 1e-12


def test_one_alpha_one_beta_textbook_matrix():
    """Distinguishable pair: <pr|H|qs> = h_pq d_rs + d_pq h_rs + (pq|rs)."""
    norb = 5
    ints = _ints(norb, 51)
    n = norb
    ref = (np.einsum("pq,rs->prqs", ints.h, np.eye(n)) + np.einsum("pq,rs->prqs", np.eye(n), ints.h)
           + np.einsum("pqrs->prqs", ints.eri)).reshape(n * n, n * n)
    alpha = np.repeat(np.uint64(1) << np.arange(n, dtype=np.uint64), n)
    beta = np.tile(np.uint64(1) << np.arange(n, dtype=np.uint64), n)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, 1, 1)
    assert np.abs(o.dense() - ref).max() < 1e-14


def test_two_alpha_antisymmetrized_matrix():
    """Same-spin pair p<r, q<s: h_pq d_rs + h_rs d_pq - h_ps d_rq - h_rq d_ps + (pq|rs) - (ps|rq)."""
    norb = 5
    ints = _ints(norb, 61)
    h, g = ints.h, ints.eri
    pairs = [(p, r) for p in range(norb) for r in range(p + 1, norb)]
    ref = np.zeros((len(pairs), len(pairs)))
    d = np.eye(norb)
    for I, (p, r) in enumerate(pairs):
        for J, (q, s) in enumerate(pairs):
            ref[I, J] = (h[p, q] * d[r, s] + h[r, s] * d[p, q] - h[p, s] * d[r, q] - h[r, q] * d[p, s]
                         + g[p, q, r, s] - g[p, s, r, q])
    alpha = np.array([(1 << p) | (1 << r) for p, r in pairs], dtype=np.uint64)
    beta = np.zeros(len(pairs), dtype=np.uint64)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, 2, 0)
    assert np.abs(o.dense() - ref).max() < 1e-14


def test_hubbard_dimer():
    vals = dict(line.split() for line in open(os.path.join(GOLD, "hubbard_dimer.txt"))
                if not line.startswith("#") and line.strip())
    t, U, E0 = float(vals["t"]), float(vals["U"]), float(vals["E0"])
    h = np.array([[0.0, -t], [-t, 0.0]])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
    alpha, beta = W.full_space(2, 1, 1)
    o = oracle.Oracle(2, 1, 1, h, eri, 0.0, alpha, beta)
    e, _ = o.lowest_eigenpair()
    assert abs(e - E0) < 1e-13
    assert abs(E0 - (U - math.sqrt(U * U + 16 * t * t)) / 2) < 1e-15


# ------------------------------------------------------------------ invariance
def test_orbital_rotation_invariance():
    norb, na, nb = 5, 2, 2
    ints = _ints(norb, 71)
    alpha, beta = W.full_space(norb, na, nb)
    e0, _ = oracle.Oracle.from_inputs(ints, alpha, beta, na, nb).lowest_eigenpair()
    q, _ = np.linalg.qr(np.random.default_rng(72).standard_normal((norb, norb)))
    e1, _ = oracle.Oracle.from_inputs(_rot_ints(ints, q), alpha, beta, na, nb).lowest_eigenpair()
    assert abs(e0 - e1) < 1e-12


def test_hermitian_and_variational_interlacing():
    ints, alpha, beta, cfg = W.config_inputs(0)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, cfg.na, cfg.nb)
    H = o.dense()
    assert np.abs(H - H.T).max() <= 1e-14 * np.abs(H).max()
    e_full, _ = o.lowest_eigenpair()
    # nested subsets: energies never go up as B grows, and bound the full space from above
    order = np.argsort(np.diag(H), kind="stable")
    prev = np.inf
    for m in (20, 50, 120, 250, 400):
        sel = np.sort(order[:m])
        om = oracle.Oracle.from_inputs(ints, alpha[sel], beta[sel], cfg.na, cfg.nb)
        em, _ = om.lowest_eigenpair()
        assert em >= e_full - 1e-12
        assert em <= prev + 1e-12
        prev = em
    assert abs(prev - e_full) < 1e-12


def test_sparse_lanczos_agrees_with_dense():
    ints, alpha, beta, cfg = W.config_inputs(1, ndet=3000)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, cfg.na, cfg.nb)
    e_dense, c_dense = o.lowest_eigenpair(dense_max=5000)
    e_lanczos, c_lanczos = o.lowest_eigenpair(dense_max=0)
    assert abs(e_dense - e_lanczos) < 1e-10
    assert abs(abs(c_dense @ c_lanczos) - 1) < 1e-9


# ------------------------------------------------------------------ sigma
def test_matrix_free_sigma_matches_matrix():
    ints, alpha, beta, cfg = W.config_inputs(1, ndet=2000)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, cfg.na, cfg.nb)
    X = W.random_block(len(alpha), 3, 5)
    rows = np.array([0, 7, 99, 1999])
    S = o.sigma_rows(X, rows)
    H = o.sparse()
    assert np.abs(S - (H @ X)[rows]).max() < 1e-12


# ------------------------------------------------------------------ couplings
def test_full_space_coupling_counts():
    """Every determinant of the full space couples to exactly the closed-form number
    of singles and doubles of each class."""
    norb, na, nb = 6, 3, 2
    ints = _ints(norb, 81)
    alpha, beta = W.full_space(norb, na, nb)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, na, nb)
    r = o.rows()
    va, vb = norb - na, norb - nb
    want = {oracle.E_1A: na * va, oracle.E_1B: nb * vb,
            oracle.E_2AA: math.comb(na, 2) * math.comb(va, 2),
            oracle.E_2BB: math.comb(nb, 2) * math.comb(vb, 2),
            oracle.E_2AB: na * va * nb * vb}
    for i in range(len(alpha)):
        et = r["etype"][r["rowptr"][i]:r["rowptr"][i + 1]]
        assert et[0] == oracle.E_DIAG
        for cls, n in want.items():
            assert int((et == cls).sum()) == n


def test_canonical_signs_against_jordan_wigner():
    norb, na, nb = 4, 2, 2
    ints = _ints(norb, 91)
    alpha, beta = W.full_space(norb, na, nb)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, na, nb)
    r = o.rows(np.arange(0, len(alpha), 5))
    x = jw.basis_index(alpha, beta, norb)
    n = norb
    checked = 0
    for t, i in enumerate(r["rows"]):
        for e in range(r["rowptr"][t] + 1, r["rowptr"][t + 1]):
            j = r["col"][e]
            et = int(r["etype"][e])
            h1, h2, p1, p2 = (int(v) for v in r["orb"][e])
            if et in (oracle.E_1A, oracle.E_1B):
                off = 0 if et == oracle.E_1A else n
                ref = jw.op_matrix_element(norb, x[i], x[j], [p1 + off], [h1 + off])
            elif et in (oracle.E_2AA, oracle.E_2BB):
                off = 0 if et == oracle.E_2AA else n
                ref = jw.op_matrix_element(norb, x[i], x[j], [p1 + off, p2 + off],
                                           [h2 + off, h1 + off])
            else:
                ref = jw.op_matrix_element(norb, x[i], x[j], [p1, p2 + n], [h2 + n, h1])
            assert ref == r["sign"][e]
            checked += 1
    assert checked > 100


def test_double_values_equal_signed_integrals():
    """Doubles carry one (opposite spin) or an antisymmetrized pair (same spin) of
    integrals times the canonical sign -- the value comes from the full operator sum."""
    ints, alpha, beta, cfg = W.config_inputs(0)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, cfg.na, cfg.nb)
    r = o.rows(np.arange(0, len(alpha), 7))
    g = ints.eri
    for e in range(len(r["col"])):
        et = r["etype"][e]
        h1, h2, p1, p2 = (int(v) for v in r["orb"][e])
        if et == oracle.E_2AB:
            assert abs(r["val"][e] - r["sign"][e] * g[p1, h1, p2, h2]) < 1e-14
        elif et in (oracle.E_2AA, oracle.E_2BB):
            v = g[p1, h1, p2, h2] - g[p1, h2, p2, h1]
            assert abs(r["val"][e] - r["sign"][e] * v) < 1e-14


# ------------------------------------------------------------------ RDMs
def test_rdm_identities():
    ints, alpha, beta, cfg = W.config_inputs(0)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, cfg.na, cfg.nb)
    e, c = o.lowest_eigenpair()
    d1, d2 = o.rdm12(c)
    N = cfg.na + cfg.nb
    assert abs(np.trace(d1) - N) < 1e-12
    assert abs(np.einsum("pprr", d2) - N * (N - 1)) < 1e-11
    assert np.abs(np.einsum("pqrr->pq", d2) - (N - 1) * d1).max() < 1e-12
    assert np.abs(d1 - d1.T).max() < 1e-13
    assert np.abs(d2 - d2.transpose(2, 3, 0, 1)).max() < 1e-13
    assert np.abs(d2 - d2.transpose(1, 0, 3, 2)).max() < 1e-13
    e_rdm = ints.e_core + np.sum(ints.h * d1) + 0.5 * np.sum(ints.eri * d2)
    assert abs(e_rdm - e) < 1e-11
    # sampled elements agree with the full tensor
    idx = np.random.default_rng(3).integers(0, cfg.norb, size=(40, 4))
    vals = o.rdm2_elements(c, idx)
    assert np.abs(vals - d2[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]]).max() < 1e-13


def test_rdm_against_jordan_wigner_expectations():
    norb, na, nb = 3, 2, 1
    ints = _ints(norb, 101)
    alpha, beta = W.sample_determinants(norb, na, nb, 7, 0.6, 0.0, 102)
    o = oracle.Oracle.from_inputs(ints, alpha, beta, na, nb)
    c = np.random.default_rng(103).standard_normal(len(alpha))
    d1, d2 = o.rdm12(c)
    M = 2 * norb
    a = jw.annihilators(M)
    x = jw.basis_index(alpha, beta, norb)
    psi = np.zeros(2 ** M)
    psi[x] = c
    for p in range(norb):
        for q in range(norb):
            ref = sum(psi @ (a[p + s * norb].T @ (a[q + s * norb] @ psi)) for s in (0, 1))
            assert abs(d1[p, q] - ref) < 1e-12
    rng = np.random.default_rng(104)
    for _ in range(30):
        p, q, r_, s_ = (int(v) for v in rng.integers(0, norb, 4))
        ref = 0.0
        for sg in (0, 1):
            for tg in (0, 1):
                v = a[q + sg * norb] @ psi
                v = a[s_ + tg * norb] @ v
                v = a[r_ + tg * norb].T @ v
                v = a[p + sg * norb].T @ v
                ref += psi @ v
        assert abs(d2[p, q, r_, s_] - ref) < 1e-12


def test_rejects_duplicates_and_bad_occupations():
    ints = _ints(4, 1)
    a = np.array([3, 3], dtype=np.uint64)
    b = np.array([3, 3], dtype=np.uint64)
    with pytest.raises(oracle.OracleError):
        oracle.Oracle.from_inputs(ints, a, b, 2, 2)
    with pytest.raises(oracle.OracleError):
        oracle.Oracle.from_inputs(ints, np.array([7], np.uint64), np.array([3], np.uint64), 2, 2)
    with pytest.raises(oracle.OracleError):
        oracle.Oracle.from_inputs(ints, np.array([3 | 16], np.uint64), np.array([3], np.uint64), 3, 2)
