"""Pins of the oracle's selection steps (paper Sec. 2.2, Steps 1' and 2): the
classical expansion of Eq. 2 and the PT2 importance of Eq. 3, checked against
an independent Jordan-Wigner construction of the Fock-space Hamiltonian, a
closed form and a combinatorial count."""
from math import comb

import numpy as np
import pytest

import oracle
import workloads as W
from tests import jw


def _small_case(norb=5, na=2, nb=2, nB=35, seed=11):
    ints = W.gen_integrals(norb, norb, -2.0, -0.5, 300 + seed)
    fa, fb = W.full_space(norb, na, nb)
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(fa), nB, replace=False)
    a, b = fa[pick], fb[pick]
    c = rng.standard_normal(nB)
    c /= np.linalg.norm(c)
    return ints, fa, fb, a, b, c


def test_pt2_matches_jordan_wigner():
    ints, fa, fb, a, b, c = _small_case()
    o = oracle.Oracle(ints.norb, 2, 2, ints.h, ints.eri, ints.e_core, a, b)
    H = jw.hamiltonian(ints.h, ints.eri, ints.e_core)
    iB = jw.basis_index(a, b, ints.norb)
    ix = jw.basis_index(fa, fb, ints.norb)
    e0 = -3.25
    num, hxx, score, absnum = o.pt2(c, e0, fa, fb, with_scale=True)
    num_ref = H[ix][:, iB] @ c
    hxx_ref = H[ix, ix].A1 if hasattr(H[ix, ix], "A1") else np.asarray(H[ix, ix]).ravel()
    scale = np.abs(H[ix][:, iB]).toarray() @ np.abs(c) + 1e-300
    assert np.all(np.abs(num - num_ref) <= 1e-12 * scale + 1e-15)
    assert np.allclose(absnum, scale, rtol=1e-12, atol=1e-15)
    assert np.allclose(hxx, hxx_ref, rtol=0, atol=1e-12)
    assert np.allclose(score, num_ref ** 2 / np.abs(e0 - hxx_ref), rtol=1e-11, atol=1e-15)
    # a member of B: the numerator is the row of H_B c, diagonal included
    HB = jw.projected(ints.h, ints.eri, ints.e_core, a, b)
    nB, hB, _ = o.pt2(c, e0, a, b)
    assert np.allclose(nB, HB @ c, rtol=0, atol=1e-12)
    assert np.allclose(hB, np.diag(HB), rtol=0, atol=1e-12)


@pytest.mark.parametrize("ntop", [1, 4, 35])
def test_expand_matches_jordan_wigner(ntop):
    ints, fa, fb, a, b, c = _small_case()
    o = oracle.Oracle(ints.norb, 2, 2, ints.h, ints.eri, ints.e_core, a, b)
    ya, yb, top = o.expand(c, ntop)
    order = sorted(range(len(c)), key=lambda i: (-abs(c[i]), i))
    assert list(top) == order[:ntop]
    H = jw.hamiltonian(ints.h, ints.eri, ints.e_core).tocsc()
    inB = set(jw.basis_index(a, b, ints.norb).tolist())
    ref = set()
    for i in order[:ntop]:
        col = H[:, int(jw.basis_index(a[i:i + 1], b[i:i + 1], ints.norb)[0])]
        for y, v in zip(col.indices, col.data):
            if abs(v) > 1e-12 and y not in inB:
                ref.add(int(y))
    lo = (1 << ints.norb) - 1
    got = [(int(x), int(y)) for x, y in zip(ya, yb)]
    assert got == sorted(got)                       # ascending (alpha, beta)
    assert len(set(got)) == len(got)                # distinct
    assert {al | (be << ints.norb) for al, be in got} == ref
    assert all((k & lo).bit_count() == 2 and (k >> ints.norb).bit_count() == 2 for k in ref)


def test_expand_reaches_every_single_and_double():
    """One determinant in B: the expansion is every single and double excitation
    of it (generic integrals make every Slater-Condon element nonzero)."""
    for norb, na, nb in ((6, 3, 3), (7, 4, 2), (5, 1, 3)):
        ints = W.gen_integrals(norb, norb, -2.0, -0.5, 40 + norb)
        a = np.array([(1 << na) - 1], dtype=np.uint64)
        b = np.array([(1 << nb) - 1], dtype=np.uint64)
        o = oracle.Oracle(norb, na, nb, ints.h, ints.eri, ints.e_core, a, b)
        ya, yb, top = o.expand(np.array([1.0]), 1)
        sa, sb = na * (norb - na), nb * (norb - nb)
        n = sa + sb + comb(na, 2) * comb(norb - na, 2) + comb(nb, 2) * comb(norb - nb, 2) + sa * sb
        assert len(ya) == n


def test_diagonal_hamiltonian_closed_form():
    """eri = 0 and diagonal h: H is diagonal, so nothing couples out of B, every
    outside numerator is 0 and H_xx = E_core + sum of the occupied h_pp."""
    norb, na, nb = 5, 2, 2
    hd = np.array([-1.0, -0.7, 0.2, 0.5, 1.1])
    h = np.diag(hd)
    eri = np.zeros((norb,) * 4)
    fa, fb = W.full_space(norb, na, nb)
    a, b = fa[:10], fb[:10]
    o = oracle.Oracle(norb, na, nb, h, eri, 0.25, a, b)
    c = np.linspace(1.0, 2.0, 10)
    ya, yb, _ = o.expand(c, 10)
    assert len(ya) == 0
    num, hxx, _ = o.pt2(c, -1.0, fa, fb)
    occ = lambda s: [p for p in range(norb) if (int(s) >> p) & 1]
    ref = np.array([0.25 + hd[occ(x)].sum() + hd[occ(y)].sum() for x, y in zip(fa, fb)])
    assert np.allclose(hxx, ref, atol=1e-14)
    assert np.allclose(num[:10], c * ref[:10], atol=1e-14)
    assert np.all(num[10:] == 0.0)


def test_expand_ties_prefer_lower_index():
    ints, fa, fb, a, b, c = _small_case()
    o = oracle.Oracle(ints.norb, 2, 2, ints.h, ints.eri, ints.e_core, a, b)
    cc = np.zeros(len(c))
    cc[[3, 7, 9, 12, 15, 20]] = [0.5, -0.5, 0.5, -0.5, 0.5, 0.25]
    _, _, top = o.expand(cc, 3)
    assert list(top) == [3, 7, 9]
    _, _, top = o.expand(cc, 6)
    assert list(top) == [3, 7, 9, 12, 15, 20]


def test_top_k_definition():
    """Hand-checked ranking: ties keep the lower index, -0.0 equals +0.0,
    infinities order at the ends, NaN is refused."""
    v = [0.5, -1.0, 0.0, -0.0, 0.5, np.inf, -np.inf, 2.0, -1.0]
    assert list(oracle.top_k(v, 4)) == [6, 1, 8, 2]
    assert list(oracle.top_k(v, 9)) == [6, 1, 8, 2, 3, 0, 4, 7, 5]
    assert list(oracle.top_k(v, 3, largest=True)) == [5, 7, 0]
    assert list(oracle.top_k(v, 9, largest=True)) == [5, 7, 0, 4, 2, 3, 1, 8, 6]
    with pytest.raises(oracle.OracleError):
        oracle.top_k([1.0, float("nan")], 1)


def test_teacher_weights_hand_example():
    """Three determinants (a1,b1), (a1,b2), (a2,b1) with c = (0.6, 0, 0.8):
    p_alpha = (0.36, 0.64), p_beta = (1.0, 0.0), so w = (0.36, 0, 0.64)."""
    a = np.array([3, 3, 5], dtype=np.uint64)
    b = np.array([3, 6, 3], dtype=np.uint64)
    w, ua, pa, ub, pb = oracle.teacher_weights(a, b, [0.6, 0.0, 0.8])
    assert list(ua) == [3, 5] and list(ub) == [3, 6]
    assert np.allclose(pa, [0.36, 0.64], rtol=0, atol=1e-15)
    assert np.allclose(pb, [1.0, 0.0], rtol=0, atol=1e-15)
    assert np.allclose(w, [0.36, 0.0, 0.64], rtol=0, atol=1e-15)
    # a sign flip or an overall scale changes nothing; one determinant gets weight 1
    w2 = oracle.teacher_weights(a, b, [-1.2, 0.0, 1.6])[0]
    assert np.allclose(w2, w, rtol=0, atol=1e-15)
    assert oracle.teacher_weights(a[:1], b[:1], [0.3])[0].tolist() == [1.0]
    with pytest.raises(oracle.OracleError):
        oracle.teacher_weights(a, b, [0.0, 0.0, 0.0])


def test_teacher_weights_product_state_is_exact():
    """On the full space a product vector c(alpha, beta) = u(alpha) v(beta) has
    marginals u^2 and v^2 (unit u, v), and the factorized weights reproduce
    |c|^2 exactly (the factorization drops nothing)."""
    norb, na, nb = 6, 2, 3
    sa = W.fci_strings(norb, na)
    sb = W.fci_strings(norb, nb)
    rng = np.random.default_rng(4)
    u = rng.standard_normal(len(sa))
    v = rng.standard_normal(len(sb))
    u /= np.linalg.norm(u)
    v /= np.linalg.norm(v)
    fa, fb = W.full_space(norb, na, nb)
    ia = np.searchsorted(sa, fa)
    ib = np.searchsorted(sb, fb)
    perm = rng.permutation(len(fa))
    c = (u[ia] * v[ib])[perm]
    w, ua, pa, ub, pb = oracle.teacher_weights(fa[perm], fb[perm], c)
    assert np.array_equal(ua, np.sort(sa)) and np.array_equal(ub, np.sort(sb))
    assert np.allclose(pa, u[np.argsort(sa)] ** 2, rtol=1e-13, atol=1e-16)
    assert np.allclose(pb, v[np.argsort(sb)] ** 2, rtol=1e-13, atol=1e-16)
    assert np.allclose(w, c ** 2, rtol=1e-12, atol=1e-17)
    assert abs(pa.sum() - 1) < 1e-14 and abs(pb.sum() - 1) < 1e-14 and abs(w.sum() - 1) < 1e-14


def test_teacher_weights_brute_force():
    """Tiny random set: every weight against a direct double loop over B."""
    norb, na, nb = 5, 2, 2
    fa, fb = W.full_space(norb, na, nb)
    rng = np.random.default_rng(8)
    pick = rng.choice(len(fa), 40, replace=False)
    a, b = fa[pick], fb[pick]
    c = rng.standard_normal(40)
    w = oracle.teacher_weights(a, b, c)[0]
    raw = []
    for i in range(40):
        pa = sum(c[j] ** 2 for j in range(40) if a[j] == a[i])
        pb = sum(c[j] ** 2 for j in range(40) if b[j] == b[i])
        raw.append(pa * pb)
    raw = np.array(raw)
    assert np.allclose(w, raw / raw.sum(), rtol=1e-13, atol=0)


def test_grow_basis_rules_hand_example():
    """Set scores (3, 1, 2, 1), candidate scores (5, 1, 4, 4), worked by hand:
    append k=2 -> candidates 0 then 2 (the tie 4 = 4 goes to the lower index);
    cap 5 -> the lowest of [3,1,2,1,5,4] is set member 1 (tied with 3);
    cap 3 -> set members 1, 3, 2 go; rebuild k=3 -> 5, 4, 4 are all
    candidates, so every set member goes; rebuild k=5 adds set members 0, 2."""
    bs = [3.0, 1.0, 2.0, 1.0]
    cs = [5.0, 1.0, 4.0, 4.0]
    assert oracle.grow_basis(bs, cs, 2) == ([0, 1, 2, 3], [0, 2])
    assert oracle.grow_basis(bs, cs, 2, b_max=5) == ([0, 2, 3], [0, 2])
    assert oracle.grow_basis(bs, cs, 2, b_max=3) == ([0], [0, 2])
    assert oracle.grow_basis(bs, cs, 3, rebuild=True) == ([], [0, 2, 3])
    kept, apps = oracle.grow_basis(bs, cs, 5, rebuild=True)
    assert kept == [0, 2] and apps == [0, 2, 3]
    # a capped append can also drop a just-chosen candidate
    assert oracle.grow_basis([9.0, 8.0], [1.0, 7.0], 2, b_max=3) == ([0, 1], [1])


def test_product_closure_definition():
    """{(a1,b1), (a2,b2)} closes to the two cross pairs; the full space closes
    to nothing; in general |closure| = |UA| |UB| - |B|."""
    a = np.array([3, 5], dtype=np.uint64)
    b = np.array([6, 9], dtype=np.uint64)
    ca, cb = oracle.product_closure(a, b)
    assert list(zip(ca.tolist(), cb.tolist())) == [(3, 9), (5, 6)]
    fa, fb = W.full_space(5, 2, 2)
    assert len(oracle.product_closure(fa, fb)[0]) == 0
    rng = np.random.default_rng(2)
    pick = rng.choice(len(fa), 30, replace=False)
    ca, cb = oracle.product_closure(fa[pick], fb[pick])
    assert len(ca) == len(set(fa[pick].tolist())) * len(set(fb[pick].tolist())) - 30
