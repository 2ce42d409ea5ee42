"""GPU parity of the selection steps around the subspace solve (Sec. 2.2):
the classical expansion (Eq. 2), the PT2 importance (Eq. 3) and the top-k
ranking, against the oracle on the same seeded inputs.

Bars:
  * expansion: the same determinant list (ascending, distinct) and the same
    chosen indices, bit for bit (integer work; every coupling value tested
    here is either generic or an exact structural zero, so the != 0 test is
    decided the same way by both sides);
  * PT2 numerator: |numer - ref| <= 1e-12 * sum_i |c_i <x_i|H|x>| (the
    oracle's own rounding scale of the sum);
  * H_xx: 1e-12 * max |H_xx| (as for the diagonal of B);
  * score: the library's score is exactly numer^2 / |e0 - H_xx| of its own
    outputs (IEEE), and matches the oracle within the bound propagated from
    the two bars above;
  * top-k: identical indices.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import log, oracle_for, solver_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hq = pytest.importorskip("paper_2606_26760_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hq.load_library()


def _coeffs(n, seed, levels=None):
    """Seeded CI-like vector: Gaussian signs and magnitudes with a decaying
    envelope over a random order (optionally quantized to `levels` distinct
    magnitudes to create ties), normalized."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n) * np.exp(-6.0 * rng.random(n))
    if levels is not None:
        c = np.sign(c) * (np.ceil(np.abs(c) / np.abs(c).max() * levels) / levels)
    return c / np.linalg.norm(c)


def _strings(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module")
def cas10():
    ints, a, b, cfg = W.config_inputs(1)
    log("selection fixture: cas10 20k determinants")
    return ints, a, b, cfg, solver_for(ints, a, b, cfg.na, cfg.nb), oracle_for(ints, a, b, cfg.na, cfg.nb)


def _check_expand(s, o, c, ntop):
    cd = torch.from_numpy(c).cuda()
    ya, yb, top = s.expand(cd, ntop)
    ra, rb, rtop = o.expand(c, ntop)
    assert np.array_equal(top.cpu().numpy(), rtop)
    assert np.array_equal(_strings(ya), ra) and np.array_equal(_strings(yb), rb), (len(ya), len(ra))
    return ra, rb


@pytest.mark.parametrize("ntop", [1, 37, 1000])
def test_expand_matches_oracle_cas10(cas10, ntop):
    ints, a, b, cfg, s, o = cas10
    log(f"expand cas10 ntop={ntop}")
    c = _coeffs(len(a), 31 + ntop)
    ra, rb = _check_expand(s, o, c, ntop)
    assert len(ra) > 0


def test_expand_ties_and_sorted_order(cas10):
    ints, a, b, cfg, s, o = cas10
    log("expand ties, sorted order")
    _check_expand(s, o, _coeffs(len(a), 5, levels=7), 300)   # many equal |c|
    c = _coeffs(len(a), 6)                                      # no ties
    ra, rb = _check_expand(s, o, c, 300)
    perm = s.permutation().cpu().numpy().astype(np.int64)       # sorted position -> caller index
    ya, yb, top = s.expand(torch.from_numpy(c[perm]).cuda(), 300, sorted_order=True)
    assert np.array_equal(_strings(ya), ra) and np.array_equal(_strings(yb), rb)
    assert np.array_equal(perm[top.cpu().numpy()], o.expand(c, 300)[2])


def test_expand_single_determinant_and_structural_zeros():
    log("expand: one determinant; diagonal Hamiltonian")
    norb, na, nb = 8, 3, 4
    ints = W.gen_integrals(norb, norb, -2.0, -0.5, 77)
    a = np.array([0b00000111], dtype=np.uint64)
    b = np.array([0b00001111], dtype=np.uint64)
    s = solver_for(ints, a, b, na, nb)
    o = oracle_for(ints, a, b, na, nb)
    ra, rb = _check_expand(s, o, np.array([1.0]), 5)
    sa, sb = na * (norb - na), nb * (norb - nb)
    assert len(ra) == sa + sb + 3 * 10 + 6 * 6 + sa * sb
    # eri = 0 and diagonal h: nothing couples
    h = np.diag(np.linspace(-1.0, 1.0, norb))
    fa, fb = W.full_space(norb, na, nb)
    s2 = hq.Hinqs()
    s2.set_integrals(h, np.zeros((norb,) * 4), 0.1)
    s2.set_determinants(fa[:50], fb[:50], na, nb)
    ya, yb, top = s2.expand(torch.ones(50, dtype=torch.float64, device="cuda"), 50)
    assert len(ya) == 0 and np.array_equal(top.cpu().numpy(), np.arange(50))


def test_expand_full_size_matches_oracle():
    ints, a, b, cfg = W.config_inputs(2)
    log("expand cas16 1e6 determinants, ntop 1000")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    c = _coeffs(len(a), 2024)
    ra, rb = _check_expand(s, o, c, 1000)
    log(f"  {len(ra)} distinct external determinants")
    # PT2 on a sample of them plus members of B, at the same size
    rng = np.random.default_rng(3)
    pick = rng.choice(len(ra), 1500, replace=False)
    inb = rng.choice(len(a), 500, replace=False)
    ca = np.concatenate([ra[pick], a[inb]])
    cb = np.concatenate([rb[pick], b[inb]])
    e0 = float(o.pt2(c, 0.0, a[:300], b[:300])[1].min()) - 0.5   # below the diagonal, as E_0 is
    _check_pt2(s, o, c, e0, ca, cb)


def _check_pt2(s, o, c, e0, ca, cb):
    num, hxx, score = s.pt2(torch.from_numpy(c).cuda(), e0, ca, cb)
    num, hxx, score = (t.cpu().numpy() for t in (num, hxx, score))
    rn, rh, rs, absnum = o.pt2(c, e0, ca, cb, with_scale=True)
    dn = 1e-12 * absnum + 1e-300
    assert np.all(np.abs(num - rn) <= dn), float(np.max(np.abs(num - rn) / dn))
    dh = 1e-12 * np.abs(rh).max()
    assert np.all(np.abs(hxx - rh) <= dh)
    assert np.array_equal(score, num * num / np.abs(e0 - hxx))
    den = np.abs(e0 - rh)
    bound = rs * (2 * dn / (np.abs(rn) + 1e-300) + dh / den) * 1.01 + 1e-300
    assert np.all(np.abs(score - rs) <= bound)
    return num, hxx, score


def test_pt2_matches_oracle_cas10(cas10):
    ints, a, b, cfg, s, o = cas10
    c = _coeffs(len(a), 8)
    ra, rb = o.expand(c, 200)[:2]
    rng = np.random.default_rng(9)
    inb = rng.choice(len(a), 3000, replace=False)
    dup = rng.choice(len(ra), 100)
    ca = np.concatenate([ra, a[inb], ra[dup]])
    cb = np.concatenate([rb, b[inb], rb[dup]])
    log(f"pt2 cas10: {len(ca)} candidates")
    e0 = float(o.pt2(c, 0.0, a[:300], b[:300])[1].min()) - 0.5
    num, hxx, score = _check_pt2(s, o, c, e0, ca, cb)
    # members of B: the numerator is the row of H_B c (diagonal included)
    assert np.count_nonzero(num) == len(num)


def test_pt2_members_matches_oracle_and_pt2(cas10):
    """PT2 of B's own members from one sigma product equals the oracle's PT2 of
    those strings (numerator: the row of H_B c with the diagonal) at the PT2
    bars, and the general kernel's results up to the order of the sums."""
    ints, a, b, cfg, s, o = cas10
    log("pt2 of the members of B (20k) via one sigma product")
    c = _coeffs(len(a), 31)
    e0 = float(o.pt2(c, 0.0, a[:300], b[:300])[1].min()) - 0.5
    cd = torch.from_numpy(c).cuda()
    num, hxx, score = (t.cpu().numpy() for t in s.pt2_members(cd, e0))
    rn, rh, rs, absnum = o.pt2(c, e0, a, b, with_scale=True)
    dn = 1e-12 * absnum + 1e-300
    assert np.all(np.abs(num - rn) <= dn)
    assert np.all(np.abs(hxx - rh) <= 1e-12 * np.abs(rh).max())
    assert np.array_equal(score, num * num / np.abs(e0 - hxx))
    gn, gh, gs = (t.cpu().numpy() for t in s.pt2(cd, e0, a, b))
    assert np.all(np.abs(num - gn) <= 2 * dn) and np.array_equal(hxx, gh)
    # sorted order: the same values permuted
    perm = s.permutation().cpu().numpy().astype(np.int64)
    n2 = s.pt2_members(torch.from_numpy(c[perm]).cuda(), e0, sorted_order=True)[0].cpu().numpy()
    assert np.array_equal(n2, num[perm])


def test_pt2_sorted_order_and_device_candidates(cas10):
    ints, a, b, cfg, s, o = cas10
    log("pt2 sorted order, device candidates")
    c = _coeffs(len(a), 12)
    perm = s.permutation().cpu().numpy().astype(np.int64)
    ya, yb, _ = s.expand(torch.from_numpy(c).cuda(), 20)
    n1, h1, s1 = s.pt2(torch.from_numpy(c).cuda(), -14.0, ya, yb)
    n2, h2, s2 = s.pt2(torch.from_numpy(c[perm]).cuda(), -14.0, ya, yb, sorted_order=True)
    assert torch.equal(n1, n2) and torch.equal(h1, h2) and torch.equal(s1, s2)
    rn = o.pt2(c, -14.0, _strings(ya), _strings(yb))[0]
    assert np.allclose(n1.cpu().numpy(), rn, rtol=0, atol=1e-12)


def test_pt2_edge_cases(cas10):
    ints, a, b, cfg, s, o = cas10
    log("pt2 edge cases")
    c = torch.from_numpy(_coeffs(len(a), 4)).cuda()
    n, h, sc = s.pt2(c, -10.0, np.zeros(0, np.uint64), np.zeros(0, np.uint64))
    assert n.numel() == 0
    # e0 equal to H_xx: division by zero gives inf (numerator nonzero)
    _, hx, _ = s.pt2(c, -10.0, a[:1], b[:1])
    _, _, sc = s.pt2(c, float(hx[0]), a[:1], b[:1])
    assert np.isinf(sc.cpu().numpy()[0])
    # wrong electron count / bits above norb: NaN outputs for those, error returned
    bad_a = np.array([a[0], a[1] | (1 << 11), a[2]], dtype=np.uint64)
    bad_b = np.array([b[0], b[1], b[2] ^ 1], dtype=np.uint64)
    with pytest.raises(hq.HinqsError) as ex:
        s.pt2(c, -10.0, bad_a, bad_b)
    assert ex.value.name == "BAD_OCCUPATION"
    with pytest.raises(hq.HinqsError) as ex:
        s.expand(torch.full((len(a),), float("nan"), dtype=torch.float64, device="cuda"), 3)
    assert ex.value.name == "NONFINITE"
    with pytest.raises(hq.HinqsError) as ex:
        s.expand(c, 0)
    assert ex.value.name == "INVALID_ARG"


@pytest.mark.parametrize("n", [1, 7, 1000, 100_003])
def test_top_k_matches_oracle(n):
    rng = np.random.default_rng(n)
    v = np.round(rng.standard_normal(n) * 4) / 4            # ties
    if n > 10:
        v[rng.choice(n, 5, replace=False)] = [np.inf, -np.inf, 0.0, -0.0, 1e300]
    s = hq.Hinqs()
    vd = torch.from_numpy(v).cuda()
    for k in sorted({1, max(1, n // 3), n}):
        for largest in (False, True):
            got = s.top_k(vd, k, largest=largest).cpu().numpy()
            assert np.array_equal(got, oracle.top_k(v, k, largest=largest)), (n, k, largest)
    with pytest.raises(hq.HinqsError) as ex:
        s.top_k(vd, n + 1)
    assert ex.value.name == "INVALID_ARG"
    v[0] = np.nan
    with pytest.raises(hq.HinqsError) as ex:
        s.top_k(torch.from_numpy(v).cuda(), 1)
    assert ex.value.name == "NONFINITE"


# ------------------------------------------------------------ teacher weights
# Bars: every marginal and weight within 1e-12 relative (sums of positive
# terms: the oracle's sequential bincount over groups of <= 2,284 entries is
# the larger rounding, <= 2.6e-13 relative); sorted and caller order bitwise
# equal after the permutation.
def _check_weights(s, a, b, c):
    w, pa, pb = s.teacher_weights(torch.from_numpy(c).cuda())
    rw, rua, rpa, rub, rpb = oracle.teacher_weights(a, b, c)
    ua, ub = s.distinct_strings()
    assert np.array_equal(_strings(ua), rua) and np.array_equal(_strings(ub), rub)
    for got, ref in ((w, rw), (pa, rpa), (pb, rpb)):
        got = got.cpu().numpy()
        assert np.all(np.abs(got - ref) <= 1e-12 * np.abs(ref)), float(np.max(np.abs(got - ref) / np.abs(ref)))
    return w


def test_teacher_weights_cas10(cas10):
    ints, a, b, cfg, s, o = cas10
    log("teacher weights cas10")
    c = _coeffs(len(a), 17)
    w = _check_weights(s, a, b, c)
    perm = s.permutation().cpu().numpy().astype(np.int64)
    ws, pas, pbs = s.teacher_weights(torch.from_numpy(c[perm]).cuda(), sorted_order=True)
    assert torch.equal(ws.cpu(), w.cpu()[perm])
    with pytest.raises(hq.HinqsError) as ex:
        s.teacher_weights(torch.zeros(len(a), dtype=torch.float64, device="cuda"))
    assert ex.value.name == "INVALID_ARG"
    bad = torch.from_numpy(c).cuda()
    bad[5] = float("inf")
    with pytest.raises(hq.HinqsError) as ex:
        s.teacher_weights(bad)
    assert ex.value.name == "NONFINITE"


def test_teacher_weights_full_space_product_state():
    """Product vector on the full CAS(6,6) space: the weights are |c|^2."""
    log("teacher weights: product state")
    ints, a, b, cfg = W.config_inputs(0)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    sa, sb = W.fci_strings(6, 3), W.fci_strings(6, 3)
    rng = np.random.default_rng(21)
    u, v = rng.standard_normal(len(sa)), rng.standard_normal(len(sb))
    c = u[np.searchsorted(sa, a)] * v[np.searchsorted(sb, b)]
    c /= np.linalg.norm(c)
    w = _check_weights(s, a, b, c).cpu().numpy()
    assert np.allclose(w, c ** 2, rtol=1e-12, atol=1e-18)


def test_teacher_weights_full_size():
    ints, a, b, cfg = W.config_inputs(2)
    log("teacher weights cas16 1e6")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    _check_weights(s, a, b, _coeffs(len(a), 99))


@pytest.mark.parametrize("norb,na,nb", [(18, 9, 8), (24, 12, 12), (32, 16, 15), (32, 3, 2)])
def test_expand_and_pt2_large_orbital_counts(norb, na, nb):
    """More than 64 alpha single moves (81, 144, 256) and, from norb 24,
    integrals read from global memory instead of LDS; norb 32 uses the top
    bit of the strings and the largest orbital fields of the descriptors."""
    log(f"expand + pt2 at norb {norb} ({na}a {nb}b)")
    ints = W.gen_integrals(norb, norb, -2.0, -0.5, 900 + norb)
    a, b = W.sample_determinants(norb, na, nb, 2000, 0.3, 0.0, 910 + norb)
    s = solver_for(ints, a, b, na, nb)
    o = oracle_for(ints, a, b, na, nb)
    c = _coeffs(len(a), norb)
    ra, rb = _check_expand(s, o, c, 3)
    rng = np.random.default_rng(norb)
    pick = rng.choice(len(ra), 300, replace=False)
    inb = rng.choice(len(a), 100, replace=False)
    ca = np.concatenate([ra[pick], a[inb]])
    cb = np.concatenate([rb[pick], b[inb]])
    e0 = float(o.pt2(c, 0.0, a[:50], b[:50])[1].min()) - 0.5
    _check_pt2(s, o, c, e0, ca, cb)


def test_expand_every_determinant_and_ntop_clamp():
    """ntop = ndet (every determinant of a 300-determinant set expanded)
    against the oracle, then the same call through the C ABI with ntop above
    ndet: the library clamps it and returns the same list."""
    import ctypes
    ints, a, b, cfg = W.config_inputs(1, ndet=300)
    log("expand all 300 determinants; ntop above ndet through the C ABI")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    c = _coeffs(len(a), 5)
    ra, rb = _check_expand(s, o, c, len(a))
    cd = torch.from_numpy(c).cuda()
    ntop = len(a) + 100
    cap = len(ra) + 1000
    out_a = torch.empty(cap, dtype=torch.int64, device="cuda")
    out_b = torch.empty(cap, dtype=torch.int64, device="cuda")
    top = torch.full((ntop,), -1, dtype=torch.int32, device="cuda")
    n = ctypes.c_int64(0)
    rc = s._lib.hinqs_expand(s._h, s._ptr(cd), ntop, cap, s._ptr(out_a), s._ptr(out_b), ctypes.byref(n),
                             s._ptr(top), 0)
    torch.cuda.synchronize()
    assert rc == 0 and n.value == len(ra)
    assert np.array_equal(_strings(out_a[:n.value]), ra) and np.array_equal(_strings(out_b[:n.value]), rb)
    t = top.cpu().numpy()
    assert np.array_equal(np.sort(t[:len(a)]), np.arange(len(a))) and np.all(t[len(a):] == -1)
