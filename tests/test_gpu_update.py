"""GPU parity of the incremental basis update (Sec. 2.2: Step 2 appends new
determinants and evicts old ones from the second iteration on; Step 3 keeps
its state and warm-starts).  After an update the context must hold exactly
the set B' = (kept determinants in caller order) + (appended ones), as the
oracle builds it from scratch:

  * couplings: per row the same (column, class, orbitals, sign) set as the
    oracle's rows of H_B' (bit-exact; entries may come in another order);
  * diagonal within 1e-12 * max |H_ii|; sigma within 1e-12 * sum_j |H_ij||X_j|
    per row and column (the FP64 sigma bar);
  * lowest eigenvalue within 1e-10 Ha of the oracle's, warm-started from the
    carried vector (kept coefficients bit-equal, appended ones zero);
  * a rejected update (repeat, bad occupation, bad index) leaves the context
    as it was.
Appended determinants come from the oracle's classical expansion of B or
from seeded draws, never from the library.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_helpers import (gpu_rows_as_tuples, log, oracle_for, oracle_rows_as_tuples, row_bound,
                               solver_for)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hq = pytest.importorskip("paper_2606_26760_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hq.load_library()


def _coeffs(n, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(n) * np.exp(-6.0 * rng.random(n))
    return c / np.linalg.norm(c)


def _new_set(a, b, evict, add_a, add_b):
    keep = np.ones(len(a), bool)
    keep[np.asarray(evict, dtype=np.int64)] = False
    return (np.concatenate([a[keep], add_a]).astype(np.uint64),
            np.concatenate([b[keep], add_b]).astype(np.uint64), keep)


def _check_set(s, o, rows, X_seed=5):
    got = gpu_rows_as_tuples(s, rows)
    want, r = oracle_rows_as_tuples(o, rows)
    for i in rows:
        assert got[int(i)] == want[int(i)], f"row {i}"
    d = s.diag().cpu().numpy()
    ref = r["val"][r["rowptr"][:-1]]
    assert np.abs(d[rows] - ref).max() <= 1e-12 * np.abs(ref).max()
    X = W.random_block(o.ndet, 8, X_seed)
    S = s.sigma(torch.from_numpy(X).cuda()).cpu().numpy()
    Sr = o.sigma_rows(X, rows)
    bound = row_bound(r, X, 8)
    assert np.all(np.abs(S[rows] - Sr) <= 1e-12 * bound + 1e-300)


@pytest.fixture(scope="module")
def cas10():
    ints, a, b, cfg = W.config_inputs(1)
    c = _coeffs(len(a), 41)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    ea, eb, _ = o.expand(c, 150)
    return ints, a, b, cfg, c, ea, eb


@pytest.mark.parametrize("n_evict,n_add", [(500, 3000), (0, 2000), (700, 0), (19_999, 5)])
def test_update_matches_fresh_oracle(cas10, n_evict, n_add):
    ints, a, b, cfg, c, ea, eb = cas10
    log(f"update cas10: evict {n_evict}, append {n_add}")
    rng = np.random.default_rng(n_evict + 7 * n_add)
    evict = rng.choice(len(a), n_evict, replace=False).astype(np.int32)
    pick = rng.choice(len(ea), n_add, replace=False)
    add_a, add_b = ea[pick], eb[pick]
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    cd = torch.from_numpy(c).cuda()
    c_new, ms = s.update_determinants(add_a, add_b, evict=evict, coeffs=cd)
    na_, nb_, keep = _new_set(a, b, evict, add_a, add_b)
    assert s.ndet == len(na_) and s.info()["ndet"] == len(na_)
    cn = c_new.cpu().numpy()
    assert np.array_equal(cn[:keep.sum()], c[keep]) and np.all(cn[keep.sum():] == 0.0)
    o2 = oracle_for(ints, na_, nb_, cfg.na, cfg.nb)
    rows = np.arange(len(na_)) if len(na_) <= 25_000 else rng.choice(len(na_), 3000, replace=False)
    _check_set(s, o2, rows)
    if 0 < len(na_) and len(na_) >= 48:
        e_ref, _ = o2.lowest_eigenpair()
        guess = c_new if np.any(cn != 0) else None
        e, cc, st = s.lowest_eigenpair(guess=guess, tol=1e-9)
        assert abs(e - e_ref) <= 1e-10, (e, e_ref)
    log(f"  update {ms:.2f} ms")


def test_update_sorted_order_and_chain(cas10):
    """Sorted-position evictions, two updates in a row, then against a fresh build."""
    ints, a, b, cfg, c, ea, eb = cas10
    log("update chain, sorted order")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    perm = s.permutation().cpu().numpy().astype(np.int64)   # sorted position -> caller index
    rng = np.random.default_rng(3)
    ev_sorted = rng.choice(len(a), 400, replace=False).astype(np.int32)
    cs = torch.from_numpy(c[perm]).cuda()
    c1, _ = s.update_determinants(ea[:1000], eb[:1000], evict=ev_sorted, coeffs=cs, sorted_order=True)
    a1, b1, keep1 = _new_set(a, b, perm[ev_sorted], ea[:1000], eb[:1000])
    # the carried vector is in the new sorted order: compare by determinant
    perm1 = s.permutation().cpu().numpy().astype(np.int64)
    carried = dict(zip(zip(a[keep1].tolist(), b[keep1].tolist()), c[keep1].tolist()))
    c1n = c1.cpu().numpy()
    for pos in range(len(a1)):
        key = (int(a1[perm1[pos]]), int(b1[perm1[pos]]))
        assert c1n[pos] == carried.get(key, 0.0)
    ev2 = rng.choice(len(a1), 300, replace=False).astype(np.int32)
    s.update_determinants(ea[1000:1800], eb[1000:1800], evict=ev2)
    a2, b2, _ = _new_set(a1, b1, ev2, ea[1000:1800], eb[1000:1800])
    _check_set(s, oracle_for(ints, a2, b2, cfg.na, cfg.nb), np.arange(len(a2)))


def test_update_rejections_leave_context_unchanged(cas10):
    ints, a, b, cfg, c, ea, eb = cas10
    log("update rejections")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    X = torch.from_numpy(W.random_block(len(a), 8, 9)).cuda()
    S0 = s.sigma(X).clone()
    cases = [
        (dict(add_alpha=a[:3], add_beta=b[:3]), "DUPLICATE"),                     # already in B
        (dict(add_alpha=ea[:2].repeat(2), add_beta=eb[:2].repeat(2)), "DUPLICATE"),  # repeated
        (dict(add_alpha=np.array([ea[0] ^ 1 ^ 2 ^ 4], np.uint64), add_beta=eb[:1]), "BAD_OCCUPATION"),
        (dict(evict=np.array([len(a)], np.int32)), "INVALID_ARG"),
        (dict(evict=np.array([3, 3], np.int32)), "INVALID_ARG"),
        (dict(evict=np.arange(len(a), dtype=np.int32)), "INVALID_ARG"),          # nothing left
    ]
    for kw, name in cases:
        with pytest.raises(hq.HinqsError) as ex:
            s.update_determinants(**kw)
        assert ex.value.name == name, (kw, ex.value)
        assert s.ndet == len(a) and torch.equal(s.sigma(X), S0)
    # a determinant that is evicted may come back in the same update
    s.update_determinants(a[:1], b[:1], evict=np.array([0], np.int32))
    a1 = np.concatenate([a[1:], a[:1]])
    b1 = np.concatenate([b[1:], b[:1]])
    _check_set(s, oracle_for(ints, a1, b1, cfg.na, cfg.nb), np.arange(len(a1)))


def test_update_full_size():
    """1e6 set: append 1e5 determinants of the classical expansion and evict
    5e4; sampled rows against the oracle on the new 1.05e6 set."""
    ints, a, b, cfg = W.config_inputs(2)
    log("update cas16 1e6: evict 5e4, append 1e5")
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    c = _coeffs(len(a), 2)
    ea, eb, _ = o.expand(c, 200)
    rng = np.random.default_rng(11)
    pick = rng.choice(len(ea), min(100_000, len(ea)), replace=False)
    evict = rng.choice(len(a), 50_000, replace=False).astype(np.int32)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    _, ms = s.update_determinants(ea[pick], eb[pick], evict=evict)
    na_, nb_, _ = _new_set(a, b, evict, ea[pick], eb[pick])
    fresh = solver_for(ints, na_, nb_, cfg.na, cfg.nb)
    inf = fresh.info()
    log(f"  update {ms:.1f} ms; fresh build {inf['ms_sort'] + inf['ms_connect'] + inf['ms_elements']:.1f} ms")
    assert s.info()["nnz"] == inf["nnz"]
    o2 = oracle_for(ints, na_, nb_, cfg.na, cfg.nb)
    _check_set(s, o2, rng.choice(len(na_), 150, replace=False))


# ------------------------------------------------------------- growth rules
def _scores(n, seed):
    """Seeded scores with ties (quantized)."""
    return np.round(np.random.default_rng(seed).exponential(1.0, n), 2)


@pytest.mark.parametrize("mode", ["append", "append_cap", "rebuild"])
def test_grow_basis_matches_oracle_rules(cas10, mode):
    ints, a, b, cfg, c, ea, eb = cas10
    log(f"grow basis: {mode}")
    cand = np.random.default_rng(5).choice(len(ea), 4000, replace=False)
    ca, cb = ea[cand], eb[cand]
    cs, bs = _scores(len(ca), 1), _scores(len(a), 2)
    k = 1500
    b_max = len(a) + 600 if mode == "append_cap" else 0
    rebuild = mode == "rebuild"
    kk = 12_000 if rebuild else k
    kept, apps = oracle.grow_basis(bs, cs, kk, b_max=b_max, rebuild=rebuild)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    c_new, s_new, ms = s.grow_basis(ca, cb, torch.from_numpy(cs).cuda(), kk,
                                    basis_score=torch.from_numpy(bs).cuda(), b_max=b_max,
                                    coeffs=torch.from_numpy(c).cuda(), rebuild=rebuild)
    na_ = np.concatenate([a[kept], ca[apps]])
    nb_ = np.concatenate([b[kept], cb[apps]])
    ga, gb = s.determinants()
    assert np.array_equal(_strs(ga), na_) and np.array_equal(_strs(gb), nb_)
    assert np.array_equal(s_new.cpu().numpy(), np.concatenate([bs[kept], cs[apps]]))
    cn = c_new.cpu().numpy()
    assert np.array_equal(cn[:len(kept)], c[kept]) and np.all(cn[len(kept):] == 0)
    if b_max:
        assert len(na_) == b_max
    _check_set(s, oracle_for(ints, na_, nb_, cfg.na, cfg.nb), np.arange(len(na_)))
    log(f"  {len(kept)} kept, {len(apps)} appended, {ms:.2f} ms")


def _strs(t):
    return t.cpu().numpy().view(np.uint64)


def test_update_large_orbital_count_and_rule_errors():
    """norb 20 (integrals read from global memory, 100 alpha single moves):
    an update against the oracle; then the growth-rule argument checks."""
    norb, na, nb = 20, 10, 9
    log(f"update at norb {norb}")
    ints = W.gen_integrals(norb, norb, -2.0, -0.5, 555)
    a, b = W.sample_determinants(norb, na, nb, 1500, 0.3, 0.0, 556)
    o = oracle_for(ints, a, b, na, nb)
    c = _coeffs(len(a), 7)
    ea, eb, _ = o.expand(c, 2)
    rng = np.random.default_rng(8)
    pick = rng.choice(len(ea), 400, replace=False)
    evict = rng.choice(len(a), 100, replace=False).astype(np.int32)
    s = solver_for(ints, a, b, na, nb)
    s.update_determinants(ea[pick], eb[pick], evict=evict)
    na_, nb_, _ = _new_set(a, b, evict, ea[pick], eb[pick])
    _check_set(s, oracle_for(ints, na_, nb_, na, nb), np.arange(len(na_)))
    cs = torch.from_numpy(_scores(20, 3)).cuda()
    with pytest.raises(hq.HinqsError) as ex:      # a capped append needs the set's scores
        s.grow_basis(ea[:20], eb[:20], cs, 10, b_max=len(na_))
    assert ex.value.name == "INVALID_ARG"
    bad = cs.clone()
    bad[3] = float("nan")
    with pytest.raises(hq.HinqsError) as ex:
        s.grow_basis(ea[:20], eb[:20], bad, 10)
    assert ex.value.name == "NONFINITE"
    assert s.ndet == len(na_)


@pytest.mark.parametrize("na,nb", [(16, 15), (3, 2)])
def test_update_top_of_orbital_range(na, nb):
    """norb 32: strings using the top bit, the largest orbital fields of the
    descriptors and (16 alpha electrons) 256 alpha single moves; an update
    with evictions and appended expansion determinants against an oracle
    built from scratch on the new set."""
    norb = 32
    log(f"update at norb {norb} ({na}a {nb}b)")
    ints = W.gen_integrals(norb, 8, -2.0, -0.5, 560 + na)
    a, b = W.sample_determinants(norb, na, nb, 1200, 0.3, 0.0, 561 + na)
    o = oracle_for(ints, a, b, na, nb)
    c = _coeffs(len(a), 9)
    ea, eb, _ = o.expand(c, 2)
    rng = np.random.default_rng(na)
    pick = rng.choice(len(ea), min(300, len(ea)), replace=False)
    evict = rng.choice(len(a), 80, replace=False).astype(np.int32)
    s = solver_for(ints, a, b, na, nb)
    s.update_determinants(ea[pick], eb[pick], evict=evict)
    na_, nb_, _ = _new_set(a, b, evict, ea[pick], eb[pick])
    _check_set(s, oracle_for(ints, na_, nb_, na, nb), np.arange(len(na_)))


def test_product_closure_and_its_energy():
    """The closure list equals the oracle's; appended with an update, the
    lowest eigenvalue on the product space matches the oracle's dense value
    and lies at or below the value on the set (variational)."""
    norb, na, nb = 8, 4, 4
    log("product-space closure")
    ints = W.gen_integrals(norb, norb, -2.0, -0.5, 71)
    a, b = W.sample_determinants(norb, na, nb, 400, 0.3, 0.0, 72)
    s = solver_for(ints, a, b, na, nb)
    ca, cb = s.product_closure()
    ra, rb = oracle.product_closure(a, b)
    assert np.array_equal(_strs(ca), ra) and np.array_equal(_strs(cb), rb)
    e_b, _, _ = s.lowest_eigenpair(tol=1e-9)
    s.update_determinants(ca, cb)
    pa, pb = np.concatenate([a, ra]), np.concatenate([b, rb])
    e_ref, _ = oracle_for(ints, pa, pb, na, nb).lowest_eigenpair()
    e_p, _, _ = s.lowest_eigenpair(tol=1e-9)
    assert abs(e_p - e_ref) <= 1e-10 and e_p <= e_b + 1e-12
    assert len(s.product_closure()[0]) == 0
    # the 20,000-determinant set: the closure is the rest of the full space
    ints, a, b, cfg = W.config_inputs(1)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    ca, cb = s.product_closure()
    ra, rb = oracle.product_closure(a, b)
    inf = s.info()
    assert np.array_equal(_strs(ca), ra) and np.array_equal(_strs(cb), rb)
    assert len(ra) == inf["n_alpha_strings"] * inf["n_beta_strings"] - len(a)
