"""GPU parity: the HIP path against the CPU oracle, element by element.

Bars (written in each test):
  * couplings, excitation class, holes/particles and sign: bit-exact;
  * FP64 sigma: |S - S_ref| <= 1e-12 * sum_j |H_ij| |X_j| per row and column;
  * FP32 sigma: the same with 2e-6 (a few FP32 ulps times the row length);
  * FP64 eigenvalue: 1e-10 Ha; eigenvector overlap >= 1 - 1e-10 (gap > 1e-6);
  * density matrices from one seeded vector: 1e-12 (atomics reorder sums).
"""
import numpy as np
import pytest

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


# ------------------------------------------------------------- Gram (MFMA)
@pytest.mark.parametrize("n,ma,nb", [(1000, 40, 8), (37, 3, 5), (4099, 96, 16), (1, 1, 1),
                                     (70001, 17, 13)])
def test_gram_matches_host(n, ma, nb):
    log(f"gram n={n} ma={ma} nb={nb}")
    rng = np.random.default_rng(n + ma)
    A = rng.standard_normal((n, ma))
    B = rng.standard_normal((n, nb))
    s = hq.Hinqs()
    G = s.gram(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()).cpu().numpy()
    ref = A.T @ B
    scale = np.abs(A).T @ np.abs(B)
    assert np.all(np.abs(G - ref) <= 1e-13 * scale + 1e-300)


# ------------------------------------------------------------- couplings
def _check_couplings(ints, alpha, beta, na, nb, rows):
    s = solver_for(ints, alpha, beta, na, nb)
    o = oracle_for(ints, alpha, beta, na, nb)
    got = gpu_rows_as_tuples(s, rows)
    want, _ = oracle_rows_as_tuples(o, rows)
    for i in rows:
        assert got[int(i)] == want[int(i)], f"row {i}"
    return s, o


def test_couplings_full_space_cas6():
    ints, a, b, cfg = W.config_inputs(0)
    log("couplings cas6 full space, all rows")
    s, _ = _check_couplings(ints, a, b, cfg.na, cfg.nb, np.arange(len(a)))
    assert s.info()["nnz"] == 400 * 117


def test_couplings_sampled_cas10_all_rows():
    ints, a, b, cfg = W.config_inputs(1)
    log("couplings cas10 20000 dets, all rows")
    _check_couplings(ints, a, b, cfg.na, cfg.nb, np.arange(len(a)))


def test_couplings_ragged_small_sets():
    # sets of a few determinants, including ones with no couplings at all
    for seed, (norb, na, nb, n) in enumerate([(5, 2, 2, 1), (5, 2, 2, 3), (7, 3, 1, 17),
                                              (8, 4, 4, 257), (6, 0, 3, 20), (6, 6, 1, 6)]):
        ints = W.gen_integrals(norb, norb, -2, -0.5, 300 + seed)
        a, b = W.sample_determinants(norb, na, nb, n, 0.5, 0.3, 400 + seed)
        log(f"couplings ragged norb={norb} na={na} nb={nb} n={n}")
        _check_couplings(ints, a, b, na, nb, np.arange(len(a)))


def test_couplings_lookup_path_forced(monkeypatch):
    """The alpha+beta lookup (binary search of each beta string one move away)
    in every group, however short: bit-exact on every row of the 20k set and
    of ragged small sets."""
    monkeypatch.setenv("HINQS_CONNECT_LOOKUP_MIN", "0")
    ints, a, b, cfg = W.config_inputs(1)
    log("couplings cas10 20000 dets, lookup path in every group")
    _check_couplings(ints, a, b, cfg.na, cfg.nb, np.arange(len(a)))
    for seed, (norb, na, nb, n) in enumerate([(5, 2, 2, 3), (7, 3, 1, 17), (8, 4, 4, 257), (6, 6, 1, 6)]):
        ints = W.gen_integrals(norb, norb, -2, -0.5, 300 + seed)
        a, b = W.sample_determinants(norb, na, nb, n, 0.5, 0.3, 400 + seed)
        _check_couplings(ints, a, b, na, nb, np.arange(len(a)))


@pytest.mark.parametrize("path", ["lookup", "scan"])
def test_couplings_dense_product_space(path, monkeypatch):
    """A product space with long alpha groups (norb 13: every one-electron alpha
    string times every 6-electron beta string, 22,308 determinants, 1,716 rows
    per group); couplings bit-exact and FP64 sigma at the row bar on 1,000
    sampled rows, with the alpha+beta partners looked up by binary search and
    with the scan."""
    monkeypatch.setenv("HINQS_CONNECT_LOOKUP_MIN", "0" if path == "lookup" else str(1 << 30))
    norb, na, nb = 13, 1, 6
    ints = W.gen_integrals(norb, 8, -2.5, -0.5, 913)
    a, b = _subset_product(list(range(norb)), na, nb)
    log(f"couplings dense product space norb={norb} n={len(a)} ({path})")
    rows = np.random.default_rng(77).choice(len(a), 1000, replace=False)
    s, o = _check_couplings(ints, a, b, na, nb, rows)
    X = W.random_block(len(a), 4, 78)
    _check_sigma(s, o, X, rows, 1e-12)


def test_couplings_1m_sampled_rows():
    ints, a, b, cfg = W.config_inputs(2)
    rows = np.random.default_rng(7).choice(len(a), 1000, replace=False)
    log("couplings cas16 1e6 dets, 1000 sampled rows")
    _check_couplings(ints, a, b, cfg.na, cfg.nb, rows)


# ------------------------------------------------------------- sigma
def _check_sigma(s, o, X, rows, tol, dtype=torch.float64, k=None):
    Xd = torch.from_numpy(X).to(dtype).cuda()
    S = s.sigma(Xd).double().cpu().numpy()
    Xr = Xd.double().cpu().numpy()
    ref = o.sigma_rows(Xr, rows)
    _, r = oracle_rows_as_tuples(o, rows)
    bound = row_bound(r, Xr, Xr.shape[1])
    err = np.abs(S[rows] - ref)
    assert np.all(err <= tol * bound + 1e-300), float((err / (bound + 1e-300)).max())


def test_diag_matches_oracle():
    ints, a, b, cfg = W.config_inputs(1, ndet=3000)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    d = s.diag().cpu().numpy()
    ref = o.diag()
    assert np.abs(d - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 3, 8, 16])
def test_sigma_fp64_cas6(k):
    ints, a, b, cfg = W.config_inputs(0)
    log(f"sigma fp64 cas6 k={k}")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    X = W.random_block(len(a), k, 11 + k)
    _check_sigma(s, o, X, np.arange(len(a)), 1e-12)


def test_sigma_every_width_both_precisions():
    """Every block width 1..16 in caller order, so each padded kernel width
    (k -> K in {1, 2, 4, 8, 16}) and its staging are used, FP64 at the 1e-12
    row bar and FP32 at 2e-6, on every row of a 3,000-determinant set."""
    ints, a, b, cfg = W.config_inputs(1, ndet=3000)
    log("sigma widths 1..16, fp64 and fp32, 3000 dets")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    rows = np.arange(len(a))
    for k in range(1, 17):
        X = W.random_block(len(a), k, 300 + k)
        _check_sigma(s, o, X, rows, 1e-12)
        _check_sigma(s, o, X, rows, 2e-6, dtype=torch.float32)


def test_sigma_fp64_cas10_all_rows():
    ints, a, b, cfg = W.config_inputs(1)
    log("sigma fp64 cas10 20000 dets k=8")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    X = W.random_block(len(a), 8, 21)
    _check_sigma(s, o, X, np.arange(len(a)), 1e-12)


def test_sigma_fp32_cas10():
    ints, a, b, cfg = W.config_inputs(1, ndet=5000)
    log("sigma fp32 cas10 5000 dets k=8")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    X = W.random_block(len(a), 8, 22)
    _check_sigma(s, o, X, np.arange(len(a)), 2e-6, dtype=torch.float32)


def test_sigma_1m_sampled_rows_fp64_and_fp32():
    ints, a, b, cfg = W.config_inputs(2)
    log("sigma cas16 1e6 dets, sampled rows")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    rows = np.random.default_rng(8).choice(len(a), 1000, replace=False)
    X = W.random_block(len(a), 8, 23)
    _check_sigma(s, o, X, rows, 1e-12)
    _check_sigma(s, o, X, rows, 2e-6, dtype=torch.float32)


def _subset_product(orbs, na, nb):
    """Every determinant whose alpha (na) and beta (nb) electrons sit in the
    orbitals `orbs`: a complete active space embedded in a larger orbital set."""
    import itertools
    strs = lambda n: [sum(1 << o for o in c) for c in itertools.combinations(orbs, n)]
    sa, sb = strs(na), strs(nb)
    a = np.array([x for x in sa for _ in sb], dtype=np.uint64)
    b = np.array([y for _ in sa for y in sb], dtype=np.uint64)
    return a, b


@pytest.mark.parametrize("norb,na,nb,kind", [
    (28, 4, 3, "cas"), (30, 5, 5, "cas"), (32, 6, 5, "cas"),
    (28, 4, 3, "sampled"), (32, 2, 2, "sampled"), (32, 31, 1, "sampled")])
def test_top_of_orbital_range(norb, na, nb, kind):
    """norb 28-32: the 5-bit orbital fields of the coupling descriptor, the
    strings' top bits and the global-memory integral path (the packed eri no
    longer fits in LDS above norb ~ 17).  "cas": all determinants of the
    lowest four and highest four orbitals (every coupling class among the top
    orbital indices); "sampled": rank-weighted draws over all orbitals.
    Couplings bit-exact on every row, FP64 sigma at the 1e-12 row bar, lowest
    eigenvalue at 1e-10 Ha."""
    ints = W.gen_integrals(norb, 8, -3.0, -0.5, 700 + norb + na)
    if kind == "cas":
        a, b = _subset_product(list(range(4)) + list(range(norb - 4, norb)), na, nb)
    else:
        n = {2: 400, 31: 64}.get(na, 3000)
        a, b = W.sample_determinants(norb, na, nb, n, 0.45, 0.2, 800 + norb + na)
    log(f"top of range norb={norb} na={na} nb={nb} {kind} n={len(a)}")
    s, o = _check_couplings(ints, a, b, na, nb, np.arange(len(a)))
    top = np.uint64(1) << np.uint64(norb - 1)
    assert np.any((a & top) != 0) and np.any((b & top) != 0)  # the highest orbital is used
    X = W.random_block(len(a), 3, 31 + norb)
    _check_sigma(s, o, X, np.arange(len(a)), 1e-12)
    e_ref, c_ref = o.lowest_eigenpair()
    e, c, st = s.lowest_eigenpair(tol=1e-9, block=4)
    log(f"  E={e!r} ref={e_ref!r} it={st['iterations']} nnz={s.info()['nnz']}")
    assert abs(e - e_ref) <= 1e-10
    w = o.spectrum(2)
    if len(w) > 1 and w[1] - w[0] > 1e-6:
        assert abs(float(np.dot(c.cpu().numpy(), c_ref))) >= 1 - 1e-9


def test_sigma_and_solve_are_bitwise_repeatable():
    """The sigma kernel hands rows out through per-XCD counters, so which team
    takes a row changes from launch to launch; every row is still summed by
    one team in a fixed order, so repeated products and solves must agree to
    the bit (1e6 set: FP64 and FP32 sigma; 20k set: the FP64 eigenpair)."""
    ints, a, b, cfg = W.config_inputs(2)
    log("bitwise repeatability: sigma at 1e6, k = 8")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    X = torch.from_numpy(W.random_block(len(a), 8, 51)).cuda()
    assert torch.equal(s.sigma(X), s.sigma(X))
    X32 = X.float()
    assert torch.equal(s.sigma(X32), s.sigma(X32))
    ints, a, b, cfg = W.config_inputs(1)
    log("bitwise repeatability: FP64 eigenpair at 20k")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    e1, c1, _ = s.lowest_eigenpair(tol=1e-9)
    e2, c2, _ = s.lowest_eigenpair(tol=1e-9)
    assert e1 == e2 and torch.equal(c1, c2)


def test_sigma_sorted_order_matches_caller_order():
    ints, a, b, cfg = W.config_inputs(1, ndet=4000)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    X = torch.from_numpy(W.random_block(len(a), 8, 24)).cuda()
    S = s.sigma(X)
    perm = s.permutation().long()
    Ss = s.sigma(X[perm].contiguous(), sorted_order=True)
    assert torch.equal(Ss, S[perm])


# ------------------------------------------------------------- eigenpairs
def _gap(o):
    w = o.spectrum(2)
    return w[1] - w[0]


def test_eigenpair_full_space_cas6_vs_dense():
    ints, a, b, cfg = W.config_inputs(0)
    log("davidson cas6 full space vs dense eigh")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    e_ref, c_ref = o.lowest_eigenpair()
    assert _gap(o) > 1e-6
    e, c, st = s.lowest_eigenpair(tol=1e-8)
    log(f"  E={e!r} ref={e_ref!r} stats={st}")
    assert abs(e - e_ref) <= 1e-10
    c = c.cpu().numpy()
    assert abs(np.dot(c, c_ref)) >= 1 - 1e-10
    assert abs(np.linalg.norm(c) - 1) < 1e-12
    assert c[np.argmax(np.abs(c))] > 0


def test_eigenpair_cas10_vs_lanczos():
    ints, a, b, cfg = W.config_inputs(1)
    log("davidson cas10 20000 dets vs oracle Lanczos")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    e_ref, c_ref = o.lowest_eigenpair(dense_max=0)
    assert _gap(o) > 1e-6
    e, c, st = s.lowest_eigenpair(tol=1e-8)
    log(f"  E={e!r} ref={e_ref!r} stats={st}")
    assert abs(e - e_ref) <= 1e-10
    assert abs(np.dot(c.cpu().numpy(), c_ref)) >= 1 - 1e-9


@pytest.mark.parametrize("e_shift", [0.0, 100.0])
def test_eigenpair_small_sets_and_tiny_spaces(e_shift):
    """Sets smaller than the block and the subspace; with e_shift = 100 every
    eigenvalue is positive, so no padding direction may pose as eigenvalue 0."""
    import dataclasses
    for seed, (norb, na, nb, n) in enumerate([(5, 2, 2, 1), (5, 2, 2, 5), (6, 3, 2, 37),
                                              (7, 3, 3, 150)]):
        ints = W.gen_integrals(norb, norb, -2, -0.5, 500 + seed)
        ints = dataclasses.replace(ints, e_core=ints.e_core + e_shift)
        a, b = W.sample_determinants(norb, na, nb, n, 0.5, 0.3, 600 + seed)
        log(f"davidson tiny norb={norb} n={n}")
        s = solver_for(ints, a, b, na, nb)
        o = oracle_for(ints, a, b, na, nb)
        e_ref, c_ref = o.lowest_eigenpair()
        e, c, st = s.lowest_eigenpair(tol=1e-9)
        assert abs(e - e_ref) <= 1e-10
        if n > 1:
            w = o.spectrum(2)
            if w[1] - w[0] > 1e-6:
                assert abs(np.dot(c.cpu().numpy(), c_ref)) >= 1 - 1e-10


def _two_copies():
    """H_B = H_A (+) H_A exactly: the full 2a+2b space of orbitals 0..3 and the
    same space moved to orbitals 4..7 (the two halves differ by four electrons,
    so nothing couples them), with the integrals of orbitals 4..7 a copy of
    those of 0..3.  Every eigenvalue is exactly twofold degenerate."""
    base = W.gen_integrals(4, 4, -2.0, -0.5, 97)
    h = np.zeros((8, 8))
    eri = np.zeros((8,) * 4)
    for o in (0, 4):
        h[o:o + 4, o:o + 4] = base.h
        eri[o:o + 4, o:o + 4, o:o + 4, o:o + 4] = base.eri
    ints = W.Integrals(8, h, eri, 0.0)
    fa, fb = W.full_space(4, 2, 2)
    a = np.concatenate([fa, fa << np.uint64(4)])
    b = np.concatenate([fb, fb << np.uint64(4)])
    return ints, a, b


@pytest.mark.parametrize("block,mixed", [(8, False), (1, False), (4, True)])
def test_exactly_degenerate_ground_state(block, mixed):
    ints, a, b = _two_copies()
    log(f"degenerate ground state, {len(a)} dets, block {block}, mixed {mixed}")
    s = solver_for(ints, a, b, 2, 2)
    o = oracle_for(ints, a, b, 2, 2)
    w = np.linalg.eigvalsh(o.dense())
    assert abs(w[1] - w[0]) <= 1e-12 * abs(w[0])  # the construction is exact
    e, c, st = s.lowest_eigenpair(tol=1e-9, block=block, mixed=mixed)
    assert abs(e - w[0]) <= (1e-8 if mixed else 1e-10)
    # the vector lies in the degenerate eigenspace: its residual is small
    H = o.dense()
    x = c.cpu().numpy()
    assert np.linalg.norm(H @ x - e * x) <= 1e-7


def test_batch_exactly_degenerate_instances():
    ints, a, b = _two_copies()
    w0 = np.linalg.eigvalsh(oracle_for(ints, a, b, 2, 2).dense())[0]
    s = hq.Hinqs()
    for _ in range(3):
        s.batch_add(ints.h, ints.eri, ints.e_core, a, b, 2, 2)
    e, c, info = s.batch_lowest_eigenpair(block=8, tol=1e-9)
    assert all(int(x) == 0 for x in info["status"])
    assert np.all(np.abs(np.asarray(e) - w0) <= 1e-10)


def test_second_projection_pass_both_ways():
    """The second pass against the basis runs only when a new direction kept
    less than half its norm in the first; both outcomes reach the oracle."""
    runs = 0
    for nd, blocks in ((100, (4, 8, 16)), (300, (8, 16))):
        ints, a, b, cfg = W.config_inputs(1, ndet=nd)
        s = solver_for(ints, a, b, cfg.na, cfg.nb)
        e_ref, _ = oracle_for(ints, a, b, cfg.na, cfg.nb).lowest_eigenpair()
        for k in blocks:
            e, _, st = s.lowest_eigenpair(tol=1e-9, block=k)
            log(f"  ndet {nd} block {k}: {st['iterations']} iterations, {st['second_passes']} second passes")
            assert abs(e - e_ref) <= 1e-10
            runs += st["second_passes"]
    assert runs >= 1  # small spaces: corrections fall largely inside the basis
    ints, a, b, cfg = W.config_inputs(1)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    e, _, st = s.lowest_eigenpair(tol=1e-8, block=8)
    log(f"  cas10 20000: {st['iterations']} iterations, {st['second_passes']} second passes")
    assert st["second_passes"] < st["iterations"]


def test_warm_start_converges_immediately():
    ints, a, b, cfg = W.config_inputs(1, ndet=5000)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    e, c, st = s.lowest_eigenpair(tol=1e-9)
    e2, c2, st2 = s.lowest_eigenpair(guess=c, tol=1e-8)
    log(f"  cold {st['iterations']} iterations, warm {st2['iterations']}")
    assert abs(e2 - e) < 1e-10
    assert st2["iterations"] <= 2


def test_warm_start_from_a_reference_dominated_vector():
    """A weakly correlated state (|c| of the lowest-diagonal determinant about
    0.98): the guess lies almost inside the span of the unit vectors at the
    lowest diagonal elements that join it in the initial block, and its own
    direction must survive the orthonormalization."""
    ints, a, b, cfg = W.config_inputs(1, ndet=5000)
    d = np.diag(np.diag(ints.h))
    ints.h = d + 0.02 * (ints.h - d)  # weak one- and two-electron coupling
    ints.eri = ints.eri * 0.02
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    e, c, st = s.lowest_eigenpair(tol=1e-10)
    cmax = float(c.abs().max())
    e2, c2, st2 = s.lowest_eigenpair(guess=c, tol=1e-8)
    log(f"  |c|max {cmax:.5f}; cold {st['iterations']} iterations, warm {st2['iterations']}")
    assert cmax > 0.97
    assert abs(e2 - e) < 1e-10
    assert st2["iterations"] <= 2


def test_not_converged_returns_best_estimate():
    ints, a, b, cfg = W.config_inputs(1, ndet=3000)
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    with pytest.raises(hq.HinqsError) as ei:
        s.lowest_eigenpair(max_iter=1, tol=1e-12)
    assert ei.value.name == "NOT_CONVERGED"
    e, c, st = s.lowest_eigenpair(max_iter=1, tol=1e-12, raise_on_not_converged=False)
    assert np.isfinite(e) and not st["converged"]


def test_mixed_precision_matches_fp64_and_oracle():
    """Mixed precision (FP32 off-diagonal products, FP64 diagonal term, residual,
    Ritz projection and orthogonalization, FP64 refinement) on a 60,000-determinant
    set drawn like the 1e6 workload (norb 16, 7+7, h_pp in [-15, 1], 5 % tail):
    the eigenvalue within 1e-8 Ha of the oracle's Lanczos value and of the FP64
    solve, most iterations in FP32."""
    ints, a, b, cfg = W.config_inputs(2, ndet=60_000)
    log("mixed vs fp64 vs oracle Lanczos, cas16 60000 dets")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    e64, c64, st64 = s.lowest_eigenpair(tol=1e-8)
    em, cm, stm = s.lowest_eigenpair(tol=1e-8, mixed=True)
    e_ref, c_ref = oracle_for(ints, a, b, cfg.na, cfg.nb).lowest_eigenpair()
    log(f"  oracle E={e_ref!r}\n  fp64 E={e64!r} {st64}\n  mixed E={em!r} {stm}\n"
        f"  |mixed - oracle| = {abs(em - e_ref):.2e}, |fp64 - oracle| = {abs(e64 - e_ref):.2e}")
    assert abs(e64 - e_ref) <= 1e-10
    assert abs(em - e_ref) <= 1e-8
    assert abs(em - e64) <= 1e-8
    # the FP32 phase runs until the residual nears the FP32 floor, not until the
    # first rise after a restart: most iterations use FP32 products
    assert 2 * stm["iterations_fp32"] >= stm["iterations"]
    assert abs(torch.dot(c64, cm).item()) >= 1 - 1e-8
    cr = torch.from_numpy(np.asarray(c_ref)).cuda()
    assert abs(torch.dot(cm, cr).item()) >= 1 - 1e-8


@pytest.mark.parametrize("e_core", [-1000.0, 1000.0])
def test_mixed_precision_with_a_large_constant(e_core):
    """A large E_core (here +-1000 Ha, beyond any FP32 resolution of the
    eigenvalue) sits on the diagonal, which the mixed path applies in FP64:
    the mixed eigenvalue stays within 1e-8 Ha of the FP64 solve and the
    oracle (10,000 determinants drawn like the 1e6 workload)."""
    import dataclasses
    ints, a, b, cfg = W.config_inputs(2, ndet=10_000)
    ints = dataclasses.replace(ints, e_core=ints.e_core + e_core)
    log(f"mixed with E_core {e_core:+.0f}, 10000 dets")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    e64, c64, _ = s.lowest_eigenpair(tol=1e-8)
    em, cm, stm = s.lowest_eigenpair(tol=1e-8, mixed=True)
    e_ref, _ = oracle_for(ints, a, b, cfg.na, cfg.nb).lowest_eigenpair()
    log(f"  oracle {e_ref!r} fp64 {e64!r} mixed {em!r} ({stm['iterations_fp32']} of {stm['iterations']} FP32)")
    assert abs(e64 - e_ref) <= 1e-10
    assert abs(em - e_ref) <= 1e-8 and abs(em - e64) <= 1e-8
    assert abs(torch.dot(c64, cm).item()) >= 1 - 1e-8


# ------------------------------------------------------------- RDMs
def test_rdm12_matches_oracle_seeded_vector():
    for idx, n in [(0, None), (3, 400)]:
        ints, a, b, cfg = W.config_inputs(idx, ndet=n)
        log(f"rdm12 config {idx} n={len(a)}")
        s = solver_for(ints, a, b, cfg.na, cfg.nb)
        o = oracle_for(ints, a, b, cfg.na, cfg.nb)
        c = W.random_block(len(a), 1, 31)[:, 0]
        d1, d2 = s.rdm12(torch.from_numpy(c).cuda())
        r1, r2 = o.rdm12(c)
        scale = float(np.sum(c * c))
        assert np.abs(d1.cpu().numpy() - r1).max() <= 1e-12 * scale * cfg.norb
        assert np.abs(d2.cpu().numpy() - r2).max() <= 1e-12 * scale * cfg.norb ** 2


@pytest.mark.parametrize("case", ["norb16_sampled", "norb28_cas", "norb32_cas"])
def test_rdm12_larger_orbital_counts(case):
    """RDMs as full tensors against the oracle where the per-workgroup tables
    still fit in LDS (norb 16) and where they go to global memory (norb 28
    and 32, the top four and bottom four orbitals of an embedded active
    space); a second call on the same context checks that the kept
    accumulation scratch starts from zero again."""
    if case == "norb16_sampled":
        ints, a, b, cfg = W.config_inputs(2, ndet=3000)
        norb, na, nb = cfg.norb, cfg.na, cfg.nb
    else:
        norb = 28 if case == "norb28_cas" else 32
        na, nb = (4, 3) if norb == 28 else (3, 3)
        ints = W.gen_integrals(norb, 8, -3.0, -0.5, 900 + norb)
        a, b = _subset_product(list(range(4)) + list(range(norb - 4, norb)), na, nb)
    log(f"rdm12 {case}: {len(a)} determinants")
    s = solver_for(ints, a, b, na, nb)
    o = oracle_for(ints, a, b, na, nb)
    c = W.random_block(len(a), 1, 77)[:, 0]
    r1, r2 = o.rdm12(c)
    scale = float(np.sum(c * c))
    for rep in range(2):
        d1, d2 = s.rdm12(torch.from_numpy(c).cuda())
        assert np.abs(d1.cpu().numpy() - r1).max() <= 1e-12 * scale * norb, rep
        assert np.abs(d2.cpu().numpy() - r2).max() <= 1e-12 * scale * norb ** 2, rep


def test_rdm12_identities_on_eigenvector_200k():
    ints, a, b, cfg = W.config_inputs(3)
    log("rdm12 identities cas12 200000 dets")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    e, c, st = s.lowest_eigenpair(tol=1e-10)
    d1, d2 = (t.cpu().numpy() for t in s.rdm12(c))
    N = cfg.na + cfg.nb
    assert abs(np.trace(d1) - N) < 1e-9
    assert abs(np.einsum("pprr", d2) - N * (N - 1)) < 1e-8
    assert np.abs(np.einsum("pqrr->pq", d2) - (N - 1) * d1).max() < 1e-9
    e_rdm = ints.e_core + np.sum(ints.h * d1) + 0.5 * np.sum(ints.eri * d2)
    assert abs(e_rdm - e) < 1e-8
    # sampled elements against the oracle, one pass over B each
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    idx = np.random.default_rng(5).integers(0, cfg.norb, size=(24, 4))
    cc = c.cpu().numpy()
    ref = o.rdm2_elements(cc, idx)
    got = d2[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]]
    assert np.abs(got - ref).max() < 1e-11


# ------------------------------------------------------------- errors
def test_error_paths():
    ints, a, b, cfg = W.config_inputs(1, ndet=500)
    s = hq.Hinqs()
    with pytest.raises(hq.HinqsError) as ei:
        s._check(s._lib.hinqs_sigma(s._h, 8, None, None, 0, 0))
    assert ei.value.name == "NOT_READY"
    with pytest.raises(hq.HinqsError) as ei:
        s.set_determinants(a, b, cfg.na, cfg.nb)
    assert ei.value.name == "NOT_READY"
    bad = ints.eri.copy()
    bad[0, 1, 2, 3] += 1e-3
    with pytest.raises(hq.HinqsError) as ei:
        s.set_integrals(ints.h, bad, 0.0)
    assert ei.value.name == "ASYMMETRIC"
    nan_h = ints.h.copy()
    nan_h[0, 0] = np.nan
    with pytest.raises(hq.HinqsError) as ei:
        s.set_integrals(nan_h, ints.eri, 0.0)
    assert ei.value.name == "NONFINITE"
    s.set_integrals(ints.h, ints.eri, 0.0)
    with pytest.raises(hq.HinqsError) as ei:
        s.set_determinants(np.concatenate([a, a[:1]]), np.concatenate([b, b[:1]]), cfg.na, cfg.nb)
    assert ei.value.name == "DUPLICATE"
    a2 = a.copy()
    a2[3] |= np.uint64(1 << 12)
    with pytest.raises(hq.HinqsError) as ei:
        s.set_determinants(a2, b, cfg.na, cfg.nb)
    assert ei.value.name == "BAD_OCCUPATION"
    s.set_determinants(a, b, cfg.na, cfg.nb)
    with pytest.raises(hq.HinqsError) as ei:
        s.sigma(torch.zeros((len(a), 17), dtype=torch.float64, device="cuda"))
    assert ei.value.name == "UNSUPPORTED"


@pytest.mark.parametrize("team,unr,occ,pipe", [(16, 2, 2, 0), (32, 4, 8, 0), (64, 2, 4, 0), (64, 4, 2, 0),
                                                (8, 2, 4, 0), (64, 2, 4, 1), (32, 4, 2, 1), (16, 2, 8, 1),
                                                (8, 4, 4, 1)])
def test_sigma_every_launch_shape(team, unr, occ, pipe, monkeypatch):
    """Every launch shape the tuner may pick gives the same products (to the bar)."""
    ints, a, b, cfg = W.config_inputs(1, ndet=5000)
    log(f"sigma launch shape team={team} unr={unr} occ={occ} pipe={pipe}")
    monkeypatch.setenv("HINQS_SIGMA_TEAM", str(team))
    monkeypatch.setenv("HINQS_SIGMA_UNR", str(unr))
    monkeypatch.setenv("HINQS_SIGMA_OCC", str(occ))
    monkeypatch.setenv("HINQS_SIGMA_PIPE", str(pipe))
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    for k in (1, 8, 16):
        X = W.random_block(len(a), k, 31 + k)
        _check_sigma(s, o, X, np.arange(len(a)), 1e-12)
    X = W.random_block(len(a), 8, 40)
    _check_sigma(s, o, X, np.arange(len(a)), 2e-6, dtype=torch.float32)


def test_autotune_then_solve():
    ints, a, b, cfg = W.config_inputs(1, ndet=8000)
    log("autotune cas10 8000 dets, then solve with the tuned shape")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    shape, ms = s.autotune(8, hq.HINQS_FP64)
    assert shape[0] in (16, 32, 64) and shape[1] in (2, 4) and shape[2] in (2, 4, 8) and ms > 0
    shape2, _ = s.autotune(8, hq.HINQS_FP64)   # cached
    assert shape2 == shape
    X = W.random_block(len(a), 8, 41)
    _check_sigma(s, o, X, np.arange(len(a)), 1e-12)
    e, c, st = s.lowest_eigenpair(tol=1e-9, autotune=True, mixed=True)
    e_ref, _ = o.lowest_eigenpair()
    assert abs(e - e_ref) <= 1e-8


@pytest.mark.parametrize("block,max_space,mixed", [(1, 8, False), (2, 12, False), (4, 24, False),
                                                   (16, 96, False), (16, 48, False), (4, 12, True)])
def test_eigenpair_every_block_size(block, max_space, mixed):
    """Every block size and subspace limit reaches the dense eigenpair (the
    tall-skinny kernels are compiled per block size)."""
    ints, a, b, cfg = W.config_inputs(1, ndet=3000)
    log(f"davidson block={block} max_space={max_space} mixed={mixed}")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    e_ref, c_ref = o.lowest_eigenpair()
    e, c, st = s.lowest_eigenpair(tol=1e-9, block=block, max_space=max_space, mixed=mixed, max_iter=600)
    assert abs(e - e_ref) <= (1e-8 if mixed else 1e-10)
    w = o.spectrum(2)
    if w[1] - w[0] > 1e-6:
        assert abs(np.dot(c.cpu().numpy(), c_ref)) >= 1 - 1e-9
    assert st["restarts"] >= 1 or st["iterations"] * block < max_space


def test_side_stream_and_interleaved_contexts():
    """A context on a stream of its own solves to the same bits as one on the
    default stream, and two contexts whose calls interleave on one GPU (each
    with its own row counters) give the products each gives alone."""
    ints, a, b, cfg = W.config_inputs(1, ndet=8000)
    log("side stream and interleaved contexts, 8000 dets")
    s0 = solver_for(ints, a, b, cfg.na, cfg.nb)
    e0, c0, _ = s0.lowest_eigenpair(tol=1e-9)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s1 = hq.Hinqs(stream=side)
        s1.set_integrals(ints.h, ints.eri, ints.e_core)
        s1.set_determinants(a, b, cfg.na, cfg.nb)
        e1, c1, _ = s1.lowest_eigenpair(tol=1e-9)
    side.synchronize()
    assert e0 == e1 and torch.equal(c0, c1)
    ints2, a2, b2, cfg2 = W.config_inputs(0)
    s2 = solver_for(ints2, a2, b2, cfg2.na, cfg2.nb)
    X0 = torch.from_numpy(W.random_block(len(a), 8, 61)).cuda()
    X2 = torch.from_numpy(W.random_block(len(a2), 8, 62)).cuda()
    ref0, ref2 = s0.sigma(X0), s2.sigma(X2)
    for _ in range(3):
        assert torch.equal(s0.sigma(X0), ref0)
        assert torch.equal(s2.sigma(X2), ref2)


def test_device_resident_determinants_match_host_input():
    """hinqs_set_determinants_device (strings already in HBM, as the outer loop
    hands them over) builds the same set as the host-array entry point:
    couplings, diagonal and sigma bitwise equal; its validation reports the
    same errors."""
    ints, a, b, cfg = W.config_inputs(1, ndet=6000)
    log("device-resident determinant input, 6000 dets")
    sh = solver_for(ints, a, b, cfg.na, cfg.nb)
    sd = hq.Hinqs()
    sd.set_integrals(ints.h, ints.eri, ints.e_core)
    da = torch.from_numpy(a.view(np.int64)).cuda()
    db = torch.from_numpy(b.view(np.int64)).cuda()
    sd.set_determinants(da, db, cfg.na, cfg.nb)
    for x, y in zip(sd.connectivity(), sh.connectivity()):
        assert torch.equal(x, y)
    assert torch.equal(sd.diag(), sh.diag())
    X = torch.from_numpy(W.random_block(len(a), 8, 71)).cuda()
    assert torch.equal(sd.sigma(X), sh.sigma(X))
    bad_a = da.clone()
    bad_a[5] = bad_a[4]
    bad_b = db.clone()
    bad_b[5] = bad_b[4]
    with pytest.raises(hq.HinqsError) as ei:
        sd.set_determinants(bad_a, bad_b, cfg.na, cfg.nb)
    assert ei.value.name == "DUPLICATE"
    bad_a = da.clone()
    bad_a[3] = bad_a[3] | (1 << 20)
    with pytest.raises(hq.HinqsError) as ei:
        sd.set_determinants(bad_a, db, cfg.na, cfg.nb)
    assert ei.value.name == "BAD_OCCUPATION"
