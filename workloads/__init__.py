"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only draws numbers: one- and two-electron integrals with the
symmetry of a real orthonormal orbital basis, and sets of occupation strings
shaped like the sampled determinant sets of the paper's selected-CI loop
(Sec. 2.2, Steps 1-3; active spaces of Table 1).  It evaluates nothing of the
method itself (no Hamiltonian element, no sign, no eigenproblem), so the GPU
path and the oracle can both consume it without sharing any of the method's
arithmetic.

Conventions
-----------
* Integrals: ``h`` is ``norb x norb`` symmetric; ``eri`` is ``norb^4`` in
  chemists' notation ``(pq|rs)`` with the 8-fold permutational symmetry of
  real orbitals; ``e_core`` plays the role of the nuclear-repulsion constant
  of the Hamiltonian in Sec. 2.2.
* Determinants: bit ``p`` of an alpha (beta) string set <=> spatial orbital
  ``p`` occupied with spin alpha (beta); strings are ``numpy.uint64``.
  Returned in draw order (not sorted), duplicates removed keeping the first
  draw, matching the de-duplication of Step 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Integrals", "gen_integrals", "fci_strings", "sample_determinants",
    "full_space", "random_block", "CONFIGS", "config_inputs",
    "batch_instance_spec",
]


@dataclass
class Integrals:
    norb: int
    h: np.ndarray          # (norb, norb) float64, symmetric
    eri: np.ndarray        # (norb, norb, norb, norb) float64, chemists' (pq|rs)
    e_core: float = 0.0


def gen_integrals(norb: int, n_l: int, lo: float, hi: float, seed: int,
                  sd_off: float = 0.1, sd_b: float = 0.15) -> Integrals:
    """Random integrals with real-orbital symmetry.

    Draw order (PCG64 ``default_rng(seed)``):
      1. a full ``norb x norb`` normal draw with standard deviation ``sd_off``;
         the strict upper triangle is kept and mirrored (off-diagonal h);
      2. ``norb`` uniform draws on ``[lo, hi)``, sorted ascending (diagonal h);
      3. for each of ``n_l`` factors a full ``norb x norb`` normal draw with
         standard deviation ``sd_b``; upper triangle incl. diagonal kept and
         mirrored;
      4. ``eri = sum_L B^L (x) B^L`` -- 8-fold symmetric and positive
         semidefinite as a pair matrix, like a density-fitted Coulomb tensor.
    """
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, sd_off, size=(norb, norb))
    h = np.triu(a, 1)
    h = h + h.T
    hpp = np.sort(rng.uniform(lo, hi, size=norb))
    h[np.arange(norb), np.arange(norb)] = hpp
    eri = np.zeros((norb, norb, norb, norb))
    for _ in range(n_l):
        b = rng.normal(0.0, sd_b, size=(norb, norb))
        b = np.triu(b) + np.triu(b, 1).T
        eri += np.multiply.outer(b, b)
    return Integrals(norb=norb, h=h, eri=eri, e_core=0.0)


def fci_strings(norb: int, nelec: int) -> np.ndarray:
    """All ``C(norb, nelec)`` strings with ``nelec`` bits set, ascending."""
    out = []
    for occ in _combinations(norb, nelec):
        s = 0
        for p in occ:
            s |= 1 << p
        out.append(s)
    return np.array(sorted(out), dtype=np.uint64)


def _combinations(n, k):
    import itertools
    return itertools.combinations(range(n), k)


def full_space(norb: int, na: int, nb: int) -> tuple[np.ndarray, np.ndarray]:
    """Every (alpha, beta) pair of the FCI space, alpha-major order."""
    sa = fci_strings(norb, na)
    sb = fci_strings(norb, nb)
    alpha = np.repeat(sa, len(sb))
    beta = np.tile(sb, len(sa))
    return alpha, beta


def _bits(n):
    return (np.uint64(1) << np.arange(n, dtype=np.uint64)).astype(np.uint64)


def _rand_subset_mask(rng, rows, n, r):
    """Boolean (rows, n) mask with exactly ``r[i]`` uniformly chosen Trues per row."""
    keys = rng.random((rows, n))
    rank = np.argsort(np.argsort(keys, axis=1), axis=1)
    return rank < np.asarray(r)[:, None]


def sample_determinants(norb: int, na: int, nb: int, ndet: int, w: float,
                        tail: float, seed: int, batch: int | None = None,
                        max_draws: int = 400_000_000) -> tuple[np.ndarray, np.ndarray]:
    """Draw ``ndet`` unique determinants, NQS-like (rank-weighted) with a uniform tail.

    Rank ``r_a + r_b`` counts alpha and beta holes relative to the aufbau
    string (the lowest ``na`` / ``nb`` orbital indices; ``h_pp`` is sorted
    ascending, so these are the lowest diagonal energies).  Each draw:
      * with probability ``tail``: a uniform alpha string times a uniform
        beta string;
      * otherwise an excitation class ``(r_a, r_b)`` with probability
        proportional to ``C(na,r_a) C(norb-na,r_a) C(nb,r_b) C(norb-nb,r_b)
        w^(r_a+r_b)`` -- i.e. every determinant of rank r carries weight w^r --
        then holes and particles uniformly within the class.
    Draws repeat until ``ndet`` distinct determinants exist; first-draw order
    is kept.
    """
    fci = math.comb(norb, na) * math.comb(norb, nb)
    if ndet > fci:
        raise ValueError(f"ndet={ndet} exceeds the FCI dimension {fci}")
    rng = np.random.default_rng(seed)
    ra_max = min(na, norb - na)
    rb_max = min(nb, norb - nb)
    cls = [(ra, rb) for ra in range(ra_max + 1) for rb in range(rb_max + 1)]
    wts = np.array([math.comb(na, ra) * math.comb(norb - na, ra) *
                    math.comb(nb, rb) * math.comb(norb - nb, rb) * w ** (ra + rb)
                    for ra, rb in cls])
    prob = wts / wts.sum()
    cls_a = np.array([c[0] for c in cls])
    cls_b = np.array([c[1] for c in cls])
    bits = _bits(norb)
    ref_a = np.uint64((1 << na) - 1)
    ref_b = np.uint64((1 << nb) - 1)

    def excite(ref_n, r, rows):
        occ_mask = _rand_subset_mask(rng, rows, ref_n, r)            # holes among 0..n-1
        vir_mask = _rand_subset_mask(rng, rows, norb - ref_n, r)     # particles among n..norb-1
        holes = (occ_mask * bits[:ref_n]).sum(axis=1, dtype=np.uint64)
        parts = (vir_mask * bits[ref_n:]).sum(axis=1, dtype=np.uint64)
        return holes, parts

    keys_all = np.empty(0, dtype=np.uint64)
    order_all = np.empty(0, dtype=np.int64)
    drawn = 0
    if batch is None:
        batch = max(4096, min(2 * ndet, 4_000_000))
    while True:
        n = batch
        is_tail = rng.random(n) < tail
        c = rng.choice(len(cls), size=n, p=prob)
        ra = cls_a[c]
        rb = cls_b[c]
        ha, pa = excite(na, ra, n)
        hb, pb = excite(nb, rb, n)
        a = (ref_a ^ ha) | pa
        b = (ref_b ^ hb) | pb
        ua = (_rand_subset_mask(rng, n, norb, np.full(n, na)) * bits).sum(axis=1, dtype=np.uint64)
        ub = (_rand_subset_mask(rng, n, norb, np.full(n, nb)) * bits).sum(axis=1, dtype=np.uint64)
        a = np.where(is_tail, ua, a)
        b = np.where(is_tail, ub, b)
        keys = (a << np.uint64(32)) | b
        keys_all = np.concatenate([keys_all, keys])
        order_all = np.concatenate([order_all, np.arange(drawn, drawn + n, dtype=np.int64)])
        drawn += n
        uniq, first = np.unique(keys_all, return_index=True)
        keys_all = uniq
        order_all = order_all[first]
        if len(keys_all) >= ndet:
            break
        if drawn > max_draws:
            raise RuntimeError("sampler made too little progress")
    sel = np.argsort(order_all, kind="stable")[:ndet]
    keys = keys_all[sel]
    alpha = (keys >> np.uint64(32)).astype(np.uint64)
    beta = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint64)
    return alpha, beta


def random_block(ndet: int, k: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Seeded ``ndet x k`` block of trial vectors (row-major, k contiguous)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ndet, k)).astype(dtype)


# --------------------------------------------------------------------------
# The five workloads.  Shapes follow the paper's N2 active-space series
# (Table 1): CAS(6,6) full space, CAS(10,10), CAS(16,14)-like, CAS(12,12),
# and a bond-scan-like batch of uneven instances.
# --------------------------------------------------------------------------
@dataclass
class Config:
    name: str
    norb: int
    na: int
    nb: int
    n_l: int
    lo: float
    hi: float
    ndet: int | None          # None -> full space
    w: float = 0.4
    tail: float = 0.0
    k: int = 8
    tol: float = 1e-8
    seed_int: int = 0
    seed_det: int = 0
    extra: dict = field(default_factory=dict)


CONFIGS = {
    0: Config("cas6_full_fp64", 6, 3, 3, 6, -2.0, -0.5, None, seed_int=1000, seed_det=2000),
    1: Config("cas10_sampled_fp64", 10, 5, 5, 10, -2.0, -0.5, 20_000, w=0.4,
              seed_int=1001, seed_det=2001),
    2: Config("cas16_1m_mixed", 16, 7, 7, 16, -15.0, 1.0, 1_000_000, w=0.35, tail=0.05,
              seed_int=1002, seed_det=2002),
    3: Config("cas12_200k_grad", 12, 6, 6, 12, -2.0, -0.5, 200_000, w=0.4,
              seed_int=1003, seed_det=2003),
}


def config_inputs(idx: int, ndet: int | None = None):
    """(Integrals, alpha, beta, Config) for workload ``idx`` (0..3).

    ``ndet`` overrides the determinant count (same sampler and seed) for
    reduced-size parity runs."""
    cfg = CONFIGS[idx]
    ints = gen_integrals(cfg.norb, cfg.n_l, cfg.lo, cfg.hi, cfg.seed_int)
    if cfg.ndet is None and ndet is None:
        alpha, beta = full_space(cfg.norb, cfg.na, cfg.nb)
        # present the full space in a scrambled caller order
        perm = np.random.default_rng(cfg.seed_det).permutation(len(alpha))
        alpha, beta = alpha[perm], beta[perm]
    else:
        n = ndet if ndet is not None else cfg.ndet
        alpha, beta = sample_determinants(cfg.norb, cfg.na, cfg.nb, n, cfg.w, cfg.tail,
                                          cfg.seed_det)
    return ints, alpha, beta, cfg


def batch_instance_spec(i: int) -> dict:
    """Instance ``i`` (0..63) of the bond-scan-like batch.

    norb = 8 + floor(9 i / 64); N = norb - 2 (even i) or norb + 2 (odd i),
    alpha gets ceil(N/2); h_pp ~ U(-2,-0.5) scaled by s_i = 0.6 + 0.8 i/63;
    n_L = norb; D_i = round(1e3 * 300^(i/63)) capped at half the FCI
    dimension; rank weight 0.4; seeds 4000+i (integrals), 5000+i (dets)."""
    norb = 8 + (9 * i) // 64
    nel = norb - 2 if i % 2 == 0 else norb + 2
    na = (nel + 1) // 2
    nb = nel - na
    s = 0.6 + 0.8 * i / 63
    fci = math.comb(norb, na) * math.comb(norb, nb)
    ndet = min(int(round(1e3 * 300 ** (i / 63))), fci // 2)
    return dict(norb=norb, na=na, nb=nb, n_l=norb, lo=-2.0 * s, hi=-0.5 * s,
                ndet=ndet, w=0.4, seed_int=4000 + i, seed_det=5000 + i)


def batch_instance(i: int, ndet_scale: float = 1.0):
    spec = batch_instance_spec(i)
    ints = gen_integrals(spec["norb"], spec["n_l"], min(spec["lo"], spec["hi"]),
                         max(spec["lo"], spec["hi"]), spec["seed_int"])
    n = max(1, int(round(spec["ndet"] * ndet_scale)))
    alpha, beta = sample_determinants(spec["norb"], spec["na"], spec["nb"], n,
                                      spec["w"], 0.0, spec["seed_det"])
    return ints, alpha, beta, spec
