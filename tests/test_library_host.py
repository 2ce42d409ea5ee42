"""CPU-side checks of the HIP library: it loads, exports every entry point the
header declares, and its host-side sign rules agree with the oracle's
operator application.  No GPU computation happens here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2606_26760_amd as hq
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "hinqs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hinqs_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = hq.load_library()
    names = _declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(hq.EXPORTED)


def test_opts_defaults_match_header():
    import ctypes
    o = hq.Opts()
    hq.load_library().hinqs_opts_default(ctypes.byref(o))
    assert (o.block, o.max_space, o.max_iter, o.tol, o.precision) == (8, 48, 200, 1e-8, 0)
    assert o.precond_floor == 1e-8 and o.mixed_switch == 1e-5 and o.flags == 0


@pytest.mark.parametrize("norb,na,nb", [(4, 2, 2), (5, 3, 2), (6, 3, 3), (6, 1, 4)])
def test_pair_descriptors_match_oracle(norb, na, nb):
    """Class, holes, particles and sign of every coupled pair of a full space,
    from the library's masked-popcount rules, equal the oracle's
    operator-string signs."""
    rng = np.random.default_rng(norb * 100 + na * 10 + nb)
    alpha, beta = W.full_space(norb, na, nb)
    h = np.eye(norb)
    eri = np.zeros((norb,) * 4)
    o = oracle.Oracle(norb, na, nb, h, eri, 0.0, alpha, beta)
    rows = rng.choice(len(alpha), size=min(len(alpha), 60), replace=False)
    r = o.rows(rows)
    n = 0
    for t, i in enumerate(r["rows"]):
        for e in range(r["rowptr"][t] + 1, r["rowptr"][t + 1]):
            j = int(r["col"][e])
            d = hq.pair_descriptor(int(alpha[i]), int(beta[i]), int(alpha[j]), int(beta[j]))
            typ, neg, h1, h2, p1, p2 = (int(v) for v in hq.decode_descriptor(d))
            et = int(r["etype"][e])
            orb = [int(v) for v in r["orb"][e]]
            assert typ == et
            assert (h1, p1) == (orb[0], orb[2])
            if et >= 3:
                assert (h2, p2) == (orb[1], orb[3])
            assert (-1 if neg else 1) == int(r["sign"][e])
            n += 1
    assert n > 0
    # pairs further apart or identical are not couplings
    assert hq.pair_descriptor(int(alpha[0]), int(beta[0]), int(alpha[0]), int(beta[0])) == 0


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        hq.Hinqs()


def test_create_rejects_half_an_allocator():
    # alloc_fn without free_fn (or the reverse) is refused before any device call
    lib = hq.load_library()
    h = ctypes.c_void_p()
    alloc = hq.ALLOC_FN(lambda n, s, u: None)
    free = hq.FREE_FN(lambda p, s, u: None)
    assert lib.hinqs_create(ctypes.byref(h), 0, None, alloc, hq.FREE_FN(), None) == -1
    assert lib.hinqs_create(ctypes.byref(h), 0, None, hq.ALLOC_FN(), free, None) == -1
    assert h.value is None
