"""hinqs_sigma_noalloc (static per-GPU scratch, no allocation) against hinqs_sigma.

Bar: |S - S_ref| <= tol * max |S_ref| per column, tol = 1e-12 (FP64) or 2e-6
(FP32); both entry points run the same kernels in the same launch shape, so
the results are also required to be bitwise equal.
Two calls in a row, the second on a smaller set, check that nothing the
previous call left in the shared array leaks into a result.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hq = pytest.importorskip("paper_2606_26760_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hq.load_library()


class CountingAllocator(hq.TorchAllocator):
    def __init__(self):
        super().__init__(0, torch.cuda.current_stream(0).cuda_stream)
        self.calls = 0

    def alloc(self, nbytes):
        self.calls += 1
        return super().alloc(nbytes)


def _solver(cfg_index, ndet=None):
    ints, a, b, cfg = W.config_inputs(cfg_index, ndet=ndet) if ndet else W.config_inputs(cfg_index)
    A = CountingAllocator()
    s = hq.Hinqs(allocator=A)
    s.set_integrals(ints.h, ints.eri, ints.e_core)
    s.set_determinants(a, b, cfg.na, cfg.nb)
    return s, A


def _compare(S, S_ref, tol):
    scale = S_ref.abs().double().amax(dim=0, keepdim=True) + 1e-300
    err = ((S.double() - S_ref.double()).abs() / scale).max().item()
    log(f"  max |S - S_ref| / max|S_ref| = {err:.3e}")
    assert err <= tol
    return err


def _call(s, A, X, sorted_order):
    out = torch.full_like(X, float("nan"))
    before = A.calls
    s.sigma_noalloc(X, out, sorted_order=sorted_order)
    torch.cuda.synchronize()
    assert A.calls == before, "the no-allocation entry point allocated"
    return out


def test_noalloc_matches_sigma_two_calls_shrinking():
    rng = np.random.default_rng(17)
    log("no-alloc sigma: 20000 determinants, k = 3, FP64, caller order")
    s1, A1 = _solver(1)
    X1 = torch.from_numpy(rng.standard_normal((s1.ndet, 3))).cuda()
    S1 = _call(s1, A1, X1, False)
    _compare(S1, s1.sigma(X1), 1e-12)
    assert torch.equal(S1, s1.sigma(X1))

    log("no-alloc sigma: 400 determinants, k = 2, FP32, caller order (smaller, after the first)")
    s2, A2 = _solver(0)
    X2 = torch.from_numpy(rng.standard_normal((s2.ndet, 2))).float().cuda()
    S2 = _call(s2, A2, X2, False)
    _compare(S2, s2.sigma(X2), 2e-6)
    assert torch.equal(S2, s2.sigma(X2))

    log("no-alloc sigma: 400 determinants, k = 1, FP64, sorted order (direct, counters only)")
    X3 = torch.from_numpy(rng.standard_normal(s2.ndet)).cuda()
    S3 = _call(s2, A2, X3, True)
    assert torch.equal(S3, s2.sigma(X3, sorted_order=True))

    log("no-alloc sigma: 20000 determinants, k = 8, FP64, sorted order, then k = 5 caller order")
    X4 = torch.from_numpy(rng.standard_normal((s1.ndet, 8))).cuda()
    S4 = _call(s1, A1, X4, True)
    assert torch.equal(S4, s1.sigma(X4, sorted_order=True))
    X5 = torch.from_numpy(rng.standard_normal((s1.ndet, 5))).cuda()
    S5 = _call(s1, A1, X5, False)
    assert torch.equal(S5, s1.sigma(X5))


def test_noalloc_rejects_staging_beyond_the_array():
    rng = np.random.default_rng(23)
    s, A = _solver(2, ndet=300_000)
    X = torch.from_numpy(rng.standard_normal((s.ndet, 16))).cuda()
    out = torch.empty_like(X)
    # caller order: 2 x 300000 x 16 x 8 bytes of staging > 64 MiB
    with pytest.raises(hq.HinqsError) as err:
        s.sigma_noalloc(X, out)
    assert err.value.code == -6 and "limit" in str(err.value)
    # sorted order needs no staging, whatever the size
    S = _call(s, A, X, True)
    assert torch.equal(S, s.sigma(X, sorted_order=True))


@pytest.mark.parametrize("k,sorted_order", [(3, False), (8, True)])
def test_noalloc_sigma_replays_in_a_captured_graph(k, sorted_order):
    """The entry point's purpose: issued under HIP graph capture (it allocates,
    clears with memset and synchronizes nothing).  The graph is replayed
    several times with new inputs written eagerly in between, and every replay
    must equal the eager hinqs_sigma."""
    ints, a, b, cfg = W.config_inputs(1)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = hq.Hinqs(stream=side)
        s.set_integrals(ints.h, ints.eri, ints.e_core)
        s.set_determinants(a, b, cfg.na, cfg.nb)
        X = torch.empty(s.ndet, k, dtype=torch.float64, device="cuda")
        out = torch.empty_like(X)
        X.normal_()
        s.sigma_noalloc(X, out, sorted_order=sorted_order)  # eager warm-up
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        s.sigma_noalloc(X, out, sorted_order=sorted_order)
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda")
    for r in range(4):
        gen.manual_seed(100 + r)
        X.normal_(generator=gen)
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = s.sigma(X, sorted_order=sorted_order)
        torch.cuda.synchronize()
        log(f"  replay {r}: k={k} sorted={sorted_order}")
        assert torch.equal(out, ref), r
