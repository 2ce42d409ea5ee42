"""Device memory through the caller's allocator (hinqs_create's alloc_fn/free_fn).

  * every buffer the library holds comes from the allocator and goes back to it
    (nothing is left outstanding after hinqs_destroy);
  * an allocator that returns NULL makes the call fail with HINQS_E_OOM, and the
    same context works normally once memory is available again;
  * repeated caller-order sigma calls allocate nothing after the first one.
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
    """PyTorch's pool, with a switch that makes every request fail."""

    def __init__(self):
        super().__init__(0, torch.cuda.current_stream(0).cuda_stream)
        self.fail = False
        self.calls = 0
        self.refused = 0
        self.live = {}

    def alloc(self, nbytes):
        self.calls += 1
        if self.fail:
            self.refused += 1
            return 0
        p = super().alloc(nbytes)
        if p:
            self.live[p] = nbytes
        return p

    def free(self, ptr):
        assert ptr in self.live, "free of a pointer the allocator did not hand out"
        del self.live[ptr]
        super().free(ptr)


def _instance():
    ints, a, b, cfg = W.config_inputs(1)
    return ints, a, b, cfg.na, cfg.nb


def test_allocator_owns_every_buffer():
    ints, a, b, na, nb = _instance()
    A = CountingAllocator()
    s = hq.Hinqs(allocator=A)
    s.set_integrals(ints.h, ints.eri, ints.e_core)
    s.set_determinants(a, b, na, nb)
    e, c, _ = s.lowest_eigenpair(tol=1e-9)
    log(f"allocator: {A.calls} allocations, {len(A.live)} live, {sum(A.live.values()) / 2**20:.1f} MiB")
    assert A.calls > 0 and len(A.live) > 0
    s.close()
    assert not A.live, f"{len(A.live)} buffers not returned"


def test_null_allocation_reports_oom_and_context_recovers():
    ints, a, b, na, nb = _instance()
    ref = hq.Hinqs(allocator="hip")
    ref.set_integrals(ints.h, ints.eri, ints.e_core)
    ref.set_determinants(a, b, na, nb)
    e_ref, c_ref, _ = ref.lowest_eigenpair(tol=1e-10)
    X = torch.from_numpy(np.random.default_rng(5).standard_normal((len(a), 3))).cuda()
    S_ref = ref.sigma(X)

    # creation itself allocates (sigma row counters)
    A0 = CountingAllocator()
    A0.fail = True
    with pytest.raises(hq.HinqsError) as err:
        hq.Hinqs(allocator=A0)
    assert err.value.code == -9
    assert not A0.live

    A = CountingAllocator()
    s = hq.Hinqs(allocator=A)
    s.set_integrals(ints.h, ints.eri, ints.e_core)
    A.fail = True
    log("building the determinant set with a failing allocator")
    with pytest.raises(hq.HinqsError) as err:
        s.set_determinants(a, b, na, nb)
    assert err.value.code == -9 and "allocator" in str(err.value)
    assert A.refused >= 1
    A.fail = False
    s.set_determinants(a, b, na, nb)
    S = s.sigma(X)
    assert torch.allclose(S, S_ref, rtol=0, atol=1e-12 * float(S_ref.abs().max()))

    # fail in the middle of a solve: the basis is allocated on its first use
    A.fail = True
    with pytest.raises(hq.HinqsError) as err:
        s.lowest_eigenpair(tol=1e-10)
    assert err.value.code == -9
    A.fail = False
    e, c, _ = s.lowest_eigenpair(tol=1e-10)
    assert abs(e - e_ref) <= 1e-10
    assert abs(float(torch.dot(c, c_ref))) >= 1 - 1e-10
    s.close()
    assert not A.live


def test_caller_order_sigma_allocates_once():
    ints, a, b, na, nb = _instance()
    A = CountingAllocator()
    s = hq.Hinqs(allocator=A)
    s.set_integrals(ints.h, ints.eri, ints.e_core)
    s.set_determinants(a, b, na, nb)
    rng = np.random.default_rng(11)
    X = torch.from_numpy(rng.standard_normal((len(a), 3))).cuda()  # k = 3: padded to 4 and staged
    S1 = s.sigma(X)
    before = A.calls
    for _ in range(3):
        S = s.sigma(X)
    assert A.calls == before, "repeated caller-order sigma allocated"
    assert torch.equal(S, S1)
    ref = hq.Hinqs(allocator="hip")
    ref.set_integrals(ints.h, ints.eri, ints.e_core)
    ref.set_determinants(a, b, na, nb)
    S_ref = ref.sigma(X)
    assert torch.allclose(S1, S_ref, rtol=0, atol=1e-12 * float(S_ref.abs().max()))


def test_batch_buffers_through_the_allocator():
    """The batch's concatenated arrays, per-instance build scratch and solve
    buffers come from the allocator too; a NULL return while adding an
    instance reports OOM, and the batch can be rebuilt and solved afterwards."""
    insts = [W.batch_instance(i, 0.1) for i in (0, 9, 20)]
    A = CountingAllocator()
    s = hq.Hinqs(allocator=A)
    for ints, a, b, spec in insts[:2]:
        s.batch_add(ints.h, ints.eri, ints.e_core, a, b, spec["na"], spec["nb"])
    A.fail = True
    ints, a, b, spec = insts[2]
    with pytest.raises(hq.HinqsError) as err:
        s.batch_add(ints.h, ints.eri, ints.e_core, a, b, spec["na"], spec["nb"])
    assert err.value.code == -9
    A.fail = False
    s.batch_clear()
    for ints, a, b, spec in insts:
        s.batch_add(ints.h, ints.eri, ints.e_core, a, b, spec["na"], spec["nb"])
    e, c, info = s.batch_lowest_eigenpair(tol=1e-9)
    assert info["converged"]
    for i, (ints, a, b, spec) in enumerate(insts):
        t = hq.Hinqs(allocator="hip")
        t.set_integrals(ints.h, ints.eri, ints.e_core)
        t.set_determinants(a, b, spec["na"], spec["nb"])
        ei, _, _ = t.lowest_eigenpair(tol=1e-9)
        assert abs(e[i] - ei) <= 1e-10
    s.close()
    assert not A.live
