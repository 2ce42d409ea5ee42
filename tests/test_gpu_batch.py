"""GPU parity of the batched solver: uneven bond-scan-like instances solved
together must give the same lowest eigenpairs as one-at-a-time solves (and
as the oracle's dense diagonalization where it is affordable).

Bars: eigenvalue within 1e-10 Ha of the sequential FP64 solve and of the
oracle (tol 1e-9 on the residual makes the eigenvalue error ~1e-18/gap);
eigenvector overlap >= 1 - 1e-10 with the sequential solve; graph replay and
plain launches bit-identical (every kernel is deterministic).
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import log, oracle_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hq = pytest.importorskip("paper_2606_26760_amd")

SUBSET = [0, 7, 18, 29, 40, 51, 62]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hq.load_library()


@pytest.fixture(scope="module")
def instances():
    return [W.batch_instance(i, 0.1) for i in SUBSET]


def _batch(instances):
    s = hq.Hinqs()
    for ints, a, b, spec in instances:
        s.batch_add(ints.h, ints.eri, ints.e_core, a, b, spec["na"], spec["nb"])
    return s


def _sequential(instances, block, tol):
    out = []
    for ints, a, b, spec in instances:
        s = hq.Hinqs()
        s.set_integrals(ints.h, ints.eri, ints.e_core)
        s.set_determinants(a, b, spec["na"], spec["nb"])
        e, c, st = s.lowest_eigenpair(block=block, tol=tol)
        out.append((e, c.cpu().numpy(), st))
    return out


@pytest.mark.parametrize("block,max_space", [(8, 48), (4, 12), (16, 64), (1, 6)])
def test_batch_matches_sequential(instances, block, max_space):
    log(f"batch of {len(instances)} instances, block {block}, max_space {max_space}")
    s = _batch(instances)
    n, off, nnz = s.batch_info()
    assert n == len(instances) and off[-1] == sum(len(x[1]) for x in instances) and nnz > 0
    e, c, info = s.batch_lowest_eigenpair(block=block, max_space=max_space, tol=1e-9, max_iter=400)
    assert info["converged"] and np.all(info["status"] == 0)
    assert info["stats"]["graphs"] >= 1 and info["stats"]["iterations"] == info["iterations"].max()
    c = c.cpu().numpy()
    seq = _sequential(instances, block, 1e-9)
    for i, (es, cs, _) in enumerate(seq):
        ci = c[off[i]:off[i + 1]]
        assert abs(e[i] - es) <= 1e-10, (i, e[i], es)
        assert abs(np.linalg.norm(ci) - 1.0) <= 1e-12
        assert abs(float(ci @ cs)) >= 1.0 - 1e-10, i
        # same gauge: the largest component is positive in both
        assert ci[np.argmax(np.abs(ci))] > 0


@pytest.fixture(scope="module")
def sequential_k8(instances):
    return _sequential(instances, 8, 1e-9)


@pytest.mark.parametrize("chunk,rr_threads", [(1024, 512), (1024, 1024), (2048, 512), (2048, 1024),
                                              (4096, 512), (4096, 1024), (8192, 512), (8192, 1024),
                                              (2048, 256)])
def test_every_batch_shape(instances, sequential_k8, chunk, rr_threads, monkeypatch):
    """Each launch shape the batch tuner can choose (chunk rows of the tall-skinny
    kernels, Rayleigh-Ritz threads) gives the sequential solves' eigenpairs."""
    monkeypatch.setenv("HINQS_BATCH_CHUNK", str(chunk))
    monkeypatch.setenv("HINQS_BATCH_RR_THREADS", str(rr_threads))
    log(f"batch shape chunk={chunk} rr_threads={rr_threads}")
    s = _batch(instances)
    e, c, info = s.batch_lowest_eigenpair(tol=1e-9)
    st = info["stats"]
    assert info["converged"] and st["chunk_rows"] == chunk and st["rr_threads"] == rr_threads
    c = c.cpu().numpy()
    off = info["offsets"]
    for i, (es, cs, _) in enumerate(sequential_k8):
        assert abs(e[i] - es) <= 1e-10, (i, e[i], es)
        assert abs(float(c[off[i]:off[i + 1]] @ cs)) >= 1.0 - 1e-10, i


def test_batch_autotune_picks_and_caches_a_shape(instances, sequential_k8):
    s = _batch(instances)
    e1, _, i1 = s.batch_lowest_eigenpair(tol=1e-9, autotune=True)
    e2, _, i2 = s.batch_lowest_eigenpair(tol=1e-9, autotune=True)
    st1, st2 = i1["stats"], i2["stats"]
    log(f"tuned shape chunk={st1['chunk_rows']} rr_threads={st1['rr_threads']} in {st1['ms_tune']:.1f} ms")
    assert st1["ms_tune"] > 0.0 and st2["ms_tune"] == 0.0   # the second call reuses the choice
    assert st1["chunk_rows"] in (1024, 2048, 4096, 8192) and st1["rr_threads"] in (512, 1024)
    assert (st2["chunk_rows"], st2["rr_threads"]) == (st1["chunk_rows"], st1["rr_threads"])
    for i, (es, _, _) in enumerate(sequential_k8):
        assert abs(e1[i] - es) <= 1e-10 and abs(e2[i] - es) <= 1e-10


def test_batch_matches_oracle_dense(instances):
    small = [x for x in instances if len(x[1]) <= 4000]
    log(f"batch vs oracle dense, {len(small)} instances")
    s = _batch(small)
    e, c, info = s.batch_lowest_eigenpair(tol=1e-9)
    c = c.cpu().numpy()
    off = info["offsets"]
    for i, (ints, a, b, spec) in enumerate(small):
        o = oracle_for(ints, a, b, spec["na"], spec["nb"])
        e_ref, c_ref = o.lowest_eigenpair()
        w = o.spectrum(2)
        assert abs(e[i] - e_ref) <= 1e-10, (i, e[i], e_ref)
        if w[1] - w[0] > 1e-6:
            assert abs(float(c[off[i]:off[i + 1]] @ c_ref)) >= 1.0 - 1e-10


def test_full_size_instance_vs_oracle_lanczos():
    """Instance 33 of the batch at full size (norb 12, 7a + 7b, 19,900
    determinants) solved inside a batch with two smaller full-size instances;
    its eigenvalue against the oracle's Lanczos at 1e-10 Ha."""
    insts = [W.batch_instance(i) for i in (33, 0, 12)]
    assert len(insts[0][1]) > 19000
    log(f"batch with a full-size instance of {len(insts[0][1])} determinants vs oracle Lanczos")
    s = _batch(insts)
    e, c, info = s.batch_lowest_eigenpair(tol=1e-9)
    assert info["converged"]
    off = info["offsets"]
    c = c.cpu().numpy()
    for i, (ints, a, b, spec) in enumerate(insts):
        o = oracle_for(ints, a, b, spec["na"], spec["nb"])
        e_ref, c_ref = o.lowest_eigenpair(dense_max=0 if i == 0 else 5000)
        log(f"  instance {i}: n={len(a)} E={e[i]!r} ref={e_ref!r}")
        assert abs(e[i] - e_ref) <= 1e-10, (i, e[i], e_ref)
        w = o.spectrum(2)
        if w[1] - w[0] > 1e-6:
            assert abs(float(c[off[i]:off[i + 1]] @ c_ref)) >= 1.0 - 1e-9


def test_graph_replays_equal_plain_launches(instances):
    """Each captured iteration graph is replayed many times; the result must be
    bit-identical to issuing the same kernels directly, and to a second call."""
    log("batch graph vs plain launches")
    s = _batch(instances)
    e1, c1, i1 = s.batch_lowest_eigenpair(tol=1e-9, graph=True)
    e2, c2, i2 = s.batch_lowest_eigenpair(tol=1e-9, graph=False)
    e3, c3, i3 = s.batch_lowest_eigenpair(tol=1e-9, graph=True)
    assert i2["stats"]["graphs"] == 0 and i1["stats"]["graphs"] >= 2
    assert i1["stats"]["iterations"] > i1["stats"]["graphs"]   # graphs were replayed
    assert np.array_equal(e1, e2) and np.array_equal(e1, e3)
    assert torch.equal(c1, c2) and torch.equal(c1, c3)
    assert np.array_equal(i1["iterations"], i2["iterations"])


def test_batch_sorted_order_and_autotune(instances):
    s = _batch(instances[:4])
    e, c, info = s.batch_lowest_eigenpair(tol=1e-9)
    es, cs, infos = s.batch_lowest_eigenpair(tol=1e-9, sorted_order=True, autotune=True)
    assert np.all(np.abs(e - es) <= 1e-10)
    off = info["offsets"]
    for i, (ints, a, b, spec) in enumerate(instances[:4]):
        t = hq.Hinqs()
        t.set_integrals(ints.h, ints.eri, ints.e_core)
        t.set_determinants(a, b, spec["na"], spec["nb"])
        perm = t.permutation().cpu().numpy()  # sorted position -> caller index
        ci = c[off[i]:off[i + 1]].cpu().numpy()
        csi = cs[off[i]:off[i + 1]].cpu().numpy()
        assert abs(float(ci[perm] @ csi)) >= 1.0 - 1e-10


def test_batch_not_converged_and_errors(instances):
    s = hq.Hinqs()
    with pytest.raises(hq.HinqsError) as ex:
        s.batch_lowest_eigenpair()
    assert ex.value.name == "NOT_READY"
    s = _batch(instances[:3])
    e, c, info = s.batch_lowest_eigenpair(max_iter=2, tol=1e-12, raise_on_not_converged=False)
    assert not info["converged"] and np.all(info["status"] == -7)
    assert np.all(np.isfinite(e)) and np.all(info["iterations"] == 2)
    off = info["offsets"]
    cc = c.cpu().numpy()
    for i in range(3):
        assert abs(np.linalg.norm(cc[off[i]:off[i + 1]]) - 1.0) <= 1e-12
    with pytest.raises(hq.HinqsError) as ex:
        s.batch_lowest_eigenpair(max_iter=2, tol=1e-12)
    assert ex.value.name == "NOT_CONVERGED"
    ints, a, b, spec = instances[0]
    s.batch_add(ints.h, ints.eri, ints.e_core, a[:20], b[:20], spec["na"], spec["nb"])
    with pytest.raises(hq.HinqsError) as ex:
        s.batch_lowest_eigenpair(max_space=48)
    assert ex.value.name == "UNSUPPORTED"
    s.batch_clear()
    assert s.batch_info()[0] == 0
    with pytest.raises(hq.HinqsError) as ex:
        s.batch_add(ints.h, ints.eri, ints.e_core, a[:5], b[:5], spec["na"] + 1, spec["nb"])
    assert ex.value.name == "BAD_OCCUPATION"


def test_batch_small_instances_and_the_size_floor():
    """Instances down to the subspace size (48 determinants at block 8; subsets
    of the 300-determinant full space of norb 6, 3a + 2b, once with negative
    and once with positive spectra) batched with a 1,381-determinant one:
    each lowest eigenvalue against the oracle's dense diagonalization.  An
    instance below that size is refused with UNSUPPORTED, and the context
    then solves the valid batch."""
    import dataclasses
    ints = W.gen_integrals(6, 6, -2.0, -0.5, 41)
    shifted = dataclasses.replace(ints, e_core=ints.e_core + 100.0)  # every eigenvalue positive
    fa, fb = W.full_space(6, 3, 2)
    rng = np.random.default_rng(42)
    insts = []
    for it in (ints, shifted):
        for n in (48, 49, 60, 300):
            idx = rng.permutation(len(fa))[:n]
            insts.append((it, fa[idx], fb[idx], {"na": 3, "nb": 2}))
    insts.append(W.batch_instance(29, 0.1))
    tiny = (ints, fa[:47], fb[:47], {"na": 3, "nb": 2})
    log("batch with small instances: " + ", ".join(str(len(x[1])) for x in insts))
    s = _batch(insts + [tiny])
    with pytest.raises(hq.HinqsError) as ex:
        s.batch_lowest_eigenpair(block=8, tol=1e-9)
    assert ex.value.name == "UNSUPPORTED" and "fewer determinants" in str(ex.value)
    s.batch_clear()
    for it, a, b, spec in insts:
        s.batch_add(it.h, it.eri, it.e_core, a, b, spec["na"], spec["nb"])
    e, c, info = s.batch_lowest_eigenpair(block=8, tol=1e-9)
    assert all(int(x) == 0 for x in info["status"])
    for i, (it, a, b, spec) in enumerate(insts):
        o = oracle_for(it, a, b, spec["na"], spec["nb"])
        e_ref = o.lowest_eigenpair()[0]
        log(f"  instance {i}: n={len(a)} E={e[i]!r} ref={e_ref!r}")
        assert abs(e[i] - e_ref) <= 1e-10
