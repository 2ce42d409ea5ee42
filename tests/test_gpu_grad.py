"""The RDM adjoint behind the autograd binding (Hellmann-Feynman gradients of
the lowest eigenvalue on a fixed determinant set with respect to the
integrals), checked three ways:

  * central finite differences of the GPU eigenvalue on 32 random integral
    entries of the 200,000-determinant norb-12 workload (step 1e-5, each
    entry moved together with all its real-orbital symmetry images):
    |FD - analytic| <= 2e-7 + 1e-6 |analytic| (the eigenvalue is solved to a
    residual of 1e-10, so its error is ~1e-20 / gap; rounding of E near
    1e2 Ha gives ~1e-13 / 1e-5 = 1e-8 of noise; the O(step^2) truncation is
    ~1e-10);
  * against the oracle's RDMs (operator by operator) on a 400-determinant
    set: grad_h = (rdm1 + rdm1^T)/2, grad_eri = 1/2 average of rdm2 over the
    8 index images, to 1e-12 relative to the largest element;
  * HinqsEnergy.apply(...).backward() returns exactly what integral_grad does.
"""
import itertools

import numpy as np
import pytest

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


def _eri_images(p, q, r, s):
    return {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
            (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}


def test_gradient_matches_central_differences():
    ints, a, b, cfg = W.config_inputs(3)
    log(f"finite differences on {len(a)} determinants, norb {cfg.norb}")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    e0, c0, st = s.lowest_eigenpair(tol=1e-10)
    gh, ge = s.integral_grad(c0)
    gh, ge = gh.cpu().numpy(), ge.cpu().numpy()
    n = cfg.norb
    rng = np.random.default_rng(33)
    step = 1e-5

    def energy(h, eri):
        s.set_integrals(h, eri, ints.e_core)
        e, _, _ = s.lowest_eigenpair(guess=c0, tol=1e-10)
        return e

    worst = 0.0
    for t in range(32):
        h, eri = ints.h.copy(), ints.eri.copy()
        dh, deri = np.zeros_like(h), np.zeros_like(eri)
        if t < 12:
            p, q = rng.integers(0, n, 2)
            dh[p, q] = dh[q, p] = 1.0
        else:
            p, q, r, u = rng.integers(0, n, 4)
            for img in _eri_images(p, q, r, u):
                deri[img] = 1.0
        analytic = float((gh * dh).sum() + (ge * deri).sum())
        ep = energy(h + step * dh, eri + step * deri)
        em = energy(h - step * dh, eri - step * deri)
        fd = (ep - em) / (2 * step)
        worst = max(worst, abs(fd - analytic) / (2e-7 + 1e-6 * abs(analytic)))
        assert abs(fd - analytic) <= 2e-7 + 1e-6 * abs(analytic), (t, fd, analytic)
    log(f"  worst |FD - analytic| / bar = {worst:.3f}")
    s.set_integrals(ints.h, ints.eri, ints.e_core)
    e1, _, _ = s.lowest_eigenpair(guess=c0, tol=1e-10)
    assert abs(e1 - e0) <= 1e-10


def test_gradient_matches_oracle_rdms():
    ints, a, b, cfg = W.config_inputs(0)
    log("integral gradient vs oracle RDMs, 400 determinants")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    o = oracle_for(ints, a, b, cfg.na, cfg.nb)
    _, c = o.lowest_eigenpair()
    gh, ge = s.integral_grad(torch.from_numpy(c).cuda())
    r1, r2 = o.rdm12(c)
    n = cfg.norb
    ref_h = 0.5 * (r1 + r1.T)
    ref_e = np.zeros_like(r2)
    for p, q, r, u in itertools.product(range(n), repeat=4):
        imgs = [(p, q, r, u), (q, p, r, u), (p, q, u, r), (q, p, u, r),
                (r, u, p, q), (u, r, p, q), (r, u, q, p), (u, r, q, p)]
        ref_e[p, q, r, u] = 0.5 * np.mean([r2[i] for i in imgs])
    gh, ge = gh.cpu().numpy(), ge.cpu().numpy()
    assert np.abs(gh - ref_h).max() <= 1e-12 * np.abs(ref_h).max()
    assert np.abs(ge - ref_e).max() <= 1e-12 * np.abs(ref_e).max()


def test_autograd_backward_equals_integral_grad():
    ints, a, b, cfg = W.config_inputs(1, ndet=5000)
    log("autograd backward")
    s = solver_for(ints, a, b, cfg.na, cfg.nb)
    h = torch.tensor(ints.h, dtype=torch.float64, requires_grad=True)
    eri = torch.tensor(ints.eri, dtype=torch.float64, requires_grad=True)
    E = hq.HinqsEnergy.apply(h, eri, s, ints.e_core, 1e-10)
    (2.5 * E).backward()
    _, c, _ = s.lowest_eigenpair(tol=1e-10)
    gh, ge = s.integral_grad(c, 2.5)
    assert np.allclose(h.grad.numpy(), gh.cpu().numpy(), rtol=0, atol=1e-12)
    assert np.allclose(eri.grad.numpy(), ge.cpu().numpy(), rtol=0, atol=1e-12)
    assert abs(float(E.detach()) - s.lowest_eigenpair(tol=1e-10)[0]) <= 1e-10
