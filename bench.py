#!/usr/bin/env python3
"""Benchmark of the selected-CI hot path on one MI355X.

One step = one pass of the whole subspace-diagonalization path of the paper's
Step 3 over the 1e6-determinant CAS(14,16)-shaped workload (norb = 16, 7
alpha + 7 beta electrons, determinants drawn with weight 0.35^rank plus a 5%
uniform tail; synthetic integrals), starting from determinant strings already
resident in HBM:
  set_integrals -> set_determinants (validate, sort, string tables, couplings,
  Slater-Condon elements) -> FP64 Davidson to 1e-8 -> mixed-precision
  Davidson to 1e-8 -> 1-/2-RDM of the FP64 eigenvector,
followed by the batched solve of a bond-scan-like family of 64 uneven
instances (norb 8..16, N = norb -+ 2, 1e3..3e5 determinants each, 3.45e6 in
all; host inputs): build every instance, then one batched FP64 Davidson to
1e-8 (one graph launch per iteration).  The same 64 instances solved one at a
time are timed once outside the timed region for comparison.

value = H.X elements per second of the FP64 block-sigma kernel on the
        1e6-determinant set ((nnz + ndet) * k per launch over its average
        launch time, from HIP events recorded around each launch on the
        library's stream during the timed FP64 solves); the "step" object
        gives the same elements summed over every block product of the step
        (both solves and the batch) over the step's wall time.
The roofline object covers that kernel: algorithmic bytes per launch
(12 nnz + 16 k ndet + 16 ndet + 8) over the same launch time.  Its traffic
is the memory-counter figure of profiles/sigma_traffic.json (FETCH_SIZE +
WRITE_SIZE per launch, scaled by the factors a copy kernel of known size
gives), used only while the sigma source is the one measured: it counts L2
requests to the memory fabric, which the Infinity Cache serves in part, so
its rate is not an HBM rate.  roofline_fp32 is the FP32 sigma kernel, timed
with HIP events on the library's stream after the timed steps.
cpu_baseline times the CPU oracle's matrix-free sigma on a bounded row sample.

After the timed steps, the "select" object times one pass of the selection
steps that follow the solve (Sec. 2.2): the classical expansion of the 1000
largest |c| of the FP64 eigenvector (Eq. 2), the PT2 score of every expanded
determinant (Eq. 3), the top 1e5 by score and the spin-marginal teacher
weights (Eqs. 5-6), with the oracle's PT2 rate on a sample beside it.  The "iteration" object then completes that outer iteration:
PT2 of the set's own members (their eviction ranking), the growth rule
(append the 1e5 best-scored, cap at 1.05e6) applied as an incremental update
of the couplings, and the FP64 Davidson warm-started from the carried vector.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sigma H·X elements/s + HBM GB/s; Davidson solve time to 1e-8 Ha, mixed vs FP64"
HBM_PEAK_GBS = 8000.0


def cpu_baseline(o, alpha, cfg, target_s=10.0):
    """The oracle's matrix-free sigma (k = 8) on a random row sample, as it stands."""
    import numpy as np

    import oracle
    import workloads as W
    X = W.random_block(len(alpha), cfg.k, 99)
    rng = np.random.default_rng(123)
    n = 256
    t0 = time.perf_counter()
    _, pairs = o.sigma_rows(X, rng.choice(len(alpha), n, replace=False), return_pairs=True)
    dt = time.perf_counter() - t0
    n2 = int(min(len(alpha), max(n, n * target_s / max(dt, 1e-3))))
    rows = rng.choice(len(alpha), n2, replace=False)
    t0 = time.perf_counter()
    _, pairs = o.sigma_rows(X, rows, return_pairs=True)
    dt = time.perf_counter() - t0
    return {"value": pairs * cfg.k / dt, "unit": "elements/s", "cores": oracle.Oracle.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"matrix-free operator-application sigma, k={cfg.k}, {n2} random rows of the "
                      f"{len(alpha)}-determinant set ({pairs} stored elements), {dt:.1f} s"}


def cpu_model():
    """Host CPU model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def fp32_sigma_launch(hq, solver, D, k, reps=20):
    """Average FP32 block-sigma launch time (ms) on the solver's set, from HIP
    events on the library's stream (the current stream)."""
    import torch
    X = torch.randn(D, k, dtype=torch.float32, device="cuda")
    S = torch.empty_like(X)
    solver.sigma(X, out=S, sorted_order=True)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        solver.sigma(X, out=S, sorted_order=True)
        b.record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / reps


def sigma_counter_run(hq, ints, alpha, beta, cfg, reps, precision="fp64"):
    """Repeated block-sigma launches on the workload (FP64 or FP32), then two
    calibration references for the memory counters, three launches each:
      copy:   an elementwise kernel reading and writing 512 MiB (128-byte
              streaming requests);
      gather: index_select of 4 Mi random 64-byte rows of a 64 MiB table
              (the access pattern of the sigma kernel's X rows), reading
              256 MiB of rows plus 32 MiB of indices and writing 256 MiB."""
    import torch
    s = hq.Hinqs(0)
    s.set_integrals(ints.h, ints.eri, ints.e_core)
    s.set_determinants(alpha, beta, cfg.na, cfg.nb)
    # the default launch shape, the one the step's solves use
    dt = torch.float64 if precision == "fp64" else torch.float32
    X = torch.randn(len(alpha), cfg.k, dtype=dt, device="cuda")
    S = torch.empty_like(X)
    for _ in range(max(1, reps)):
        s.sigma(X, out=S, sorted_order=True)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    del src, dst
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    table = torch.ones(1 << 20, 8, dtype=torch.float64, device="cuda")
    idx = torch.randint(0, 1 << 20, (4 << 20,), device="cuda", generator=g)
    out = torch.empty(4 << 20, 8, dtype=torch.float64, device="cuda")
    for _ in range(3):
        torch.index_select(table, 0, idx, out=out)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "sigma", "precision": precision, "ndet": len(alpha), "nnz": s.info()["nnz"],
                      "launches": reps, "shape": "default"}))


def solve_run(hq, ints, alpha, beta, cfg, reps):
    """FP64 and mixed Davidson solves of the workload, `reps` each after one
    untimed solve of each (for per-kernel traces of the solver alone)."""
    import torch
    s = hq.Hinqs(0)
    s.set_integrals(ints.h, ints.eri, ints.e_core)
    s.set_determinants(alpha, beta, cfg.na, cfg.nb)
    out = {"mode": "solve", "ndet": len(alpha), "nnz": s.info()["nnz"]}
    for mixed in (False, True):
        s.lowest_eigenpair(tol=cfg.tol, block=cfg.k, mixed=mixed)
        torch.cuda.synchronize()
        ms, st = [], None
        for _ in range(max(1, reps)):
            t0 = time.perf_counter()
            e, _, st = s.lowest_eigenpair(tol=cfg.tol, block=cfg.k, mixed=mixed)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        key = "mixed" if mixed else "fp64"
        out[key] = {"energy": e, "ms": min(ms), "iterations": st["iterations"],
                    "iterations_fp32": st["iterations_fp32"], "ms_sigma": st["ms_sigma"],
                    "sigma_blocks": st["sigma_blocks"]}
        print(json.dumps({key: out[key]}), flush=True)
    out["mixed_over_fp64"] = out["mixed"]["ms"] / out["fp64"]["ms"]
    out["abs_dE"] = abs(out["mixed"]["energy"] - out["fp64"]["energy"])
    print(json.dumps(out), flush=True)


def batch_inputs(n=64):
    import workloads as W
    return [W.batch_instance(i) for i in range(n)]


def sequential_batch(hq, insts, block, tol):
    """The batch's instances solved one at a time with the plain FP64 solver."""
    import torch
    t_build = t_solve = 0.0
    energies = []
    for ints, a, b, spec in insts:
        s = hq.Hinqs(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_integrals(ints.h, ints.eri, ints.e_core)
        s.set_determinants(a, b, spec["na"], spec["nb"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e, _, _ = s.lowest_eigenpair(block=block, tol=tol)
        torch.cuda.synchronize()
        t_build += t1 - t0
        t_solve += time.perf_counter() - t1
        energies.append(e)
        s.close()
    return t_build, t_solve, energies


def selection_pass(hq, solver, c, e0, ntop, keep, reps=3):
    """One pass of the selection steps that follow the solve, on the solved
    determinant set: classical expansion of the ntop largest |c| (Eq. 2),
    PT2 scores of every expanded determinant (Eq. 3), the top `keep` of
    them, and the spin-marginal teacher weights of c (Eqs. 5-6).  Median wall time of each phase over `reps` passes (each call
    synchronizes the library's stream)."""
    import numpy as np
    import torch
    times = {"expand": [], "pt2": [], "top_k": [], "weights": []}
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ya, yb, _ = solver.expand(c, ntop)
        t1 = time.perf_counter()
        num, hxx, score = solver.pt2(c, e0, ya, yb)
        t2 = time.perf_counter()
        k = min(keep, len(ya))
        idx = solver.top_k(score, k, largest=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        solver.teacher_weights(c)
        torch.cuda.synchronize()
        times["weights"].append(time.perf_counter() - t3)
        times["expand"].append(t1 - t0)
        times["pt2"].append(t2 - t1)
        times["top_k"].append(t3 - t2)
    med = {kk: float(np.median(v)) * 1e3 for kk, v in times.items()}
    n = len(ya)
    return {"ntop": ntop, "candidates": n, "keep": k,
            "ms_expand": med["expand"], "ms_pt2": med["pt2"], "ms_top_k": med["top_k"],
            "ms_teacher_weights": med["weights"],
            "pt2_candidates_per_s": n / (med["pt2"] * 1e-3),
            "max_score": float(score[idx[0]].item()) if n else None}, (ya, yb)


def outer_iteration(hq, solver, solver_integrals, c, e0, ya, yb, cand_score, keep, b_max, k, tol):
    """The rest of one outer iteration after scoring (Sec. 2.2, Steps 2-3 at
    t >= 2): PT2 scores of the current set (its eviction ranking), the growth
    rule (append the `keep` best candidates, cap at b_max), then the FP64
    Davidson warm-started from the carried eigenvector."""
    import torch
    a_b, b_b = solver.determinants()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, bscore = solver.pt2_members(c, e0)   # PT2 of the set's own members: one sigma product
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c_new, _, ms_upd = solver.grow_basis(ya, yb, cand_score, keep, basis_score=bscore, b_max=b_max, coeffs=c)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    e1, _, st = solver.lowest_eigenpair(guess=c_new, tol=tol, block=k)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    # sigma on the patched couplings against a from-scratch build of the same set
    def sigma_ms(s, reps=5):
        X = torch.ones(s.ndet, k, dtype=torch.float64, device="cuda")
        S = torch.empty_like(X)
        s.sigma(X, out=S, sorted_order=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            s.sigma(X, out=S, sorted_order=True)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3
    a_n, b_n = solver.determinants()
    fresh = hq.Hinqs(0)
    fresh.set_integrals(*solver_integrals)
    fresh.set_determinants(a_n, b_n, solver.na, solver.nb)
    out = {"ndet_new": solver.ndet, "nnz_new": solver.info()["nnz"], "ms_rescore_set": (t1 - t0) * 1e3,
           "ms_grow_update": (t2 - t1) * 1e3, "ms_update_kernels": ms_upd, "ms_warm_solve": (t3 - t2) * 1e3,
           "warm_iterations": st["iterations"], "energy": e1, "energy_drop": e0 - e1,
           "ms_fresh_build": fresh.info()["ms_sort"] + fresh.info()["ms_connect"] + fresh.info()["ms_elements"],
           "ms_sigma_patched": sigma_ms(solver), "ms_sigma_fresh": sigma_ms(fresh)}
    fresh.close()
    return out


def cpu_pt2_rate(o, c, e0, ya, yb, n=40000):
    """The oracle's PT2 (Eq. 3) on a sample of the expanded determinants, as it stands."""
    import oracle
    m = min(n, len(ya))
    t0 = time.perf_counter()
    o.pt2(c, e0, ya[:m], yb[:m])
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "candidates/s", "cores": oracle.Oracle.num_threads(), "kind": "oracle",
            "sample": f"first {m} expanded determinants, {dt:.2f} s"}


def copy_peak_gbs(nbytes=2 << 30, reps=10):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of
    a 2 GiB buffer (larger than the Infinity Cache): the streaming rate this
    HBM reaches with a plain copy, next to the 8 TB/s spec."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * nbytes / t / 1e9


def recorded_traffic():
    """Fabric bytes per FP64 sigma launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
    from the committed counter summary, or None when the sigma kernel source
    has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sigma_traffic.json")
    src = os.path.join(ROOT, "paper_2606_26760_amd", "csrc", "sigma.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("sigma_source_sha256") != sha:
        return None
    return float(rec["bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ndet", type=int, default=None, help="override the determinant count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="leave the batched instances out of the step")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--ntop", type=int, default=1000, help="determinants expanded by the selection pass")
    ap.add_argument("--keep", type=int, default=100000, help="candidates kept by score in the selection pass")
    ap.add_argument("--sigma-precision", choices=["fp64", "fp32"], default="fp64",
                    help="precision of the launches of --mode sigma")
    ap.add_argument("--mode", choices=["step", "sigma", "solve"], default="step",
                    help="sigma: only repeated FP64 sigma launches plus a copy kernel of known "
                         "size (for hardware-counter runs); solve: only FP64 and mixed Davidson "
                         "solves of the workload (for per-kernel traces of the solver)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU path is "
              "not part of this library", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2606_26760_amd as hq
    import workloads as W

    ints, alpha, beta, cfg = W.config_inputs(2, ndet=args.ndet)
    D = len(alpha)
    if args.mode == "sigma":
        sigma_counter_run(hq, ints, alpha, beta, cfg, args.steps, args.sigma_precision)
        return
    if args.mode == "solve":
        solve_run(hq, ints, alpha, beta, cfg, args.steps)
        return
    dev = torch.device("cuda", 0)
    a_d = torch.from_numpy(alpha.view(np.int64).copy()).to(dev)
    b_d = torch.from_numpy(beta.view(np.int64).copy()).to(dev)
    solver = hq.Hinqs(0)
    stream = torch.cuda.current_stream(dev)
    insts = None if args.no_batch else batch_inputs()
    bsolver = None if args.no_batch else hq.Hinqs(0)

    last = {}

    def step():
        t = {}
        t0 = time.perf_counter()
        solver.set_integrals(ints.h, ints.eri, ints.e_core)
        solver.set_determinants(a_d, b_d, cfg.na, cfg.nb)
        t1 = time.perf_counter()
        e64, c64, st64 = solver.lowest_eigenpair(tol=cfg.tol, block=cfg.k)
        last["c64"] = c64
        t2 = time.perf_counter()
        em, cm, stm = solver.lowest_eigenpair(tol=cfg.tol, block=cfg.k, mixed=True)
        t3 = time.perf_counter()
        d1, d2 = solver.rdm12(c64)
        stream.synchronize()
        t4 = time.perf_counter()
        t.update(build=t1 - t0, fp64=t2 - t1, mixed=t3 - t2, rdm=t4 - t3)
        bres = None
        if insts is not None:
            bsolver.batch_clear()
            for bi, ba, bb, spec in insts:
                bsolver.batch_add(bi.h, bi.eri, bi.e_core, ba, bb, spec["na"], spec["nb"])
            stream.synchronize()
            t5 = time.perf_counter()
            be, _, binfo = bsolver.batch_lowest_eigenpair(tol=cfg.tol, block=cfg.k, autotune=True)
            stream.synchronize()
            t6 = time.perf_counter()
            t.update(batch_build=t5 - t4, batch_solve=t6 - t5)
            bres = (be, binfo)
        return t, (e64, st64), (em, stm), bres

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    info = solver.info()
    nnz = info["nnz"]
    cols = sum(r[1][1]["sigma_columns"] + r[2][1]["sigma_columns"] for r in res)
    elements = (nnz + D) * cols
    if insts is not None:
        elements += sum(r[3][1]["stats"]["sigma_elements"] for r in res)
    step_value = elements / elapsed
    # FP64 sigma launches of the FP64 solves: one kernel per event pair
    ms_sig = sum(r[1][1]["ms_sigma"] for r in res)
    n_sig = sum(r[1][1]["sigma_blocks"] for r in res)
    t_launch = ms_sig / n_sig * 1e-3
    k = cfg.k
    alg_bytes = 12 * nnz + 16 * k * D + 8 * (D + 1) + 8 * D
    achieved = alg_bytes / t_launch / 1e9
    value = (nnz + D) * k / t_launch
    traffic = recorded_traffic()
    ms32 = fp32_sigma_launch(hq, solver, D, k)
    alg32 = 8 * nnz + 8 * k * D + 8 * (D + 1) + 4 * D
    med = lambda xs: float(np.median(xs))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cas16_{D}: norb=16, 7a+7b electrons, {D} determinants sampled "
                               "with weight 0.35^rank + 5% uniform tail, random integrals "
                               "(h_pp in [-15,1], 16 eri factors), Davidson block k=8, tol 1e-8"
                               + ("" if insts is None else
                                  "; then a 64-instance bond-scan batch (norb 8-16, 3.45e6 determinants)"),
                   "ndet": D, "nnz": nnz, "block": k, "tol": cfg.tol,
                   "batch_instances": 0 if insts is None else len(insts)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_level": "L2-to-fabric requests (FETCH_SIZE + WRITE_SIZE, copy-calibrated); "
                                      "Infinity Cache hits and HBM are not separable by these counters",
                     "kernel": "k_sigma (FP64 block sigma, k=8)",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": t_launch * 1e3},
        "roofline_fp32": {"bound": "hbm", "achieved": alg32 / ms32 / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": alg32 / ms32 / 1e6 / HBM_PEAK_GBS, "kernel": "k_sigma (FP32 block sigma, k=8)",
                          "alg_bytes_per_launch": alg32, "avg_launch_ms": ms32,
                          "elements_per_s": (nnz + D) * k / (ms32 * 1e-3)},
        "sigma_kernel": {"elements_per_s": value, "rows_per_s": D * k / t_launch,
                         "launches": n_sig,
                         "fabric_traffic_gbs": None if traffic is None else traffic / t_launch / 1e9,
                         "device_copy_gbs": copy_peak_gbs()},
        "step": {"elements_per_s": step_value, "elements": elements,
                 "what": "H.X elements of every block product of the step (both solves and the batch) "
                         "over the step's wall time"},
        "solve_ms": {"fp64": med([r[0]["fp64"] for r in res]) * 1e3,
                     "mixed": med([r[0]["mixed"] for r in res]) * 1e3,
                     "mixed_over_fp64": med([r[0]["mixed"] for r in res]) / med([r[0]["fp64"] for r in res])},
        "build_ms": med([r[0]["build"] for r in res]) * 1e3,
        "rdm_ms": med([r[0]["rdm"] for r in res]) * 1e3,
        "energy": {"fp64": res[-1][1][0], "mixed": res[-1][2][0],
                   "abs_diff": abs(res[-1][1][0] - res[-1][2][0])},
        "iterations": {"fp64": res[-1][1][1]["iterations"], "mixed": res[-1][2][1]["iterations"],
                       "mixed_fp32": res[-1][2][1]["iterations_fp32"]},
        "build_breakdown_ms": {"sort_tables": info["ms_sort"], "couplings": info["ms_connect"],
                               "elements": info["ms_elements"]},
    }
    if insts is not None:
        be, binfo = res[-1][3]
        bst = binfo["stats"]
        # the same batch with the untuned launch shape (2048-row chunks, 1024 Rayleigh-Ritz threads)
        os.environ["HINQS_BATCH_CHUNK"], os.environ["HINQS_BATCH_RR_THREADS"] = "2048", "1024"
        try:
            _, _, dinfo = bsolver.batch_lowest_eigenpair(tol=cfg.tol, block=cfg.k, autotune=True)
        finally:
            del os.environ["HINQS_BATCH_CHUNK"], os.environ["HINQS_BATCH_RR_THREADS"]
        dst = dinfo["stats"]
        sb, ss, se = sequential_batch(hq, insts, cfg.k, cfg.tol)
        ms_solve = med([r[0]["batch_solve"] for r in res]) * 1e3
        out["batch"] = {
            "workload": f"bond-scan batch: 64 instances, norb 8-16, N = norb -+ 2, 1e3-3e5 determinants "
                        f"({bst['ndet']} in all), FP64 Davidson k={cfg.k} to {cfg.tol}",
            "instances": bst["instances"], "ndet": bst["ndet"], "nnz": bst["nnz"],
            "ms_build": med([r[0]["batch_build"] for r in res]) * 1e3, "ms_solve": ms_solve,
            "iterations": bst["iterations"], "graphs": bst["graphs"],
            "ms_per_iteration": bst["ms_iterations"] / max(1, bst["iterations"]),
            "sigma_shape": [bst["sigma_team"], bst["sigma_unroll"], bst["sigma_occupancy"]],
            "tuned_shape": {"chunk_rows": bst["chunk_rows"], "rr_threads": bst["rr_threads"]},
            "default_shape_ms_per_iteration": dst["ms_iterations"] / max(1, dst["iterations"]),
            "default_shape_iterations": dst["iterations"],
            "sequential_ms_build": sb * 1e3, "sequential_ms_solve": ss * 1e3,
            "solve_speedup_vs_sequential": ss * 1e3 / ms_solve,
            "max_abs_dE_vs_sequential": float(np.max(np.abs(np.asarray(se) - be))),
        }
    # the selection steps after the solve, on the last FP64 eigenpair (outside the timed region)
    e_sel = res[-1][1][0]
    sel, (ya, yb) = selection_pass(hq, solver, last["c64"], e_sel, args.ntop, args.keep)
    out["select"] = dict(sel, workload=f"expansion of the {args.ntop} largest |c| of the FP64 eigenvector "
                                       f"of the {D}-determinant set, PT2 of every expanded determinant, "
                                       f"top {args.keep} by score")
    _, _, score = solver.pt2(last["c64"], e_sel, ya, yb)
    out["iteration"] = dict(outer_iteration(hq, solver, (ints.h, ints.eri, ints.e_core), last["c64"], e_sel,
                                            ya, yb, score, args.keep,
                                            D + args.keep // 2, cfg.k, cfg.tol),
                            workload=f"append the {args.keep} best-scored expanded determinants, cap at "
                                     f"{D + args.keep // 2} (the lowest PT2 scores of the set and the "
                                     f"appended ones go), FP64 Davidson to {cfg.tol} from the carried vector; "
                                     f"cold FP64 solve of the original set: {res[-1][1][1]['iterations']} iterations")
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.Oracle.from_inputs(ints, alpha, beta, cfg.na, cfg.nb)
        out["cpu_baseline"] = cpu_baseline(o, alpha, cfg, args.cpu_seconds)
        out["select"]["cpu_pt2"] = cpu_pt2_rate(o, last["c64"].cpu().numpy(), e_sel,
                                                ya.cpu().numpy().view(np.uint64),
                                                yb.cpu().numpy().view(np.uint64))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
