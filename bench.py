"""Benchmark: QMC integration of the two-loop massless planar double box.

Workload: all sectors of the planar double box (7 propagators, 6 integration
variables), Euclidean point s = -3, t = -1, eps-expansion to eps^0, a rank-1
Korobov lattice of prime size n (default 1000003) with 16 random shifts,
FP64.  One step is one pass of the whole path: every sector at every shift
and lattice point (integrand kernels, fixed-order reduction, copy of the
per-shift sums and the Laurent assembly), with the inputs already resident
on the device.  The JSON line reports integrand evaluations per second, the
roofline position of the integrand kernels, time to 1e-3 relative error
under lattice doubling and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("integrand evals/s (FP64 vs FP32) + time to 1e-3 rel err; "
          "serve p50/p99 ms")
PEAK_FP64_VALU = 78.6e12     # 256 CU x 4 SIMD x 16 lanes x 2 (fma) x 2.4 GHz
# growing prime lattices for the time to 1e-3 (CBC vectors exist up to 10^7)
DOUBLING_PRIMES = [4099, 10007, 65521, 131071, 262139, 524287, 1048573, 2097143,
                   4194301, 8388593]


# Section IV workloads with the integration times the paper reports on one
# Tesla K20 (context only): the Table 1 columns of the off-shell double box
# (Euclidean, s = t = -2/3) and the gg -> HH double boxes of Tables 2-3.
# (label, problem, kinematics, lambda, paper seconds)
PAPER_WORKLOADS = [
    ("I_B legs 1,4", "doublebox_off14", {"s": -2 / 3, "t": -2 / 3, "p1sq": -1.0, "p4sq": -1.0},
     0.0, 2.2),
    ("I_B legs 2,4", "doublebox_off24", {"s": -2 / 3, "t": -2 / 3, "p2sq": -1.0, "p4sq": -1.0},
     0.0, 0.84),
    ("I_B legs 3,4", "doublebox_off34", {"s": -2 / 3, "t": -2 / 3, "p3sq": -1.0, "p4sq": -1.0},
     0.0, 2.2),
    ("I_C", "hh_planar", None, 1.0, 19.0),
    ("I_D", "hh_nonplanar", None, 0.5, 20.0),
]


def max_rel_err(r):
    """Largest err/|mean| over the orders of point 0 (absolute against the
    largest order where an order is below 1e-3 of it)."""
    import numpy as np

    mean = r["mean"][0]
    err = np.hypot(r["err_re"][0], r["err_im"][0])
    scale = np.abs(mean)
    rel = np.where(scale > 1e-3 * scale.max(), err / np.maximum(scale, 1e-300),
                   err / scale.max())
    return float(rel.max())


def paper_workloads(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log, m=16):
    """Time to 1e-3 on every order for the paper's Section IV integrals,
    geometric sectors, growing prime lattices, m shifts (host planning
    reported apart, not timed)."""
    import torch
    from seeded_inputs.problems import HH_POINT

    out = {}
    for label, name, kin_vals, lam, paper_s in PAPER_WORKLOADS:
        tp = time.perf_counter()
        secs, info = fe.decompose(PROBLEMS[name], "geometric")
        plan = ctx.plan(fe.sector_arrays(secs, info), info, 0, fe.prefactor_series(info, 12),
                        lam=lam)
        plan_s = time.perf_counter() - tp
        kin = fe.kin_vector(info, HH_POINT if kin_vals is None else kin_vals)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = {"seconds": None, "sectors": len(secs), "host_planning_seconds": plan_s,
               "paper_seconds_k20": paper_s}
        for nn in DOUBLING_PRIMES:
            r = plan.integrate(kin, (nn, lattice(nn)), shift_table(0, m, 8))
            rel = max_rel_err(r)
            log(f"paper workload {label}: n={nn} max rel err {rel:.2e}")
            if rel <= 1e-3:
                res.update({"seconds": time.perf_counter() - t1, "n": nn, "max_rel_err": rel,
                            "violations": int(r["violations"])})
                break
        plan.close()
        out[label] = res
    return out


def kernel_source_hash():
    """SHA-256 over the library's device and host sources (csrc/), so a
    counter figure can be matched to the kernel build it was taken on."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_1508_02512_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(poles, width, n, m, ppl, variant):
    """HBM bytes (read + written) per launch of one integrand kernel class of
    this workload in one launch shape (points per lane, occupancy build),
    from the rocprofv3 FETCH_SIZE and WRITE_SIZE passes recorded in
    profiles/traffic.json (each calibrated with a 256 MiB device copy).  None
    when no pass was taken for that launch, or when the kernel sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, "no counter record"
    if rec.get("source_hash") != kernel_source_hash():
        return None, "counters predate the current kernel sources"
    for e in rec.get("entries", []):
        if (e["poles"], e["width"], e["n"], e["m"], e.get("points_per_lane"),
                e.get("variant")) == (poles, width, n, m, ppl, variant):
            return e["read_bytes"] + e["write_bytes"], "rocprofv3 FETCH_SIZE + WRITE_SIZE"
    return None, "launch shape not in the counter record"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1000003)
    ap.add_argument("--shifts", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-target", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-pole-methods", action="store_true",
                    help="skip the double box with its poles integrated by parts")
    ap.add_argument("--pole-methods-n", type=int, default=131071,
                    help="lattice size of the FP32/FP64 comparison of both pole methods")
    ap.add_argument("--pole-methods-ttt", action="store_true",
                    help="also time the poles-by-parts plan to 1e-3 (about a minute)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="bind the main workload with the library's default launch shapes")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the non-planar vertex, the 512-point batch and the s-scan")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (calibrates HBM counters)")
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="arrival rate of the saturating serving leg")
    ap.add_argument("--serve-burst", type=int, default=400,
                    help="requests of the saturating leg")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the steady-state batched FP32 leg")
    ap.add_argument("--serve-requests-fp64", type=int, default=300)
    ap.add_argument("--serve-requests-plain", type=int, default=150)
    ap.add_argument("--serve-sectors", choices=("iterated", "geometric"), default="geometric")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    return ap.parse_args()


def cpu_threads():
    """Host threads the oracle may use: this process's CPU share, at most 16
    (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(target_seconds):
    """The oracle on a bounded, stratified sample of the benchmark workload:
    every 147th of the 882 sectors (6 sectors of several pole counts), 16
    shifts, n = 100003.  Each sector call splits into 16 shifts x 2 chunks
    of 2^16 indices = 32 jobs, so every thread has work.  The same sectors
    at n = 10007 on one thread give the single-thread rate (the cost of one
    evaluation does not depend on n), so the ratio of the two is the
    parallel efficiency of the threads reported."""
    from oracle import qmc as oq
    from oracle.decompose import decompose as odec
    from seeded_inputs.lattice import lattice
    from seeded_inputs.problems import PROBLEMS
    from seeded_inputs.rng import shift_table

    secs, info = odec(PROBLEMS["doublebox"])
    kin = {"s": -3.0, "t": -1.0}
    nums = [oq.NumericSector(s, info, kin) for s in secs]
    m = 16
    sh = shift_table(0, m, 8)
    threads = cpu_threads()

    def run(sample, n, nthreads, budget):
        z = lattice(n)
        evals, done, t0 = 0, 0, time.perf_counter()
        for ns in sample:
            oq.sector_sums(ns, n, z, sh, 2, 0.0, -4, 5, nthreads=nthreads)
            evals += n * m
            done += 1
            if time.perf_counter() - t0 > budget:
                break
        return evals / (time.perf_counter() - t0), done

    sample = nums[::147]
    rate, done = run(sample, 100003, threads, target_seconds)
    rate1, done1 = run(sample[:done], 10007, 1, target_seconds)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": rate, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "single_thread_value": rate1,
            "parallel_efficiency": rate / (threads * rate1),
            "single_thread_sample": f"the same {done1} sectors, n=10007, m={m}, 1 thread",
            "cpu_model": model,
            "sample": f"planar double box s=-3 t=-1, {done} sectors (every 147th of "
                      f"{len(nums)}), n=100003, m={m} shifts, FP64 oracle, {threads} threads"}


# masses of Section IV (GeV^2) for the physical two-loop planar box I_C
MT2, MH2 = 172.0 ** 2, 125.0 ** 2


def serve_kinematics(rng, kind):
    """Seeded physical kinematics of one serving request."""
    if kind == 2:
        return "np_vertex", {"s": float(rng.uniform(4.2, 8.0)), "msq": 1.0}
    if kind == 0:
        sv = float(rng.uniform(1.0, 10.0))
        return "box", {"s": sv, "t": float(rng.uniform(-sv + 0.1, -0.1))}
    # gg -> HH above the top-pair threshold: s in [1.3e5, 2.5e5] GeV^2,
    # scattering angle cos(theta) in [-0.8, 0.8]
    sv = float(rng.uniform(1.3e5, 2.5e5))
    beta = (1.0 - 4.0 * MH2 / sv) ** 0.5
    t = MH2 - 0.5 * sv * (1.0 - beta * float(rng.uniform(-0.8, 0.8)))
    return "hh_planar", {"s": sv, "t": t, "mtsq": MT2, "mhsq": MH2}


def serve_bench(qmc, fe, PROBLEMS, lattice, n_req, rate, fp32, slots, log,
                strategy="geometric", seed=0):
    """Poisson request stream (seeded) mixing the one-loop box, the planar
    two-loop box of Section IV.C (I_C) and the non-planar vertex, all at
    physical kinematics, target 1e-3 relative; embedded lattices
    n = 2^14 .. 2^22 doubling, 8 shifts, up to 4 deformation back-offs;
    sectors from the given decomposition strategy.  n_req requests arrive
    at `rate` per second; latency is submit to completion."""
    import numpy as np

    rng = np.random.default_rng(seed)
    prec = qmc.QMC_FP32_EVAL if fp32 else qmc.QMC_FP64
    ctx = qmc.Context(0, max_slots=slots)
    plans = {}
    for name, lam in (("box", 0.5), ("hh_planar", 1.0), ("np_vertex", 0.5)):
        secs, info = fe.decompose(PROBLEMS[name], strategy)
        plans[name] = (ctx.plan(fe.sector_arrays(secs, info), info, 0,
                                fe.prefactor_series(info, 12), lam=lam, precision=prec), info)
    from seeded_inputs.lattice import embedded_lattice
    z = embedded_lattice()
    gaps = rng.exponential(1.0 / rate, size=n_req)
    kinds = rng.integers(0, 3, size=n_req)
    reqs = []
    t0 = time.perf_counter()
    t_next = t0
    for i in range(n_req):
        t_next += gaps[i]
        while time.perf_counter() < t_next:
            time.sleep(min(1e-3, max(0.0, t_next - time.perf_counter())))
        name, vals = serve_kinematics(rng, int(kinds[i]))
        plan, info = plans[name]
        reqs.append((name, qmc.submit(plan, fe.kin_vector(info, vals), 1e-3, 1 << 14, 1 << 22,
                                      8, 1000 + i, z, lambda_halvings=4)))
    t_arrived = time.perf_counter() - t0
    lat, evals, status = [], 0, {}
    per = {}
    for name, r in reqs:
        out = r.wait(900)
        if out is None:
            status["timeout"] = status.get("timeout", 0) + 1
            continue
        lat.append(out["latency_ms"])
        evals += out["evals"]
        status[out["rc"]] = status.get(out["rc"], 0) + 1
        d = per.setdefault(name, {"n": 0, "ok": 0, "latency_ms": [], "n_final": [], "halv": 0})
        d["n"] += 1
        d["ok"] += out["rc"] == 0
        d["halv"] += out["lambda_halvings"]
        d["latency_ms"].append(out["latency_ms"])
        d["n_final"].append(out["n_final"])
        r.release()
    wall = time.perf_counter() - t0
    for plan, _ in plans.values():
        plan.close()
    ctx.close()
    lat = np.array(lat)
    res = {"requests": n_req, "rate_req_s": rate, "slots": slots,
           "precision": "fp32-eval" if fp32 else "fp64",
           "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
           "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
           "completed_req_s": len(lat) / wall, "evals_per_s": evals / wall,
           "arrival_s": t_arrived, "wall_s": wall,
           "status_counts": {str(k): v for k, v in status.items()},
           "per_problem": {k: {"requests": v["n"], "converged": v["ok"],
                               "p50_ms": float(np.percentile(v["latency_ms"], 50)),
                               "p99_ms": float(np.percentile(v["latency_ms"], 99)),
                               "median_n_final": int(np.median(v["n_final"])),
                               "lambda_halvings": v["halv"]}
                           for k, v in per.items()}}
    log(f"serve ({res['precision']}, slots {slots}, {n_req} at {rate:.1f}/s): p50 "
        f"{res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms, "
        f"{res['completed_req_s']:.1f} req/s")
    return res


def serve_suite(qmc, fe, PROBLEMS, lattice, args, log):
    """The serving comparison: the batched mixed-precision form (64 slots,
    FP32-eval) against the plain FP64 form (one slot), plus batched FP64 (64
    slots) to separate batching from precision.  The batched FP32 form runs
    once at 200 req/s (saturating: its completion rate is the sustainable
    rate) and then with >= 1000 requests at 70% of that rate (steady state);
    the two FP64 forms run at the same 70% rate, fewer requests."""
    out = {"sectors": args.serve_sectors,
           "mix": "one-loop box, planar two-loop box of Section IV.C (I_C, top-quark loop), "
                  "non-planar two-loop vertex; physical kinematics; target 1e-3"}
    # the massless planar double box at physical kinematics: plan refused
    ctx = qmc.Context(0)
    secs, info = fe.decompose(PROBLEMS["doublebox"], args.serve_sectors)
    try:
        ctx.plan(fe.sector_arrays(secs, info), info, 0, fe.prefactor_series(info, 12),
                 lam=0.25).close()
        out["massless_planar_double_box"] = "planned"
    except qmc.QMCError as e:
        out["massless_planar_double_box"] = {
            "planned": False, "error": str(e),
            "reason": "deformed sectors with 3-4 poles are refused (corner differences "
                      "below FP64 accuracy); the mix serves the paper's planar two-loop "
                      "box I_C instead"}
    ctx.close()
    burst = serve_bench(qmc, fe, PROBLEMS, lattice, args.serve_burst, args.serve_rate, True, 64,
                        log, args.serve_sectors, seed=1)
    sustained = max(burst["completed_req_s"], 1.0)
    steady_rate = 0.7 * sustained
    out["batched_fp32_at_200_req_s"] = burst
    out["sustainable_req_s"] = sustained
    out["batched_fp32"] = serve_bench(qmc, fe, PROBLEMS, lattice, args.serve_requests,
                                      steady_rate, True, 64, log, args.serve_sectors)
    out["batched_fp64"] = serve_bench(qmc, fe, PROBLEMS, lattice, args.serve_requests_fp64,
                                      steady_rate, False, 64, log, args.serve_sectors)
    out["plain_fp64"] = serve_bench(qmc, fe, PROBLEMS, lattice, args.serve_requests_plain,
                                    steady_rate, False, 1, log, args.serve_sectors)
    return out


def launch_roofline(job, peak=PEAK_FP64_VALU):
    """One eager, profiled run of a bound job: the dominant kernel-class
    launch (the longest), its algorithmic flops over its HIP-event time,
    against the vector peak."""
    job.profile(True)
    job.run()
    r = job.fetch()
    st = job.class_stats()
    dom = max(st, key=lambda c: c["ms"])
    achieved = dom["algo_flops"] / (dom["ms"] / 1e3)
    job.profile(False)
    kind = (f"qmc_eval_real<poles={dom['poles']}>" if dom["width"] == 0 else
            f"qmc_eval_cplx<width={dom['width']}, poles={dom['poles']}>")
    return {"bound": "alu", "kernel": kind, "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak, "launch_ms": dom["ms"],
            "points_per_lane": dom["points_per_lane"], "grid": dom["grid"],
            "occupancy_variant": dom["variant"],
            "step_kernel_ms": r["kernel_ms"],
            "step_frac": r["algo_flops"] / (r["kernel_ms"] / 1e3) / peak}, r


def sizing_primes(lo, hi):
    from seeded_inputs.lattice import PRIME_SIZES
    return [p for p in PRIME_SIZES if lo <= p <= hi]


def vertex_bench(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log, n_avg=10000019):
    """Non-planar two-loop vertex with a massive loop, s = 4.5 (physical),
    lambda = 0.5, 32 shifts, per-sector lattice sizes from the library's
    variance-weighted sizing (pilot at n = 65521) for an average of
    n_avg points per sector."""
    import torch

    secs, info = fe.decompose(PROBLEMS["np_vertex"])
    plan = ctx.plan(fe.sector_arrays(secs, info), info, 0, fe.prefactor_series(info, 12),
                    lam=0.5)
    kin = fe.kin_vector(info, {"s": 4.5, "msq": 1.0})
    sh = shift_table(0, 32, 8)
    sizes = qmc.size_lattices(plan, kin, n_avg * plan.n_sectors, sizing_primes(10007, 10 ** 8),
                              65521, lattice(65521), shift_table(1, 8, 8))
    lats = [(n, lattice(n)) for n in sizes]
    job = plan.bind(kin, None, sh, lat_per_sector=lats)
    roof, _ = launch_roofline(job)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job.run()
    r = job.fetch()
    wall = time.perf_counter() - t0
    job.close()
    plan.close()
    out = {"workload": "non-planar two-loop vertex, massive loop, s=4.5, lambda=0.5, "
                       "32 shifts, variance-weighted sector lattices",
           "value": r["evals"] / wall, "unit": "evals/s", "seconds": wall,
           "evals": r["evals"], "kernel_ms": r["kernel_ms"],
           "achieved_tflops": r["algo_flops"] / r["kernel_ms"] / 1e9,
           "eps0": [float(r["mean"][0, -1].real), float(r["mean"][0, -1].imag)],
           "err": [float(r["err_re"][0, -1]), float(r["err_im"][0, -1])],
           "violations": int(r["violations"]), "n_min": min(sizes), "n_max": max(sizes),
           "n_mean": sum(sizes) / len(sizes), "roofline": roof}
    log(f"np_vertex: {out['value']:.3e} evals/s, dominant launch {roof['frac']:.3f} of peak")
    return out


def hh_box_scan(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log):
    """Section IV.A workload: the one-loop gg -> HH box at 1000 points
    s = 70000 .. 500000 GeV^2 (t = -6000, M_t = 172, M_H = 125) in one
    batched bind, n = 262139, 8 shifts, lambda = 0.5."""
    import numpy as np
    import torch

    secs, info = fe.decompose(PROBLEMS["hh_box"])
    plan = ctx.plan(fe.sector_arrays(secs, info), info, 0, fe.prefactor_series(info, 12),
                    lam=0.5)
    svals = np.linspace(70000.0, 500000.0, 1000)
    kin = np.stack([fe.kin_vector(info, {"s": float(v), "t": -6000.0, "mtsq": MT2,
                                         "mhsq": MH2}) for v in svals])
    n = 262139
    job = plan.bind(kin, (n, lattice(n)), shift_table(0, 8, 8))
    job.run()
    job.fetch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job.run()
    r = job.fetch()
    wall = time.perf_counter() - t0
    job.close()
    plan.close()
    mean = r["mean"][:, 0]
    rel = np.hypot(r["err_re"][:, 0], r["err_im"][:, 0]) / np.abs(mean)
    out = {"points": len(svals), "seconds": wall, "ms_per_point": wall / len(svals) * 1e3,
           "evals_per_s": r["evals"] / wall, "max_rel_err": float(rel.max()),
           "points_rel_err_below_1e-4": int((rel < 1e-4).sum()),
           "violations": int(r["violations"])}
    log(f"hh_box scan: {out['ms_per_point']:.2f} ms/point, max rel err {out['max_rel_err']:.1e}, "
        f"{out['points_rel_err_below_1e-4']} points below 1e-4")
    return out


def batch_bench(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log, fp32):
    """512 kinematic points of the all-massive two-loop planar vertex,
    s uniform in [-10, 10] without |s - 4| < 0.05 (numpy PCG64 seed 0),
    geometric sectors, 4 shifts, every sector with its own lattice size in
    [1e5, 1e7] from the library's variance-weighted sizing at s = 6 (average
    1e6 points per sector); launch shapes (points per lane, persistent grid,
    occupancy build) from the autotuner; the whole launch sequence captured
    in one HIP graph and replayed."""
    import numpy as np
    import torch

    rng = np.random.default_rng(0)
    svals = []
    while len(svals) < 512:
        v = float(rng.uniform(-10.0, 10.0))
        if abs(v - 4.0) >= 0.05:
            svals.append(v)
    secs, info = fe.decompose(PROBLEMS["triangle2l"], "geometric")
    prec = qmc.QMC_FP32_EVAL if fp32 else qmc.QMC_FP64
    plan = ctx.plan(fe.sector_arrays(secs, info), info, 0, fe.prefactor_series(info, 12),
                    lam=0.25, precision=prec)
    kin = np.stack([fe.kin_vector(info, {"s": v, "msq": 1.0}) for v in svals])
    sizes = qmc.size_lattices(plan, fe.kin_vector(info, {"s": 6.0, "msq": 1.0}),
                              10 ** 6 * plan.n_sectors, sizing_primes(10 ** 5, 10 ** 7), 65521,
                              lattice(65521), shift_table(1, 8, 8))
    lats = [(n, lattice(n)) for n in sizes]
    sh = shift_table(0, 4, 8)
    choices = plan.autotune(kin[:8], None, shift_table(0, 2, 8), lat_per_sector=lats)
    job = plan.bind(kin, None, sh, lat_per_sector=lats)
    roof, _ = launch_roofline(job)
    job.use_graph(True)
    job.run()
    job.fetch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job.run()
    r = job.fetch()
    wall = time.perf_counter() - t0
    job.close()
    plan.close()
    out = {"workload": "two-loop massive planar vertex, 512 points s in [-10, 10], 22 "
                       "geometric sectors, uneven lattices, 4 shifts, one graph replay",
           "value": r["evals"] / wall, "unit": "evals/s", "seconds": wall, "evals": r["evals"],
           "precision": "fp32-eval" if fp32 else "fp64", "points": len(svals),
           "n_min": min(sizes), "n_max": max(sizes), "autotune": choices,
           "violations": int(r["violations"]), "roofline": roof}
    log(f"batch ({out['precision']}): {out['value']:.3e} evals/s in {wall:.2f} s, "
        f"dominant launch {roof['frac']:.3f} of peak")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the integration of one problem is "
              "not sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1508_02512_amd import frontend as fe
    from paper_1508_02512_amd import qmc
    from seeded_inputs.lattice import lattice
    from seeded_inputs.problems import PROBLEMS
    from seeded_inputs.rng import shift_table

    assert torch.cuda.is_available(), "needs a GPU"
    stream = torch.cuda.current_stream().cuda_stream
    if args.copy_probe:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    kin_vals = {"s": -3.0, "t": -1.0}
    secs, info = fe.decompose(PROBLEMS["doublebox"])
    arrs = fe.sector_arrays(secs, info)
    ctx = qmc.Context(0, stream=stream)
    plan = ctx.plan(arrs, info, 0, fe.prefactor_series(info, 12))
    kin = fe.kin_vector(info, kin_vals)
    n, m = args.n, args.shifts
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    tuned = None
    if not args.no_autotune:
        # launch shape per kernel class (points per lane, persistent grid,
        # occupancy build) timed on the same lattice with 4 shifts
        t_tune = time.perf_counter()
        tuned = plan.autotune(kin, (n, lattice(n)), shift_table(0, 4, 8))
        log(f"autotune ({time.perf_counter() - t_tune:.1f} s): {tuned}")
    job = plan.bind(kin, (n, lattice(n)), shift_table(0, m, 8))
    job.profile(True)          # HIP events around every kernel-class launch

    log(f"bench: {plan.n_sectors} sectors, n={n}, m={m}, warmup {args.warmup}")
    for _ in range(args.warmup):
        job.run()
        job.fetch()
    torch.cuda.synchronize()
    kernel_ms, step_stats = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        job.run()
        res = job.fetch()
        kernel_ms.append(res["kernel_ms"])
        step_stats.append(job.class_stats())
        log(f"step {len(kernel_ms)}: kernels {res['kernel_ms']:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evals_per_step = res["evals"]
    value = evals_per_step * args.steps / wall
    avg_kernel_s = float(np.mean(kernel_ms)) / 1e3
    achieved_step = res["algo_flops"] / avg_kernel_s
    # dominant kernel: the class launch with the largest share of the step,
    # its time averaged over the timed steps
    stats = step_stats
    dom = max(range(len(stats[0])), key=lambda i: stats[0][i]["ms"])
    dom_ms = float(np.mean([st[dom]["ms"] for st in stats]))
    dom_stat = stats[0][dom]
    achieved = dom_stat["algo_flops"] / (dom_ms / 1e3)

    def time_to_target(pl, label, kind="korobov"):
        """Wall time of the growing prime lattices until every order has
        err/|mean| <= 1e-3 (absolute against the largest order where an
        order is below 1e-3 of it); kind picks the stored generating
        vectors (Korobov or CBC)."""
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for nn in DOUBLING_PRIMES:
            r = pl.integrate(kin, (nn, lattice(nn, kind)), shift_table(0, m, 8))
            rel = max_rel_err(r)
            log(f"time-to-target ({label}): n={nn} max rel err {rel:.2e}")
            if rel <= 1e-3:
                return {"seconds": time.perf_counter() - t1, "n": nn, "max_rel_err": rel}, r
        return None, r

    ttt = ttt_cbc = ttt_geo = None
    if not args.no_time_to_target:
        ttt, r64 = time_to_target(plan, "fp64")
        ttt_cbc, _ = time_to_target(plan, "fp64, CBC vectors", "cbc")
        # the same integral over the geometric sectors (planning not timed)
        tp = time.perf_counter()
        gsecs, ginfo = fe.decompose(PROBLEMS["doublebox"], "geometric")
        plang = ctx.plan(fe.sector_arrays(gsecs, ginfo), ginfo, 0,
                         fe.prefactor_series(ginfo, 12))
        plan_s = time.perf_counter() - tp
        ttt_geo, _ = time_to_target(plang, "fp64, geometric sectors")
        if ttt_geo is not None:
            ttt_geo.update({"sectors": len(gsecs), "host_planning_seconds": plan_s})
            # full-size steps over the geometric sectors (same n, m)
            jg = plang.bind(kin, (n, lattice(n)), shift_table(0, m, 8))
            jg.run()
            jg.fetch()
            torch.cuda.synchronize()
            tg = time.perf_counter()
            for _ in range(args.steps):
                jg.run()
                rg = jg.fetch()
            torch.cuda.synchronize()
            wg = (time.perf_counter() - tg) / args.steps
            ttt_geo["full_step"] = {"evals_per_s": rg["evals"] / wg, "ms_per_step": wg * 1e3,
                                    "evals_per_step": rg["evals"]}
            jg.close()
        plang.close()

    # FP32-evaluation mode on the same workload
    fp32 = None
    if not args.no_fp32:
        plan32 = ctx.plan(arrs, info, 0, fe.prefactor_series(info, 12),
                          precision=qmc.QMC_FP32_EVAL)
        tuned32 = None
        if not args.no_autotune:
            tuned32 = plan32.autotune(kin, (n, lattice(n)), shift_table(0, 4, 8))
        job32 = plan32.bind(kin, (n, lattice(n)), shift_table(0, m, 8))
        job32.run()
        job32.fetch()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        k32 = []
        for _ in range(args.steps):
            job32.run()
            res32 = job32.fetch()
            k32.append(res32["kernel_ms"])
        torch.cuda.synchronize()
        wall32 = time.perf_counter() - t2
        dev = np.abs(res32["mean"][0] - res["mean"][0]) / np.maximum(
            np.hypot(res["err_re"][0], res["err_im"][0]), 1e-300)
        rel = np.abs(res32["mean"][0] - res["mean"][0]) / np.maximum(
            np.abs(res["mean"][0]), 1e-300)
        fp32 = {"value": res32["evals"] * args.steps / wall32, "unit": "evals/s",
                "ms_per_step": wall32 / args.steps * 1e3,
                "kernel_ms_per_step": float(np.mean(k32)),
                "achieved_tflops": res32["algo_flops"] / (float(np.mean(k32)) / 1e3) / 1e12,
                "autotune": tuned32,
                "max_dev_vs_fp64_in_sigma": float(dev.max()),
                "rel_dev_vs_fp64_per_order": [float(x) for x in rel]}
        if not args.no_time_to_target:
            fp32["time_to_1e-3"], _ = time_to_target(plan32, "fp32")
        job32.close()
        plan32.close()
        log(f"fp32: {fp32['value']:.3e} evals/s")

    # the poles integrated by parts (Eq. 13) instead of subtracted (Eq. 11):
    # rates, errors and the FP32-evaluation deviation from FP64 of both pole
    # methods on one lattice (the by-parts time to 1e-3 on request)
    poles_ibp = None
    if not args.no_pole_methods:
        tp = time.perf_counter()
        pl_i = ctx.plan(arrs, info, 0, fe.prefactor_series(info, 12),
                        pole_method=qmc.QMC_POLES_IBP)
        poles_ibp = {"sectors": pl_i.n_sectors, "host_planning_seconds":
                     time.perf_counter() - tp,
                     "flops_per_point": pl_i.info.flops_per_point,
                     "flops_per_point_subtraction": plan.info.flops_per_point}
        if not args.no_autotune:
            pl_i.autotune(kin, (131071, lattice(131071)), shift_table(0, 4, 8))
        if args.pole_methods_ttt:
            poles_ibp["time_to_1e-3"], _ = time_to_target(pl_i, "fp64, poles by parts")
        nb = args.pole_methods_n
        dev = {}
        for label, pm in (("subtraction", qmc.QMC_POLES_SUBTRACT),
                          ("by_parts", qmc.QMC_POLES_IBP)):
            r = {}
            for prec in (qmc.QMC_FP64, qmc.QMC_FP32_EVAL):
                pq = pl_i if (pm, prec) == (qmc.QMC_POLES_IBP, qmc.QMC_FP64) else ctx.plan(
                    arrs, info, 0, fe.prefactor_series(info, 12), precision=prec,
                    pole_method=pm)
                r[prec] = pq.integrate(kin, (nb, lattice(nb)), shift_table(0, m, 8))
                if pq is not pl_i:
                    pq.close()
            a, b = r[qmc.QMC_FP64], r[qmc.QMC_FP32_EVAL]
            sig = np.hypot(a["err_re"][0], a["err_im"][0])
            dev[label] = {"evals_per_s_fp64": a["evals"] / (a["kernel_ms"] / 1e3),
                          "evals_per_s_fp32": b["evals"] / (b["kernel_ms"] / 1e3),
                          "max_rel_err_fp64": max_rel_err(a),
                          "fp32_rel_dev_per_order":
                              [float(x) for x in np.abs(b["mean"][0] - a["mean"][0])
                               / np.abs(a["mean"][0])],
                          "fp32_dev_in_sigma_per_order":
                              [float(x) for x in np.abs(b["mean"][0] - a["mean"][0]) / sig]}
        poles_ibp["fp32_vs_fp64_at_n"] = nb
        poles_ibp["methods"] = dev
        pl_i.close()
        log(f"poles by parts: {poles_ibp}")

    workloads = None
    if not args.no_workloads:
        workloads = {
            "np_vertex": vertex_bench(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log),
            "batch_fp64": batch_bench(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log, False),
            "batch_fp32": batch_bench(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log, True),
            "hh_box_scan": hh_box_scan(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log)}

    paper = None
    if not args.no_time_to_target:
        paper = paper_workloads(qmc, fe, PROBLEMS, lattice, shift_table, ctx, log)

    serve = None
    if not args.no_serve:
        serve = serve_suite(qmc, fe, PROBLEMS, lattice, args, log)

    traffic, traffic_src = measured_traffic(dom_stat["poles"], dom_stat["width"], n, m,
                                            dom_stat["points_per_lane"], dom_stat["variant"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "planar double box (7 props, 6 dims), Euclidean "
                               "s=-3 t=-1, all sectors, eps^-4..eps^0, Korobov r=2",
                   "sectors": plan.n_sectors, "lattice_n": n, "shifts": m,
                   "evals_per_step": evals_per_step, "precision": "fp64"},
        "launch_shapes": tuned,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                     "traffic": traffic, "traffic_source": traffic_src,
                     "kernel": f"qmc_eval_real<poles={dom_stat['poles']}, double>"
                               if dom_stat["width"] == 0 else
                               f"qmc_eval_cplx<width={dom_stat['width']}, "
                               f"poles={dom_stat['poles']}>",
                     "launch_ms": dom_ms, "algo_flops_per_launch": dom_stat["algo_flops"],
                     "evals_per_launch": dom_stat["evals"],
                     "grid": dom_stat["grid"], "points_per_lane": dom_stat["points_per_lane"],
                     "occupancy_variant": dom_stat["variant"],
                     "step": {"kernel_ms": avg_kernel_s * 1e3,
                              "algo_flops": res["algo_flops"],
                              "achieved": achieved_step / 1e12,
                              "frac": achieved_step / PEAK_FP64_VALU,
                              "launches": [{"poles": c["poles"], "width": c["width"],
                                            "ms": c["ms"], "tflops": c["algo_flops"] /
                                            max(c["ms"], 1e-9) / 1e9}
                                           for c in stats[-1]]}},
        "time_to_1e-3": ttt,
        "time_to_1e-3_cbc_vectors": ttt_cbc,
        "time_to_1e-3_geometric_sectors": ttt_geo,
        "fp32_eval": fp32,
        "poles_by_parts": poles_ibp,
        "paper_workloads_time_to_1e-3": paper,
        "serve": serve,
        "workloads": workloads,
        "result_eps0": [float(res["mean"][0, -1].real), float(res["err_re"][0, -1])],
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    job.close()
    plan.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
