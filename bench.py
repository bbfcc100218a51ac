#!/usr/bin/env python3
"""Benchmark: batched Jacobian-vector products of the implicit-Coriolis IMEX step on one MI355X.

Workload (the metric's shell): L = M = 128, m0 = 10, N = 48, Ek = 1e-5, Pr = 1,
Ra = 1.2 * 6.5 Ek^(-1/3) = 362.0, dt = 200; a seeded synthetic base state (kinetic-energy
density ~25, coefficients decaying as l^-3, conductive temperature profile added) and 200
seeded unit Krylov-like vectors (decay l^-1).  One step = one sc_jvp call on a batch of
nvec vectors (the whole hot path: transforms, products, projections, implicit solve and,
where the precision asks for it, refinement).  Inputs are resident in HBM before the timed region.

Prints one JSON line.  `value` is mixed-precision jvp/s (FP32 transforms, one FP64 solve); the
FP64 path, and the mixed path with an FP32 solve plus FP64 refinement, are timed the same way
and reported beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

WORKLOADS = {
    # the shell the metric is quoted on
    "c3": dict(L=128, M=128, m0=10, N=48, Ek=1e-5, Pr=1.0, Ra=362.0, dt=200.0),
    # the throughput-stress shell (context only: no oracle baseline, no Newton run)
    "stress": dict(L=255, M=255, m0=12, N=64, Ek=3e-6, Pr=1.0, Ra=541.0, dt=200.0),
}
WORKLOAD = WORKLOADS["c3"]
RI_RO = (0.35 / 0.65, 1.0 / 0.65)   # inner and outer radius, gap 1
BASE_AMP = (8.0, 8.0, 0.1)   # e, f amplitudes give kinetic-energy density ~25 at this shell
PEAK = {"hbm": 8000.0, "fp32": 157.3, "fp64": 78.6}   # GB/s, TFLOP/s (MI355X published)


# single-kernel stages of the mixed path at this workload and the kernel each one launches
SINGLE_KERNEL_STAGES = {
    "ring": "sc::k_ring_reg<float, 0, 8, 5, 32>",      # N_phi = 40 = 8 x 5, 32 rings per workgroup
    "legendre_synth": "sc::k_synth<float>",
    "legendre_anal": "sc::k_anal<float, 5>",           # up to 5 column tiles per degree parity
    "radial_prep": "sc::k_radial_prep<float, 3>",
    "project_rhs": "sc::k_project_rhs<float, false, 3>",
}


def stage_kernels(tuning, N=48):
    """The kernel of each single-kernel stage under the autotuner's choices (FP32 transforms)."""
    k = dict(SINGLE_KERNEL_STAGES)
    rt = (N + 15) // 16
    k["radial_prep"] = f"sc::k_radial_prep<float, {rt}>"
    k["project_rhs"] = f"sc::k_project_rhs<float, false, {rt}>"
    if tuning is not None:
        if tuning["ring_fp32"] >= 0:
            k["ring"] = "sc::k_ring<float, 0>"
        else:   # register ring of shape -1 - v: 32, 24 or 16 rings per workgroup
            k["ring"] = f"sc::k_ring_reg<float, 0, 8, 5, {(32, 24, 16)[-1 - tuning['ring_fp32']]}>"
        if not tuning["anal_folded"]:
            k["legendre_anal"] = "sc::k_gemm_batched<float>"
    return k
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "hbm_traffic_L128_N48_nvec16.json")


def sources_sha256():
    """Hash of the kernel sources' code: comments and runs of white space are dropped first, so
    that an edited comment does not discard counters taken on the same code."""
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in ("paper_2508_16635_amd/csrc/kernels.h", "paper_2508_16635_amd/csrc/api.hip"):
        with open(os.path.join(here, f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)   # block comments
        src = re.sub(r"//[^\n]*", " ", src)                  # line comments
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by the plain-copy calibration), or None if the summary is missing or was
    taken on other sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != sources_sha256() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["bytes"]


def stage_work(lay, nvec, prec_bytes, factor_bytes, nblocks, refine, dp_only=True):
    """Algorithmic flops and bytes per launch of each stage: the work the method defines (each
    operand read once, each result written once), not what a kernel happens to move."""
    L, N, Np, nth, nphi, K1, S = (lay["L"], lay["N"], lay["Np"], lay["ntheta"], lay["nphi"],
                                  lay["K"] + 1, lay["S"])
    m0 = lay["m0"]
    nl = [L - k * m0 + 1 for k in range(K1)]
    w = {}
    # Legendre synthesis: per m, (6 Np nvec x nl) . (nl x nth) and (10 Np nvec x nl) . (nl x 2 nth),
    # counted with the equatorial split (even and odd degrees on half the nodes: half the flops);
    # it writes 6 scalar and 12 vector-field rows of nth per (vec, r_p, m)
    fl = sum(2.0 * Np * nvec * n * (6 * nth + 10 * 2 * nth) for n in nl) / 2
    by = prec_bytes * (Np * nvec * 16 * S + (K1 * Np * nvec * (6 * nth + 12 * nth)) + 3 * nth * S)
    w["legendre_synth"] = (fl, by)
    # Legendre analysis: (4 Np nvec x nth) . (nth x nl) and (4 Np nvec x 2 nth) . (2 nth x nl) per m,
    # counted with the mirror folding (each degree parity contracts over the northern half); the
    # vector inputs are read once (their m P/sin half is derived from the dP half)
    fl = sum(2.0 * Np * nvec * n * (4 * nth + 4 * 2 * nth) for n in nl) / 2
    by = prec_bytes * (K1 * Np * nvec * (4 * nth + (4 if dp_only else 8) * nth) + Np * nvec * 8 * S + 3 * nth * S // 2)
    w["legendre_anal"] = (fl, by)
    rings = Np * nth * nvec
    # ring: reads 18 rows (6 scalar sums, 12 vector fields) and writes 8 rows (4 scalar, 4 vector;
    # 12 when the batched-GEMM analysis needs both halves of the vector rows) per (ring,
    # harmonic), plus the 9 base fields per (r_p, node, point) in the linear mode
    w["ring"] = (rings * (2.0 * 13 * K1 * nphi * 2 + 60 * nphi),
                 prec_bytes * (rings * (18 + (8 if dp_only else 12)) * K1 + Np * nth * 9 * nphi))
    nreal = 6 * N * S
    w["radial_prep"] = (nvec * Np * S * 7 * N * 4.0, 8.0 * nvec * nreal + prec_bytes * nvec * Np * 16 * S)
    w["project_rhs"] = (nvec * S * 2 * (Np * Np + 3 * N * Np + N * N) * 2.0,
                        prec_bytes * nvec * Np * 8 * S + 8.0 * nvec * nreal * 3)
    solves = 1 + refine
    nvg = (nvec + 15) // 16
    w["chain_solve"] = (solves * nvec * nblocks * 3 * N * N * 8.0,
                        solves * (nvg * factor_bytes + 8.0 * nvec * nreal * 4 / 3 * 2))
    w["T_solve"] = (solves * nvec * S * N * N * 4.0, solves * 8.0 * nvec * nreal / 3 * 2)
    w["residual64"] = (refine * nvec * 3 * S * N * N * 2 * 10.0, refine * 8.0 * nvec * nreal * 3)
    return w


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def run(args):
    import torch
    import paper_2508_16635_amd as sc
    import seeded_inputs as si

    dev = torch.device("cuda:0")
    W = WORKLOAD
    nvec = args.nvec
    mixed_solve = sc.SC_MIXED_SOLVE_FP32 if args.mixed_solve == "fp32" else sc.SC_MIXED_SOLVE_FP64
    plan = sc.Plan(W["L"], W["M"], W["m0"], W["N"], Ek=W["Ek"], Ra=W["Ra"], Pr=W["Pr"], dt=W["dt"],
                   nvec_max=nvec, refine_mixed=args.refine_mixed, mixed_solve=mixed_solve)
    lay_d = plan.layout
    lay = si.Layout(W["L"], W["M"], W["m0"], W["N"])
    assert lay.n_real == plan.n_real
    log("factor")
    t0 = time.time()
    plan.factor()
    t_factor = time.time() - t0
    ri, ro = RI_RO
    X = si.random_state(lay, 301, amp=BASE_AMP, p=3.0, t_offset=lambda x: ro * ri / ((x + ri + ro) / 2) - ri)
    J = si.default_phase_slot(lay, X)
    C = 0.5
    Xd = torch.from_numpy(X).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    plan.set_base(Xd, C, J)
    torch.cuda.synchronize()
    t_base = time.time() - t0
    # kernel choice by measurement at this shell and batch (sc_autotune, timing the Jacobian
    # action's linear products on this base state), before any timing
    # 20 timed passes per candidate: the register ring's shapes differ by a few per cent
    tuning = None if args.no_autotune else plan.autotune(nvec, reps=20)
    nv_total = max(args.nvectors, nvec)
    V = torch.from_numpy(si.random_vectors(lay, range(3001, 3001 + nv_total))).to(dev)
    Y = torch.empty((nvec, plan.n_real), dtype=torch.float64, device=dev)
    nb = nv_total // nvec

    def batch(i):
        b = i % nb
        return V[b * nvec:(b + 1) * nvec]

    def timed(pl, prec):
        # the timed loop runs without instrumentation; a second, profiled loop of the same
        # length gives the per-stage times (HIP events around every stage)
        for i in range(args.warmup):
            pl.jvp(batch(i), Y, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            pl.jvp(batch(i), Y, prec)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t0
        pl.profile(True)
        torch.cuda.synchronize()
        for i in range(args.steps):
            pl.jvp(batch(i), Y, prec)
        prof = pl.profile_read()
        pl.profile(False)
        return dict(seconds=dt_, jvps=args.steps * nvec, prof=prof)

    log("timing the mixed and FP64 paths")
    results = {"mixed": timed(plan, sc.SC_MIXED), "fp64": timed(plan, sc.SC_FP64)}
    # the other implicit solve of the mixed path, on a plan of its own (same shell and base)
    other = None
    if not args.no_alt_solve:
        log("the other mixed-path solve")
        alt = "fp64" if args.mixed_solve == "fp32" else "fp32"
        plan2 = sc.Plan(W["L"], W["M"], W["m0"], W["N"], Ek=W["Ek"], Ra=W["Ra"], Pr=W["Pr"], dt=W["dt"], nvec_max=nvec,
                        refine_mixed=args.refine_mixed,
                        mixed_solve=sc.SC_MIXED_SOLVE_FP32 if alt == "fp32" else sc.SC_MIXED_SOLVE_FP64)
        plan2.factor()
        plan2.set_base(Xd, C, J)
        if not args.no_autotune:
            plan2.autotune(nvec, reps=20)
        r2 = timed(plan2, sc.SC_MIXED)
        Y2 = torch.empty_like(Y)
        plan2.jvp(batch(0), Y2, sc.SC_MIXED)
        plan2.close()
        other = {"mixed_solve": alt, "refine_mixed": args.refine_mixed if alt == "fp32" else 0,
                 "jvp_per_s": r2["jvps"] / r2["seconds"],
                 "stages": {k: v[0] / max(args.steps, 1) for k, v in r2["prof"].items() if v[1]}}

    # mixed vs FP64 on the same batch (GPU vs GPU, a consistency figure)
    Y64 = torch.empty_like(Y)
    plan.jvp(batch(0), Y, sc.SC_MIXED)
    plan.jvp(batch(0), Y64, sc.SC_FP64)
    torch.cuda.synchronize()
    mixed_vs_fp64 = float(((Y - Y64).norm(dim=1) / Y64.norm(dim=1)).max())
    if other is not None:
        other["mixed_vs_fp64_max_rel"] = float(((Y2 - Y64).norm(dim=1) / Y64.norm(dim=1)).max())

    mixed = results["mixed"]
    fp64 = results["fp64"]
    value = mixed["jvps"] / mixed["seconds"]
    # roofline of the dominant stage of the mixed path
    N = W["N"]
    nblocks = sum(W["L"] - max(k * W["m0"], 1) + 1 for k in range(lay_d["K"] + 1)) * 2
    fbytes = 3 * nblocks * N * N * (8 if args.mixed_solve == "fp32" else 16)
    work = stage_work(lay_d, nvec, 4, fbytes, nblocks, refine=args.refine_mixed if args.mixed_solve == "fp32" else 0,
                      dp_only=tuning is None or bool(tuning["anal_folded"]))
    prof = mixed["prof"]
    # the dominant single-kernel stage of the mixed path (the chain solve is five kernels and
    # the temperature solve runs beside it on a second stream)
    kernels = stage_kernels(tuning, W["N"])
    dom = max((k for k in kernels if k in prof and prof[k][1]), key=lambda k: prof[k][0])
    ms, cnt = prof[dom]
    avg_s = ms / 1e3 / max(cnt, 1)
    # launches per jvp call differ per stage; the work table is per call
    per_call = cnt / max(args.steps, 1)
    fl, by = work.get(dom, (0.0, 0.0))
    fl /= max(per_call, 1)
    by /= max(per_call, 1)
    kname = kernels[dom]
    traffic = measured_traffic(kname) if args.workload == "c3" else None   # counters taken on that shell
    if dom in ("legendre_synth", "legendre_anal"):
        roof = {"bound": "mfma", "achieved": fl / avg_s / 1e12, "peak": PEAK["fp32"], "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": by / avg_s / 1e9, "peak": PEAK["hbm"], "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic
    roof["kernel"] = kname
    roof["stage"] = dom
    roof["algorithmic_per_launch"] = fl if roof["bound"] == "mfma" else by
    roof["avg_launch_us"] = avg_s * 1e6
    stages = {k: {"ms_per_step": v[0] / max(args.steps, 1), "launches_per_step": v[1] / max(args.steps, 1)}
              for k, v in prof.items() if v[1]}
    out = {
        "metric": "Jacobian-vector products/s at L=128,N=48; mixed vs FP64 at 1e-10 residual"
                  if args.workload == "c3" else f"Jacobian-vector products/s at L={W['L']},N={W['N']} (stress shell)",
        "value": value,
        "unit": "jvp/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"rotating-shell jvp L=M={W['L']} m0={W['m0']} N={W['N']} Ek={W['Ek']:g} "
                               f"Ra={W['Ra']:g} dt={W['dt']:g}",
                   "nvec": nvec, "mixed_solve": args.mixed_solve,
                   "refine_mixed": args.refine_mixed if args.mixed_solve == "fp32" else 0, "N_p": lay_d["Np"], "N_theta": lay_d["ntheta"], "N_phi": lay_d["nphi"],
                   "n_real": plan.n_real},
        "fp64_jvp_per_s": fp64["jvps"] / fp64["seconds"],
        "mixed_vs_fp64_max_rel": mixed_vs_fp64,
        "mixed_other_solve": other,
        "factor_s": t_factor,
        "tuning": tuning,
        "set_base_s": t_base,
        "roofline": roof,
        "stages_mixed": stages,
        "stages_fp64": {k: {"ms_per_step": v[0] / max(args.steps, 1)} for k, v in fp64["prof"].items() if v[1]},
    }
    log("single-vector rates")
    if not args.no_single_vector:
        out["nvec1_jvp_per_s"] = single_vector_rates(args, plan, batch, sc)
    if args.batch_scaling and args.workload == "c3":
        log("larger batches")
        out["batch_scaling_jvp_per_s"] = batch_scaling(args, W, Xd, C, J, V, sc)
    if not args.no_newton:
        log("Newton runs")
        out["newton"] = newton_runs(args, plan, C, lay)
    if not args.no_c4 and args.workload == "c3":
        log("batched Newton of 32 uneven problems")
        out["c4_batch"] = c4_batch(args)
    if not args.no_cpu_baseline:
        log("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(args, X, C, J, lay)
    return out


def newton_runs(args, plan, C, lay):
    """Manufactured Newton problem on the timed state: X* = the seeded base state the jvp is timed
    on (BASE_AMP, kinetic-energy density ~25), forcing F* = -R(X*), start X* + 1e-3 |X*| d (seeded
    d, phase slot kept) with C* + 1e-3; every run must drive ||R_F|| to 1e-10.  The mixed Jacobian
    runs with GMRES tolerance 1e-6 (its FP32 transforms give ~1e-7 per action); FP64 runs with the
    paper's 1e-10 and with the same 1e-6.  Reports steps, Jacobian actions, final residual, errors
    of X and C against the root, wall time and Jacobian actions per second (one vector per action,
    as GMRES applies them)."""
    import torch
    import paper_2508_16635_amd as sc
    import seeded_inputs as si
    dev = torch.device("cuda:0")
    ri, ro = RI_RO
    X = si.random_state(lay, 301, amp=BASE_AMP, p=3.0, t_offset=lambda x: ro * ri / ((x + ri + ro) / 2) - ri)
    J = si.default_phase_slot(lay, X)
    Xs = torch.from_numpy(X).to(dev)
    F = torch.empty_like(Xs)
    plan.newton_residual(Xs, C, F)
    F.neg_()
    d = si.random_state(lay, 3999, p=2.0)
    d[lay.nonphysical_mask()] = 0.0
    d[J] = 0.0
    d *= 1e-3 * np.linalg.norm(X) / np.linalg.norm(d)
    res = {"state": f"the timed base state (seed 301, amplitudes {BASE_AMP}, p = 3, conductive T profile)",
           "restart": args.restart, "tol": 1e-10}
    for name, prec, gtol in (("mixed", sc.SC_MIXED, 1e-6), ("fp64", sc.SC_FP64, 1e-10),
                             ("fp64_gmres_tol_1e-6", sc.SC_FP64, 1e-6)):
        x = torch.from_numpy(X + d).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Cf, rep = plan.newton(x, C + 1e-3, J, tol=1e-10, gmres_tol=gtol, restart=args.restart,
                              max_newton=8, max_matvec=args.max_matvec, prec=prec, forcing=F)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t0
        err = float((x - Xs).norm() / Xs.norm())
        res[name] = {"converged": rep["converged"], "newton_steps": rep["newton_steps"], "matvecs": rep["matvecs"],
                     "rnorm_final": rep["rnorm"][-1], "rnorm_history": rep["rnorm"], "seconds": dt_,
                     "matvecs_per_s": rep["matvecs"] / dt_, "rel_err_vs_root": err, "C_err": abs(Cf - C),
                     "gmres_tol": gtol}
    res["mixed_speedup_vs_fp64"] = res["fp64"]["seconds"] / res["mixed"]["seconds"]
    return res


def batch_scaling(args, W, Xd, C, J, V, sc):
    """jvp/s of both paths with 32 and 64 vectors per call (a plan sized for 64, the plan's
    default kernels), context for the 16-vector headline."""
    import torch
    plan = sc.Plan(W["L"], W["M"], W["m0"], W["N"], Ek=W["Ek"], Ra=W["Ra"], Pr=W["Pr"], dt=W["dt"], nvec_max=64)
    plan.factor()
    plan.set_base(Xd, C, J)
    out = {}
    for nv in (32, 64):
        v = V[:nv]
        y = torch.empty_like(v)
        for name, prec in (("mixed", sc.SC_MIXED), ("fp64", sc.SC_FP64)):
            for _ in range(2):
                plan.jvp(v, y, prec)
            torch.cuda.synchronize()
            reps = max(args.steps // 2, 3)
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.jvp(v, y, prec)
            torch.cuda.synchronize()
            out[f"{name}_nvec{nv}"] = reps * nv / (time.perf_counter() - t0)
    plan.close()
    return out


def single_vector_rates(args, plan, batch, sc):
    """jvp/s with one vector per call (the way GMRES applies the Jacobian), both precisions."""
    import torch
    v = batch(0)[:1]
    y = torch.empty_like(v)
    out = {}
    for name, prec in (("mixed", sc.SC_MIXED), ("fp64", sc.SC_FP64)):
        for _ in range(3):
            plan.jvp(v, y, prec)
        torch.cuda.synchronize()
        n = max(args.steps, 10)
        t0 = time.perf_counter()
        for _ in range(n):
            plan.jvp(v, y, prec)
        torch.cuda.synchronize()
        out[name] = n / (time.perf_counter() - t0)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, X, C, J, lay):
    """The FP64 oracle timed on the host cores on a bounded sample of the same workload, with the
    BLAS threads it gets by default and with one thread."""
    import seeded_inputs as si
    from oracle.solver import Problem
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count()
    W = WORKLOAD
    p = Problem(W["L"], W["M"], W["m0"], W["N"], Ek=W["Ek"], Ra=W["Ra"], Pr=W["Pr"], dt=W["dt"])
    p.factor()
    p.set_base(X, C, J)
    V = si.random_vectors(lay, range(3001, 3001 + args.cpu_sample))
    p.jvp(V[0])   # warm-up
    t0 = time.perf_counter()
    for i in range(args.cpu_sample):
        p.jvp(V[i])
    dt_ = time.perf_counter() - t0
    out = {"value": args.cpu_sample / dt_, "unit": "jvp/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"{args.cpu_sample} single-vector jvps of the same shell and base state "
                     f"(oracle factor and base setup excluded)"}
    if threadpool_limits is not None and args.cpu_sample_1t > 0:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            for i in range(args.cpu_sample_1t):
                p.jvp(V[i])
            out["value_1thread"] = args.cpu_sample_1t / (time.perf_counter() - t0)
            out["sample_1thread"] = f"{args.cpu_sample_1t} single-vector jvps with one BLAS thread"
        # the oracle's small dense products run faster on one thread: report the faster setting
        out["value_default_threads"] = out["value"]
        out["cores_default_threads"] = cores
        if out["value_1thread"] > out["value"]:
            out["value"], out["cores"] = out["value_1thread"], 1
            out["sample"] = out["sample_1thread"] + " (faster than the default threads)"
    return out


def action_study(args):
    """Jacobian actions per continuation point, implicit vs explicit Coriolis (Sec. 5, Figs. 8-10),
    for the rotating wave RW4 (m0 = 4) along a branch in Ek with Ra = 7.8 Ek^(-1/3) (Ra = 78 at
    Ek = 1e-3; the paper's path is 6.5 Ek^(-1/3)), and sector (m0 = 4) vs full domain (m0 = 1).
    GMRES runs with the largest restart the library takes (1024 vectors), i.e. unrestarted for
    every implicit solve.

    Route: the oracle's RW4 of the tiny shell, carried to L = M = 47, N = 46 and converged
    (Newton); continuation in log10 Ek with refinement (threshold 1e-6) down to Ek <= 1e-4 and up
    to Ek >= 1e-2.  At each Ek point: three steps of Ra continuation (first step +2 % of Ra) with
    implicit Coriolis, then the same from the explicit variant's own root; the actions of the
    three Newton-GMRES solves are averaged (GMRES tolerance 1e-10, restart 300)."""
    import torch
    import paper_2508_16635_amd as sc
    import seeded_inputs as si
    here = os.path.dirname(os.path.abspath(__file__))
    d = np.load(os.path.join(here, "tests", "golden", "rw4_L16_m4_N16.npz"), allow_pickle=False)
    m0, L, N, coef = 4, 47, 46, 78.0 * 1e-3 ** (1.0 / 3.0)
    newton_kw = dict(tol=1e-10, gmres_tol=1e-10, restart=1024, max_newton=10, max_matvec=args.study_max_matvec)
    tiny = sc.Plan(16, 16, m0, 16, Ek=1e-3, Ra=78.0, nvec_max=1)
    base = sc.Plan(L, L, m0, N, Ek=1e-3, Ra=78.0, dt=200.0, nvec_max=1)
    base.factor()
    x = torch.empty(base.n_real, dtype=torch.float64, device="cuda")
    sc.interpolate(tiny, torch.from_numpy(d["X"]).cuda(), base, x)
    J = si.default_phase_slot(si.Layout(L, L, m0, N), x.cpu().numpy())
    C, rep = base.newton(x, float(d["C"]), J, **newton_kw)
    points = [(1e-3, L, N, x.clone(), C, J)]
    for dp in (-0.25, 0.25):
        pl = sc.Plan(L, L, m0, N, Ek=1e-3, Ra=78.0, dt=200.0, nvec_max=1)
        pl.factor()
        cont = sc.Continuation(pl, x, C, J, param=sc.SC_CONT_EK, n_opt=3, gamma=450.0, ra_coef=coef,
                               refine_tol=1e-6, refine_growth=1.2, **newton_kw)
        last = [1e-3]
        for _ in range(12):
            pt = cont.step(dp_first=dp)
            log(f"Ek continuation: {json.dumps({k: pt[k] for k in ('Ek', 'Ra', 'C', 'L', 'N', 'converged', 'refined')})}")
            if not pt["converged"]:
                break
            last.append(pt["Ek"])
            if len(last) > 3 and abs(np.log10(last[-1] / last[-3])) < 0.01:
                break     # the branch turns (a fold in Ek along this Ra path): stop there
            xs, Cs = cont.state()
            lay = cont.layout()
            points.append((pt["Ek"], lay["L"], lay["N"], xs, Cs, si.default_phase_slot(
                si.Layout(lay["L"], lay["L"], m0, lay["N"]), xs.cpu().numpy())))
            if (dp < 0 and pt["Ek"] <= 1.0001e-4) or (dp > 0 and pt["Ek"] >= 0.9999e-2):
                break
        cont.close()
    # sector vs full domain at Ek = 1e-3: the RW4 embedded in the full-domain layout (m0 = 1)
    lay4, lay1 = si.Layout(L, L, 4, N), si.Layout(L, L, 1, N)
    x4 = points[0][3].cpu().numpy()
    x1 = np.zeros(lay1.n_real)
    for fld in range(3):
        for k, m in enumerate(lay4.ms):
            o4, o1, n = lay4.offset(fld, k, m), lay1.offset(fld, m, m), 2 * N * (L - m + 1)
            x1[o1:o1 + n] = x4[o4:o4 + n]
    # the same phase slot as the sector's (an m = 4 entry; the full layout's m = 1 entries are 0)
    J4 = points[0][5]
    node4 = J4 // 2
    fld4, lm4, j4 = node4 // (N * lay4.S), (node4 // N) % lay4.S, node4 % N
    k4 = max(k for k in range(len(lay4.ms)) if lay4.lm_base[k] <= lm4)
    l4 = lay4.ms[k4] + lm4 - lay4.lm_base[k4]
    J1 = lay1.offset(fld4, lay4.ms[k4], l4, j4) + 1
    dom = {}
    for name, mm, xx, JJ in (("sector_m0_4", 4, x4, J4), ("full_m0_1", 1, x1, J1)):
        pl = sc.Plan(L, L, mm, N, Ek=1e-3, Ra=78.0, dt=200.0, nvec_max=1)
        pl.factor()
        cont = sc.Continuation(pl, torch.from_numpy(xx).cuda(), points[0][4], JJ, param=sc.SC_CONT_RA, n_opt=4,
                               gamma=50.0, **newton_kw)
        mv, Cs_ = [], []
        for _ in range(3):
            pt = cont.step(dp_first=2.0)
            mv.append(pt["matvecs"])
            Cs_.append(pt["C"])
            log(f"{name}: Ra {pt['Ra']:.3f} C {pt['C']:.6f} actions {pt['matvecs']} converged {pt['converged']}")
        cont.close()
        dom[name] = {"actions": mv, "C": Cs_}
        pl.close()
    rows = []
    for Ek, Lp, Np, xs, Cs, Jp in sorted(points, key=lambda t: -t[0]):
        row = {"Ek": Ek, "Ra": coef * Ek ** (-1.0 / 3.0), "L": Lp, "N": Np}
        for name, cor in (("implicit", sc.SC_CORIOLIS_IMPLICIT), ("explicit", sc.SC_CORIOLIS_EXPLICIT)):
            if name == "explicit" and Ek < args.study_explicit_min_ek:
                row[name] = {"actions_per_point": None,
                             "skipped": f"below Ek = {args.study_explicit_min_ek:g} (tens of thousands of actions per point)"}
                continue
            pl = sc.Plan(Lp, Lp, m0, Np, Ek=Ek, Ra=row["Ra"], dt=200.0, nvec_max=1, coriolis=cor)
            pl.factor()
            t0 = time.perf_counter()
            mv, C_first = [], None
            try:
                cont = sc.Continuation(pl, xs, Cs, Jp, param=sc.SC_CONT_RA, n_opt=4, gamma=50.0, **newton_kw)
                C_first = cont.first["C"]
                for _ in range(3):
                    pt = cont.step(dp_first=0.02 * row["Ra"])
                    log(f"Ek={Ek:.3g} {name}: Ra {pt['Ra']:.3f} actions {pt['matvecs']} converged {pt['converged']}")
                    if not pt["converged"]:
                        break
                    mv.append(pt["matvecs"])
                cont.close()
            except Exception as e:   # a Newton that does not converge within the caps
                log(f"{name} at Ek={Ek:g}: {e}")
            row[name] = {"actions_per_point": float(np.mean(mv)) if len(mv) == 3 else None, "actions": mv,
                         "seconds": time.perf_counter() - t0, "C_first": C_first}
            pl.close()
        a, b = row["implicit"]["actions_per_point"], row["explicit"]["actions_per_point"]
        row["explicit_over_implicit"] = b / a if a and b else None
        rows.append(row)
    return {"study": "Jacobian actions per Newton-GMRES solve, RW4 branch", "rows": rows, "domain": dom,
            "newton": newton_kw, "ra_coef": coef}


def c4_problems():
    """The batched-continuation workload: 32 problems of uneven truncation, i = 0..31:
    Ek = (3e-5, 1e-4)[i // 16], Ra = Ra_ref(Ek) 3^((i % 16)/15) with Ra_ref = 6.5 Ek^(-1/3),
    L = M = (64, 80, 96)[i % 3], N = (32, 40)[(i // 3) % 2], m0 = 4 + i % 9, seed 4001 + i."""
    out = []
    for i in range(32):
        Ek = (3e-5, 1e-4)[i // 16]
        Ra = 6.5 * Ek ** (-1.0 / 3.0) * 3.0 ** ((i % 16) / 15.0)
        L = (64, 80, 96)[i % 3]
        N = (32, 40)[(i // 3) % 2]
        out.append(dict(i=i, Ek=Ek, Ra=Ra, L=L, M=L, N=N, m0=4 + i % 9, seed=4001 + i))
    return out


def c4_state(si, lay, pr):
    """X* of problem pr, a rotating-wave-like guess: the conductive profile, the order m0 at
    amplitude 1e-2 with coefficients decaying as (l+1)^-2 (random phases), the orders 2 m0 and
    above at 1e-4, nothing else at m = 0."""
    ri, ro = RI_RO
    X = si.random_state(lay, pr["seed"], amp=(1.0, 1.0, 1.0), p=2.0, t_offset=lambda x: ro * ri / ((x + ri + ro) / 2) - ri)
    Xc = si.random_state(lay, pr["seed"], amp=(0.0, 0.0, 0.0), p=2.0, t_offset=lambda x: ro * ri / ((x + ri + ro) / 2) - ri)
    for fld in range(3):
        for k, m in enumerate(lay.ms):
            o = lay.offset(fld, k, m)
            n = 2 * lay.N * lay.nl[k]
            X[o:o + n] = Xc[o:o + n] if k == 0 else X[o:o + n] * (1e-2 if k == 1 else 1e-4)
    return X


def c4_batch(args):
    """All 32 problems' manufactured Newton-GMRES solves (root X*, forcing -R(X*), start
    X* + 1e-3 |X*| d) in one sc_batch_newton call: every plan on its own stream branch, driven by
    a host thread of its own, its Arnoldi steps on the device in chunks of 8 between host checks.
    Mixed Jacobian actions (GMRES tolerance 1e-6), Newton residual in FP64 to 1e-10.  Reports the
    aggregate Jacobian actions per second."""
    import torch
    import paper_2508_16635_amd as sc
    import seeded_inputs as si
    probs = c4_problems()
    plans, xs, Cs, Js, Fs, Xs = [], [], [], [], [], []
    t0 = time.perf_counter()
    for pr in probs:
        p = sc.Plan(pr["L"], pr["M"], pr["m0"], pr["N"], Ek=pr["Ek"], Ra=pr["Ra"], Pr=1.0, dt=200.0, nvec_max=1)
        p.factor()
        lay = si.Layout(pr["L"], pr["M"], pr["m0"], pr["N"])
        X = c4_state(si, lay, pr)
        J = si.default_phase_slot(lay, X)
        Xd = torch.from_numpy(X).cuda()
        F = torch.empty_like(Xd)
        p.newton_residual(Xd, 0.5, F)
        F.neg_()
        d = si.random_state(lay, pr["seed"] + 1000, p=2.0)
        d[lay.nonphysical_mask()] = 0.0
        d[J] = 0.0
        d *= 1e-3 * np.linalg.norm(X) / np.linalg.norm(d)
        plans.append(p)
        xs.append(torch.from_numpy(X + d).cuda())
        Cs.append(0.501)
        Js.append(J)
        Fs.append(F)
        Xs.append(Xd)
    t_setup = time.perf_counter() - t0
    log(f"C4: 32 plans factored in {t_setup:.1f} s")
    b = sc.Batch(plans)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = b.newton(xs, Cs, Js, tol=1e-10, gmres_tol=1e-6, restart=args.c4_restart, max_newton=8,
                   max_matvec=2000, prec=sc.SC_MIXED, forcings=Fs)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    b.close()
    mv = sum(rep["matvecs"] for _, rep in out)
    errs = [float((x - X).norm() / X.norm()) for x, X in zip(xs, Xs)]
    res = {"problems": 32, "converged": sum(rep["converged"] for _, rep in out), "jacobian_actions": mv,
           "seconds": secs, "jvp_per_s": mv / secs, "setup_s": t_setup, "restart": args.c4_restart,
           "max_rel_err_vs_root": max(errs), "max_final_rnorm": max(rep["rnorm"][-1] for _, rep in out),
           "newton_steps": [rep["newton_steps"] for _, rep in out], "actions": [rep["matvecs"] for _, rep in out]}
    for p in plans:
        p.close()
    return res


def _csv_rows(d, suffix):
    """Rows of every rocprofv3 CSV under directory d whose name ends with suffix."""
    import csv
    rows = []
    for root, _, files in os.walk(d):
        for f in sorted(files):
            if f.endswith(suffix):
                with open(os.path.join(root, f), newline="") as fh:
                    rows.extend(csv.DictReader(fh))
    return rows


def _kname(s):
    """Kernel name without the return type and the argument list."""
    s = s.strip()
    if s.startswith("void "):
        s = s[5:]
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return s[:i]
    return s


def _counters(d):
    """{kernel: {"launches": n, counter: mean per dispatch, "vgpr", "lds"}} from counter CSVs."""
    per = {}
    for r in _csv_rows(d, "counter_collection.csv"):
        k, c = _kname(r["Kernel_Name"]), r["Counter_Name"]
        disp = per.setdefault(k, {})
        e = disp.setdefault(r["Dispatch_Id"], {"vgpr": r.get("VGPR_Count"), "agpr": r.get("Accum_VGPR_Count"),
                                                "lds": r.get("LDS_Block_Size"), "wg": r.get("Workgroup_Size")})
        e[c] = e.get(c, 0.0) + float(r["Counter_Value"])
    out = {}
    for k, disp in per.items():
        names = {c for e in disp.values() for c in e if c not in ("vgpr", "agpr", "lds", "wg")}
        first = next(iter(disp.values()))
        out[k] = {"launches": len(disp), "vgpr": first["vgpr"], "agpr": first["agpr"], "lds": first["lds"],
                  "wg": first["wg"]}
        for c in names:
            out[k][c] = sum(e.get(c, 0.0) for e in disp.values()) / len(disp)
    return out


def summarize_profiles(d):
    """Turns the rocprofv3 runs under d (stats/, fetch/, write/, probe_fetch/, probe_write/,
    sq_mfma/, sq_lds/, sq_time/, any of them may be missing) into the committed traffic file and prints
    Markdown tables.  FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by the
    ratio of the bytes a plain copy moves to what the same counter reads for it."""
    md = []
    stats = {}
    for r in _csv_rows(os.path.join(d, "stats"), "kernel_stats.csv"):
        stats[_kname(r["Name"])] = {"calls": int(r["Calls"]), "total_us": float(r["TotalDurationNs"]) / 1e3,
                            "avg_us": float(r["AverageNs"]) / 1e3, "pct": float(r["Percentage"])}
    if stats:
        md += ["kernel | calls | total us | avg us | % of GPU time", "---|---|---|---|---"]
        for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["total_us"]):
            md.append(f"{k} | {v['calls']} | {v['total_us']:.1f} | {v['avg_us']:.1f} | {v['pct']:.2f}")
        md.append("")
    fetch, write = _counters(os.path.join(d, "fetch")), _counters(os.path.join(d, "write"))
    pf, pw = _counters(os.path.join(d, "probe_fetch")), _counters(os.path.join(d, "probe_write"))
    if fetch and write and pf and pw:
        probe = lambda t, c: next(v[c] for k, v in t.items() if "Mul" in k)
        nbytes = 256 * (1 << 20)
        kib = {"FETCH_SIZE": probe(pf, "FETCH_SIZE"), "WRITE_SIZE": probe(pw, "WRITE_SIZE")}
        scale = {c: nbytes / (kib[c] * 1024.0) for c in kib}
        ker = {}
        for k in set(fetch) & set(write):
            fb = fetch[k]["FETCH_SIZE"] * 1024.0 * scale["FETCH_SIZE"]
            wb = write[k]["WRITE_SIZE"] * 1024.0 * scale["WRITE_SIZE"]
            ker[k] = {"launches": fetch[k]["launches"], "fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb}
        traffic = {"copy_probe_kib_per_launch": kib, "scale": scale, "kernels": ker,
                   "sources_sha256": sources_sha256()}
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(traffic, fh, indent=1, sort_keys=True)
        md += [f"Calibration: the plain copy (256 MiB read, 256 MiB written) reads FETCH_SIZE = "
               f"{kib['FETCH_SIZE']:.0f} KiB and WRITE_SIZE = {kib['WRITE_SIZE']:.0f} KiB per launch: scale "
               f"{scale['FETCH_SIZE']:.3f} and {scale['WRITE_SIZE']:.3f}.", "",
               "kernel | launches | read MB/launch | written MB/launch | total MB/launch", "---|---|---|---|---"]
        for k, v in sorted(ker.items(), key=lambda kv: -kv[1]["bytes"]):
            md.append(f"{k} | {v['launches']} | {v['fetch_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} | "
                      f"{v['bytes'] / 1e6:.1f}")
        md.append("")
    mf = _counters(os.path.join(d, "sq_mfma"))
    if mf:
        # SQ_BUSY_CYCLES sums the cycles of the 32 shader engines (4 per XCD), the MFMA busy
        # cycles those of the 1024 SIMDs
        md += ["kernel | launches | MFMA FLOP/launch | MFMA TFLOP/s (trace avg) | of peak | MFMA busy per SIMD-cycle | "
               "VALU insts/wave | waves/launch",
               "---|---|---|---|---|---|---|---"]
        for k, v in sorted(mf.items(), key=lambda kv: -stats.get(kv[0], {}).get("total_us", 0.0)):
            if not k.startswith("sc::"):
                continue
            f32 = v.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) * 512
            f64 = v.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512
            fl, peak = (f64, PEAK["fp64"]) if f64 > f32 else (f32, PEAK["fp32"])
            avg = stats.get(k, {}).get("avg_us")
            rate = fl / (avg * 1e-6) / 1e12 if avg and fl else 0.0
            busy = v.get("SQ_BUSY_CYCLES", 0.0)
            mb = v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (busy / 32.0 * 1024.0) if busy else 0.0
            waves = v.get("SQ_WAVES", 0.0)
            vi = v.get("SQ_INSTS_VALU", 0.0) / waves if waves else 0.0
            md.append(f"{k} | {v['launches']} | {fl:.3e} | {rate:.1f} | {rate / peak:.3f} | {mb:.3f} | {vi:.0f} | "
                      f"{waves:.0f}")
        md.append("")
    ld = _counters(os.path.join(d, "sq_lds"))
    if ld:
        md += ["kernel | LDS insts/wave | bank-conflict cycles / LDS active cycles | LDS wait / LDS active | "
               "VMEM rd insts/wave",
               "---|---|---|---|---"]
        for k, v in sorted(ld.items(), key=lambda kv: -stats.get(kv[0], {}).get("total_us", 0.0)):
            if not k.startswith("sc::"):
                continue
            waves = v.get("SQ_WAVES", 0.0) or 1.0
            act = v.get("SQ_LDS_IDX_ACTIVE", 0.0)
            bc = v.get("SQ_LDS_BANK_CONFLICT", 0.0) / act if act else 0.0
            aw = v.get("SQ_ACTIVE_INST_LDS", 0.0)
            wt = v.get("SQ_WAIT_INST_LDS", 0.0) / aw if aw else 0.0
            md.append(f"{k} | {v.get('SQ_INSTS_LDS', 0.0) / waves:.0f} | {bc:.3f} | {wt:.2f} | "
                      f"{v.get('SQ_INSTS_VMEM_RD', 0.0) / waves:.0f}")
        md.append("")
    tm = _counters(os.path.join(d, "sq_time"))
    if tm:
        # per-wave time split (wave-cycles, quad-cycle units cancel in the ratios)
        md += ["kernel | waiting on anything / wave time | issuing any / wave time | VALU issue / wave time | "
               "LDS issue / wave time | VMEM issue / wave time",
               "---|---|---|---|---|---"]
        for k, v in sorted(tm.items(), key=lambda kv: -stats.get(kv[0], {}).get("total_us", 0.0)):
            if not k.startswith("sc::"):
                continue
            wc = v.get("SQ_WAVE_CYCLES", 0.0) or 1.0
            md.append(f"{k} | {v.get('SQ_WAIT_ANY', 0.0) / wc:.2f} | {v.get('SQ_ACTIVE_INST_ANY', 0.0) / wc:.2f} | "
                      f"{v.get('SQ_ACTIVE_INST_VALU', 0.0) / wc:.2f} | {v.get('SQ_ACTIVE_INST_LDS', 0.0) / wc:.2f} | "
                      f"{v.get('SQ_ACTIVE_INST_VMEM', 0.0) / wc:.2f}")
        md.append("")
    print("\n".join(md), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nvec", type=int, default=16)
    ap.add_argument("--nvectors", type=int, default=200)
    ap.add_argument("--cpu-sample", type=int, default=20)
    ap.add_argument("--cpu-sample-1t", type=int, default=10, help="oracle jvps timed with one BLAS thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-solve", choices=("fp64", "fp32"), default="fp64",
                    help="implicit solve of the mixed path: one FP64 solve, or an FP32 solve plus refinement")
    ap.add_argument("--refine-mixed", type=int, default=1,
                    help="with --mixed-solve fp32: FP64 refinement passes (FP64 residual + FP64 correction)")
    ap.add_argument("--no-alt-solve", action="store_true", help="do not time the other mixed-path solve")
    ap.add_argument("--no-newton", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default kernel choices")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c3",
                    help="c3: the metric's shell; stress: L=M=255, N=64 (no oracle baseline, no Newton run)")
    ap.add_argument("--restart", type=int, default=1000,
                    help="GMRES restart of the Newton runs (GMRES(40) stagnates on the timed state)")
    ap.add_argument("--max-matvec", type=int, default=3000)
    ap.add_argument("--study", choices=("actions",), default=None,
                    help="actions: Jacobian actions per continuation point, implicit vs explicit Coriolis and "
                         "sector vs full domain (prints its own JSON line instead of the benchmark)")
    ap.add_argument("--study-max-matvec", type=int, default=8000)
    ap.add_argument("--study-explicit-min-ek", type=float, default=1.1e-4)
    ap.add_argument("--no-single-vector", action="store_true", help="skip the one-vector-per-call rates")
    ap.add_argument("--no-c4", action="store_true", help="skip the 32-problem batched Newton leg")
    ap.add_argument("--batch-scaling", type=int, default=1, help="also time 32 and 64 vectors per call (0: skip)")
    ap.add_argument("--c4-restart", type=int, default=1000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy (y = 1.0 * x, fp32) of MIB MiB five times: the reference "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None,
                    help="only summarize the rocprofv3 runs under DIR (stats/, fetch/, write/, probe_fetch/, "
                         "probe_write/, sq_mfma/, sq_lds/, sq_time/): rewrite the traffic file, print Markdown tables")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5}), flush=True)
        return
    if args.study == "actions":
        print(json.dumps(action_study(args)), flush=True)
        return
    global WORKLOAD
    WORKLOAD = WORKLOADS[args.workload]
    if args.workload != "c3":   # the oracle and the Newton problem are sized for the metric's shell
        args.no_cpu_baseline = True
        args.no_newton = True
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    out = run(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    main()
