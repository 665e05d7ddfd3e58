#!/usr/bin/env python
"""Benchmark of the Wilson-clover propagator solve on one MI355X.

Workload of the timed step (the value): the 32^3x64 propagator -- links
exp(i 0.2 H) (Gaussian traceless Hermitian H, seed 3), periodic space /
antiperiodic time, kappa = 0.135, csw = 1.9, the 12 spin-colour point
sources at the origin solved together as one 12-rhs even-odd preconditioned
CG with BF16-storage operands (links, clover blocks and the iterated
spinors in BF16, FP32 arithmetic) and reliable updates (true residual in
FP64, the recursion's restart residual through the FP32 operators) on a
tenfold drop of |r| and at least every 100 iterations, to a true relative
residual of 1e-10 recomputed in FP64.  Each
step runs the whole path: clover term (built once per gauge field and
parameters, then cached), source preparation, CG on Dhat^+ Dhat in hipGraph
chunks, odd-site reconstruction and the FP64 full-lattice residual check.
Inputs are resident in HBM before the timed region; kernels are autotuned
before it.  Beside it, the same 12 sources solved one at a time by the FP64
CG (the metric's "solves/s mixed vs FP64") and with FP32 inner precision.

The JSON line (stdout) also carries
* "roofline": the dominant kernel of the step, the BF16 12-rhs e->o hop, bound
  by FP32 vector arithmetic (algorithmic flops per launch / average launch
  time, launches replayed from one graph, HIP events on its stream, against
  the FP32 vector peak without dual issue), with its HBM rate beside it; the
  FP64 one-rhs hop of the baseline at the same size (HBM bound);
* "c2": the 16^3x32 propagator (kappa 0.1345), FP64 one source at a time and
  12 rhs per solve in FP64/FP32/BF16 inner precision;
* "mixed_c4": the 24^3x48 Schroedinger-functional propagator (kappa 0.134,
  csw 1.8, 12 point sources at t = 1), FP64 one source at a time vs one
  multi-RHS mixed solve;
* "c3": the 32^3x64 Z2-noise solve (kappa 0.135) in FP64, FP32 and BF16 inner
  precision, and the meson contraction of the propagator;
* "dw_hbm": the hop kernels at 32^3x64 (working set > 1 GB, beyond the 256 MB
  last-level cache) in FP64/FP32/BF16, one and 12 rhs;
* "serving": a Poisson stream of mixed propagator requests through the
  serving loop (kernels tuned before it starts), p50/p99 latency and
  solves/s at the offered rate, then at 0.7x the measured capacity (where the
  latencies describe the service and not a growing backlog);
* "cpu_baseline": the FP64 CPU oracle on a bounded sample of the step's
  workload, with the host's CPU model.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-hbm] [--no-cpu]
       [--no-mixed] [--no-serve] [--serve-requests N] [--serve-rate R]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dw GB/s (% HBM peak); solves/s mixed vs FP64 at 1e-10; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
CSW, EPS, TOL = 1.9, 0.2, 1e-10
THETA = (1, 1, 1, -1)
# the step: 32^3x64 propagator (12 point sources at the origin)
L_STEP, KAPPA_STEP, SEED_STEP = (32, 32, 32, 64), 0.135, 3
# the 16^3x32 propagator
L_C2, KAPPA, SEED = (16, 16, 16, 32), 0.1345, 2
# algorithmic traffic per lattice site V (reals): each input read once, each
# output written once.  Links: 4 per site of 12 reals stored as two rows
# (paper Sec. 2.2; 18 reals with full links); clover blocks 36, spinors 12 per
# parity.
LINK_REALS = {True: 48, False: 72}  # per site V, two-row / full links


def hop_reals(op, nrhs=1, two_row=True, tm=False):
    """Algorithmic reals per site V of one hop launch (or of the full Dw);
    tm: twisted mass, whose e->o launch also reads A_oo (36 reals per V)."""
    u = LINK_REALS[two_row]
    if op == "hop_oe":   # U + psi_o + psi_e + A_ee + out
        return u + 36 + 36 * nrhs
    if op == "hop_eo":   # U + psi_e + A_oo^-1 (+ A_oo) + out
        return u + 36 + (36 if tm else 0) + 24 * nrhs
    return u + 72 + 48 * nrhs  # full Dw: U + A + psi + out


# Algorithmic flops per output site and rhs of one hop launch (the standard
# Wilson-clover count): eight hops of 168 flops (spin projection 12, SU(3)
# times a two-spinor 132, reconstruction 24) less the 24 of the first
# accumulation = 1320; the -1/2 scale 24; two Hermitian 6x6 blocks times a
# 6-vector 2 x 252 = 504; o->e adds the self term (24 more).
FLOPS_PER_SITE_RHS = {"hop_eo": 1320 + 24 + 504, "hop_oe": 1320 + 24 + 504 + 24}
# FP32 vector peak without packed (dual) FP32 issue, which this build disables
# for correctness: 256 CUs x 64 FMA lanes per clock x 2 flop x 2.4 GHz
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12  # 78.6
BYTES_PER_REAL = {0: 8, 1: 4, 2: 2}
PREC_NAME = {0: "f64", 1: "f32", 2: "bf16"}
# hop tuning of the 16^3x32 FP64 one-at-a-time solves (nr_tile, block_order,
# rhs_lanes, nt_store, cached_gauge, occ_cap, dir_split): cached gauge loads
# keep links and clover in the last-level cache, which holds this lattice's
# whole working set; the direction split gives the 65536 sites of a parity two
# waves each
STEP_TUNING = (1, 1, 1, True, True, 0, True)
# gauge fields of every leg store two rows per link
TWO_ROW = True
# twisted mass of the twisted-mass leg (32^3x64 Z2 source)
TM_MU = 0.01
ROOFLINE_LAUNCHES = 100
KERNEL_SOURCES = ["paper_2503_16994_amd/csrc/k_dslash.hip", "paper_2503_16994_amd/csrc/lqcd_dev.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


COUNTERS_JSON = os.path.join(ROOT, "profiles", "hop_kernels_32x32x32x64_counters.json")


def stored_traffic(op, prec, nrhs, tuning):
    """HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE) of the hop launch
    (op, prec, nrhs) from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source in the same tuning; else None."""
    try:
        with open(COUNTERS_JSON) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    for e in d.get("launches", []):
        if e.get("op") == op and e.get("prec") == prec and e.get("nrhs") == nrhs and e.get("tuning") == tuning:
            return e.get("hbm_bytes_per_launch")
    return None


def graph_launch_ms(fn, n, stream):
    """Average time of fn's launch(es): n calls captured in one graph,
    replayed once untimed and once timed with HIP events on `stream` (eager
    launches through Python would time the host for short kernels)."""
    import torch
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for _ in range(n):
            fn()
    graph.replay()
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    graph.replay()
    e1.record(stream)
    e1.synchronize()
    del graph
    return e0.elapsed_time(e1) / n


def internal_vectors(lat_, prec, nrhs):
    """Random input and an output internal-layout vector (finite BF16 pairs)."""
    import torch

    from paper_2503_16994_amd import lqcd
    vb = lqcd.vec_bytes(lat_, prec, nrhs, 2)
    if prec == lqcd.BF16:
        x = torch.randn(vb // 2, device="cuda").to(torch.bfloat16).view(torch.uint8)
    elif prec == lqcd.F64:
        x = torch.randn(vb // 8, device="cuda", dtype=torch.float64).view(torch.uint8)
    else:
        x = torch.randn(vb // 4, device="cuda").view(torch.uint8)
    return x, torch.empty(vb, dtype=torch.uint8, device="cuda")


def hop_roofline(g, lat_, ws, d, op_name, prec, nrhs, stream, launches):
    """Roofline entry of one hop launch in the workspace's tuning."""
    from paper_2503_16994_amd import lqcd
    x, y = internal_vectors(lat_, prec, nrhs)
    op = {"hop_eo": lqcd.OP_HOP_EO, "hop_oe": lqcd.OP_HOP_OE}[op_name]
    ms = graph_launch_ms(lambda: lqcd.dw_apply_internal(g, d, x, y, op, prec, nrhs, ws, stream=stream),
                         launches, stream)
    tr = bool(g.pmask & lqcd.PM_TWO_ROW)
    alg = hop_reals(op_name, nrhs, tr) * BYTES_PER_REAL[prec] * lat_.volume
    achieved = alg / (ms * 1e-3) / 1e9
    tune = lqcd.get_tuning(ws, prec)
    traffic = stored_traffic(op_name, PREC_NAME[prec], nrhs, tune)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "traffic_vs_alg": round(traffic / alg, 3) if traffic else None,
            "kernel": f"{op_name} {PREC_NAME[prec]} {nrhs} rhs", "lattice": list(lat_.L),
            "avg_launch_us": round(ms * 1e3, 2), "alg_bytes_per_launch": alg, "tuning": tune,
            "links": "two rows per link" if tr else "full"}


def alu_roofline(h, op_name, nrhs, lat_):
    """Roofline entry of a hop launch bound by FP32 vector arithmetic (the
    reduced-precision multi-rhs launches: rocprofv3 counts their VALU
    instructions at ~90% of the issue slots of the launch): algorithmic
    flops per launch / average launch time against the FP32 vector peak; the
    HBM figures of the same launch are kept beside it."""
    flops = FLOPS_PER_SITE_RHS[op_name] * (lat_.volume // 2) * nrhs
    achieved = flops / (h["avg_launch_us"] * 1e-6) / 1e12
    out = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
           "frac": round(achieved / ALU_PEAK_TFLOPS, 4), "traffic": h["traffic"],
           "flops_per_launch": flops, "hbm_achieved_GBps": h["achieved"], "hbm_frac": h["frac"],
           "peak_note": "FP32 FMA without packed-FP32 dual issue (disabled in this build): "
                        "256 CUs x 64 lanes x 2 flop x 2.4 GHz; the published 157.3 TFLOP/s counts dual issue"}
    for k in ("traffic_vs_alg", "kernel", "lattice", "avg_launch_us", "alg_bytes_per_launch", "tuning", "links"):
        if k in h:
            out[k] = h[k]
    return out


def time_launches(fn, reps, stream):
    import torch
    for _ in range(3):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps  # ms


def hop_rates(g, lat_, ws, d, prec, nrhs, stream, reps=30):
    """Average launch time and algorithmic GB/s of the two hop kernels (and,
    for one FP64 rhs, of the full-lattice Dw) on random internal vectors."""
    import torch

    from paper_2503_16994_amd import lqcd
    vb = lqcd.vec_bytes(lat_, prec, nrhs, 2)
    if prec == lqcd.BF16:  # finite bf16 pairs
        x = torch.randn(vb // 2, device="cuda").to(torch.bfloat16).view(torch.uint8)
    else:
        x = torch.randn(vb // 4, device="cuda").view(torch.uint8)
    y = torch.empty(vb, dtype=torch.uint8, device="cuda")
    tr = bool(g.pmask & lqcd.PM_TWO_ROW)
    tm = d.mu != 0.0
    ops = [(lqcd.OP_HOP_EO, "hop_eo", hop_reals("hop_eo", nrhs, tr, tm)),
           (lqcd.OP_HOP_OE, "hop_oe", hop_reals("hop_oe", nrhs, tr))]
    if prec == lqcd.F64 and nrhs == 1:
        ops.append((lqcd.OP_DW, "dw_full", hop_reals("dw_full", 1, tr)))
    out = {}
    for op, name, reals in ops:
        ms = time_launches(lambda op=op: lqcd.dw_apply_internal(g, d, x, y, op, prec, nrhs, ws, stream=stream),
                           reps, stream)
        gbs = reals * BYTES_PER_REAL[prec] * lat_.volume / (ms * 1e-3) / 1e9
        out[name] = {"us": round(ms * 1e3, 1), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del x, y
    return out


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-hbm", action="store_true", help="skip the other 32^3x64 legs (Z2 solve, kernel rates)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 16^3x32 and 24^3x48 SF legs")
    ap.add_argument("--no-ctx", action="store_true", help="skip the 32^4 context leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=60)
    ap.add_argument("--serve-rate", type=float, default=50.0, help="mean arrivals per second")
    ap.add_argument("--profile-kernel", action="store_true",
                    help="only calibration copy/sum and hop-kernel launches (profiler runs)")
    ap.add_argument("--profile-step", action="store_true",
                    help="only the step (tuned beforehand), for a kernel trace of the solve")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent propagators shard across GPUs with no communication between them)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2503_16994_amd import inputs, lqcd

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    if args.profile_kernel:
        profile_kernels(stream)
        return
    load_tuning_table()
    pm = lqcd.PM_F64 | lqcd.PM_F32 | lqcd.PM_BF16
    gpm = pm | lqcd.PM_TWO_ROW  # gauge fields store two rows per link

    # ---- the step: 32^3x64, 12 sources in one BF16-inner solve -------------
    L = L_STEP
    U3 = inputs.gauge_field(L, EPS, seed=SEED_STEP)
    lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, THETA)
    g3 = lqcd.GaugeField(lat, torch.from_numpy(U3), gpm, stream=stream)
    d3 = lqcd.dirac(KAPPA_STEP, CSW)
    etap = torch.from_numpy(inputs.point_sources_12(L, (0, 0, 0, 0))).cuda()
    prop = torch.empty_like(etap)
    ws12 = lqcd.Workspace(lat, pm, 12)

    def tune_mixed(ws, g, d, ip, nrhs):
        """the tuning of the inner precision, of FP64 (the hops of the
        reliable updates) and, for BF16, of FP32 (the reliable updates'
        Dhat^+ for the recursion) for nrhs rhs: from the committed table, else
        autotuned"""
        precs = (ip, lqcd.F64) + ((lqcd.F32,) if ip == lqcd.BF16 else ())
        for prec in precs:
            t = lqcd.tune_cache_find(g, prec, nrhs)
            if t is None:
                t, _ = lqcd.autotune(g, d, prec, nrhs, ws, stream=stream)
            else:
                lqcd.set_tuning(ws, prec, **t)
            if prec == ip:
                tune = t
        return tune

    def solve12(ip, ws):
        return lqcd.solve(g3, etap, KAPPA_STEP, CSW, tol=TOL, solver=lqcd.SOLVER_CG_EO, inner_prec=ip,
                          reliable_every=100, use_graph=True, ws=ws, stream=stream, psi=prop,
                          raise_on_noconv=False)

    def summary(r, dt):
        rho = max(i["true_residual"] for i in r.info)
        return {"solves_per_s": round(12 / dt, 3), "ms_per_12": round(dt * 1e3, 2),
                "converged": bool(r.status == 0 and rho <= TOL), "max_true_residual": rho,
                "iters": max(i["iters"] for i in r.info),
                "reliable_updates": max(i["reliable_updates"] for i in r.info),
                "fp64_from": max(i["fp64_from"] for i in r.info)}

    tune_bf16 = tune_mixed(ws12, g3, d3, lqcd.BF16, 12)
    torch.cuda.synchronize()
    if args.profile_step:
        timed(lambda: solve12(lqcd.BF16, ws12), 2, 1)
        return
    dt, r = timed(lambda: solve12(lqcd.BF16, ws12), args.steps, args.warmup)
    ms_step, value = dt * 1e3, 12 / dt
    step = summary(r, dt)
    step["tuning"] = tune_bf16
    assert step["converged"], r.info
    log(f"step: 32^3x64 12-rhs BF16 inner: {step}")
    # the same 12 sources, FP32 inner (12 rhs) and FP64 one at a time
    tune_f32 = tune_mixed(ws12, g3, d3, lqcd.F32, 12)
    dt32, r32 = timed(lambda: solve12(lqcd.F32, ws12), 1, 1)
    step_f32 = dict(summary(r32, dt32), tuning=tune_f32)
    log(f"32^3x64 12-rhs FP32 inner: {step_f32}")
    # roofline of the step's dominant kernel (the BF16 12-rhs e->o hop, two
    # launches per iteration) in the step's tuning
    roofline = alu_roofline(hop_roofline(g3, lat, ws12, d3, "hop_eo", lqcd.BF16, 12, stream, 20), "hop_eo", 12, lat)
    roofline["o_to_e_same_tuning"] = {
        k: v for k, v in alu_roofline(hop_roofline(g3, lat, ws12, d3, "hop_oe", lqcd.BF16, 12, stream, 20),
                                      "hop_oe", 12, lat).items()
        if k in ("achieved", "frac", "avg_launch_us", "traffic", "traffic_vs_alg", "hbm_achieved_GBps", "hbm_frac")}
    del ws12
    torch.cuda.empty_cache()
    ws1 = lqcd.Workspace(lat, pm, 1)
    tune64 = lqcd.tune_cache_find(g3, lqcd.F64, 1, dir_split=True)
    if tune64 is None:
        lqcd.set_tuning(ws1, lqcd.F64, dir_split=True)
        tune64, _ = lqcd.autotune(g3, d3, lqcd.F64, 1, ws1, stream=stream)
    else:
        lqcd.set_tuning(ws1, lqcd.F64, **tune64)

    def f64_one():
        return [lqcd.solve(g3, etap[j:j + 1], KAPPA_STEP, CSW, tol=TOL, inner_prec=lqcd.F64, use_graph=True,
                           ws=ws1, stream=stream, psi=prop[j:j + 1]).info[0] for j in range(12)]
    dt64, infos64 = timed(f64_one, 1, 1)
    fp64 = {"solves_per_s": round(12 / dt64, 3), "ms_per_12": round(dt64 * 1e3, 1),
            "iters": max(i["iters"] for i in infos64),
            "max_true_residual": max(i["true_residual"] for i in infos64), "tuning": tune64}
    assert fp64["max_true_residual"] <= TOL
    log(f"32^3x64 FP64 one at a time: {fp64}")
    # the baseline's dominant kernel: the FP64 one-rhs o->e hop with A_ee
    roofline["fp64_one_rhs_hop_oe"] = {k: v for k, v in hop_roofline(g3, lat, ws1, d3, "hop_oe", lqcd.F64, 1,
                                                                      stream, 50).items()
                                       if k in ("achieved", "frac", "avg_launch_us", "traffic", "traffic_vs_alg",
                                                "tuning", "alg_bytes_per_launch")}
    log(f"roofline: {roofline}")
    del ws1
    torch.cuda.empty_cache()
    step_cfg = {"bf16_inner_12rhs": step, "f32_inner_12rhs": step_f32, "fp64_one_at_a_time": fp64,
                "bf16_vs_fp64": round(value / fp64["solves_per_s"], 3),
                "f32_vs_fp64": round(step_f32["solves_per_s"] / fp64["solves_per_s"], 3)}

    c2 = mixed_c4 = c3 = dw_hbm = serving = ctx = None
    # ---- 32^3x64: Z2 solve, meson contraction, the kernels' HBM rates --------
    if not args.no_hbm:
        c3, dw_hbm = c3_leg(stream, pm, g3, lat, prop)
    del g3, etap, prop
    torch.cuda.empty_cache()
    # ---- 16^3x32 and the 24^3x48 SF propagator --------------------------------
    if not args.no_mixed:
        c2 = c2_leg(stream, pm, gpm, mixed_leg)
        mixed_c4 = c4_leg(stream, pm, gpm, mixed_leg, 1)
    if not args.no_ctx:
        ctx = ctx_leg(stream, gpm & (lqcd.PM_F64 | lqcd.PM_TWO_ROW))

    # ---- serving -------------------------------------------------------------
    if not args.no_serve:
        serving = serve_legs(args.serve_requests, args.serve_rate)

    # ---- CPU oracle baseline (bounded sample of the step's workload) -----------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(U3)
        log(f"cpu_baseline: {cpu}")
    del U3

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "32^3x64 Wilson-clover propagator: the 12 point sources at the origin in one "
                               "12-rhs even-odd CG, BF16-storage operands with FP32 arithmetic, FP64 reliable "
                               "updates (on a tenfold drop of |r|, at least every 100 iterations), true residual "
                               "1e-10",
                   "lattice": list(L), "kappa": KAPPA_STEP, "csw": CSW, "bc": "periodic/antiperiodic",
                   "link_eps": EPS, "link_seed": SEED_STEP, "sources": 12, "tol": TOL,
                   "storage": "bf16 (links, clover, p/q/t spinors); f32 recursion; f64 solution and residuals",
                   "links": "two rows per link (third rebuilt in registers)", "hop_tuning": tune_bf16},
        "step": step_cfg, "roofline": roofline, "c2": c2, "mixed_c4": mixed_c4, "c3": c3, "dw_hbm": dw_hbm,
        "ctx": ctx, "serving": serving, "cpu_baseline": cpu,
    }
    if os.environ.get("LQCD_SAVE_TUNING"):
        lqcd.tune_cache_save(os.environ["LQCD_SAVE_TUNING"])
    print(json.dumps(line), flush=True)


def mixed_leg(stream, g, lat_, ws, etas, kappa, csw, fp64_sps, steps, warmup, tag, precs=("f64", "f32", "bf16")):
    """12 rhs in one solve per inner precision (autotuned kernels; the FP64
    hops of the reliable updates in the 12-rhs FP64 tuning), vs fp64_sps."""
    from paper_2503_16994_amd import lqcd
    res = {}
    pmap = {"f64": lqcd.F64, "f32": lqcd.F32, "bf16": lqcd.BF16}
    for name in precs:
        ip = pmap[name]
        # the FP64 tuning of the workspace stays the 12-rhs one of the f64
        # leg: the reliable updates of the mixed solves run in it
        tune, _ = lqcd.autotune(g, lqcd.dirac(kappa, csw), ip, 12, ws, stream=stream)

        def mstep():
            return lqcd.solve(g, etas, kappa, csw, tol=TOL, solver=lqcd.SOLVER_CG_EO, inner_prec=ip,
                              reliable_every=100, use_graph=True, ws=ws, stream=stream,
                              raise_on_noconv=False)
        mdt, r = timed(mstep, steps, warmup)
        rho = max(i["true_residual"] for i in r.info)
        sps = 12 / mdt
        res[name] = {"solves_per_s": round(sps, 2), "ms_per_12": round(mdt * 1e3, 2),
                     "vs_fp64_one_at_a_time": round(sps / fp64_sps, 3),
                     "converged": bool(r.status == 0 and rho <= TOL),
                     "iters": max(i["iters"] for i in r.info), "max_true_residual": rho,
                     "reliable_updates": max(i["reliable_updates"] for i in r.info), "tuning": tune}
        if name != "f64":
            res[name]["fp64_from"] = [i["fp64_from"] for i in r.info]
        log(f"12-rhs {tag} {name}: {res[name]}")
    return res


def c2_leg(stream, pm, gpm, mixed_leg):
    """16^3x32 propagator: 12 sources one at a time in FP64 (the benchmark
    step's tuning: cached gauge loads, direction split) vs 12 rhs per solve."""
    import torch

    from paper_2503_16994_amd import inputs, lqcd
    U2 = inputs.gauge_field(L_C2, EPS, seed=SEED)
    lat = lqcd.Lattice(L_C2, lqcd.BC_PERIODIC, THETA)
    g = lqcd.GaugeField(lat, torch.from_numpy(U2), gpm, stream=stream)
    del U2
    eta = torch.from_numpy(inputs.point_sources_12(L_C2, (0, 0, 0, 0))).cuda()
    psi = torch.empty_like(eta)
    ws1 = lqcd.Workspace(lat, pm, 1)
    lqcd.set_tuning(ws1, lqcd.F64, *STEP_TUNING)

    def one():
        return [lqcd.solve(g, eta[j:j + 1], KAPPA, CSW, tol=TOL, inner_prec=lqcd.F64, use_graph=True, ws=ws1,
                           stream=stream, psi=psi[j:j + 1]).info[0] for j in range(12)]
    dt, infos = timed(one, 5, 2)
    out = {"lattice": list(L_C2), "kappa": KAPPA,
           "fp64_one_at_a_time": {"solves_per_s": round(12 / dt, 2), "ms_per_12": round(dt * 1e3, 2),
                                  "iters": [i["iters"] for i in infos],
                                  "max_true_residual": max(i["true_residual"] for i in infos),
                                  "tuning": lqcd.get_tuning(ws1, lqcd.F64)}}
    log(f"16^3x32 FP64 one at a time: {out['fp64_one_at_a_time']}")
    del ws1
    ws12 = lqcd.Workspace(lat, pm, 12)
    out["multi_rhs_12"] = mixed_leg(stream, g, lat, ws12, eta, KAPPA, CSW, 12 / dt, 3, 1, "16^3x32")
    del ws12, g
    torch.cuda.empty_cache()
    return out


def c4_leg(stream, pm, gpm, mixed_leg, steps):
    """24^3x48 SF propagator: FP64 one source at a time vs mixed multi-RHS."""
    import torch

    from paper_2503_16994_amd import inputs, lqcd
    L4 = (24, 24, 24, 48)
    kappa, csw = 0.134, 1.8
    U4 = inputs.gauge_field(L4, EPS, seed=4, bc=lqcd.BC_SF)
    lat4 = lqcd.Lattice(L4, lqcd.BC_SF, (1, 1, 1, 1))
    g4 = lqcd.GaugeField(lat4, torch.from_numpy(U4), gpm, stream=stream)
    del U4
    eta4 = torch.from_numpy(inputs.point_sources_12(L4, (0, 0, 0, 1))).cuda()
    ws1 = lqcd.Workspace(lat4, pm, 1)
    lqcd.set_tuning(ws1, lqcd.F64, dir_split=True)
    lqcd.autotune(g4, lqcd.dirac(kappa, csw), lqcd.F64, 1, ws1, stream=stream)

    def fstep():
        return [lqcd.solve(g4, eta4[j:j + 1], kappa, csw, tol=TOL, inner_prec=lqcd.F64, use_graph=True,
                           ws=ws1, stream=stream).info[0] for j in range(12)]
    dt, infos = timed(fstep, steps, 1)
    fp64 = 12 / dt
    out = {"lattice": list(L4), "bc": "SF", "kappa": kappa, "csw": csw, "sources": "12 point at t=1",
           "fp64_one_at_a_time": {"solves_per_s": round(fp64, 2), "ms_per_12": round(dt * 1e3, 2),
                                  "iters": max(i["iters"] for i in infos),
                                  "max_true_residual": max(i["true_residual"] for i in infos)}}
    log(f"C4 FP64: {out['fp64_one_at_a_time']}")
    del ws1
    torch.cuda.empty_cache()
    ws12 = lqcd.Workspace(lat4, pm, 12)
    out["multi_rhs_12"] = mixed_leg(stream, g4, lat4, ws12, eta4, kappa, csw, fp64, steps, 1, "24^3x48 SF")
    del eta4
    # f_P, f_A: boundary source, 12-rhs FP64 solve, contraction (one call)
    t0 = time.perf_counter()
    fP, fA, H, infos = lqcd.sf_correlators(g4, kappa, csw, tol=TOL, inner_prec=lqcd.F64, use_graph=True,
                                           ws=ws12, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fP, fA = fP.real.cpu().numpy(), fA.real.cpu().numpy()
    out["sf_correlators"] = {"seconds": round(dt, 3), "iters": max(i["iters"] for i in infos),
                             "max_true_residual": max(i["true_residual"] for i in infos),
                             "x0": [1, 2, 12, 24, 36, 47],
                             "f_P": [float(fP[t]) for t in (1, 2, 12, 24, 36, 47)],
                             "f_A": [float(fA[t]) for t in (1, 2, 12, 24, 36, 47)]}
    log(f"SF f_P/f_A: {out['sf_correlators']}")
    del ws12, g4, H
    torch.cuda.empty_cache()
    return out


def c3_leg(stream, pm, g3, lat3, prop):
    """32^3x64: the hop kernels' HBM rates (one and 12 rhs, autotuned), the
    Z2-noise solve in FP64/FP32/BF16 inner precision (also with a twisted
    mass), and the meson contraction of the step's propagator `prop`."""
    import torch

    from paper_2503_16994_amd import inputs, lqcd
    L3 = tuple(lat3.L)
    kappa = KAPPA_STEP
    ws3 = lqcd.Workspace(lat3, pm, 1)
    d3 = lqcd.dirac(kappa, CSW)
    dw_hbm = {"lattice": list(L3)}
    for prec, pname in ((lqcd.F64, "f64"), (lqcd.F32, "f32"), (lqcd.BF16, "bf16")):
        lqcd.set_tuning(ws3, prec, dir_split=True)
        tune, _ = lqcd.autotune(g3, d3, prec, 1, ws3, stream=stream)
        for k, v in hop_rates(g3, lat3, ws3, d3, prec, 1, stream).items():
            dw_hbm[f"{k}_{pname}"] = dict(v, tuning=tune)
    log(f"dw_hbm: {dw_hbm}")
    c3 = {"lattice": list(L3), "kappa": kappa, "csw": CSW, "source": "Z2 complex noise"}
    eta3 = torch.from_numpy(inputs.z2_noise(L3, seed=3)).cuda()
    precs = ((lqcd.F64, "f64"), (lqcd.F32, "f32"), (lqcd.BF16, "bf16"))
    for ip, name in precs:
        def s3():
            return lqcd.solve(g3, eta3, kappa, CSW, tol=TOL, inner_prec=ip, reliable_every=100, use_graph=True,
                              ws=ws3, stream=stream, raise_on_noconv=False)
        dt, r = timed(s3, 2, 1)
        c3[name] = {"seconds": round(dt, 4), "iters": r.info[0]["iters"],
                    "reliable_updates": r.info[0]["reliable_updates"],
                    "true_residual": r.info[0]["true_residual"], "status": r.status}
        if name != "f64":
            c3[name]["vs_fp64"] = round(c3["f64"]["seconds"] / dt, 3)
    # twisted mass D(mu) = Dw + i mu g5, same source
    c3["twisted"] = {"mu": TM_MU}
    for ip, name in precs:
        def s3m():
            return lqcd.solve(g3, eta3, kappa, CSW, tol=TOL, inner_prec=ip, reliable_every=100, use_graph=True,
                              ws=ws3, stream=stream, raise_on_noconv=False, mu=TM_MU)
        dt, r = timed(s3m, 2, 1)
        c3["twisted"][name] = {"seconds": round(dt, 4), "iters": r.info[0]["iters"],
                               "true_residual": r.info[0]["true_residual"], "status": r.status}
        if name != "f64":
            c3["twisted"][name]["vs_fp64"] = round(c3["twisted"]["f64"]["seconds"] / dt, 3)
    d3m = lqcd.dirac(kappa, CSW, 1.0, TM_MU)
    for k, v in hop_rates(g3, lat3, ws3, d3m, lqcd.F64, 1, stream).items():
        dw_hbm[f"{k}_f64_twisted"] = dict(v, tuning=lqcd.get_tuning(ws3, lqcd.F64))
    log(f"C3: {c3}")
    del eta3
    # meson two-point functions of the step's propagator (16 diagonal Gamma pairs)
    pairs = [(m, m) for m in range(16)]
    ms_meson = time_launches(lambda: lqcd.meson(lat3, prop, pairs, ws3, stream=stream), 10, stream)
    C, _ = lqcd.meson(lat3, prop, pairs, ws3, want_G=False, stream=stream)
    torch.cuda.synchronize()
    mb = 12 * 12 * 16 * lat3.volume  # the propagator, read once
    c3["meson"] = {"us": round(ms_meson * 1e3, 1), "alg_bytes": mb,
                   "GB/s": round(mb / (ms_meson * 1e-3) / 1e9, 1),
                   "frac": round(mb / (ms_meson * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "pion_t0_t1_tmid": [float(C[15, 0].real), float(C[15, 1].real), float(C[15, 32].real)]}
    log(f"meson: {c3['meson']}")
    del C, ws3
    torch.cuda.empty_cache()
    # the hop kernels with 12 rhs, each precision autotuned
    ws12 = lqcd.Workspace(lat3, pm, 12)
    for prec, pname in ((lqcd.F64, "f64"), (lqcd.F32, "f32"), (lqcd.BF16, "bf16")):
        tune, _ = lqcd.autotune(g3, d3, prec, 12, ws12, stream=stream)
        for k, v in hop_rates(g3, lat3, ws12, d3, prec, 12, stream, reps=10).items():
            dw_hbm[f"{k}_{pname}_12rhs"] = dict(v, tuning=tune)
    log(f"dw_hbm with 12 rhs: { {k: v for k, v in dw_hbm.items() if k.endswith('12rhs')} }")
    del ws12
    torch.cuda.empty_cache()
    return c3, dw_hbm


def ctx_leg(stream, gpm):
    """The shape of the paper's CG timing: 1000 FP64 full-lattice CG
    iterations on a 32^4 lattice (periodic space, antiperiodic time, one
    point source).  Context only: the paper's fields, parameters and
    boundary conditions are not stated."""
    import torch

    from paper_2503_16994_amd import inputs, lqcd
    L = (32, 32, 32, 32)
    U = inputs.gauge_field(L, EPS, seed=5)
    lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, THETA)
    g = lqcd.GaugeField(lat, torch.from_numpy(U), gpm, stream=stream)
    del U
    ws = lqcd.Workspace(lat, lqcd.PM_F64, 1)
    eta = torch.from_numpy(inputs.point_source(L)[None]).cuda()
    lqcd.set_tuning(ws, lqcd.F64, dir_split=True)
    lqcd.autotune(g, lqcd.dirac(KAPPA, CSW), lqcd.F64, 1, ws, stream=stream)

    def run():
        return lqcd.solve(g, eta, KAPPA, CSW, tol=1e-30, solver=lqcd.SOLVER_CG_FULL, maxiter=1000,
                          use_graph=True, ws=ws, stream=stream, raise_on_noconv=False)
    dt, r = timed(run, 1, 1)
    out = {"lattice": list(L), "solver": "FP64 full-lattice CG on Dw^+Dw", "iterations": r.info[0]["iters"],
           "seconds": round(dt, 3), "ms_per_iteration": round(dt / r.info[0]["iters"] * 1e3, 3),
           "paper_context": {"A100_s": 13.9, "H100_s": 6.46,
                             "note": "1000 CG iterations at L/a=32 (paper Sec. 3.4 table); fields and "
                                     "parameters differ"}}
    log(f"ctx: {out}")
    del g, ws
    torch.cuda.empty_cache()
    return out


SERVE_LATS = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]


def serve_legs(n_requests, rate):
    """The serving loop on the C5 mix: gauge fields {8^4, 16^3x32, 24^3x48,
    32^3x64} x {open, periodic/antiperiodic} resident in the arena, kernels
    autotuned for every (field, FP32 inner, 1 or 12 rhs) before the first
    request (lqcd_server_warmup; requests never tune), then a Poisson stream
    of n_requests at `rate`, then 20 requests at 0.7x the capacity measured in
    the first run."""
    import numpy as np

    from paper_2503_16994_amd import inputs, lqcd
    pm = lqcd.PM_F64 | lqcd.PM_F32 | lqcd.PM_TWO_ROW
    srv = lqcd.Server(200 << 30, max_streams=4)
    gids, etas = {}, {}
    t0 = time.perf_counter()
    for i, L in enumerate(SERVE_LATS):
        U = inputs.gauge_field(L, EPS, seed=50 + i)
        gids[(L, lqcd.BC_PERIODIC)] = srv.add_gauge(L, lqcd.BC_PERIODIC, THETA, U, pm)
        gids[(L, lqcd.BC_OPEN)] = srv.add_gauge(L, lqcd.BC_OPEN, (1, 1, 1, 1), U, pm)
        del U
        src = inputs.point_sources_12(L, (0, 0, 0, 0))
        etas[(L, 12)] = (src, np.empty_like(src))
        etas[(L, 1)] = (src[:1].copy(), np.empty_like(src[:1]))
    t_fields = time.perf_counter() - t0
    t0 = time.perf_counter()
    for gid in gids.values():
        for nrhs in (1, 12):
            srv.warmup(gid, lqcd.F32, nrhs)
    t_tune = time.perf_counter() - t0
    log(f"serving: {len(gids)} gauge fields in {t_fields:.1f} s, warm-up tuning {t_tune:.1f} s")
    out = {"setup": {"gauge_fields": len(gids), "import_s": round(t_fields, 2), "warmup_tuning_s": round(t_tune, 2),
                     "note": "kernels tuned per (field, precision, rhs count) before the first request"}}
    out["offered"] = serve_run(srv, gids, etas, n_requests, rate, seed=99)
    cap = out["offered"]["requests_per_s"]
    out["at_0.7_capacity"] = serve_run(srv, gids, etas, 20, 0.7 * cap, seed=98)
    out["peak_arena_gib"] = round(srv.peak_bytes() / 2**30, 2)
    srv.close()
    return out


def serve_run(srv, gids, etas, n_requests, rate, seed):
    """Poisson stream of propagator requests through lqcd_submit/lqcd_poll:
    lattice and boundary type uniform over the resident fields, kappa uniform
    in [0.125, 0.136], csw 1.9, 1 or 12 point sources, FP32 inner precision.
    Latency = completion - submission (server clock); requests are submitted
    at their arrival times."""
    import numpy as np

    from paper_2503_16994_amd import lqcd
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, n_requests)
    reqs = []
    for k in range(n_requests):
        L = SERVE_LATS[int(rng.integers(0, 4))]
        bc = lqcd.BC_OPEN if rng.integers(0, 2) else lqcd.BC_PERIODIC
        kappa = float(rng.uniform(0.125, 0.136))
        nrhs = 12 if rng.integers(0, 2) else 1
        reqs.append((L, bc, kappa, nrhs))
    t0 = time.perf_counter()
    arrival = np.cumsum(gaps)
    tickets = []
    for k, (L, bc, kappa, nrhs) in enumerate(reqs):
        wait = arrival[k] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        p = lqcd.Server.params(kappa, 1.9, tol=TOL, inner_prec=lqcd.F32, nrhs=nrhs)
        e, ps = etas[(L, nrhs)]
        tickets.append(srv.submit(gids[(L, bc)], p, e, ps))
    done = {}
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
                    if len(done) % 10 == 0:
                        log(f"serving: {len(done)}/{len(tickets)} requests done "
                            f"({time.perf_counter() - t0:.1f} s)")
        time.sleep(0.001)
    wall = time.perf_counter() - t0
    lat_s = np.array([done[t][2][2] - done[t][2][0] for t in tickets])
    wait_s = np.array([done[t][2][1] - done[t][2][0] for t in tickets])
    svc_s = np.array([done[t][2][2] - done[t][2][1] for t in tickets])
    ok = sum(1 for t in tickets if done[t][0] == lqcd.OK)
    nsolves = sum(r[3] for r in reqs)
    worst = max(i["true_residual"] for t in tickets for i in done[t][1])
    out = {"requests": n_requests, "rate_per_s": round(rate, 3), "ok": ok, "solves": int(nsolves),
           "p50_latency_s": round(float(np.percentile(lat_s, 50)), 4),
           "p99_latency_s": round(float(np.percentile(lat_s, 99)), 4),
           "mean_admission_wait_s": round(float(wait_s.mean()), 4),
           "mean_service_s": round(float(svc_s.mean()), 4),
           "solves_per_s": round(nsolves / wall, 2), "requests_per_s": round(n_requests / wall, 3),
           "wall_s": round(wall, 3), "max_true_residual": worst,
           "statuses": sorted(set(int(done[t][0]) for t in tickets)),
           "fp64_continuations": int(sum(1 for t in tickets for i in done[t][1] if i["fp64_from"] > 0))}
    log(f"serving: {out}")
    return out


def step_tunings(g, ws12, ws1, stream):
    """The tunings of the step's kernels: from the committed tuning table of
    this GPU if it has them (so that the profiled launches and the bench use
    the same configuration), else autotuned (and added to the process cache)."""
    from paper_2503_16994_amd import lqcd
    d = lqcd.dirac(KAPPA_STEP, CSW)
    out = {}
    for ws, prec, nrhs, split in ((ws12, lqcd.BF16, 12, False), (ws12, lqcd.F32, 12, False),
                                  (ws1, lqcd.F64, 1, True)):
        if ws is None:
            continue
        t = lqcd.tune_cache_find(g, prec, nrhs, dir_split=split)
        if t is None:
            lqcd.set_tuning(ws, prec, dir_split=split)
            t, _ = lqcd.autotune(g, d, prec, nrhs, ws, stream=stream)
        out[(prec, nrhs)] = t
    return out


def profile_kernels(stream):
    """Launch sequence for rocprofv3 runs: a plain 1 GiB device copy (to
    calibrate FETCH_SIZE/WRITE_SIZE against known bytes, and the copy rate), a
    1 GiB fill and a 1 GiB read-only sum, then, at 32^3x64 on two-row links in
    the step's tunings (the committed tuning table), 20 launches of each hop
    kernel of the step and its baseline: BF16 and FP32 with 12 rhs, FP64 with
    one rhs (e->o, then o->e, then the full-lattice Dw); then 10 meson
    contractions of a random 12-column field."""
    import torch

    from paper_2503_16994_amd import inputs, lqcd

    n = 1 << 30
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    for _ in range(3):
        b.fill_(1.0)
    for _ in range(3):
        a.sum()
    torch.cuda.synchronize()
    del a, b
    load_tuning_table()
    pm = lqcd.PM_F64 | lqcd.PM_F32 | lqcd.PM_BF16
    L = L_STEP
    U = inputs.gauge_field(L, EPS, seed=SEED_STEP)
    lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, THETA)
    g = lqcd.GaugeField(lat, torch.from_numpy(U), pm | lqcd.PM_TWO_ROW, stream=stream)
    del U
    d = lqcd.dirac(KAPPA_STEP, CSW)
    ws12 = lqcd.Workspace(lat, pm, 12)
    ws1 = lqcd.Workspace(lat, pm, 1)
    tunes = step_tunings(g, ws12, ws1, stream)
    for (prec, nrhs), t in tunes.items():
        ws = ws12 if nrhs == 12 else ws1
        lqcd.set_tuning(ws, prec, **t)
        x, y = internal_vectors(lat, prec, nrhs)
        # the two hops, then (FP64, one rhs) the full-lattice Dw of the
        # residual checks
        ops = (lqcd.OP_HOP_EO, lqcd.OP_HOP_OE) + ((lqcd.OP_DW,) if prec == lqcd.F64 else ())
        for op in ops:
            for _ in range(20):
                lqcd.dw_apply_internal(g, d, x, y, op, prec, nrhs, ws, stream=stream)
        torch.cuda.synchronize()
        log(f"profiled {L} {PREC_NAME[prec]} nrhs {nrhs} tuning {t}")
        del x, y
    shape = (12,) + lat.spinor_shape()
    prop = torch.complex(torch.randn(shape, dtype=torch.float64, device="cuda"),
                         torch.randn(shape, dtype=torch.float64, device="cuda"))
    for _ in range(10):
        lqcd.meson(lat, prop, [(m, m) for m in range(16)], ws1, want_G=False, stream=stream)
    torch.cuda.synchronize()
    log(f"profiled meson {L}")


TUNING_TABLE = os.path.join(ROOT, "paper_2503_16994_amd", "tuning", "gfx950.txt")


def load_tuning_table():
    from paper_2503_16994_amd import lqcd
    if os.path.exists(TUNING_TABLE):
        lqcd.tune_cache_load(TUNING_TABLE)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(U):
    """Oracle (plain FP64 full-lattice Dw and CG, OpenMP over sites) on the
    host, on a bounded sample of the step's workload (32^3x64, kappa 0.135):
    one clover build, a few Dw applications (full-Dw GB/s in the 1536 B/site
    FP64 model: psi 24 + U 72 + A 72 + out 24 reals) and ~10 s of CG
    iterations on the first point source; scaled to 12 solves x the oracle's
    own iteration count to 1e-10 (oracle/c3_reference.json)."""
    from oracle import oracle as orc
    from paper_2503_16994_amd import inputs

    L = L_STEP
    with open(os.path.join(ROOT, "oracle", "c3_reference.json")) as f:
        ref = json.load(f)
    assert tuple(ref["lattice"]) == L and ref["kappa"] == KAPPA_STEP
    n_iter = int(ref["iterations"])
    t0 = time.perf_counter()
    A = orc.clover_matrix(L, orc.PERIODIC, U, orc.m0_from_kappa(KAPPA_STEP), CSW)
    t_clover = time.perf_counter() - t0
    eta = inputs.point_source(L, (0, 0, 0, 0), 0, 0)
    t0 = time.perf_counter()
    nd = 3
    for _ in range(nd):
        orc.dw(L, orc.PERIODIC, THETA, U, A, eta)
    t_dw = (time.perf_counter() - t0) / nd
    V = L[0] * L[1] * L[2] * L[3]
    done_iters, t_cg = 0, 0.0
    while t_cg < 10.0 and done_iters < 100:
        t0 = time.perf_counter()
        orc.cg_fixed(L, orc.PERIODIC, THETA, U, A, eta, 2)
        t_cg += time.perf_counter() - t0
        done_iters += 2
    t_iter = t_cg / done_iters
    t_step = t_clover + 12 * n_iter * t_iter
    return {"value": round(12 / t_step, 5), "unit": "solves/s", "cores": orc.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"one clover build ({t_clover:.1f} s), {nd} full Dw applications and {done_iters} "
                      f"full-lattice FP64 CG iterations ({t_cg:.1f} s) on source (0,0,0,0; s0,c0) of the "
                      f"32^3x64 step workload; scaled to 12 solves x {n_iter} iterations (the oracle's own "
                      f"count to 1e-10, oracle/c3_reference.json)",
            "s_per_cg_iter": round(t_iter, 4), "dw_full_s": round(t_dw, 4),
            "dw_full_GBps": round(1536 * V / t_dw / 1e9, 2)}


if __name__ == "__main__":
    main()
