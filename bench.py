#!/usr/bin/env python
"""Benchmark of the Wilson-clover propagator solve on one MI355X.

Workload of the timed step (the value): the 16^3x32 propagator -- links
exp(i 0.2 H) (Gaussian traceless Hermitian H, seed 2), periodic space /
antiperiodic time, kappa = 0.1345, csw = 1.9, the 12 spin-colour point
sources at the origin solved one at a time with the FP64 even-odd
preconditioned CG to a true relative residual of 1e-10.  Each solve runs the
whole path: clover term (built once per gauge field and parameters, then
cached), source preparation, CG on Dhat^+ Dhat in hipGraph chunks, odd-site
reconstruction and the FP64 full-lattice residual check.  Inputs are
resident in HBM before the timed region.

The JSON line (stdout) also carries
* "mixed": the same 12 sources as one multi-RHS solve, FP32 or BF16 inner
  precision with FP64 reliable updates (autotuned kernels), vs FP64;
* "mixed_c4": the 24^3x48 Schroedinger-functional propagator (kappa 0.134,
  csw 1.8, 12 point sources at t = 1), FP64 one source at a time vs one
  multi-RHS mixed solve;
* "c3": the 32^3x64 Z2-noise solve (kappa 0.135) in FP64, FP32 and BF16 inner
  precision;
* "roofline": the dominant kernel of the step (the FP64 odd->even hop with
  the clover block), algorithmic bytes per launch / average launch time
  (100 launches replayed from one graph, HIP events on its stream);
* "dw_hbm": the hop kernels at 32^3x64 (working set > 1 GB, beyond the 256 MB
  last-level cache) in FP64/FP32/BF16;
* "serving": a Poisson stream of mixed propagator requests through the
  serving loop, p50/p99 latency and solves/s (with --serve-full also a run at
  0.7x the measured capacity, where the latencies describe the service and
  not a growing backlog);
* "cpu_baseline": the FP64 CPU oracle on a bounded sample.

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
L_C2 = (16, 16, 16, 32)
KAPPA, CSW, EPS, SEED, TOL = 0.1345, 1.9, 0.2, 2, 1e-10
THETA = (1, 1, 1, -1)
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


BYTES_PER_REAL = {0: 8, 1: 4, 2: 2}
# the dominant kernel: the FP64 o->e hop with the clover block, direction split
DOMINANT_KERNEL = "k_hop<double2,double2,double2,PRE_CLOV,POST_NONE,HOP,1,1,SPLIT>"
# hop tuning of the benchmark step and of its roofline measurement
# (nr_tile, block_order, rhs_lanes, nt_store, cached_gauge, occ_cap,
# dir_split): cached gauge loads keep links and clover in the last-level
# cache, which holds this lattice's whole working set; the direction split
# gives the 65536 sites of a parity two waves each
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


def stored_traffic(name, tuning=None):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel source in the same tuning."""
    path = os.path.join(ROOT, "profiles", "hop_oe_fp64_16x16x16x32_counters.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != name:
        return None
    if tuning is not None and d.get("tuning") != tuning:
        return None
    return d.get("hbm_bytes_per_launch")


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
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-hbm", action="store_true", help="skip the 32^3x64 legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision legs")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=16)
    ap.add_argument("--serve-full", action="store_true",
                    help="longer serving run: 60 requests at the offered rate, then 20 at 0.7x the measured capacity")
    ap.add_argument("--serve-rate", type=float, default=50.0, help="mean arrivals per second")
    ap.add_argument("--profile-kernel", action="store_true",
                    help="only calibration copy/sum and hop-kernel launches (profiler runs)")
    args = ap.parse_args()
    if args.serve_full and args.serve_requests == 16:
        args.serve_requests = 60
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
    pm = lqcd.PM_F64 | lqcd.PM_F32 | lqcd.PM_BF16
    gpm = pm | (lqcd.PM_TWO_ROW if TWO_ROW else 0)  # gauge fields

    # ---- the step: 16^3x32, 12 sources, FP64 eo-CG one at a time -------------
    U2 = inputs.gauge_field(L_C2, EPS, seed=SEED)
    lat = lqcd.Lattice(L_C2, lqcd.BC_PERIODIC, THETA)
    gauge = lqcd.GaugeField(lat, torch.from_numpy(U2), gpm, stream=stream)
    eta = torch.from_numpy(inputs.point_sources_12(L_C2, (0, 0, 0, 0))).cuda()
    psi = torch.empty_like(eta)
    ws1 = lqcd.Workspace(lat, pm, 1)
    ws12 = lqcd.Workspace(lat, pm, 12)
    d = lqcd.dirac(KAPPA, CSW)
    lqcd.set_tuning(ws1, lqcd.F64, *STEP_TUNING)
    tune64 = lqcd.get_tuning(ws1, lqcd.F64)
    torch.cuda.synchronize()

    def step():
        out = []
        for j in range(12):
            r = lqcd.solve(gauge, eta[j:j + 1], KAPPA, CSW, tol=TOL, solver=lqcd.SOLVER_CG_EO,
                           inner_prec=lqcd.F64, use_graph=True, ws=ws1, stream=stream,
                           psi=psi[j:j + 1])
            out.append(r.info[0])
        return out

    dt, infos = timed(step, args.steps, args.warmup)
    ms_step = dt * 1e3
    value = 12 / dt
    rho_max = max(i["true_residual"] for i in infos)
    iters = [i["iters"] for i in infos]
    assert all(i["status"] == 0 for i in infos) and rho_max <= TOL, infos
    log(f"FP64 eo-CG 16^3x32: {ms_step:.2f} ms / 12 solves, {value:.1f} solves/s, iters {iters}, "
        f"max rho {rho_max:.2e}, tuning {tune64}")

    # ---- roofline of the dominant kernel (FP64 odd->even hop + clover) -------
    vb = lqcd.vec_bytes(lat, lqcd.F64, 1, 2)
    vin = (torch.randn(vb // 8, device="cuda", dtype=torch.float64)).view(torch.uint8)
    vout = torch.empty(vb, dtype=torch.uint8, device="cuda")

    tune_roof = lqcd.get_tuning(ws1, lqcd.F64)  # the step's configuration

    def hop_oe():
        lqcd.dw_apply_internal(gauge, d, vin, vout, lqcd.OP_HOP_OE, lqcd.F64, 1, ws1, stream=stream)

    # 100 launches captured in one graph: at this size a launch (~25 us) is
    # shorter than a call through Python, so eager launches would time the host
    for _ in range(3):
        hop_oe()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for _ in range(ROOFLINE_LAUNCHES):
            hop_oe()
    graph.replay()
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    graph.replay()
    e1.record(stream)
    e1.synchronize()
    ms_oe = e0.elapsed_time(e1) / ROOFLINE_LAUNCHES
    del graph
    alg_bytes = hop_reals("hop_oe", 1, TWO_ROW) * BYTES_PER_REAL[0] * lat.volume
    achieved = alg_bytes / (ms_oe * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": stored_traffic(DOMINANT_KERNEL, tune_roof),
                "kernel": DOMINANT_KERNEL, "avg_launch_us": round(ms_oe * 1e3, 2),
                "alg_bytes_per_launch": alg_bytes, "tuning": tune_roof,
                "links": "two rows per link" if TWO_ROW else "full",
                "note": "16^3x32 working set (~130 MB) fits the 256 MB last-level cache; "
                        "HBM-resident figures in dw_hbm"}
    log(f"roofline: {roofline}")
    del vin, vout

    # ---- mixed precision, 12 rhs in one solve ---------------------------------
    def mixed_leg(g, lat_, ws, etas, kappa, csw, fp64_sps, steps, warmup, tag, precs=("f64", "f32", "bf16"),
                  hbm=None):
        """12 rhs in one solve per inner precision (autotuned kernels); with a
        dict `hbm`, also the 12-rhs hop-kernel rates in each precision."""
        res = {}
        pmap = {"f64": lqcd.F64, "f32": lqcd.F32, "bf16": lqcd.BF16}
        for name in precs:
            ip = pmap[name]
            tune, _ = lqcd.autotune(g, lqcd.dirac(kappa, csw), ip, 12, ws, stream=stream)
            if ip != lqcd.F64:
                # the FP64 hops of the reliable updates run one rhs per thread:
                # with the direction split they are ~25% faster
                t64 = lqcd.get_tuning(ws, lqcd.F64)
                t64["dir_split"] = True
                lqcd.set_tuning(ws, lqcd.F64, **t64)
            if hbm is not None:
                for k, v in hop_rates(g, lat_, ws, lqcd.dirac(kappa, csw), ip, 12, stream).items():
                    hbm[f"{k}_{name}_12rhs"] = dict(v, tuning=tune)

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

    mixed = mixed_c4 = c3 = dw_hbm = serving = None
    if not args.no_mixed:
        mixed = mixed_leg(gauge, lat, ws12, eta, KAPPA, CSW, value, args.steps, args.warmup, "16^3x32")
        del ws12
        torch.cuda.empty_cache()
        mixed_c4 = c4_leg(stream, pm, gpm, mixed_leg, 1)

    # ---- 32^3x64: Z2 solve, 12-source propagator and the kernels' HBM rates --
    ctx = None
    if not args.no_hbm:
        c3, dw_hbm = c3_leg(stream, pm, gpm, args.no_mixed, mixed_leg)
        ctx = ctx_leg(stream, gpm & (lqcd.PM_F64 | lqcd.PM_TWO_ROW))

    # ---- serving -------------------------------------------------------------
    if not args.no_serve:
        serving = {"offered": serve_leg(args.serve_requests, args.serve_rate, U2)}
        if args.serve_full:
            cap = serving["offered"]["requests_per_s"]
            serving["at_0.7_capacity"] = serve_leg(20, 0.7 * cap, U2, seed=98)

    # ---- CPU oracle baseline (bounded sample) ----------------------------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline()
        log(f"cpu_baseline: {cpu}")

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "16^3x32 Wilson-clover propagator: 12 point sources solved one at a "
                               "time, FP64 even-odd CG, tol 1e-10",
                   "lattice": list(L_C2), "kappa": KAPPA, "csw": CSW, "bc": "periodic/antiperiodic",
                   "link_eps": EPS, "sources": 12, "tol": TOL, "solver": "eo-CG FP64, hipGraph chunks",
                   "links": "two rows per link (third rebuilt in registers)" if TWO_ROW else "full",
                   "hop_tuning": tune64},
        "iters_per_solve": iters, "max_true_residual": rho_max,
        "roofline": roofline, "mixed": mixed, "mixed_c4": mixed_c4, "c3": c3, "dw_hbm": dw_hbm, "ctx": ctx,
        "serving": serving, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


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
    out["multi_rhs_12"] = mixed_leg(g4, lat4, ws12, eta4, kappa, csw, fp64, steps, 1, "24^3x48 SF")
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


def c3_leg(stream, pm, gpm, no_mixed, mixed_leg):
    """32^3x64: Z2-noise solve in FP64/FP32/BF16, the 12-source propagator
    (FP64 one source at a time vs 12 rhs in one solve) and the hop kernels'
    HBM rates."""
    import torch

    from paper_2503_16994_amd import inputs, lqcd
    L3 = (32, 32, 32, 64)
    kappa = 0.135
    U3 = inputs.gauge_field(L3, EPS, seed=3)
    lat3 = lqcd.Lattice(L3, lqcd.BC_PERIODIC, THETA)
    g3 = lqcd.GaugeField(lat3, torch.from_numpy(U3), gpm, stream=stream)
    del U3
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
    precs = ((lqcd.F64, "f64"),) if no_mixed else ((lqcd.F64, "f64"), (lqcd.F32, "f32"), (lqcd.BF16, "bf16"))
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
    # 12 point sources at the origin: FP64 one at a time, then 12 rhs per solve
    etap = torch.from_numpy(inputs.point_sources_12(L3, (0, 0, 0, 0))).cuda()
    lqcd.autotune(g3, d3, lqcd.F64, 1, ws3, stream=stream)

    prop = torch.empty_like(etap)

    def f64_one():
        return [lqcd.solve(g3, etap[j:j + 1], kappa, CSW, tol=TOL, inner_prec=lqcd.F64, use_graph=True, ws=ws3,
                           stream=stream, psi=prop[j:j + 1]).info[0] for j in range(12)]
    dt, infos = timed(f64_one, 1, 1)
    fp64 = 12 / dt
    c3["propagator_12"] = {"fp64_one_at_a_time": {"solves_per_s": round(fp64, 2), "ms_per_12": round(dt * 1e3, 1),
                                                  "iters": max(i["iters"] for i in infos),
                                                  "max_true_residual": max(i["true_residual"] for i in infos)}}
    # meson two-point functions of that propagator (16 diagonal Gamma pairs)
    pairs = [(m, m) for m in range(16)]
    ms_meson = time_launches(lambda: lqcd.meson(lat3, prop, pairs, ws3, stream=stream), 10, stream)
    C, _ = lqcd.meson(lat3, prop, pairs, ws3, want_G=False, stream=stream)
    torch.cuda.synchronize()
    mb = 12 * 12 * 16 * lat3.volume  # the propagator, read once
    c3["propagator_12"]["meson"] = {"us": round(ms_meson * 1e3, 1), "alg_bytes": mb,
                                    "GB/s": round(mb / (ms_meson * 1e-3) / 1e9, 1),
                                    "frac": round(mb / (ms_meson * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                    "pion_t0_t1_tmid": [float(C[15, 0].real), float(C[15, 1].real),
                                                        float(C[15, 32].real)]}
    log(f"meson: {c3['propagator_12']['meson']}")
    del prop, C
    del ws3
    torch.cuda.empty_cache()
    if not no_mixed:
        ws12 = lqcd.Workspace(lat3, pm, 12)
        c3["propagator_12"]["multi_rhs_12"] = mixed_leg(g3, lat3, ws12, etap, kappa, CSW, fp64, 1, 1, "32^3x64",
                                                        hbm=dw_hbm)
        log(f"dw_hbm with 12 rhs: { {k: v for k, v in dw_hbm.items() if k.endswith('12rhs')} }")
        del ws12
    log(f"C3 propagator: {c3['propagator_12']}")
    del g3, etap
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


def serve_leg(n_requests, rate, U16, seed=99):
    """Poisson stream of propagator requests through lqcd_submit/lqcd_poll:
    lattices {8^4, 16^3x32, 24^3x48, 32^3x64} x {open, periodic}, kappa uniform
    in [0.125, 0.136], csw 1.9, 1 or 12 point sources, FP32 inner precision,
    gauge fields resident.  Latency = completion - submission (server clock);
    requests are submitted at their arrival times."""
    import numpy as np

    from paper_2503_16994_amd import inputs, lqcd
    lats = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]
    pm = lqcd.PM_F64 | lqcd.PM_F32
    srv = lqcd.Server(200 << 30, max_streams=4)
    gids = {}
    etas = {}
    for i, L in enumerate(lats):
        U = U16 if L == L_C2 else inputs.gauge_field(L, EPS, seed=50 + i)
        gpm = pm | (lqcd.PM_TWO_ROW if TWO_ROW else 0)
        gids[(L, lqcd.BC_PERIODIC)] = srv.add_gauge(L, lqcd.BC_PERIODIC, THETA, U, gpm)
        gids[(L, lqcd.BC_OPEN)] = srv.add_gauge(L, lqcd.BC_OPEN, (1, 1, 1, 1), U, gpm)
        del U
        src = inputs.point_sources_12(L, (0, 0, 0, 0))
        etas[(L, 12)] = (src, np.empty_like(src))
        etas[(L, 1)] = (src[:1].copy(), np.empty_like(src[:1]))
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, n_requests)
    reqs = []
    for k in range(n_requests):
        L = lats[int(rng.integers(0, 4))]
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
    ok = sum(1 for t in tickets if done[t][0] == lqcd.OK)
    nsolves = sum(r[3] for r in reqs)
    peak = srv.peak_bytes()
    srv.close()
    out = {"requests": n_requests, "rate_per_s": rate, "ok": ok, "solves": int(nsolves),
           "p50_latency_s": round(float(np.percentile(lat_s, 50)), 4),
           "p99_latency_s": round(float(np.percentile(lat_s, 99)), 4),
           "mean_admission_wait_s": round(float(wait_s.mean()), 4),
           "solves_per_s": round(nsolves / wall, 2), "requests_per_s": round(n_requests / wall, 3),
           "wall_s": round(wall, 3), "peak_arena_gib": round(peak / 2**30, 2),
           "statuses": sorted(set(int(done[t][0]) for t in tickets)),
           "fp64_continuations": int(sum(1 for t in tickets for i in done[t][1] if i["fp64_from"] > 0))}
    log(f"serving: {out}")
    return out


def profile_kernels(stream):
    """Launch sequence for rocprofv3 runs: a plain 1 GiB device copy (to
    calibrate FETCH_SIZE/WRITE_SIZE against known bytes, and the copy rate), a
    1 GiB read-only sum (read rate), then 20 launches of each hop kernel, all
    on two-row links: FP64 at 16^3x32 and at 32^3x64, FP32 and BF16 at
    32^3x64 (one rhs), and FP32 with 12 rhs at 32^3x64 (rhs tile 3); at
    16^3x32 in the benchmark step's tuning, at 32^3x64 with block order 2,
    non-temporal stores and (one rhs) the direction split; then 10 meson
    contractions of a random 12-column field at 32^3x64."""
    import torch

    from paper_2503_16994_amd import inputs, lqcd

    n = 1 << 30
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    for _ in range(3):
        a.sum()
    torch.cuda.synchronize()
    del a, b
    pm = lqcd.PM_F64 | lqcd.PM_F32 | lqcd.PM_BF16
    for L in (L_C2, (32, 32, 32, 64)):
        big = L[3] == 64
        U = inputs.gauge_field(L, EPS, seed=SEED)
        lat = lqcd.Lattice(L, lqcd.BC_PERIODIC, THETA)
        g = lqcd.GaugeField(lat, torch.from_numpy(U), (pm if big else lqcd.PM_F64) | lqcd.PM_TWO_ROW,
                            stream=stream)
        del U
        nr = 12 if big else 1
        ws = lqcd.Workspace(lat, pm if big else lqcd.PM_F64, nr)
        d = lqcd.dirac(KAPPA, CSW)
        # (nr_tile, block_order, rhs_lanes, nt_store, cached_gauge, occ_cap, dir_split)
        one = (1, 2, 1, True, False, 0, True)
        cases = [(lqcd.F64, 1, STEP_TUNING if not big else one)]
        if big:
            cases += [(lqcd.F32, 1, one), (lqcd.BF16, 1, one), (lqcd.F32, 12, (3, 2, 1, True))]
        for prec, nrhs, tune in cases:
            lqcd.set_tuning(ws, prec, *tune)
            vb = lqcd.vec_bytes(lat, prec, nrhs, 2)
            if prec == lqcd.BF16:
                x = torch.randn(vb // 2, device="cuda").to(torch.bfloat16).view(torch.uint8)
            else:
                x = torch.randn(vb // 4, device="cuda").view(torch.uint8)
            y = torch.empty(vb, dtype=torch.uint8, device="cuda")
            for op in (lqcd.OP_HOP_OE, lqcd.OP_HOP_EO):
                for _ in range(20):
                    lqcd.dw_apply_internal(g, d, x, y, op, prec, nrhs, ws, stream=stream)
            torch.cuda.synchronize()
            log(f"profiled {L} prec {prec} nrhs {nrhs} tuning {tune}")
            del x, y
        if big:  # meson contraction of a 12-column field, 16 diagonal pairs
            shape = (12,) + lat.spinor_shape()
            prop = torch.complex(torch.randn(shape, dtype=torch.float64, device="cuda"),
                                 torch.randn(shape, dtype=torch.float64, device="cuda"))
            for _ in range(10):
                lqcd.meson(lat, prop, [(m, m) for m in range(16)], ws, want_G=False, stream=stream)
            torch.cuda.synchronize()
            log(f"profiled meson {L}")
            del prop
        del g, ws
        torch.cuda.empty_cache()


def cpu_baseline():
    """Oracle (plain FP64 full-lattice CG, OpenMP over sites) on the host."""
    from oracle import oracle as orc
    from paper_2503_16994_amd import inputs

    ref_path = os.path.join(ROOT, "oracle", "c2_reference.json")
    with open(ref_path) as f:
        ref = json.load(f)
    n_iter = int(ref["iterations"])
    U = inputs.gauge_field(L_C2, EPS, seed=SEED)
    t0 = time.perf_counter()
    A = orc.clover_matrix(L_C2, orc.PERIODIC, U, orc.m0_from_kappa(KAPPA), CSW)
    t_clover = time.perf_counter() - t0
    eta = inputs.point_source(L_C2, (0, 0, 0, 0), 0, 0)
    done_iters, t_cg = 0, 0.0
    while t_cg < 10.0 and done_iters < 200:
        t0 = time.perf_counter()
        orc.cg_fixed(L_C2, orc.PERIODIC, THETA, U, A, eta, 5)
        t_cg += time.perf_counter() - t0
        done_iters += 5
    t_iter = t_cg / done_iters
    t_step = t_clover + 12 * n_iter * t_iter
    return {"value": round(12 / t_step, 4), "unit": "solves/s", "cores": orc.num_threads(),
            "kind": "oracle",
            "sample": f"one clover build + {done_iters} full-lattice FP64 CG iterations on source "
                      f"(0,0,0,0; s0,c0) of the 16^3x32 workload ({t_clover + t_cg:.1f} s); scaled to "
                      f"12 solves x {n_iter} iterations (the oracle's own count to 1e-10, "
                      f"oracle/c2_reference.json)",
            "s_per_iter": round(t_iter, 4)}


if __name__ == "__main__":
    main()
