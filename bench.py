#!/usr/bin/env python3
"""Benchmark: staggered Dslash throughput and even-odd CG time to a 1e-10
true residual, mixed precision against FP64, on one MI355X.

Workload (the paper's large single-GPU case, Sec. 4.1-4.2): 64^3 x 16
lattice, smooth links U = exp(i eps H) with eps = 0.3 (seed 1002), Gaussian
even source (seed 2002), m = 0.01, synthetic data.

A timed step is one complete solve of M x = b (M = m^2 - D_eo D_oe) from
x = 0 to ||b - Mx|| / ||b|| <= 1e-10 (FP64 residual) with the mixed-precision
solver: FP16-storage / FP32-arithmetic inner CG on 12-real links (third row
rebuilt in the kernel) with FP64 residual updates on the full 18-real links.
`value` is the mean seconds per solve (lower is better), timed as a caller
runs the solver (HIP graphs on, no per-launch events).  The same run also
times the plain FP64 solve (for the mixed-vs-FP64 ratio), the standalone hop
in every link format (GB/s, GFLOP/s, fraction of 8 TB/s), and one complete
solve of the same system by the CPU oracle, whose x every GPU solve is
compared with.

Right after the timed steps the same solves run again with every hop launch
bracketed by HIP events recorded on the stream it is launched on; `roofline`
reports the dominant kernel of the step from that pass, with the algorithmic
bytes per launch (links, each input vector once, the output), and beside them
the paper's model bytes (every neighbour read counted, Sec. 4.3) and the HBM
traffic rocprofv3 measured on the same kernel source.  Options --only-hop /
--only-copy run the launches a rocprofv3 counter pass needs and nothing else.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
DIMS = (64, 64, 64, 16)
MASS = 0.01
TOL = 1e-10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inner", default="f16", choices=["f16", "f32"])
    ap.add_argument("--recon", type=int, default=12, choices=[18, 12])
    ap.add_argument("--reliable", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hop-reps", type=int, default=20)
    ap.add_argument("--only-hop", default=None, help="prec:recon, e.g. f64:18 -- hop launches only (profiling)")
    ap.add_argument("--only-copy", action="store_true", help="plain copy kernel only (counter calibration)")
    ap.add_argument("--only-solve", action="store_true",
                    help="one mixed-precision solve with the timed step's settings and nothing else (profiling)")
    ap.add_argument("--hop-nrhs", type=int, default=1, help="right-hand sides of the --only-hop launches")
    ap.add_argument("--no-temporal", action="store_true", help="skip the temporal-gauge solves")
    ap.add_argument("--dims", default=None, help="override lattice, e.g. 32,32,32,8")
    ap.add_argument("--suite", action="store_true",
                    help="measure the other workloads (size sweep, multi-RHS, batches, force); one JSON line each")
    ap.add_argument("--suite-dims", default=None,
                    help="lattices of the hop and CG size sweeps, e.g. '48,48,48,48;64,64,64,64'")
    ap.add_argument("--suite-only", default=None,
                    help="comma-separated suite sections: hop_sweep, cg_sweep, nmulti, temporal, multishift, "
                         "block_cg, uneven, small_cg, reliable, force, oracle, hmc")
    return ap.parse_args()


# Sources that define a kernel's code (the standalone hop unless an entry of the
# counter summary names others): counter readings taken on other sources are
# not reported.
HOP_SOURCES = ["dev.hpp", "hop.hpp", "dslash.hip"]


def src_hash(sources=None):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2502_03249_amd", "csrc")
    for name in sources or HOP_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key, launches_sites):
    """HBM bytes per launch from the committed counter summary, if taken on this source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel_key)
    if not e or e.get("src_hash") != src_hash(e.get("sources")):
        return None
    return e["bytes_per_launch"]


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2502_03249_amd as lqs
    from paper_2502_03249_amd import model
    import synth

    dims = tuple(int(v) for v in a.dims.split(",")) if a.dims else DIMS
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    if a.suite:
        run_suite(a)
        return

    if a.only_copy:
        n = 1 << 28   # 2 GiB of float64, copied 10 times
        x = torch.ones(n, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": n * 8, "copy_bytes_written_per_launch": n * 8}))
        return

    t_setup = time.time()
    U = synth.gauge(dims, "smooth", seed=1002, eps=0.3)
    b = synth.source(dims, 0, seed=2002)
    # Default launch shapes (256-thread blocks, one right-hand side per thread,
    # streaming link loads at this link footprint), so that the timed kernels
    # are the ones the counter passes (--only-hop) measure; the autotuner is
    # exercised by --suite.
    ctx = lqs.Context(0, tuning=False)
    Ud = torch.from_numpy(U).to(dev)
    g = lqs.Gauge(ctx, dims, Ud, lqs.FMT_ALL)
    bf = lqs.Field.from_lex(ctx, torch.from_numpy(b).to(dev), 0)
    xf = bf.like().zero_()
    torch.cuda.synchronize()
    del Ud
    setup_s = time.time() - t_setup
    vh = int(np.prod(dims)) // 2

    def hop_rate(prec, recon, reps, nrhs=1):
        """Standalone hop D_eo on nrhs random odd fields; HIP events on the launch stream."""
        pr = lqs.PREC[prec]
        src = synth.source(dims, 1, seed=7) if nrhs == 1 else \
            np.stack([synth.source(dims, 1, seed=7 + k) for k in range(nrhs)])
        xin = lqs.Field.from_lex(ctx, torch.from_numpy(src).to(dev), 1, pr)
        out = xin.like(parity=0)
        for _ in range(3):
            lqs.dslash_apply(ctx, g, xin, out, recon=recon)
        lqs.profile_hops(ctx, True)
        for _ in range(reps):
            lqs.dslash_apply(ctx, g, xin, out, recon=recon)
        torch.cuda.synchronize()
        n, ms, sites = lqs.profile_hops_result(ctx, pr, recon)
        lqs.profile_hops(ctx, False)
        mb = model.hop_model_bytes(pr, recon, nrhs) * vh
        nb = model.hop_min_bytes(pr, recon, nrhs) * vh
        r = {"prec": prec, "recon": recon, "ms": ms, "model_GBps": mb / ms / 1e6, "min_GBps": nb / ms / 1e6,
             "frac_hbm_min": nb / ms / 1e6 / PEAK_HBM_GBPS,
             "GFLOPs": model.FLOPS_PER_SITE * nrhs * vh / ms / 1e6, "frac_hbm": mb / ms / 1e6 / PEAK_HBM_GBPS,
             "model_bytes_per_site": model.hop_model_bytes(pr, recon, nrhs),
             "min_bytes_per_site": model.hop_min_bytes(pr, recon, nrhs), "launches": n}
        if nrhs > 1:
            r["nrhs"] = nrhs
        return r

    if a.only_hop:
        prec, recon = a.only_hop.split(":")
        r = hop_rate(prec, int(recon), a.hop_reps, a.hop_nrhs)
        print(json.dumps(r))
        return

    inner = lqs.PREC[a.inner]

    if a.only_solve:
        st = lqs.cg_solve(ctx, [(g, MASS, bf, xf)], tol=TOL, max_iter=20000, inner_prec=inner,
                          inner_recon=a.recon, reliable_interval=a.reliable)
        torch.cuda.synchronize()
        print(json.dumps(st[0]))
        return

    def solve(prec, recon, reliable):
        xf.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = lqs.cg_solve(ctx, [(g, MASS, bf, xf)], tol=TOL, max_iter=20000, inner_prec=prec,
                          inner_recon=recon, reliable_interval=reliable)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st[0]

    # warmup (also pages in code objects and workspaces)
    for _ in range(a.warmup):
        solve(inner, a.recon, a.reliable)

    # timed steps: mixed-precision solves as a caller runs them (HIP graphs on,
    # no per-launch events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(a.steps):
        st = lqs.cg_solve(ctx, [(g, MASS, bf, xf)], tol=TOL, max_iter=20000, inner_prec=inner,
                          inner_recon=a.recon, reliable_interval=a.reliable)
        stats.append(st[0])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mixed_s = elapsed / a.steps
    x_mixed = xf.to_lex(ctx)  # solution of the last timed solve, compared below with the FP64 ones
    ok = all(s["status"] == 0 and s["true_rel_residual"] <= TOL for s in stats)

    # profiled pass right after the timed steps: the same solves with every hop
    # launch bracketed by HIP events on its stream (graphs are off while hops
    # are profiled).  Launches queued after a solve converged return at once
    # (a few us); only launches longer than 20 us are counted (one working hop
    # per iteration).
    prof_steps = max(1, min(a.steps, 3))
    lqs.profile_hops(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prof_stats = []
    for _ in range(prof_steps):
        st = lqs.cg_solve(ctx, [(g, MASS, bf, xf)], tol=TOL, max_iter=20000, inner_prec=inner,
                          inner_recon=a.recon, reliable_interval=a.reliable)
        prof_stats.append(st[0])
    torch.cuda.synchronize()
    eager_s = (time.perf_counter() - t0) / prof_steps
    n_hop, hop_ms, _ = lqs.profile_hops_result(ctx, inner, a.recon, min_ms=0.02)
    lqs.profile_hops(ctx, False)
    working = sum(s["iters"] for s in prof_stats)
    ok = ok and all(s["status"] == 0 and s["true_rel_residual"] <= TOL for s in prof_stats)

    # FP64 solve on the same system (untimed by the step loop, timed on its own)
    other = lqs.F32 if inner == lqs.F16 else lqs.F16
    for p_, r_, k_ in ((lqs.F64, 18, 0), (lqs.F64, 12, 0), (other, a.recon, a.reliable)):
        solve(p_, r_, k_)  # warmup / tuning
    fp64 = [solve(lqs.F64, 18, 0) for _ in range(2)]
    fp64_s = min(t for t, _ in fp64)
    fp64_st = fp64[0][1]
    x_fp64 = xf.to_lex(ctx)
    fp64_12 = [solve(lqs.F64, 12, 0) for _ in range(2)]
    fp64_12_s = min(t for t, _ in fp64_12)
    other_t, other_st = solve(other, a.recon, a.reliable)
    x_other = xf.to_lex(ctx)

    def rel_err(x):
        # ||x - x_FP64|| / ||x_FP64||: the solve's error against the FP64 solution of the same
        # system (the FP64 solver itself is checked against the oracle by the test suite)
        return float(torch.linalg.vector_norm(x - x_fp64) / torch.linalg.vector_norm(x_fp64))

    err_mixed, err_other = rel_err(x_mixed), rel_err(x_other)
    # kept on the device for the comparison with the oracle's solution below
    x_mixed_keep, x_other_keep, x_t_keep = x_mixed, x_other, None

    # The paper's storage (Sec. 4.3): the same system in temporal gauge, U' = G U G^dag with
    # U'_t = 1 off the last slice, b' = G b; the hop then reads 6 + 2/Nt links per site.
    # |b' - M' x'| = |b - M x| (G is unitary per site), so the stop test is the same.
    temporal = None
    if not a.no_temporal:
        Ud = torch.from_numpy(U).to(dev)
        Uf, G = lqs.gauge_fix_temporal(ctx, dims, Ud)
        del Ud
        gt = lqs.Gauge(ctx, dims, Uf, lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
        del Uf
        bt = (G * torch.from_numpy(b).to(dev).unsqueeze(-2)).sum(-1)
        btf = lqs.Field.from_lex(ctx, bt, 0)
        del bt
        xtf = btf.like()

        def solve_t(prec, recon, reliable):
            xtf.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = lqs.cg_solve(ctx, [(gt, MASS, btf, xtf)], tol=TOL, max_iter=20000, inner_prec=prec,
                              inner_recon=recon, reliable_interval=reliable)
            torch.cuda.synchronize()
            return time.perf_counter() - t0, st[0]

        solve_t(inner, 12, a.reliable)
        tm = [solve_t(inner, 12, a.reliable) for _ in range(2)]
        # x = G^dag x' maps the fixed-gauge solution back
        xt = (G.conj().transpose(-1, -2) * xtf.to_lex(ctx)[0].unsqueeze(-2)).sum(-1)
        err_t = rel_err(xt.unsqueeze(0))
        x_t_keep = xt.unsqueeze(0)
        del xt, G
        solve_t(lqs.F64, 12, 0)
        t64 = solve_t(lqs.F64, 12, 0)
        temporal = {"mixed_s": round(min(t for t, _ in tm), 5), "mixed_iters": tm[0][1]["iters"],
                    "mixed_true_res": tm[0][1]["true_rel_residual"], "mixed_x_rel_err_vs_fp64": err_t,
                    "fp64_recon12_s": round(t64[0], 5), "fp64_iters": t64[1]["iters"],
                    "fp64_true_res": t64[1]["true_rel_residual"],
                    "converged": all(st["status"] == 0 and st["true_rel_residual"] <= TOL
                                     for st in [tm[0][1], tm[1][1], t64[1]])}
        del gt, btf, xtf

    # standalone hop in every format
    hops = [hop_rate(p, r, a.hop_reps) for p in ("f64", "f32", "f16") for r in (18, 12)]

    # roofline of the dominant kernel of the step: the inner-precision hop.  achieved counts the
    # algorithmic (minimum) bytes: links, each input vector once, the output; the paper's model
    # bytes (every neighbour read counted) are reported beside it.
    min_site = model.hop_min_bytes(inner, a.recon)
    mb_site = model.hop_model_bytes(inner, a.recon)
    achieved = min_site * vh / hop_ms / 1e6
    key = f"hop_{a.inner}_{a.recon}"
    traffic = traffic_for(key, vh)
    roof = {"bound": "hbm", "kernel": key, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic,
            "bytes_per_launch": min_site * vh, "bytes_per_site": min_site, "avg_launch_ms": round(hop_ms, 5),
            "launches_timed": n_hop, "working_launches": working,
            "model_bytes_per_site": mb_site, "model_GBps": round(mb_site * vh / hop_ms / 1e6, 1),
            "traffic_GBps": round(traffic / hop_ms / 1e6, 1) if traffic else None}
    h64 = [h for h in hops if h["prec"] == "f64" and h["recon"] == 18][0]

    cpu = None
    oracle_err = None
    if not a.no_cpu_baseline:
        import oracle
        # One complete FP64 oracle solve of the same 64^3 x 16 system, timed on
        # the host with every thread the oracle's OpenMP regions use; its x is
        # the reference every GPU solve of this run is compared with.
        t1 = time.perf_counter()
        x_ora, st_ora, it_ora, tr_ora = oracle.cg(dims, U, MASS, b, tol=TOL, max_iter=20000)
        dt = time.perf_counter() - t1
        cpu = {"value": round(dt, 2), "unit": "s", "cores": oracle.threads(), "kind": "oracle",
               "sample": f"one complete FP64 CG solve of the 64^3x16 system to a {TOL:g} true residual "
                         f"({it_ora} iterations, status {st_ora}, true residual {tr_ora:.3e})"}
        xo = torch.from_numpy(x_ora).to(dev).unsqueeze(0)
        del x_ora

        def err_ora(x):
            return float(torch.linalg.vector_norm(x - xo) / torch.linalg.vector_norm(xo))

        oracle_err = {"mixed": err_ora(x_mixed_keep), "fp64": err_ora(x_fp64),
                      f"{'f32' if other == lqs.F32 else 'f16'}_mixed": err_ora(x_other_keep)}
        if x_t_keep is not None:
            oracle_err["temporal_gauge_mixed"] = err_ora(x_t_keep)
        del xo

    line = {
        "metric": "Dslash GB/s & GFLOP/s (% HBM roofline); CG s-to-1e-10, mixed vs FP64",
        "value": round(mixed_s, 5), "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1000 * mixed_s, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{a.inner}-storage/f32 inner, f64 residual",
        "data": "synthetic",
        "config": {"workload": "64^3x16 even-odd staggered CG to 1e-10, m=0.01, smooth links eps=0.3",
                   "dims": list(dims), "mass": MASS, "tol": TOL, "inner": a.inner, "recon": a.recon,
                   "reliable_interval": a.reliable,
                   "reliable_delta": 0.05 if a.inner == "f16" else 0.02, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "cg": {"mixed_s": round(mixed_s, 5), "mixed_eager_profiled_s": round(eager_s, 5),
               "mixed_iters": stats[-1]["iters"],
               "mixed_reliable_updates": stats[-1]["reliable_updates"],
               "mixed_gflops": round(stats[-1]["gflops"], 1), "mixed_gbytes_per_s": round(stats[-1]["gbytes_per_s"], 1),
               "mixed_true_res": stats[-1]["true_rel_residual"], "mixed_x_rel_err_vs_fp64": err_mixed,
               "x_rel_err_vs_oracle": oracle_err,
               "all_converged": ok,
               "fp64_s": round(fp64_s, 5), "fp64_iters": fp64_st["iters"], "fp64_true_res": fp64_st["true_rel_residual"],
               "fp64_recon12_s": round(fp64_12_s, 5),
               "speedup_mixed_vs_fp64": round(fp64_s / mixed_s, 3),
               "speedup_mixed_vs_best_fp64": round(min(fp64_s, fp64_12_s) / mixed_s, 3),
               f"{'f32' if other == lqs.F32 else 'f16'}_mixed_s": round(other_t, 5),
               f"{'f32' if other == lqs.F32 else 'f16'}_mixed_iters": other_st["iters"],
               f"{'f32' if other == lqs.F32 else 'f16'}_mixed_x_rel_err_vs_fp64": err_other,
               "temporal_gauge": temporal},
        "dslash": {"fp64_18_model_GBps": round(h64["model_GBps"], 1), "fp64_18_GFLOPs": round(h64["GFLOPs"], 1),
                   "fp64_18_frac_hbm": round(h64["frac_hbm"], 4),
                   "formats": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in h.items()} for h in hops]},
        "setup_s": round(setup_s, 1),
    }
    print(json.dumps(line))


def run_suite(a):
    """The other workloads, one JSON line per measurement (not the contract line).

    hop and CG size sweeps (Fig. 3 analogue) | multi-vector hop on 32^4 and 32^3x8 (Table 2
    analogue), default and autotuned shapes | 16-RHS block CG vs 16 single solves |
    uneven three-lattice batch, persistent vs separate | 4^4 and 32^3x8 FP64 CG |
    24^4 action, adjoint and force | the oracle's hop and CG on the host | 24^4 plaquette force and
    HMC trajectories.
    """
    import numpy as np
    import torch

    import paper_2502_03249_amd as lqs
    from paper_2502_03249_amd import model
    import synth

    dev = torch.device("cuda", 0)

    def emit(d):
        print(json.dumps(d), flush=True)

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def event_ms(fn, reps):
        # Warm up for about 30 ms of back-to-back calls first: after an idle
        # spell (context or field set-up) the first launches run slower for
        # several milliseconds (measured on the 16-vector hop at 64^3x16:
        # 717, then 617, then 599 us in three consecutive 10-call batches).
        torch.cuda.synchronize()
        t_w = time.perf_counter()
        for k in range(1000):
            fn()
            if k % 4 == 3:
                torch.cuda.synchronize()
                if time.perf_counter() - t_w > 0.03:
                    break
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps

    import tempfile
    # the suite's tuned shapes persist across sections (and runs) in this JSON cache
    tune_cache = os.environ.get("LQS_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "lqs_tune_suite.json"))
    ctx = lqs.Context(0, tune_cache=tune_cache)
    only = set(a.suite_only.split(",")) if a.suite_only else None

    def want(name):
        return only is None or name in only

    def setup(dims, kind, lseed, sseeds, mass=None, formats=lqs.FMT_ALL):
        U = synth.gauge(dims, kind, seed=lseed, eps=0.3)
        g = lqs.Gauge(ctx, dims, torch.from_numpy(U).to(dev), formats)
        srcs = np.stack([synth.source(dims, 0, seed=s) for s in sseeds])
        b = lqs.Field.from_lex(ctx, torch.from_numpy(srcs).to(dev), 0)
        torch.cuda.synchronize()
        return U, g, b

    sweep_dims = [(4, 4, 4, 4), (8, 8, 8, 8), (16, 16, 16, 16), (24, 24, 24, 8), (32, 32, 32, 8), (24, 24, 24, 24),
                  (32, 32, 32, 32), (48, 48, 48, 12), (64, 64, 64, 16), (48, 48, 48, 48), (64, 64, 64, 64)]
    if a.suite_dims:
        sweep_dims = [tuple(int(v) for v in d.split(",")) for d in a.suite_dims.split(";")]

    def temporal_gauge(dims, U):
        """The same links fixed to temporal gauge (U_t = 1 off the last slice), the paper's storage."""
        Ud = torch.from_numpy(U).to(dev)
        Uf, G = lqs.gauge_fix_temporal(ctx, dims, Ud)
        del Ud
        gt = lqs.Gauge(ctx, dims, Uf, lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
        del Uf
        return gt, G

    # 1. hop size sweep (Fig. 3 analogue): the hop at every format, standalone, stream events;
    #    then the paper's storage (temporal gauge, 12 reals: 6 + 2/Nt links read per site)
    if want("hop_sweep"):
        for dims in sweep_dims:
            U, g, _ = setup(dims, "smooth", 1002, [7])
            vh = int(np.prod(dims)) // 2
            src = torch.from_numpy(synth.source(dims, 1, seed=7)).to(dev)

            def one(gauge_, prec, recon, lps, storage):
                pr = lqs.PREC[prec]
                x = lqs.Field.from_lex(ctx, src, 1, pr)
                y = x.like(parity=0)
                ms = event_ms(lambda: lqs.dslash_apply(ctx, gauge_, x, y, recon=recon), 20)
                mb = model.hop_model_bytes(pr, recon, 1, lps)
                nb = model.hop_min_bytes(pr, recon, 1, lps)
                emit({"suite": "hop_size_sweep", "dims": dims, "storage": storage, "prec": prec, "recon": recon,
                      "us": round(1e3 * ms, 2), "GFLOPs": round(570 * vh / ms / 1e6, 1),
                      "model_GBps": round(mb * vh / ms / 1e6, 1), "alg_GBps": round(nb * vh / ms / 1e6, 1),
                      "alg_frac_8TBps": round(nb * vh / ms / 1e6 / PEAK_HBM_GBPS, 3),
                      "note": "links fit in the 256 MB MALL" if 8 * model.link_bytes(pr, recon) * vh < 2.5e8 else "HBM"})

            for prec, recon in [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12), ("f16", 18), ("f16", 12)]:
                one(g, prec, recon, 8, "ungauged")
            g.close()
            gt, G = temporal_gauge(dims, U)
            del G, U
            for prec in ("f64", "f32", "f16"):
                one(gt, prec, 12, 6 + 2 / dims[3], "temporal_gauge")
            gt.close()
            torch.cuda.empty_cache()

    # 1b. CG size sweep (the CG curve of Fig. 3): time per iteration and algorithmic GB/s of the
    #     FP64 solver and the FP16-mixed solver, 8^4 .. 64^4, m 0.05; from 32^4 on also in the
    #     paper's storage (temporal gauge, 12-real links), the source transformed with the gauge
    if want("cg_sweep"):
        for dims in [d for d in sweep_dims if int(np.prod(d)) >= 8 ** 4]:
            U, g, b = setup(dims, "smooth", 1002, [2002])
            vh = int(np.prod(dims)) // 2
            x = b.like()

            def sweep(gauge_, bb, xx, inner, recon, storage, lps):
                pr = lqs.PREC[inner]
                lqs.cg_solve(ctx, [(gauge_, 0.05, bb, xx.zero_())], tol=TOL, inner_prec=pr, inner_recon=recon,
                             reliable_interval=100)
                st = []
                t = timed(lambda: st.append(lqs.cg_solve(ctx, [(gauge_, 0.05, bb, xx.zero_())], tol=TOL, inner_prec=pr,
                                                         inner_recon=recon, reliable_interval=100)), 2)
                it = st[-1][0]["iters"]
                by = model.cg_iteration_bytes(pr, lqs.F64 if pr == lqs.F64 else lqs.F32, recon, lps) * vh
                emit({"suite": "cg_size_sweep", "dims": dims, "storage": storage, "inner": inner, "recon": recon,
                      "s": round(t, 5), "iters": it, "us_per_iter": round(1e6 * t / it, 2),
                      "device_us_per_iter": round(1e6 * st[-1][0]["device_seconds"] / it, 2),
                      "alg_GBps": round(by * it / t / 1e9, 1), "true_res": st[-1][0]["true_rel_residual"],
                      "converged": st[-1][0]["status"] == 0})

            for inner, recon in (("f64", 18), ("f16", 12)):
                sweep(g, b, x, inner, recon, "ungauged", 8)
            g.close()
            if int(np.prod(dims)) >= 32 ** 4:
                gt, G = temporal_gauge(dims, U)
                bsrc = torch.from_numpy(synth.source(dims, 0, seed=2002)).to(dev)
                bt = lqs.Field.from_lex(ctx, (G * bsrc.unsqueeze(-2)).sum(-1), 0)
                del G, bsrc
                xt = bt.like()
                for inner in ("f64", "f16"):
                    sweep(gt, bt, xt, inner, 12, "temporal_gauge", 6 + 2 / dims[3])
                gt.close()
            del U
            torch.cuda.empty_cache()

    # 2. multi-vector hop: 32^4 (the paper's Table 2 lattice), 32^3x8 and 64^3x16 with 16 sources
    if want("nmulti"):
        for dims in [(32, 32, 32, 32), (32, 32, 32, 8), (64, 64, 64, 16)]:
            U, g, _ = setup(dims, "smooth", 1001, [7])
            vh = int(np.prod(dims)) // 2
            srcs = np.stack([synth.source(dims, 1, seed=2100 + k) for k in range(16)])
            ns = (1, 2, 4, 8, 16) if dims[3] == 16 else (1, 2, 3, 4, 6, 8, 10, 12, 14, 16)
            for prec, recon in [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12), ("f16", 12)]:
                pr = lqs.PREC[prec]
                for n in ns:
                    x = lqs.Field.from_lex(ctx, torch.from_numpy(srcs[:n]).to(dev), 1, pr)
                    y = x.like(parity=0)
                    for tuned in (False, True):
                        ctx.set_tuning(tuned)
                        ms = event_ms(lambda: lqs.dslash_apply(ctx, g, x, y, recon=recon), 10)
                        emit({"suite": "nmulti", "dims": dims, "prec": prec, "recon": recon, "n": n, "tuned": tuned,
                              "us": round(1e3 * ms, 2), "TFLOPs": round(570 * n * vh / ms / 1e9, 3),
                              "model_GBps": round(model.hop_model_bytes(pr, recon, n) * vh / ms / 1e6, 1),
                              "alg_frac_8TBps": round(model.hop_min_bytes(pr, recon, n) * vh / ms / 1e6 / PEAK_HBM_GBPS,
                                                      3)})
                    ctx.set_tuning(False)
            g.close()

    # 2b. the paper's Table 2 storage: 32^4 in temporal gauge, 12-real links (6 links read per
    if want("temporal"):
        #     site off the last time slice), FP64 and FP32, n = 1..16, tuned shapes
        dims = (32, 32, 32, 32)
        U = synth.gauge(dims, "smooth", seed=1001, eps=0.3)
        Uf, _ = lqs.gauge_fix_temporal(ctx, dims, torch.from_numpy(U).to(dev))
        g = lqs.Gauge(ctx, dims, Uf, lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
        vh = int(np.prod(dims)) // 2
        srcs = np.stack([synth.source(dims, 1, seed=2100 + k) for k in range(16)])
        lps = 6 + 2 / dims[3]
        ctx.set_tuning(True)
        for prec, recon in [("f64", 12), ("f32", 12), ("f64", 18), ("f32", 18), ("f16", 12)]:
            pr = lqs.PREC[prec]
            for n in (1, 2, 3, 4, 6, 8, 10, 12, 14, 16):
                x = lqs.Field.from_lex(ctx, torch.from_numpy(srcs[:n]).to(dev), 1, pr)
                y = x.like(parity=0)
                ms = event_ms(lambda: lqs.dslash_apply(ctx, g, x, y, recon=recon), 10)
                emit({"suite": "nmulti_temporal", "dims": dims, "prec": prec, "recon": recon, "n": n,
                      "us": round(1e3 * ms, 2), "TFLOPs": round(570 * n * vh / ms / 1e9, 3),
                      "model_GBps": round(model.hop_model_bytes(pr, recon, n, lps) * vh / ms / 1e6, 1)})
        ctx.set_tuning(False)
        g.close()
        del Uf

    # 2c. several masses on one Krylov space vs one solve per mass (64^3x16, FP64)
    if want("multishift"):
        dims = DIMS
        U, g, b = setup(dims, "smooth", 1002, [2002])
        masses = [0.01, 0.02, 0.05, 0.1, 0.2, 0.5, 1.0, 2.0]
        xs = [b.like() for _ in masses]
        st = []
        t_ms = timed(lambda: st.append(lqs.cg_solve_multishift(ctx, g, masses, b, xs, tol=TOL)), 2)
        t_sep = 0.0
        for m_, x_ in zip(masses, xs):
            t_sep += timed(lambda: lqs.cg_solve(ctx, [(g, m_, b, x_.zero_())], tol=TOL, inner_prec=lqs.F64), 1)
        emit({"suite": "multishift", "dims": dims, "masses": masses, "multishift_s": round(t_ms, 4),
              "separate_fp64_s": round(t_sep, 4), "speedup": round(t_sep / t_ms, 2),
              "iters": [r["iters"] for r in st[-1]], "true_res": [r["true_rel_residual"] for r in st[-1]],
              "all_converged": all(r["status"] == 0 for r in st[-1])})
        # the recurrence in FP32 / FP16 storage (12-real links), every mass refined to the FP64 residual
        for inner in ("f32", "f16"):
            stm = []
            lqs.cg_solve_multishift(ctx, g, masses, b, xs, tol=TOL, inner_prec=inner, inner_recon=12)
            t_mix = timed(lambda: stm.append(lqs.cg_solve_multishift(ctx, g, masses, b, xs, tol=TOL,
                                                                     inner_prec=inner, inner_recon=12)), 2)
            emit({"suite": "multishift_mixed", "dims": dims, "masses": masses, "inner": inner, "recon": 12,
                  "multishift_s": round(t_mix, 4), "fp64_multishift_s": round(t_ms, 4),
                  "speedup_vs_fp64_multishift": round(t_ms / t_mix, 2),
                  "iters": [r["iters"] for r in stm[-1]], "true_res": [r["true_rel_residual"] for r in stm[-1]],
                  "all_converged": all(r["status"] == 0 for r in stm[-1])})
        g.close()

    # 3. 16-RHS block CG on 32^3x8 (m 0.02) vs 16 single solves, FP32 inner + FP64 reliable updates
    if want("block_cg"):
        dims, mass = (32, 32, 32, 8), 0.02
        U, g, b = setup(dims, "smooth", 1001, [2100 + k for k in range(16)])
        x = b.like()
        for prec in ("f32", "f16", "f64"):
            # tune the 16-vector and the single-vector shapes (hop and fused normal kernel) first
            ctx.set_tuning(True)
            lqs.cg_solve(ctx, [(g, mass, b, x.zero_())], tol=TOL, inner_prec=lqs.PREC[prec], reliable_interval=100)
            b0 = lqs.Field(dims, lqs.F64, 0, 1, data=b.data[:lqs.field_bytes(dims, lqs.F64)])
            lqs.cg_solve(ctx, [(g, mass, b0, b0.like())], tol=TOL, inner_prec=lqs.PREC[prec], reliable_interval=100)
            ctx.set_tuning(False)
            st = []
            t = timed(lambda: st.append(lqs.cg_solve(ctx, [(g, mass, b, x.zero_())], tol=TOL, inner_prec=lqs.PREC[prec],
                                                     reliable_interval=100)), 2)
            singles = 0.0
            for k in range(16):
                bk = lqs.Field(dims, lqs.F64, 0, 1, data=b.data[k * lqs.field_bytes(dims, lqs.F64):
                                                              (k + 1) * lqs.field_bytes(dims, lqs.F64)])
                xk = bk.like()
                singles += timed(lambda: lqs.cg_solve(ctx, [(g, mass, bk, xk.zero_())], tol=TOL,
                                                      inner_prec=lqs.PREC[prec], reliable_interval=100), 1)
            s = st[-1]
            emit({"suite": "block_cg_16rhs", "dims": dims, "mass": mass, "inner": prec, "shapes": "tuned",
                  "block_s": round(t, 4),
                  "sixteen_singles_s": round(singles, 4), "speedup": round(singles / t, 2),
                  "iters": [r["iters"] for r in s], "max_true_res": max(r["true_rel_residual"] for r in s),
                  "all_converged": all(r["status"] == 0 for r in s)})
        g.close()

    # 4. uneven batch: one persistent launch vs three multi-kernel solves
    if want("uneven"):
        specs = [((16, 16, 16, 16), 0.05, 1031, 2031), ((24, 24, 24, 8), 0.02, 1032, 2032),
                 ((32, 32, 32, 8), 0.01, 1033, 2033)]
        probs = []
        for d_, m_, ls, ss in specs:
            _, g_, b_ = setup(d_, "smooth", ls, [ss])
            probs.append((g_, m_, b_, b_.like()))
        for prec, tuned in (("f32", False), ("f32", True), ("f16", False), ("f16", True), ("f64", False)):
            pr = lqs.PREC[prec]
            st = []
            ctx.set_tuning(tuned)
            # one untimed call first: it runs the shape search when tuning is on
            lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_()) for g_, m_, b_, x_ in probs], tol=TOL, inner_prec=pr,
                         reliable_interval=100, persistent=True)
            tp = timed(lambda: st.append(lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_()) for g_, m_, b_, x_ in probs],
                                                      tol=TOL, inner_prec=pr, reliable_interval=100,
                                                      persistent=True)), 3)
            ctx.set_tuning(False)
            # one call, multi-kernel: the lattices run concurrently on side streams
            # HIP events on the stream of the cooperative launch (cg_solve returns after it)
            ev_ms = event_ms(lambda: st.append(lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_()) for g_, m_, b_, x_ in probs],
                                                            tol=TOL, inner_prec=pr, reliable_interval=100,
                                                            persistent=True)), 3)
            pst = st[-1]
            stc = []
            # one untimed call of each path first (workspaces of the concurrent and single solves)
            lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_()) for g_, m_, b_, x_ in probs], tol=TOL, inner_prec=pr,
                         reliable_interval=100)
            ts = timed(lambda: stc.append(lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_()) for g_, m_, b_, x_ in probs],
                                                       tol=TOL, inner_prec=pr, reliable_interval=100)), 3)

            def sequential():
                for g_, m_, b_, x_ in probs:
                    lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_())], tol=TOL, inner_prec=pr, reliable_interval=100)
            sequential()
            tq = timed(sequential, 3)
            emit({"suite": "uneven_batch", "lattices": [s_[0] for s_ in specs], "masses": [s_[1] for s_ in specs],
                  "inner": prec, "persistent_tuned": tuned, "persistent_event_ms": round(ev_ms, 4),
                  "persistent_group_ms": [round(1e3 * r["device_seconds"], 4) for r in pst],
                  "persistent_us_per_iter": [round(1e6 * r["device_seconds"] / max(r["iters"], 1), 2) for r in pst],
                  "concurrent_us_per_iter": [round(1e6 * r["device_seconds"] / max(r["iters"], 1), 2)
                                             for r in stc[-1]],
                  "persistent_s": round(tp, 5),
                  "concurrent_multikernel_s": round(ts, 5), "sequential_s": round(tq, 5),
                  "persistent_vs_sequential": round(tq / tp, 2), "concurrent_vs_sequential": round(tq / ts, 2),
                  "iters": [r["iters"] for r in st[-1]],
                  "true_res": [r["true_rel_residual"] for r in st[-1]],
                  "all_converged": all(r["status"] == 0 for r in st[-1])})
        for g_, _, _, _ in probs:
            g_.close()

    # 4b. many small lattices: 64 lattices of 4^4 / 4^3x6 / 6x4^3 (m 0.1 .. 0.73), one persistent launch
    #     (one block per lattice) vs one multi-kernel call (side streams) vs one call per lattice
    if want("uneven"):
        shapes = [(4, 4, 4, 4), (4, 4, 4, 6), (6, 4, 4, 4)]
        probs = []
        for k in range(64):
            _, g_, b_ = setup(shapes[k % 3], "smooth", 1300 + k, [2300 + k])
            probs.append((g_, 0.1 + 0.01 * k, b_, b_.like()))
        for prec in ("f64", "f16"):
            pr = lqs.PREC[prec]
            st = []
            tp = timed(lambda: st.append(lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_()) for g_, m_, b_, x_ in probs],
                                                      tol=TOL, inner_prec=pr, reliable_interval=100,
                                                      persistent=True)), 3)
            tc = timed(lambda: lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_()) for g_, m_, b_, x_ in probs], tol=TOL,
                                            inner_prec=pr, reliable_interval=100), 3)

            def sequential():
                for g_, m_, b_, x_ in probs:
                    lqs.cg_solve(ctx, [(g_, m_, b_, x_.zero_())], tol=TOL, inner_prec=pr, reliable_interval=100)
            tq = timed(sequential, 1)
            emit({"suite": "many_small_batch", "lattices": 64, "shapes": shapes, "inner": prec,
                  "persistent_s": round(tp, 5), "concurrent_multikernel_s": round(tc, 5), "sequential_s": round(tq, 5),
                  "persistent_vs_sequential": round(tq / tp, 2), "persistent_vs_concurrent": round(tc / tp, 2),
                  "max_iters": max(r["iters"] for r in st[-1]),
                  "all_converged": all(r["status"] == 0 for r in st[-1])})
        for g_, _, _, _ in probs:
            g_.close()

    # 5. small-lattice and 32^3x8 FP64 CG (multi-kernel and persistent)
    if want("small_cg"):
        for dims, kind, ls, ss, mass in [((4, 4, 4, 4), "haar", 1000, 2000, 0.1), ((32, 32, 32, 8), "smooth", 1001, 2001, 0.02)]:
            U, g, b = setup(dims, kind, ls, [ss])
            x = b.like()
            for persistent in (False, True):
                st = []
                t = timed(lambda: st.append(lqs.cg_solve(ctx, [(g, mass, b, x.zero_())], tol=TOL, inner_prec=lqs.F64,
                                                         persistent=persistent)), 3)
                emit({"suite": "cg_fp64", "dims": dims, "mass": mass, "persistent": persistent, "s": round(t, 5),
                      "iters": st[-1][0]["iters"], "true_res": st[-1][0]["true_rel_residual"]})
            tm = timed(lambda: st.append(lqs.cg_solve(ctx, [(g, mass, b, x.zero_())], tol=TOL, inner_prec=lqs.F16,
                                                      reliable_interval=100, inner_recon=12)), 3)
            emit({"suite": "cg_mixed_f16", "dims": dims, "mass": mass, "s": round(tm, 5), "iters": st[-1][0]["iters"],
                  "true_res": st[-1][0]["true_rel_residual"]})
            g.close()

    # 6. reliable-update interval K and threshold delta for the 64^3x16 FP16 solve
    if want("reliable"):
        dims, mass = DIMS, MASS
        U, g, b = setup(dims, "smooth", 1002, [2002])
        x = b.like()
        for K in (50, 100, 200, 400):
            for delta in (0.1, 0.05, 0.01):
                st = []
                t = timed(lambda: st.append(lqs.cg_solve(ctx, [(g, mass, b, x.zero_())], tol=TOL, inner_prec=lqs.F16,
                                                         inner_recon=12, reliable_interval=K, reliable_delta=delta)), 2)
                r = st[-1][0]
                emit({"suite": "reliable_sweep", "dims": dims, "K": K, "delta": delta, "s": round(t, 5),
                      "iters": r["iters"], "reliable_updates": r["reliable_updates"],
                      "true_res": r["true_rel_residual"], "status": r["status"]})
        g.close()

    # 7. differentiation: 24^4, m 0.05: action (CG), adjoint force
    if want("force"):
        from paper_2502_03249_amd.autograd import staggered_action
        dims, mass = (24, 24, 24, 24), 0.05
        U = synth.gauge(dims, "smooth", seed=1004, eps=0.3)
        Ut = torch.from_numpy(U).to(dev).requires_grad_(True)
        phi = torch.from_numpy(synth.source(dims, 0, seed=2004)).to(dev).requires_grad_(True)

        def fwd_bwd():
            Ut.grad = None
            phi.grad = None
            S = staggered_action(Ut, phi, mass, ctx, project=True, tol=1e-10)
            S.backward()
        t = timed(fwd_bwd, 3)
        g = lqs.Gauge(ctx, dims, Ut.detach(), lqs.fmt("f64", 18))
        X = lqs.Field.from_lex(ctx, phi.detach(), 0)
        out = torch.empty_like(Ut.detach())
        ms = event_ms(lambda: lqs.fermion_force(ctx, g, X, None, 1.0, 0, out), 10)
        emit({"suite": "force_24x4", "action_forward_backward_s": round(t, 4), "fermion_force_call_ms": round(ms, 4),
              "note": "fermion_force = one D_oe hop + the outer-product/projection kernel"})
        del g, X, out

    # 7b. the oracle on the host: hop at 32^3x8, 24^4 and 64^3x16 with one thread and all threads,
    #     CG at 4^4 (full) -- the CPU baseline of the GPU numbers above
    if want("oracle"):
        import oracle
        nthr = oracle.threads()
        for dh in [(32, 32, 32, 8), (24, 24, 24, 24), (64, 64, 64, 16)]:
            Uh = synth.gauge(dh, "smooth", seed=1001, eps=0.3)
            xh = synth.source(dh, 1, seed=7)
            res = {}
            for nt_ in (1, nthr):
                oracle.set_threads(nt_)
                t0 = time.perf_counter()
                oracle.dslash(dh, Uh, xh, 0)
                res[nt_] = time.perf_counter() - t0
            oracle.set_threads(nthr)
            vhh = int(np.prod(dh)) // 2
            emit({"suite": "oracle_hop", "dims": dh, "s_1_thread": round(res[1], 4), "s_all": round(res[nthr], 4),
                  "threads": nthr, "GFLOPs_all": round(570 * vhh / res[nthr] / 1e9, 3),
                  "model_GBps_all": round(1584 * vhh / res[nthr] / 1e9, 3)})
            del Uh, xh
        U4 = synth.gauge((4, 4, 4, 4), "haar", seed=1000)
        b4 = synth.source((4, 4, 4, 4), 0, seed=2000)
        t0 = time.perf_counter()
        _, st4, it4, tr4 = oracle.cg((4, 4, 4, 4), U4, 0.1, b4, tol=TOL)
        emit({"suite": "oracle_cg_4x4", "s": round(time.perf_counter() - t0, 4), "iters": it4, "true_res": tr4,
              "threads": nthr})
        # the oracle's whole FP64 CG on the 32^3x8 (m 0.02) and 24^4 (m 0.05) systems, all threads,
        # beside the GPU's FP64 and mixed solves of the same systems
        for dh, mh, us, bs in (((32, 32, 32, 8), 0.02, 1001, 2001), ((24, 24, 24, 24), 0.05, 1004, 2004)):
            Uh = synth.gauge(dh, "smooth", seed=us, eps=0.3)
            bh = synth.source(dh, 0, seed=bs)
            t0 = time.perf_counter()
            _, _, ith, trh = oracle.cg(dh, Uh, mh, bh, tol=TOL)
            t_or = time.perf_counter() - t0
            gh = lqs.Gauge(ctx, dh, torch.from_numpy(Uh).to(dev), lqs.FMT_ALL)
            bf = lqs.Field.from_lex(ctx, torch.from_numpy(bh).to(dev), 0)
            xg = bf.like()
            gpu = {}
            for name, prec, rc in (("fp64", lqs.F64, 18), ("f16_mixed", lqs.F16, 12)):
                lqs.cg_solve(ctx, [(gh, mh, bf, xg.zero_())], tol=TOL, inner_prec=prec, inner_recon=rc)
                gpu[name] = timed(lambda: lqs.cg_solve(ctx, [(gh, mh, bf, xg.zero_())], tol=TOL, inner_prec=prec,
                                                       inner_recon=rc), 2)
            emit({"suite": "oracle_cg", "dims": dh, "mass": mh, "oracle_s": round(t_or, 3), "oracle_iters": ith,
                  "oracle_true_res": trh, "threads": nthr, "gpu_fp64_s": round(gpu["fp64"], 5),
                  "gpu_f16_mixed_s": round(gpu["f16_mixed"], 5),
                  "speedup_gpu_fp64": round(t_or / gpu["fp64"], 1)})
            gh.close()
            del Uh, bh

    # 8. HMC on 24^4 (beta 5.5, m 0.05, tau 1): the plaquette force kernel alone, and whole
    #    trajectories with FP64 and mixed-precision solves (warm-started), Omelyan, 10 steps
    if want("hmc"):
        dims = (24, 24, 24, 24)
        Ud = torch.from_numpy(synth.gauge(dims, "smooth", seed=1004, eps=0.2)).to(dev)
        Qd = torch.from_numpy(synth.momenta(dims, seed=3005)).to(dev)
        vol = int(np.prod(dims))
        Fd = torch.empty_like(Qd)
        ms = event_ms(lambda: lqs.gauge_force(ctx, dims, Ud, 5.5, 1.0, out=Fd, accumulate=True), 10)
        links = 4 * vol
        # minimum traffic: every link read once, the momentum read and written (144 B each)
        emit({"suite": "gauge_force_24x4", "ms": round(ms, 4), "links": links,
              "min_GBps": round(links * 3 * 144 / ms / 1e6, 1),
              "GFLOPs_fp64": round(links * (13 * 198 + 40) / ms / 1e6, 1),
              "note": "per link 12 SU(3) products for the 6 staples + U V (198 flop each) + TA"})
        # Thermalisation: molecular-dynamics trajectories from the smooth start whose proposal is
        # kept whatever dH (fresh momenta and pseudofermion noise for each).  Then a step-size
        # scan (one trajectory per step count), and timed trajectories with the Metropolis
        # decision (u uniform) at the smallest step count whose |dH| stayed below 1.
        def traj(U_, k, u, nsteps, inner, recon, ftol, proposal=None):
            Q0 = torch.from_numpy(synth.momenta(dims, seed=4000 + k)).to(dev)
            eta = torch.from_numpy(synth.source(dims, -1, seed=5000 + k) / np.sqrt(2)).to(dev)
            return lqs.hmc_trajectory(ctx, dims, U_, Q0, eta, u=u, beta=5.5, mass=0.05, tau=1.0, nsteps=nsteps,
                                      integrator=lqs.OMELYAN, fermions=1, tol=1e-10, inner_prec=lqs.PREC[inner],
                                      inner_recon=recon, use_x0=True, force_tol=ftol, proposal=proposal)

        n_therm, ns_therm = 20, 40
        P = torch.empty_like(Ud)
        t_th = time.perf_counter()
        dhs = []
        for k in range(n_therm):
            st = traj(Ud, k, 0.0, ns_therm, "f16", 12, 1e-7, proposal=P)
            Ud.copy_(P)
            dhs.append(st["dH"])
        torch.cuda.synchronize()
        emit({"suite": "hmc_24x4_thermalisation", "trajectories": n_therm, "nsteps": ns_therm,
              "s": round(time.perf_counter() - t_th, 2), "dH_first_last": [dhs[0], dhs[-1]],
              "plaquette": 1.0 - lqs.gauge_action(ctx, dims, Ud, 1.0) / (6 * vol),
              "note": "proposal kept whatever dH (molecular dynamics with momentum refresh), FP16 inner, "
                      "force solves to 1e-7; plaquette = 1 - S_g(beta=1) / (6 V)"})
        scan = {}
        for ns in (20, 40, 80, 160):
            U0 = Ud.clone()
            st = traj(U0, 100 + ns, 0.0, ns, "f16", 12, 1e-7)
            scan[ns] = st["dH"]
        nsel = min([ns for ns in scan if abs(scan[ns]) < 1.0] or [160])
        emit({"suite": "hmc_24x4_step_scan", "dH_by_nsteps": scan, "chosen_nsteps": nsel})
        rng = np.random.default_rng(3100)
        for inner, recon, ftol in (("f64", 18, 0.0), ("f32", 12, 0.0), ("f16", 12, 0.0), ("f32", 12, 1e-7),
                                   ("f16", 12, 1e-7)):
            res = []
            for k in range(2):
                U0 = Ud.clone()
                u = float(rng.uniform())
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = traj(U0, 200 + k, u, nsel, inner, recon, ftol)
                torch.cuda.synchronize()
                res.append((time.perf_counter() - t0, st))
            emit({"suite": "hmc_24x4", "inner": inner, "recon": recon, "force_tol": ftol, "nsteps": nsel,
                  "s_per_trajectory": round(float(np.mean([t_ for t_, _ in res])), 4),
                  "cg_solves": res[-1][1]["cg_solves"], "cg_iters": res[-1][1]["cg_iters"],
                  "dH": [r_["dH"] for _, r_ in res], "accepted": [r_["accepted"] for _, r_ in res],
                  "plaquette": res[-1][1]["plaquette"], "status": res[-1][1]["status"],
                  "note": "thermalised links, Omelyan, tau 1, beta 5.5, m 0.05, solves to 1e-10 "
                          "(force solves to force_tol if set), warm-started"})


if __name__ == "__main__":
    main()
