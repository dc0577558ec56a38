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
`value` is the mean seconds per solve (lower is better).  The same run also
times the plain FP64 solve (for the mixed-vs-FP64 ratio), the standalone hop
in every link format (GB/s, GFLOP/s, fraction of 8 TB/s), and the CPU oracle.

The hop kernels are timed with HIP events recorded on the stream they are
launched on, inside the timed region; `roofline` reports the dominant kernel
of the step.  Options --only-hop / --only-copy run the launches a rocprofv3
counter pass needs and nothing else.
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
    ap.add_argument("--dims", default=None, help="override lattice, e.g. 32,32,32,8")
    return ap.parse_args()


# Sources that define the hop kernel: counter readings taken on other sources
# are not reported.
HOP_SOURCES = ["dev.hpp", "hop.hpp", "dslash.hip", "lqs_impl.hpp"]


def src_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2502_03249_amd", "csrc")
    for name in HOP_SOURCES:
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
    if not e or e.get("src_hash") != src_hash():
        return None
    return e["bytes_per_launch"]


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
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
    ctx = lqs.Context(0)
    Ud = torch.from_numpy(U).to(dev)
    g = lqs.Gauge(ctx, dims, Ud, lqs.FMT_ALL)
    bf = lqs.Field.from_lex(ctx, torch.from_numpy(b).to(dev), 0)
    xf = bf.like().zero_()
    torch.cuda.synchronize()
    del Ud
    setup_s = time.time() - t_setup
    vh = int(np.prod(dims)) // 2

    def hop_rate(prec, recon, reps):
        """Standalone hop D_eo on a random odd field; HIP events on the launch stream."""
        pr = lqs.PREC[prec]
        xin = lqs.Field.from_lex(ctx, torch.from_numpy(synth.source(dims, 1, seed=7)).to(dev), 1, pr)
        out = xin.like(parity=0)
        for _ in range(3):
            lqs.dslash_apply(ctx, g, xin, out, recon=recon)
        lqs.profile_hops(ctx, True)
        for _ in range(reps):
            lqs.dslash_apply(ctx, g, xin, out, recon=recon)
        torch.cuda.synchronize()
        n, ms, sites = lqs.profile_hops_result(ctx, pr, recon)
        lqs.profile_hops(ctx, False)
        mb = model.hop_model_bytes(pr, recon) * vh
        return {"prec": prec, "recon": recon, "ms": ms, "model_GBps": mb / ms / 1e6,
                "GFLOPs": model.FLOPS_PER_SITE * vh / ms / 1e6, "frac_hbm": mb / ms / 1e6 / PEAK_HBM_GBPS,
                "model_bytes_per_site": model.hop_model_bytes(pr, recon),
                "min_bytes_per_site": model.hop_min_bytes(pr, recon), "launches": n}

    if a.only_hop:
        prec, recon = a.only_hop.split(":")
        r = hop_rate(prec, int(recon), a.hop_reps)
        print(json.dumps(r))
        return

    inner = lqs.PREC[a.inner]

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

    # timed steps: mixed-precision solves, hop launches event-timed
    lqs.profile_hops(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(a.steps):
        st = lqs.cg_solve(ctx, [(g, MASS, bf, xf)], tol=TOL, max_iter=20000, inner_prec=inner,
                          inner_recon=a.recon, reliable_interval=a.reliable)
        stats.append(st[0])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # Launches queued after a solve converged return at once (a few us); only
    # launches longer than 20 us are counted (one working hop per iteration).
    n_hop, hop_ms, _ = lqs.profile_hops_result(ctx, inner, a.recon, min_ms=0.02)
    lqs.profile_hops(ctx, False)
    working = sum(s["iters"] for s in stats)
    mixed_s = elapsed / a.steps
    ok = all(s["status"] == 0 and s["true_rel_residual"] <= TOL for s in stats)

    # FP64 solve on the same system (untimed by the step loop, timed on its own)
    fp64 = [solve(lqs.F64, 18, 0) for _ in range(2)]
    fp64_s = min(t for t, _ in fp64)
    fp64_st = fp64[0][1]
    fp64_12 = [solve(lqs.F64, 12, 0) for _ in range(2)]
    fp64_12_s = min(t for t, _ in fp64_12)
    other = lqs.F32 if inner == lqs.F16 else lqs.F16
    other_t, other_st = solve(other, a.recon, a.reliable)

    # standalone hop in every format
    hops = [hop_rate(p, r, a.hop_reps) for p in ("f64", "f32", "f16") for r in (18, 12)]

    # roofline of the dominant kernel of the step: the inner-precision hop
    mb_site = model.hop_model_bytes(inner, a.recon)
    achieved = mb_site * vh / hop_ms / 1e6
    key = f"hop_{a.inner}_{a.recon}"
    traffic = traffic_for(key, vh)
    roof = {"bound": "hbm", "kernel": key, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic,
            "bytes_per_launch": mb_site * vh, "avg_launch_ms": round(hop_ms, 5), "launches_timed": n_hop,
            "working_launches": working}
    h64 = [h for h in hops if h["prec"] == "f64" and h["recon"] == 18][0]

    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        # Bounded sample: 6 CG iterations of the oracle on the same 64^3 x 16
        # system, scaled to the FP64 iteration count of the GPU solve.
        bl = b.copy()
        t1 = time.perf_counter()
        _, _, it, _ = oracle.cg(dims, U, MASS, bl, tol=TOL, max_iter=6)
        dt = time.perf_counter() - t1
        # the call also pays two FP64 M applications (initial residual and final check)
        per_it = dt / (it + 2)
        cpu = {"value": round(per_it * fp64_st["iters"], 2), "unit": "s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"{it} FP64 CG iterations of the 64^3x16 system (+2 operator applications) in "
                         f"{dt:.1f} s, scaled to the {fp64_st['iters']} iterations of a full solve"}

    line = {
        "metric": "Dslash GB/s & GFLOP/s (% HBM roofline); CG s-to-1e-10, mixed vs FP64",
        "value": round(mixed_s, 5), "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1000 * mixed_s, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{a.inner}-storage/f32 inner, f64 residual",
        "data": "synthetic",
        "config": {"workload": "64^3x16 even-odd staggered CG to 1e-10, m=0.01, smooth links eps=0.3",
                   "dims": list(dims), "mass": MASS, "tol": TOL, "inner": a.inner, "recon": a.recon,
                   "reliable_interval": a.reliable, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "cg": {"mixed_s": round(mixed_s, 5), "mixed_iters": stats[-1]["iters"],
               "mixed_reliable_updates": stats[-1]["reliable_updates"],
               "mixed_true_res": stats[-1]["true_rel_residual"], "all_converged": ok,
               "fp64_s": round(fp64_s, 5), "fp64_iters": fp64_st["iters"], "fp64_true_res": fp64_st["true_rel_residual"],
               "fp64_recon12_s": round(fp64_12_s, 5),
               "speedup_mixed_vs_fp64": round(fp64_s / mixed_s, 3),
               "speedup_mixed_vs_best_fp64": round(min(fp64_s, fp64_12_s) / mixed_s, 3),
               f"{'f32' if other == lqs.F32 else 'f16'}_mixed_s": round(other_t, 5),
               f"{'f32' if other == lqs.F32 else 'f16'}_mixed_iters": other_st["iters"]},
        "dslash": {"fp64_18_model_GBps": round(h64["model_GBps"], 1), "fp64_18_GFLOPs": round(h64["GFLOPs"], 1),
                   "fp64_18_frac_hbm": round(h64["frac_hbm"], 4),
                   "formats": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in h.items()} for h in hops]},
        "setup_s": round(setup_s, 1),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
