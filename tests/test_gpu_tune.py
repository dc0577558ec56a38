"""Autotuner: the sweep writes a cache, later contexts reuse it, results do not change."""
import json

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import field, gauge, lex_of, rel

pytestmark = pytest.mark.gpu

lqs = pytest.importorskip("paper_2502_03249_amd")


def test_tuning_cache_roundtrip_and_identical_results(tmp_path):
    dims, mass = (8, 8, 8, 16), 0.05
    U = synth.gauge(dims, "smooth", seed=91, eps=0.3)
    srcs = np.stack([synth.source(dims, 1, seed=910 + k) for k in range(4)])
    cache = str(tmp_path / "tune.json")

    plain = lqs.Context(0)
    g0 = gauge(plain, dims, U)
    ref = lex_of(plain, lqs.dslash_apply(plain, g0, field(plain, dims, srcs, 1)), squeeze=False)

    tuned = lqs.Context(0, tune_cache=cache, tuning=True)
    g1 = gauge(tuned, dims, U)
    got = lex_of(tuned, lqs.dslash_apply(tuned, g1, field(tuned, dims, srcs, 1)), squeeze=False)
    # a hop computes every site independently: the launch shape cannot change a bit
    assert np.array_equal(got, ref)
    b = synth.source(dims, 0, seed=92)
    bf = field(tuned, dims, b, 0)
    xf = bf.like().zero_()
    st = lqs.cg_solve(tuned, [(g1, mass, bf, xf)], tol=1e-10, inner_prec=lqs.F32, reliable_interval=100)
    assert st[0]["status"] == 0
    assert oracle.true_residual(dims, U, mass, b, lex_of(tuned, xf)) <= 1e-10
    tuned.close()

    entries = json.load(open(cache))
    keys = list(entries)
    assert any("|hop|8x8x8x16|p0|r18|n4" in k for k in keys)
    assert any("|normal_dot|8x8x8x16|p1|r18|n1" in k for k in keys)
    for v in entries.values():
        blk, k, st, sl, ld, pf, tr = (int(t) for t in v.split(","))
        assert blk in (64, 128, 256, 512) and k in (1, 2, 4) and st in (0, 1) and sl in (-1, 0, 1, 2, 3)
        assert ld in (0, 1) and pf in (0, 1) and (pf == 0 or ld == 0) and tr in (-1, 0, 2, 4, 8)

    # the persistent multi-lattice solve tunes its resident blocks per compute unit
    tuned = lqs.Context(0, tune_cache=cache, tuning=True)
    dims2 = (4, 6, 8, 10)
    U2 = synth.gauge(dims2, "haar", seed=93)
    b2 = synth.source(dims2, 0, seed=94)
    probs = []
    for d_, U_, b_ in ((dims, U, b), (dims2, U2, b2)):
        gg = gauge(tuned, d_, U_)
        bb = field(tuned, d_, b_, 0)
        probs.append((gg, 0.1, bb, bb.like().zero_()))
    st = lqs.cg_solve(tuned, probs, tol=1e-10, inner_prec=lqs.F32, reliable_interval=100, persistent=True)
    assert all(s["status"] == 0 for s in st)
    for (gg, m_, bb, xx), (d_, U_, b_) in zip(probs, ((dims, U, b), (dims2, U2, b2))):
        assert oracle.true_residual(d_, U_, m_, b_, lex_of(tuned, xx)) <= 1e-10
    tuned.close()
    entries = json.load(open(cache))
    pkeys = [k for k in entries if "|persistent|p1|r18|8x8x8x16|4x6x8x10" in k]
    assert len(pkeys) == 1
    blk, bpc = (int(t) for t in entries[pkeys[0]].split(",")[:2])
    assert blk in (256, 512, 1024) and bpc in (1, 2, 4)

    # a new context loads the cache and does not need to tune again
    again = lqs.Context(0, tune_cache=cache, tuning=True)
    g2 = gauge(again, dims, U)
    got2 = lex_of(again, lqs.dslash_apply(again, g2, field(again, dims, srcs, 1)), squeeze=False)
    assert np.array_equal(got2, ref)
    # every stored persistent shape (a 1024-thread one included) is read back, not re-tuned
    again.close()
    entries[pkeys[0]] = "1024,1,0"
    with open(cache, "w") as f:
        json.dump(entries, f)
    again = lqs.Context(0, tune_cache=cache, tuning=True)
    probs = []
    for d_, U_, b_ in ((dims, U, b), (dims2, U2, b2)):
        gg = gauge(again, d_, U_)
        bb = field(again, d_, b_, 0)
        probs.append((gg, 0.1, bb, bb.like().zero_()))
    st = lqs.cg_solve(again, probs, tol=1e-10, inner_prec=lqs.F32, reliable_interval=100, persistent=True)
    assert all(s_["status"] == 0 for s_ in st)
    again.close()
    assert json.load(open(cache)) == entries


@pytest.mark.parametrize("prec,recon,bound", [(lqs.F64, 18, 1e-12), (lqs.F32, 12, 2e-6), (lqs.F16, 12, 4e-3)])
def test_streaming_link_loads(tmp_path, prec, recon, bound):
    """Cached and streaming link loads read the same words: the hop agrees with the oracle either way
    and the two give the same bits (the products are fused in one fixed order in both kernels), and
    so do the CG solutions."""
    dims, mass = (8, 8, 8, 16), 0.05
    U = synth.gauge(dims, "haar", seed=95)
    srcs = np.stack([synth.source(dims, 1, seed=950 + k) for k in range(2)])
    b = synth.source(dims, 0, seed=96)
    want = np.stack([oracle.dslash(dims, U, srcs[k], 0) for k in range(2)])
    out = []
    for st in (0, 1):
        cache = str(tmp_path / f"tune{st}.json")
        key_arch = torch.cuda.get_device_properties(0).gcnArchName.replace('"', "_")
        entries = {}
        for kern, n in (("hop", 2), ("hop", 1), ("normal_dot", 1)):
            entries[f"{key_arch}|{kern}|8x8x8x16|p{prec}|r{recon}|n{n}"] = f"128,{n},{st}"
        with open(cache, "w") as f:
            json.dump(entries, f)
        ctx = lqs.Context(0, tune_cache=cache, tuning=False)
        g = gauge(ctx, dims, U)
        y = lex_of(ctx, lqs.dslash_apply(ctx, g, field(ctx, dims, srcs, 1, prec), recon=recon), squeeze=False)
        for k in range(2):
            assert rel(y[k], want[k]) <= bound
        bf = field(ctx, dims, b, 0)
        xf = bf.like().zero_()
        res = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=prec, inner_recon=recon,
                           reliable_interval=100)
        assert res[0]["status"] == 0
        x = lex_of(ctx, xf)
        assert oracle.true_residual(dims, U, mass, b, x) <= 1e-10
        out.append((y, x))
        ctx.close()
        assert json.load(open(cache)) == entries
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_xcd_maps_give_identical_results(tmp_path):
    """Both block -> tile maps (round robin over the XCDs, one slab per XCD)
    cover every (site tile, right-hand-side group) once: hops are bit-identical,
    and so is a CG solve, whose <p, q> partials are indexed by tile."""
    dims, mass = (6, 8, 10, 12), 0.07  # 2880 sites per parity: ragged tiles of 64
    U = synth.gauge(dims, "haar", seed=95)
    srcs = np.stack([synth.source(dims, 1, seed=950 + k) for k in range(3)])
    b = synth.source(dims, 0, seed=96)
    cache = str(tmp_path / "tune.json")
    tuned = lqs.Context(0, tune_cache=cache, tuning=True)
    g = gauge(tuned, dims, U)
    lqs.dslash_apply(tuned, g, field(tuned, dims, srcs, 1))
    lqs.dslash_apply(tuned, g, field(tuned, dims, srcs[0], 1))
    bf = field(tuned, dims, b, 0)
    lqs.cg_solve(tuned, [(g, mass, bf, bf.like().zero_())], tol=1e-10, inner_prec=lqs.F32, reliable_interval=50)
    tuned.close()
    entries = json.load(open(cache))
    keys = {n: [k for k in entries if f"|{n}|6x8x10x12|" in k] for n in ("hop", "normal_dot")}
    assert len(keys["hop"]) >= 2 and keys["normal_dot"]

    outs = []
    for sl in (0, 1):
        for k in keys["hop"]:
            entries[k] = "64,1,0,%d" % sl if k.endswith("|n1") else "64,2,0,%d" % sl
        for k in keys["normal_dot"]:
            entries[k] = "64,1,0,%d" % sl
        with open(cache, "w") as f:
            json.dump(entries, f)
        ctx = lqs.Context(0, tune_cache=cache)
        gg = gauge(ctx, dims, U)
        h3 = lex_of(ctx, lqs.dslash_apply(ctx, gg, field(ctx, dims, srcs, 1)), squeeze=False)
        h1 = lex_of(ctx, lqs.dslash_apply(ctx, gg, field(ctx, dims, srcs[0], 1)))
        bb = field(ctx, dims, b, 0)
        xx = bb.like().zero_()
        st = lqs.cg_solve(ctx, [(gg, mass, bb, xx)], tol=1e-10, inner_prec=lqs.F32, reliable_interval=50)
        assert st[0]["status"] == 0
        x = lex_of(ctx, xx)
        assert oracle.true_residual(dims, U, mass, b, x) <= 1e-10
        outs.append((h3, h1, x, st[0]["iters"]))
        ctx.close()
    (a3, a1, ax, ai), (b3, b1, bx, bi) = outs
    assert np.array_equal(a3, b3) and np.array_equal(a1, b1)
    assert ai == bi and np.array_equal(ax, bx)
    assert rel(a1, oracle.dslash(dims, U, srcs[0], 0)) <= 1e-14


@pytest.mark.parametrize("dims", [(6, 8, 10, 12), (2, 4, 2, 6)])
def test_lds_staged_hop_is_bit_identical(tmp_path, dims):
    """The hop whose x and y neighbours come from an LDS window of the block's input sites
    (other neighbours and the periodic wraps from memory) equals the plain hop bit for bit (the
    products are fused in one fixed order in every kernel variant), for one and several
    right-hand sides per thread, in every precision; both match the oracle."""
    U = synth.gauge(dims, "haar", seed=97)
    srcs = np.stack([synth.source(dims, 1, seed=970 + k) for k in range(3)])
    cache = str(tmp_path / "tune.json")
    tuned = lqs.Context(0, tune_cache=cache, tuning=True)
    g = gauge(tuned, dims, U)
    for prec in (lqs.F64, lqs.F32, lqs.F16):
        lqs.dslash_apply(tuned, g, field(tuned, dims, srcs, 1, prec))
        lqs.dslash_apply(tuned, g, field(tuned, dims, srcs[0], 1, prec))
    tuned.close()
    entries = json.load(open(cache))
    keys = [k for k in entries if "|hop|" in k]
    assert len(keys) >= 6
    outs = []
    for ld in (0, 1):
        for k in keys:
            entries[k] = "64,1,0,-1,%d" % ld if k.endswith("|n1") else "64,2,1,0,%d" % ld
        with open(cache, "w") as f:
            json.dump(entries, f)
        ctx = lqs.Context(0, tune_cache=cache)
        gg = gauge(ctx, dims, U)
        res = []
        for prec in (lqs.F64, lqs.F32, lqs.F16):
            res.append(lex_of(ctx, lqs.dslash_apply(ctx, gg, field(ctx, dims, srcs, 1, prec)), squeeze=False))
            res.append(lex_of(ctx, lqs.dslash_apply(ctx, gg, field(ctx, dims, srcs[0], 1, prec))))
            res.append(lex_of(ctx, lqs.dslash_dagger(ctx, gg, field(ctx, dims, srcs, 1, prec)), squeeze=False))
        outs.append(res)
        ctx.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    for k in range(3):
        want = oracle.dslash(dims, U, srcs[k], 0)
        assert rel(outs[1][0][k], want) <= 1e-12 and rel(outs[1][3][k], want) <= 2e-6
        assert rel(outs[1][6][k], want) <= 4e-3


def test_lds_staged_normal_kernel_in_cg(tmp_path):
    """A multi-vector mixed-precision CG whose hop and fused normal kernel both stage their
    input through LDS converges to the FP64 true residual, column by column, and gives the
    unstaged solve's bits and iteration counts."""
    dims, mass = (6, 8, 10, 12), 0.1
    U = synth.gauge(dims, "smooth", seed=98, eps=0.3)
    b = np.stack([synth.source(dims, 0, seed=980 + k) for k in range(3)])
    cache = str(tmp_path / "tune.json")
    tuned = lqs.Context(0, tune_cache=cache, tuning=True)
    g = gauge(tuned, dims, U)
    bf = field(tuned, dims, b, 0)
    lqs.cg_solve(tuned, [(g, mass, bf, bf.like().zero_())], tol=1e-10, inner_prec=lqs.F32, reliable_interval=50)
    tuned.close()
    entries = json.load(open(cache))
    keys = [k for k in entries if ("|hop|" in k or "|normal_dot|" in k) and k.endswith("|n3")]
    assert len(keys) == 2
    xs = []
    for ld in (0, 1):
        for k in keys:
            entries[k] = "64,2,0,-1,%d" % ld
        with open(cache, "w") as f:
            json.dump(entries, f)
        ctx = lqs.Context(0, tune_cache=cache)
        gg = gauge(ctx, dims, U)
        bb = field(ctx, dims, b, 0)
        xx = bb.like().zero_()
        st = lqs.cg_solve(ctx, [(gg, mass, bb, xx)], tol=1e-10, inner_prec=lqs.F32, reliable_interval=50)
        assert all(s_["status"] == 0 for s_ in st)
        x = lex_of(ctx, xx, squeeze=False)
        for k in range(3):
            assert oracle.true_residual(dims, U, mass, b[k], x[k]) <= 1e-10
        xs.append((x, [s_["iters"] for s_ in st]))
        ctx.close()
    assert np.array_equal(xs[1][0], xs[0][0]) and xs[1][1] == xs[0][1]


def test_lds_staged_temporal_gauge_hop(tmp_path):
    """LDS staging combined with the temporal-gauge hop (unit t-links by site index): equal to
    the unstaged temporal hop bit for bit and to the oracle on the gauge-fixed links."""
    dims = (4, 6, 8, 10)  # 96-site time slices: wavefronts straddle slices
    U = synth.gauge(dims, "haar", seed=99)
    ctx0 = lqs.Context(0)
    Uf = lqs.gauge_fix_temporal(ctx0, dims, torch.from_numpy(U).to("cuda"))[0].cpu().numpy()
    ctx0.close()
    srcs = np.stack([synth.source(dims, 1, seed=990 + k) for k in range(3)])
    cache = str(tmp_path / "tune.json")
    tuned = lqs.Context(0, tune_cache=cache, tuning=True)
    g = lqs.Gauge(tuned, dims, torch.from_numpy(Uf).to("cuda"), lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
    for prec in (lqs.F64, lqs.F32):
        lqs.dslash_apply(tuned, g, field(tuned, dims, srcs, 1, prec), recon=12)
    tuned.close()
    entries = json.load(open(cache))
    keys = [k for k in entries if "|hop_tg|" in k]
    assert len(keys) == 2
    outs = []
    for ld in (0, 1):
        for k in keys:
            entries[k] = "64,2,1,0,%d" % ld
        with open(cache, "w") as f:
            json.dump(entries, f)
        ctx = lqs.Context(0, tune_cache=cache)
        gg = lqs.Gauge(ctx, dims, torch.from_numpy(Uf).to("cuda"), lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
        outs.append([lex_of(ctx, lqs.dslash_apply(ctx, gg, field(ctx, dims, srcs, 1, prec), recon=12),
                            squeeze=False) for prec in (lqs.F64, lqs.F32)])
        ctx.close()
    assert np.array_equal(outs[1][0], outs[0][0]) and np.array_equal(outs[1][1], outs[0][1])
    for k in range(3):
        want = oracle.dslash(dims, Uf, srcs[k], 0)
        assert rel(outs[1][0][k], want) <= 1e-12 and rel(outs[1][1][k], want) <= 2e-6


@pytest.mark.parametrize("prec,recon", [(lqs.F16, 12), (lqs.F64, 18)])
def test_lds_staged_hop_in_cg_two_columns(tmp_path, prec, recon):
    """A CG whose hop stages its input through LDS gives the unstaged solve's bits, iteration
    counts and reliable updates in FP16 storage and FP64, for two columns that converge at
    different iterations (the first idles behind its FP64 check while the other continues)."""
    dims, mass = (8, 8, 8, 16), 0.05
    U = synth.gauge(dims, "smooth", seed=96, eps=0.3)
    b = np.stack([synth.source(dims, 0, seed=960), 1e-3 * synth.source(dims, 0, seed=961)])
    cache = str(tmp_path / "tune.json")
    runs = []
    for ld in (0, 1):
        key = "|".join([torch.cuda.get_device_properties(0).gcnArchName, "hop", "8x8x8x16", "p%d" % prec,
                        "r%d" % recon, "n2"])
        with open(cache, "w") as f:
            json.dump({key: "128,2,0,-1,%d" % ld}, f)
        ctx = lqs.Context(0, tune_cache=cache)
        g = gauge(ctx, dims, U)
        bf = field(ctx, dims, b, 0)
        xf = bf.like().zero_()
        st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=prec, inner_recon=recon,
                          reliable_interval=100)
        x = lex_of(ctx, xf, squeeze=False)
        for k in range(2):
            assert st[k]["status"] == 0
            assert oracle.true_residual(dims, U, mass, b[k], x[k]) <= 1e-10
        runs.append((x, [(s_["iters"], s_["reliable_updates"]) for s_ in st]))
        ctx.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and runs[0][1] == runs[1][1]


def _arch():
    return torch.cuda.get_device_properties(0).gcnArchName


@pytest.mark.parametrize("dims", [(8, 8, 8, 16), (4, 6, 8, 10)])
def test_prefetch_hop_is_bit_identical(tmp_path, dims):
    """The one-vector hop that requests all words of a site before its products (LF_PREFETCH)
    gives the bits of the plain hop in all six link formats, with cached and streaming link
    loads, and in temporal gauge (unit t-links by site index); both agree with the oracle."""
    U = synth.gauge(dims, "haar", seed=97)
    ctx0 = lqs.Context(0)
    Uf = lqs.gauge_fix_temporal(ctx0, dims, torch.from_numpy(U).to("cuda"))[0].cpu().numpy()
    ctx0.close()
    src = synth.source(dims, 1, seed=970)
    tag = "x".join(str(d) for d in dims)
    cache = str(tmp_path / "tune.json")
    fmts = [(pr, rc) for pr in (lqs.F64, lqs.F32, lqs.F16) for rc in (18, 12)]
    bound = {lqs.F64: 1e-12, lqs.F32: 2e-6, lqs.F16: 4e-3}
    for st in (0, 1):
        outs = []
        for pf in (0, 1):
            entries = {}
            for kern in ("hop", "hop_tg"):
                for pr, rc in fmts:
                    entries["|".join([_arch(), kern, tag, "p%d" % pr, "r%d" % rc, "n1"])] = "64,1,%d,-1,0,%d" % (st, pf)
            with open(cache, "w") as f:
                json.dump(entries, f)
            ctx = lqs.Context(0, tune_cache=cache)
            g = gauge(ctx, dims, U)
            gt = lqs.Gauge(ctx, dims, torch.from_numpy(Uf).to("cuda"), lqs.FMT_ALL | lqs.TEMPORAL_GAUGE)
            y = [lex_of(ctx, lqs.dslash_apply(ctx, g, field(ctx, dims, src, 1, pr), recon=rc)) for pr, rc in fmts]
            yt = [lex_of(ctx, lqs.dslash_apply(ctx, gt, field(ctx, dims, src, 1, pr), recon=12))
                  for pr in (lqs.F64, lqs.F32, lqs.F16)]
            outs.append((y, yt))
            ctx.close()
            assert json.load(open(cache)) == entries
        for a, b in zip(outs[0][0] + outs[0][1], outs[1][0] + outs[1][1]):
            assert np.array_equal(a, b)
        want, want_t = oracle.dslash(dims, U, src, 0), oracle.dslash(dims, Uf, src, 0)
        for (pr, rc), y in zip(fmts, outs[1][0]):
            assert rel(y, want) <= bound[pr], (pr, rc)
        for pr, y in zip((lqs.F64, lqs.F32, lqs.F16), outs[1][1]):
            assert rel(y, want_t) <= bound[pr], pr


@pytest.mark.parametrize("prec,recon", [(lqs.F16, 12), (lqs.F32, 12), (lqs.F64, 18)])
def test_prefetch_in_cg(tmp_path, prec, recon):
    """A CG whose hop and fused normal kernel prefetch (LF_PREFETCH) gives the plain solve's bits,
    iteration count and reliable updates."""
    dims, mass = (8, 8, 8, 16), 0.05
    U = synth.gauge(dims, "smooth", seed=98, eps=0.3)
    b = synth.source(dims, 0, seed=980)
    cache = str(tmp_path / "tune.json")
    runs = []
    for pf in (0, 1):
        entries = {"|".join([_arch(), kern, "8x8x8x16", "p%d" % pr, "r%d" % rc, "n1"]): "256,1,0,-1,0,%d" % pf
                   for kern in ("hop", "normal_dot") for pr in (lqs.F64, prec) for rc in (18, recon)}
        with open(cache, "w") as f:
            json.dump(entries, f)
        ctx = lqs.Context(0, tune_cache=cache)
        g = gauge(ctx, dims, U)
        bf = field(ctx, dims, b, 0)
        xf = bf.like().zero_()
        st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=prec, inner_recon=recon,
                          reliable_interval=100)
        x = lex_of(ctx, xf)
        assert st[0]["status"] == 0
        assert oracle.true_residual(dims, U, mass, b, x) <= 1e-10
        runs.append((x, st[0]["iters"], st[0]["reliable_updates"]))
        ctx.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and runs[0][1:] == runs[1][1:]


@pytest.mark.parametrize("prec,recon,bound", [(lqs.F64, 18, 1e-12), (lqs.F32, 12, 2e-6), (lqs.F16, 12, 4e-3)])
def test_prefetch_multi_rhs_bit_identical(tmp_path, prec, recon, bound):
    """Several vectors per thread with prefetched words: every column equals the one-vector plain
    hop bit for bit (five vectors, so the last group of four is partly empty), and a five-column
    block CG gives the plain block CG's bits and iteration counts."""
    dims, mass, n = (8, 8, 8, 16), 0.05, 5
    U = synth.gauge(dims, "smooth", seed=99, eps=0.3)
    srcs = np.stack([synth.source(dims, 1, seed=990 + k) for k in range(n)])
    b = np.stack([synth.source(dims, 0, seed=995 + k) for k in range(n)])
    cache = str(tmp_path / "tune.json")
    key = lambda kern, pr, rc, nn: "|".join([_arch(), kern, "8x8x8x16", "p%d" % pr, "r%d" % rc, "n%d" % nn])
    # the CG runs only for 256-thread shapes: the block size sets the tiles whose partials the
    # dot products add, so solves at other block sizes agree only to rounding
    shapes = ["256,4,0,2,0,0", "128,4,0,2,0,1", "256,4,0,2,0,1", "64,2,1,-1,0,1", "256,4,1,0,0,1"]
    outs, sols = [], []
    for sh in ["256,1,0,-1,0,0"] + shapes:
        ents = {key("hop", prec, recon, nn): sh if nn == n else "256,1,0,-1,0,0" for nn in (1, n)}
        ents.update({key("normal_dot", prec, recon, n): sh})
        with open(cache, "w") as f:
            json.dump(ents, f)
        ctx = lqs.Context(0, tune_cache=cache)
        g = gauge(ctx, dims, U)
        if sh.startswith("256,1,"):
            y = np.stack([lex_of(ctx, lqs.dslash_apply(ctx, g, field(ctx, dims, srcs[k], 1, prec), recon=recon))
                          for k in range(n)])
        else:
            y = lex_of(ctx, lqs.dslash_apply(ctx, g, field(ctx, dims, srcs, 1, prec), recon=recon), squeeze=False)
        outs.append(y)
        if prec != lqs.F64 and sh.startswith("256,"):
            bf = field(ctx, dims, b, 0)
            xf = bf.like().zero_()
            st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=prec, inner_recon=recon,
                              reliable_interval=100)
            assert all(s_["status"] == 0 for s_ in st)
            sols.append((lex_of(ctx, xf, squeeze=False), [s_["iters"] for s_ in st]))
        ctx.close()
    for y in outs[1:]:
        assert np.array_equal(y, outs[0])
    for k in range(n):
        assert rel(outs[0][k], oracle.dslash(dims, U, srcs[k], 0)) <= bound
    for x, it in sols[1:]:
        assert np.array_equal(x, sols[0][0]) and it == sols[0][1]
    if sols:
        for k in range(n):
            assert oracle.true_residual(dims, U, mass, b[k], sols[0][0][k]) <= 1e-10


@pytest.mark.parametrize("dims", [(32, 16, 4, 8), (32, 32, 4, 6)])
@pytest.mark.parametrize("prec,recon,bound", [(lqs.F64, 18, 1e-12), (lqs.F16, 12, 4e-3)])
def test_tile_maps_and_time_runs_bit_identical(tmp_path, dims, prec, recon, bound):
    """Time-inner and pencil block -> tile maps, over all time slices and in runs of 2 and 4, on
    lattices whose z planes hold one or two whole 256-site tiles (32x32x4x6: two bands, and runs
    of 4 over 6 slices end with a shorter run): the hop of five vectors (4 per thread, 2 groups)
    and a one-vector solve give the round-robin map's bits and iteration counts."""
    mass, n = 0.05, 5
    tag = "x".join(str(d) for d in dims)
    U = synth.gauge(dims, "smooth", seed=101, eps=0.3)
    srcs = np.stack([synth.source(dims, 1, seed=1010 + k) for k in range(n)])
    b = synth.source(dims, 0, seed=1020)
    cache = str(tmp_path / "tune.json")
    key = lambda kern, nn: "|".join([_arch(), kern, tag, "p%d" % prec, "r%d" % recon, "n%d" % nn])
    maps = ["0,0", "2,0", "2,2", "3,0", "3,4", "3,2"]
    outs, sols = [], []
    for m in maps:
        ents = {key("hop", n): "256,4,0,%s,0,1,%s" % tuple(m.split(",")),
                key("hop", 1): "256,1,0,%s,0,0,%s" % tuple(m.split(",")),
                key("normal_dot", 1): "256,1,0,%s,0,1,%s" % tuple(m.split(","))}
        with open(cache, "w") as f:
            json.dump(ents, f)
        ctx = lqs.Context(0, tune_cache=cache)
        g = gauge(ctx, dims, U)
        outs.append(lex_of(ctx, lqs.dslash_apply(ctx, g, field(ctx, dims, srcs, 1, prec), recon=recon), squeeze=False))
        bf = field(ctx, dims, b, 0)
        xf = bf.like().zero_()
        st = lqs.cg_solve(ctx, [(g, mass, bf, xf)], tol=1e-10, inner_prec=prec, inner_recon=recon,
                          reliable_interval=100)
        assert st[0]["status"] == 0
        sols.append((lex_of(ctx, xf), st[0]["iters"]))
        ctx.close()
    for y in outs[1:]:
        assert np.array_equal(y, outs[0])
    for x, it in sols[1:]:
        assert np.array_equal(x, sols[0][0]) and it == sols[0][1]
    for k in range(n):
        assert rel(outs[0][k], oracle.dslash(dims, U, srcs[k], 0)) <= bound
    assert oracle.true_residual(dims, U, mass, b, sols[0][0]) <= 1e-10
