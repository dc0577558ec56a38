// tune.cpp -- launch-shape autotuner with a persistent cache.
//
// For a (device, kernel, lattice, precision, link format, nrhs) key the tuner
// times every candidate shape (threads per block x right-hand sides per
// thread x cached or streaming link loads x prefetched words, then the other
// block -> XCD maps, with runs of time slices, and LDS staging of the input
// window for the best of these)
// with HIP events on the caller's stream (bursts of back-to-back launches),
// keeps the one with the lowest median time if it beats the default again in
// a second, alternating timing, and stores it in a flat JSON object
// {"key": "block,rhs_per_thread,stream_links,xcd_slab,lds,prefetch,trun", ...} that
// later runs load.  Tuning runs
// write only into library scratch buffers, never into caller memory.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <fstream>
#include <sstream>

#include "hop.hpp"
#include "lqs_impl.hpp"

namespace lqs {

void launch_normal_dot_shape(const Gauge &gauge, const CgVectors &v, LaunchShape sh, hipStream_t s);

Tuner::Tuner(const char *p)
{
    if (!p) return;
    path = p;
    std::ifstream in(path);
    if (!in) return;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string txt = ss.str();
    // entries look like "key": "value"; keys and values hold no quotes
    size_t pos = 0;
    while (true) {
        size_t k0 = txt.find('"', pos);
        if (k0 == std::string::npos) break;
        size_t k1 = txt.find('"', k0 + 1);
        size_t v0 = txt.find('"', k1 + 1);
        size_t v1 = v0 == std::string::npos ? v0 : txt.find('"', v0 + 1);
        if (k1 == std::string::npos || v1 == std::string::npos) break;
        cache[txt.substr(k0 + 1, k1 - k0 - 1)] = txt.substr(v0 + 1, v1 - v0 - 1);
        pos = v1 + 1;
    }
}

// On a hit the stored fields replace those of `out`; an entry without the
// third to seventh field keeps out.stream_links, out.xcd_slab, out.lds,
// out.prefetch or out.trun.
bool Tuner::lookup(const std::string &key, LaunchShape &out, int max_block) const
{
    auto it = cache.find(key);
    if (it == cache.end()) return false;
    int b = 0, k = 0, st = out.stream_links, sl = out.xcd_slab, ld = out.lds, pf = out.prefetch, tr = out.trun;
    const int n = std::sscanf(it->second.c_str(), "%d,%d,%d,%d,%d,%d,%d", &b, &k, &st, &sl, &ld, &pf, &tr);
    if (n < 2) return false;
    if (b < 64 || b > max_block || (b & 63) || !(k == 1 || k == 2 || k == 4) || !(st == 0 || st == 1) ||
        !(sl >= -1 && sl <= 3) || !(ld == 0 || ld == 1) || !(pf == 0 || pf == 1) || tr < -1)
        return false;
    out.block = b;
    out.rhs_per_thread = k;
    out.stream_links = st;
    out.xcd_slab = sl;
    out.lds = ld;
    out.prefetch = pf;
    out.trun = tr;
    return true;
}

void Tuner::store(const std::string &key, const LaunchShape &v)
{
    cache[key] = std::to_string(v.block) + "," + std::to_string(v.rhs_per_thread) + "," +
                 std::to_string(v.stream_links) + "," + std::to_string(v.xcd_slab) + "," + std::to_string(v.lds) +
                 "," + std::to_string(v.prefetch) + "," + std::to_string(v.trun);
}

void Tuner::save() const
{
    if (path.empty()) return;
    std::ofstream out(path + ".tmp");
    if (!out) return;
    out << "{\n";
    size_t i = 0;
    for (const auto &kv : cache) {
        out << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++i < cache.size() ? ",\n" : "\n");
    }
    out << "}\n";
    out.close();
    std::rename((path + ".tmp").c_str(), path.c_str());
}

std::string tune_key(const Ctx &ctx, const char *kernel, const Geom &g, int prec, int recon, int nrhs)
{
    std::ostringstream k;
    k << ctx.prop.gcnArchName << "|" << kernel << "|" << g.n[0] << "x" << g.n[1] << "x" << g.n[2] << "x" << g.n[3]
      << "|p" << prec << "|r" << recon << "|n" << nrhs;
    std::string s = k.str();
    std::replace(s.begin(), s.end(), '"', '_');
    return s;
}

static std::vector<LaunchShape> candidates(int nrhs)
{
    std::vector<LaunchShape> c;
    for (int k : {1, 2, 4}) {
        if (k > nrhs) break;
        for (int b : {64, 128, 256, 512})
            for (int st : {0, 1}) {
                c.push_back({b, k, st});
                LaunchShape pf{b, k, st};
                pf.prefetch = 1;
                c.push_back(pf);
            }
    }
    return c;
}

void autotune(Ctx &ctx, const Gauge &gauge, const char *kernel, int prec, int recon, int nrhs, hipStream_t s)
{
    if (!ctx.tuner) return;
    // temporal-gauge links get their own entries (a different kernel variant)
    const std::string key =
        tune_key(ctx, (std::string(kernel) + (gauge.temporal ? "_tg" : "")).c_str(), gauge.g, prec, recon, nrhs);
    LaunchShape found;
    if (ctx.tuner->lookup(key, found)) return;
    const bool is_dot = std::strcmp(kernel, "normal_dot") == 0;
    const Geom &g = gauge.g;
    const int64_t fb = field_bytes(g, prec, nrhs);
    void *in = ctx.workspace("tune.in", fb);
    void *out = ctx.workspace("tune.out", fb);
    void *aux = ctx.workspace("tune.aux", fb);
    // Non-zero, finite inputs in every precision (bytes 0x3C: binary16 1.06, FP32 0.0115,
    // FP64 1.6e-18): an all-zero FP16 site takes a shorter store path and would flatter
    // the shapes tried on it.
    LQS_HIP(hipMemsetAsync(in, 0x3C, fb, s));
    LQS_HIP(hipMemsetAsync(aux, 0x3C, fb, s));
    CgVectors v{};
    CgState *st = nullptr;
    std::vector<CgState> tmpl(nrhs);
    if (is_dot) {
        v.prec = prec;
        v.recon = recon;
        v.nrhs = nrhs;
        v.mass = 0.1;
        v.t = in;
        v.p = aux;
        v.q = out;
        v.max_blocks = cg_partials_needed(gauge, nrhs);
        v.partials = (double *)ctx.workspace("tune.partials", sizeof(double) * (size_t)v.max_blocks * nrhs);
        st = (CgState *)ctx.workspace("tune.state", sizeof(CgState) * nrhs);
        for (auto &S : tmpl) {
            S = CgState{};
            S.phase = CG_RUNNING;
            S.rho = 1.0;
            S.m2 = v.mass * v.mass;
        }
        v.state = st;
    }
    hipEvent_t e0, e1;
    LQS_HIP(hipEventCreate(&e0));
    LQS_HIP(hipEventCreate(&e1));
    const LinkRef L = gauge.ref(prec, recon);
    auto launch_once = [&](const LaunchShape &c) {
        if (is_dot) launch_normal_dot_shape(gauge, v, c, s);
        else launch_hop_gated(g, L, prec, recon, 0, 1, nrhs, in, out, nullptr, 0, c, s);
    };
    // Launches are timed in bursts of back to back calls, as a solver issues
    // them: one launch between two events also counts its own start, which on
    // lattices whose launches take 10-20 us had favoured shapes that are
    // slower in a stream of launches.  The normal kernel only reads the state
    // records (gate and mass), so they are set once.
    constexpr int BURST = 4;
    auto time_shape = [&](const LaunchShape &c) {
        if (is_dot) LQS_HIP(hipMemcpyAsync(st, tmpl.data(), sizeof(CgState) * nrhs, hipMemcpyHostToDevice, s));
        launch_once(c);
        launch_once(c);
        std::vector<float> t;
        for (int rep = 0; rep < 5; ++rep) {
            LQS_HIP(hipEventRecord(e0, s));
            for (int k = 0; k < BURST; ++k) launch_once(c);
            LQS_HIP(hipEventRecord(e1, s));
            LQS_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            LQS_HIP(hipEventElapsedTime(&ms, e0, e1));
            t.push_back(ms / BURST);
        }
        std::sort(t.begin(), t.end());
        return t[t.size() / 2];
    };
    // A shape replaces the current best only when it is faster by more than
    // MARGIN: shapes within the run-to-run spread of a few percent would
    // otherwise be picked by noise (measured: a 64-thread FP16 hop chosen
    // this way made the 64^3 x 16 solve 1 % slower than the default).
    constexpr float MARGIN = 0.98f;
    LaunchShape best_shape = default_hop_shape(L, nrhs);
    // After an idle spell the first launches run slower for several
    // milliseconds; the default shape, timed first, would be measured cold
    // against candidates timed warm.  Run it back to back for about 20 ms
    // first (the normal kernel's gate is set to running for every launch).
    {
        const auto w0 = std::chrono::steady_clock::now();
        if (is_dot) LQS_HIP(hipMemcpyAsync(st, tmpl.data(), sizeof(CgState) * nrhs, hipMemcpyHostToDevice, s));
        for (int i = 0; i < 500; ++i) {
            launch_once(best_shape);
            if ((i & 3) == 3) {
                LQS_HIP(hipStreamSynchronize(s));
                if (std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count() > 0.02) break;
            }
        }
        LQS_HIP(hipStreamSynchronize(s));
    }
    float best = time_shape(best_shape);
    auto consider = [&](const LaunchShape &c) {
        const float med = time_shape(c);
        if (med < MARGIN * best) {
            best = med;
            best_shape = c;
        }
    };
    for (const LaunchShape &c : candidates(nrhs)) consider(c);
    // the candidates use the map the lattice shape selects; try the other
    LaunchShape flip = best_shape;
    flip.xcd_slab = xcd_slab_auto(g, flip.block) ? 0 : 1;
    consider(flip);
    // and the time-inner and pencil maps, where whole tiles make up a time
    // slice or a z plane, over all time slices and in runs of 8, 4 and 2
    const LaunchShape base = best_shape;
    for (int mode : {2, 3})
        for (int run : {0, 8, 4, 2}) {
            if (run >= g.n[3]) continue;
            LaunchShape m = base;
            m.xcd_slab = mode;
            m.trun = run;
            if (m.xcd_slab == base.xcd_slab && m.trun == base.trun) continue;
            if (tile_map(g, m.block, mode, run).kind == (mode == 2 ? TM_TIME : TM_PENCIL)) consider(m);
        }
    // then the kernel with its x/y neighbours staged through LDS, where the window fits
    LaunchShape staged = best_shape;
    staged.lds = 1;
    staged.prefetch = 0;
    if (hop_lds_bytes(g, prec, staged.rhs_per_thread, staged) > 0) consider(staged);
    // Confirm a winner against the default with fresh timings, the two
    // alternating: on lattices whose launches take 10-20 us one noisy median
    // had picked shapes up to 34 % slower than the default.
    const LaunchShape def = default_hop_shape(L, nrhs);
    auto same = [](const LaunchShape &a, const LaunchShape &b) {
        return a.block == b.block && a.rhs_per_thread == b.rhs_per_thread && a.stream_links == b.stream_links &&
               a.xcd_slab == b.xcd_slab && a.lds == b.lds && a.prefetch == b.prefetch && a.trun == b.trun;
    };
    if (!same(best_shape, def)) {
        float td = 0.f, tb = 0.f;
        for (int k = 0; k < 3; ++k) {
            td += time_shape(def);
            tb += time_shape(best_shape);
        }
        if (!(tb < MARGIN * td)) best_shape = def;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx.tuner->store(key, best_shape);
    ctx.tuner->save();
}

}  // namespace lqs
