// capi.cpp -- the extern "C" boundary declared in include/lqs.h: argument
// validation before any launch, C++ exceptions mapped to lqs_status, and the
// lifetime of contexts, gauge objects and workspaces.
#include <cmath>
#include <cstring>
#include <string>

#include "lqs_impl.hpp"

namespace lqs {

void autotune(Ctx &ctx, const Gauge &gauge, const char *kernel, int prec, int recon, int nrhs, hipStream_t s);

static thread_local std::string g_last_error;

Geom make_geom(const int32_t dims[4])
{
    Geom g;
    for (int i = 0; i < 4; ++i) g.n[i] = dims[i];
    g.vh = (int32_t)(((int64_t)dims[0] * dims[1] * dims[2] * dims[3]) / 2);
    return g;
}

int64_t field_bytes(const Geom &g, int prec, int nrhs)
{
    return spinor_bytes_per_site(prec) * (int64_t)g.vh * nrhs;
}

void *Ctx::workspace(const std::string &slot, size_t bytes)
{
    auto it = ws.find(slot);
    if (it != ws.end() && it->second.second >= bytes) return it->second.first;
    if (it != ws.end()) {
        LQS_HIP(hipDeviceSynchronize());
        LQS_HIP(hipFree(it->second.first));
        ws.erase(it);
    }
    void *p = nullptr;
    LQS_HIP(hipMalloc(&p, bytes < 256 ? 256 : bytes));
    ws[slot] = {p, bytes};
    return p;
}

void *Ctx::pinned(const std::string &slot, size_t bytes)
{
    auto it = pinned_ws.find(slot);
    if (it != pinned_ws.end() && it->second.second >= bytes) return it->second.first;
    if (it != pinned_ws.end()) {
        LQS_HIP(hipDeviceSynchronize());
        LQS_HIP(hipHostFree(it->second.first));
        pinned_ws.erase(it);
    }
    void *p = nullptr;
    LQS_HIP(hipHostMalloc(&p, bytes < 256 ? 256 : bytes, hipHostMallocDefault));
    pinned_ws[slot] = {p, bytes};
    return p;
}

hipStream_t Ctx::side_stream(int i)
{
    while ((int)side_streams.size() <= i) {
        hipStream_t st = nullptr;
        LQS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        side_streams.push_back(st);
    }
    return side_streams[i];
}

Ctx::~Ctx()
{
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    for (auto &kv : ws) (void)hipFree(kv.second.first);
    for (auto &kv : pinned_ws) (void)hipHostFree(kv.second.first);
    for (hipStream_t st : side_streams) (void)hipStreamDestroy(st);
    for (auto &e : prof_events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (tuner) tuner->save();
}

Gauge::~Gauge()
{
    for (auto &row : fmt)
        for (auto &p : row)
            if (p) (void)hipFree(p);
}

}  // namespace lqs

using namespace lqs;

// ---------------------------------------------------------------------------
// validation helpers

static void check_dims(const int32_t *dims)
{
    LQS_REQUIRE(dims != nullptr, LQS_EINVAL, "dims is NULL");
    int64_t v = 1;
    for (int i = 0; i < 4; ++i) {
        LQS_REQUIRE(dims[i] >= 2 && dims[i] % 2 == 0, LQS_EINVAL, "every extent must be even and >= 2");
        v *= dims[i];
    }
    LQS_REQUIRE(v <= (int64_t(1) << 30), LQS_EINVAL, "volume above 2^30 sites");
}

static void check_ptr(const void *p, const char *what)
{
    LQS_REQUIRE(p != nullptr, LQS_EINVAL, std::string(what) + " is NULL");
    LQS_REQUIRE(((uintptr_t)p & 15) == 0, LQS_EINVAL, std::string(what) + " is not 16-byte aligned");
}

static void check_field(const lqs_field *f, const char *what)
{
    LQS_REQUIRE(f != nullptr, LQS_EINVAL, std::string(what) + " is NULL");
    check_ptr(f->data, what);
    LQS_REQUIRE(f->prec >= 0 && f->prec <= 2, LQS_EINVAL, std::string(what) + ": bad precision");
    LQS_REQUIRE(f->parity == 0 || f->parity == 1, LQS_EINVAL, std::string(what) + ": parity must be 0 or 1");
    LQS_REQUIRE(f->nrhs >= 1 && f->nrhs <= 16, LQS_EINVAL, std::string(what) + ": nrhs must be in 1..16");
}

template <typename F> static lqs_status guard(F &&f)
{
    try {
        f();
        return LQS_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return LQS_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return LQS_EHIP;
    } catch (...) {
        g_last_error = "unknown error";
        return LQS_EHIP;
    }
}

static hipStream_t as_stream(void *s) { return (hipStream_t)s; }

// ---------------------------------------------------------------------------

extern "C" {

const char *lqs_strerror(lqs_status s)
{
    switch (s) {
    case LQS_OK: return "success";
    case LQS_ENOTCONV: return "not converged within max_iter";
    case LQS_EINVAL: return "invalid argument";
    case LQS_EHIP: return "HIP runtime error";
    case LQS_ENOMEM: return "out of device memory";
    case LQS_EBREAKDOWN: return "CG breakdown (p.Mp <= 0)";
    case LQS_ENONFINITE: return "non-finite value in CG";
    case LQS_EUNSUPPORTED: return "unsupported format or option";
    default: return "unknown status";
    }
}

const char *lqs_last_error(void) { return g_last_error.c_str(); }

lqs_status lqs_ctx_create(int32_t device, const char *tune_cache_path, lqs_ctx **out)
{
    return guard([&] {
        LQS_REQUIRE(out != nullptr, LQS_EINVAL, "out is NULL");
        int n = 0;
        LQS_HIP(hipGetDeviceCount(&n));
        LQS_REQUIRE(device >= 0 && device < n, LQS_EINVAL, "no such device");
        LQS_HIP(hipSetDevice(device));
        auto *c = new lqs_ctx();
        c->device = device;
        hipError_t e = hipGetDeviceProperties(&c->prop, device);
        if (e != hipSuccess) {
            delete c;
            LQS_HIP(e);
        }
        c->num_cu = c->prop.multiProcessorCount;
        try {
            c->noalloc_scratch = noalloc_scratch(device);
            c->tuner.reset(new Tuner(tune_cache_path));
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
    });
}

void lqs_ctx_destroy(lqs_ctx *ctx) { delete ctx; }

lqs_status lqs_set_tuning(lqs_ctx *ctx, int32_t enable)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        ctx->tuning = enable != 0;
    });
}

lqs_status lqs_set_graphs(lqs_ctx *ctx, int32_t enable)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        ctx->graphs = enable != 0;
    });
}

lqs_status lqs_field_bytes(const int32_t dims[4], int32_t prec, int32_t nrhs, size_t *bytes)
{
    return guard([&] {
        check_dims(dims);
        LQS_REQUIRE(prec >= 0 && prec <= 2, LQS_EINVAL, "bad precision");
        LQS_REQUIRE(nrhs >= 1 && nrhs <= 16, LQS_EINVAL, "nrhs must be in 1..16");
        LQS_REQUIRE(bytes != nullptr, LQS_EINVAL, "bytes is NULL");
        *bytes = (size_t)field_bytes(make_geom(dims), prec, nrhs);
    });
}

lqs_status lqs_gauge_create(lqs_ctx *ctx, const int32_t dims[4], const double *links, uint32_t formats, void *stream,
                            lqs_gauge **out)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr && out != nullptr, LQS_EINVAL, "ctx or out is NULL");
        check_dims(dims);
        check_ptr(links, "links");
        LQS_REQUIRE((formats & ~(LQS_FMT_ALL | LQS_TEMPORAL_GAUGE)) == 0, LQS_EINVAL, "unknown format bits");
        LQS_HIP(hipSetDevice(ctx->device));
        const bool temporal = (formats & LQS_TEMPORAL_GAUGE) != 0;
        if (temporal) {
            const double v = temporal_gauge_violation(*ctx, make_geom(dims), links, as_stream(stream));
            LQS_REQUIRE(v <= 1e-12, LQS_EINVAL, "links are not in temporal gauge (U_t != 1 off the last slice)");
        }
        formats = (formats & LQS_FMT_ALL) | LQS_FMT(LQS_F64, 18);
        auto *g = new lqs_gauge();
        try {
            g->ctx = ctx;
            g->g = make_geom(dims);
            g->vh = g->g.vh;
            g->temporal = temporal;
            g->pitch = temporal ? g->vh + TEMPORAL_PAD : g->vh;
            for (int prec = 0; prec < 3; ++prec)
                for (int rc = 0; rc < 2; ++rc) {
                    const int recon = rc ? 12 : 18;
                    if (!(formats & LQS_FMT(prec, recon))) continue;
                    const size_t bytes = (size_t)link_block_bytes_per_site(prec, recon) * g->pitch * 8;
                    LQS_HIP(hipMalloc(&g->fmt[prec][rc], bytes));
                    launch_pack_links(g->g, links, prec, recon, g->pitch, g->fmt[prec][rc], as_stream(stream));
                    if (temporal) launch_unit_link(g->g, prec, recon, g->pitch, g->fmt[prec][rc], as_stream(stream));
                }
        } catch (...) {
            delete g;
            throw;
        }
        *out = g;
    });
}

void lqs_gauge_destroy(lqs_gauge *g)
{
    if (!g) return;
    (void)hipDeviceSynchronize();
    delete g;
}

lqs_status lqs_gauge_fix_temporal(lqs_ctx *ctx, const int32_t dims[4], const double *links, double *out, double *G,
                                  void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        check_dims(dims);
        check_ptr(links, "links");
        check_ptr(out, "out");
        check_ptr(G, "G");
        const Geom g = make_geom(dims);
        const int64_t lb = 2 * (int64_t)g.vh * 4 * 9 * 16;
        const char *a = (const char *)links, *o = (const char *)out;
        LQS_REQUIRE(a + lb <= o || o + lb <= a, LQS_EINVAL, "links and out overlap");
        LQS_HIP(hipSetDevice(ctx->device));
        launch_gauge_fix_temporal(g, links, out, G, as_stream(stream));
    });
}

lqs_status lqs_field_pack(lqs_ctx *ctx, const int32_t dims[4], const double *lex, const lqs_field *out, void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        check_dims(dims);
        check_ptr(lex, "lex");
        check_field(out, "out");
        launch_field_pack(make_geom(dims), lex, *out, as_stream(stream));
    });
}

lqs_status lqs_field_unpack(lqs_ctx *ctx, const int32_t dims[4], const lqs_field *in, double *lex, void *stream)
{
    return lqs_field_unpack_scaled(ctx, dims, in, 1.0, lex, stream);
}

lqs_status lqs_field_unpack_scaled(lqs_ctx *ctx, const int32_t dims[4], const lqs_field *in, double scale, double *lex,
                                   void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        check_dims(dims);
        check_ptr(lex, "lex");
        check_field(in, "in");
        LQS_REQUIRE(std::isfinite(scale), LQS_EINVAL, "scale must be finite");
        launch_field_unpack(make_geom(dims), *in, scale, lex, as_stream(stream));
    });
}

lqs_status lqs_field_dot(lqs_ctx *ctx, const int32_t dims[4], const lqs_field *a, const lqs_field *b, double *out,
                         void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        check_dims(dims);
        check_field(a, "a");
        check_field(b, "b");
        check_ptr(out, "out");
        LQS_REQUIRE(a->prec == LQS_F64 && b->prec == LQS_F64, LQS_EUNSUPPORTED, "dot takes FP64 fields");
        LQS_REQUIRE(a->nrhs == b->nrhs && a->parity == b->parity, LQS_EINVAL, "fields differ in nrhs or parity");
        launch_field_dot(*ctx, make_geom(dims), a->nrhs, a->data, b->data, out, as_stream(stream));
    });
}

static lqs_status dslash_common(lqs_ctx *ctx, const lqs_gauge *g, int32_t recon, const lqs_field *in, lqs_field *out,
                                void *stream, int dagger)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr && g != nullptr, LQS_EINVAL, "ctx or gauge is NULL");
        check_field(in, "in");
        check_field(out, "out");
        LQS_REQUIRE(recon == 18 || recon == 12, LQS_EINVAL, "recon must be 18 or 12");
        LQS_REQUIRE(in->prec == out->prec, LQS_EINVAL, "in and out precision differ");
        LQS_REQUIRE(in->nrhs == out->nrhs, LQS_EINVAL, "in and out nrhs differ");
        LQS_REQUIRE(in->parity == 1 - out->parity, LQS_EINVAL, "in and out must have opposite parity");
        const int64_t bytes = field_bytes(g->g, in->prec, in->nrhs);
        const char *a = (const char *)in->data, *b = (const char *)out->data;
        LQS_REQUIRE(a + bytes <= b || b + bytes <= a, LQS_EINVAL, "in and out overlap");
        (void)g->ref(in->prec, recon);
        if (ctx->tuning) autotune(*ctx, *g, "hop", in->prec, recon, in->nrhs, as_stream(stream));
        launch_hop(*ctx, *g, in->prec, recon, dagger, out->parity, in->nrhs, in->data, out->data, as_stream(stream),
                   nullptr);
    });
}

lqs_status dslash_apply(lqs_ctx *ctx, const lqs_gauge *g, int32_t recon, const lqs_field *in, lqs_field *out,
                        void *stream)
{
    return dslash_common(ctx, g, recon, in, out, stream, 0);
}

lqs_status dslash_dagger(lqs_ctx *ctx, const lqs_gauge *g, int32_t recon, const lqs_field *in, lqs_field *out,
                         void *stream)
{
    return dslash_common(ctx, g, recon, in, out, stream, 1);
}

static void check_cg_params(const lqs_cg_params &p)
{
    LQS_REQUIRE(p.tol > 0 && std::isfinite(p.tol), LQS_EINVAL, "tol must be positive");
    LQS_REQUIRE(p.max_iter >= 1, LQS_EINVAL, "max_iter must be >= 1");
    LQS_REQUIRE(p.inner_prec >= 0 && p.inner_prec <= 2, LQS_EINVAL, "bad inner precision");
    LQS_REQUIRE(p.inner_recon == 18 || p.inner_recon == 12, LQS_EINVAL, "inner_recon must be 18 or 12");
    LQS_REQUIRE(p.reliable_interval >= 0 && p.reliable_delta >= 0 && p.reliable_delta < 1, LQS_EINVAL,
                "bad reliable-update parameters");
}

static void check_problem(const lqs_problem &pb, const lqs_cg_params &p)
{
    LQS_REQUIRE(pb.gauge != nullptr, LQS_EINVAL, "problem without gauge");
    LQS_REQUIRE(pb.nrhs >= 1 && pb.nrhs <= 16, LQS_EINVAL, "nrhs must be in 1..16");
    LQS_REQUIRE(std::isfinite(pb.mass) && pb.mass >= 0, LQS_EINVAL, "mass must be finite and >= 0");
    check_ptr(pb.b, "b");
    check_ptr(pb.x, "x");
    (void)pb.gauge->ref(p.inner_prec, p.inner_recon);
    if (p.persistent) LQS_REQUIRE(pb.nrhs == 1, LQS_EUNSUPPORTED, "persistent solve needs nrhs == 1");
}

// The worst per-right-hand-side status: errors before warnings before OK.
static lqs_status worst_status(const lqs_cg_stats *stats, int n)
{
    lqs_status worst = LQS_OK;
    for (int i = 0; i < n; ++i) {
        const lqs_status si = stats[i].status;
        if (si < 0 && (worst >= 0 || si < worst)) worst = si;
        else if (worst == LQS_OK && si > 0) worst = si;
    }
    return worst;
}

lqs_status cg_solve(lqs_ctx *ctx, int32_t nprob, const lqs_problem *probs, const lqs_cg_params *params,
                    lqs_cg_stats *stats, void *stream)
{
    lqs_status worst = LQS_OK;
    lqs_status st = guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        LQS_REQUIRE(nprob >= 1 && probs != nullptr, LQS_EINVAL, "need at least one problem");
        LQS_REQUIRE(params != nullptr && stats != nullptr, LQS_EINVAL, "params or stats is NULL");
        const lqs_cg_params &p = *params;
        check_cg_params(p);
        for (int i = 0; i < nprob; ++i) check_problem(probs[i], p);
        LQS_HIP(hipSetDevice(ctx->device));
        hipStream_t s = as_stream(stream);
        if (p.persistent) {
            std::vector<PersistentProblem> pp;
            for (int i = 0; i < nprob; ++i) pp.push_back({probs[i].gauge, probs[i].mass, probs[i].b, probs[i].x});
            persistent_solve(*ctx, pp, p, stats, s);
        } else {
            if (ctx->tuning)
                for (int i = 0; i < nprob; ++i) {
                    autotune(*ctx, *probs[i].gauge, "hop", p.inner_prec, p.inner_recon, probs[i].nrhs, s);
                    autotune(*ctx, *probs[i].gauge, "normal_dot", p.inner_prec, p.inner_recon, probs[i].nrhs, s);
                }
            if (nprob == 1) cg_solve_one(*ctx, probs[0], p, stats, s);
            else cg_solve_concurrent(*ctx, nprob, probs, p, stats, s);
        }
        int n = 0;
        for (int i = 0; i < nprob; ++i) n += probs[i].nrhs;
        worst = worst_status(stats, n);
    });
    return st != LQS_OK ? st : worst;
}

lqs_status cg_solve_noalloc(lqs_ctx *ctx, const lqs_problem *prob, const lqs_cg_params *params,
                            lqs_cg_stats *stats, void *stream)
{
    lqs_status worst = LQS_OK;
    lqs_status st = guard([&] {
        LQS_REQUIRE(ctx != nullptr && prob != nullptr, LQS_EINVAL, "ctx or problem is NULL");
        LQS_REQUIRE(params != nullptr && stats != nullptr, LQS_EINVAL, "params or stats is NULL");
        check_cg_params(*params);
        check_problem(*prob, *params);
        LQS_REQUIRE(!params->persistent, LQS_EUNSUPPORTED, "cg_solve_noalloc has no persistent mode");
        LQS_HIP(hipSetDevice(ctx->device));
        cg_solve_noalloc_impl(*ctx, *prob, *params, stats, as_stream(stream));
        worst = worst_status(stats, prob->nrhs);
    });
    return st != LQS_OK ? st : worst;
}

lqs_status cg_solve_multishift(lqs_ctx *ctx, const lqs_gauge *g, int32_t nmass, const double *masses, const double *b,
                               double *const *x, const lqs_cg_params *params, lqs_cg_stats *stats, void *stream)
{
    lqs_status worst = LQS_OK;
    lqs_status st = guard([&] {
        LQS_REQUIRE(ctx != nullptr && g != nullptr, LQS_EINVAL, "ctx or gauge is NULL");
        LQS_REQUIRE(nmass >= 1 && nmass <= 17, LQS_EINVAL, "nmass must be in 1..17");
        LQS_REQUIRE(masses != nullptr && x != nullptr && params != nullptr && stats != nullptr, LQS_EINVAL,
                    "masses, x, params or stats is NULL");
        const lqs_cg_params &p = *params;
        LQS_REQUIRE(p.tol > 0 && std::isfinite(p.tol), LQS_EINVAL, "tol must be positive");
        LQS_REQUIRE(p.max_iter >= 1, LQS_EINVAL, "max_iter must be >= 1");
        LQS_REQUIRE(p.inner_recon == 18 || p.inner_recon == 12, LQS_EINVAL, "inner_recon must be 18 or 12");
        LQS_REQUIRE(p.inner_prec == LQS_F64 || p.inner_prec == LQS_F32 || p.inner_prec == LQS_F16, LQS_EINVAL,
                    "inner_prec must be LQS_F64, LQS_F32 or LQS_F16");
        LQS_REQUIRE(!p.persistent, LQS_EUNSUPPORTED, "multi-shift CG has no persistent form");
        check_ptr(b, "b");
        for (int i = 0; i < nmass; ++i) {
            LQS_REQUIRE(std::isfinite(masses[i]) && masses[i] >= 0, LQS_EINVAL, "masses must be finite and >= 0");
            check_ptr(x[i], "x[i]");
            for (int j = 0; j < i; ++j) LQS_REQUIRE(x[i] != x[j], LQS_EINVAL, "solution fields must be distinct");
        }
        (void)g->ref(p.inner_prec, p.inner_recon);
        LQS_HIP(hipSetDevice(ctx->device));
        multishift_solve(*ctx, *g, nmass, masses, b, x, p, stats, as_stream(stream));
        for (int i = 0; i < nmass; ++i) {
            const lqs_status si = stats[i].status;
            if (si < 0 && (worst >= 0 || si < worst)) worst = si;
            else if (worst == LQS_OK && si > 0) worst = si;
        }
    });
    return st != LQS_OK ? st : worst;
}

lqs_status fermion_force(lqs_ctx *ctx, const lqs_gauge *g, const double *X, const double *Y, double coeff,
                         int32_t mode, double *force, void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr && g != nullptr, LQS_EINVAL, "ctx or gauge is NULL");
        check_ptr(X, "X");
        if (Y) check_ptr(Y, "Y");
        check_ptr(force, "force");
        LQS_REQUIRE(mode >= 0 && mode <= 2, LQS_EINVAL, "mode must be 0, 1 or 2");
        LQS_REQUIRE(std::isfinite(coeff), LQS_EINVAL, "coeff must be finite");
        hipStream_t s = as_stream(stream);
        const int64_t fb = field_bytes(g->g, F64, 1);
        double *psx = (double *)ctx->workspace("force.psx", fb);
        double *psy = psx;
        const LinkRef L = g->ref(F64, 18);
        const LaunchShape sh = default_hop_shape(L, 1);
        launch_hop_gated(g->g, L, F64, 18, 0, 1, 1, X, psx, nullptr, 0, sh, s);
        if (Y && Y != X) {
            psy = (double *)ctx->workspace("force.psy", fb);
            launch_hop_gated(g->g, L, F64, 18, 0, 1, 1, Y, psy, nullptr, 0, sh, s);
        }
        launch_force(g->g, L, X, Y ? Y : X, psx, psy, coeff, mode, force, s);
    });
}

lqs_status gauge_action(lqs_ctx *ctx, const int32_t dims[4], const double *links, double beta, double *S,
                        void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr && S != nullptr, LQS_EINVAL, "ctx or S is NULL");
        check_dims(dims);
        check_ptr(links, "links");
        LQS_REQUIRE(std::isfinite(beta), LQS_EINVAL, "beta must be finite");
        LQS_HIP(hipSetDevice(ctx->device));
        hipStream_t s = as_stream(stream);
        double *d = (double *)ctx->workspace("api.scalar", sizeof(double) * 2);
        launch_gauge_action(*ctx, make_geom(dims), links, beta, d, 0, s);
        LQS_HIP(hipMemcpyAsync(S, d, sizeof(double), hipMemcpyDeviceToHost, s));
        LQS_HIP(hipStreamSynchronize(s));
    });
}

lqs_status gauge_force(lqs_ctx *ctx, const int32_t dims[4], const double *links, double beta, double coeff,
                       int32_t accumulate, double *out, void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        check_dims(dims);
        check_ptr(links, "links");
        check_ptr(out, "out");
        LQS_REQUIRE(out != links, LQS_EINVAL, "out must not overlap links");
        LQS_REQUIRE(accumulate == 0 || accumulate == 1, LQS_EINVAL, "accumulate must be 0 or 1");
        LQS_REQUIRE(std::isfinite(beta) && std::isfinite(coeff), LQS_EINVAL, "beta and coeff must be finite");
        LQS_HIP(hipSetDevice(ctx->device));
        launch_gauge_force(make_geom(dims), links, beta, coeff, accumulate, out, as_stream(stream));
    });
}

lqs_status link_update(lqs_ctx *ctx, const int32_t dims[4], double *links, const double *mom, double eps,
                       void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        check_dims(dims);
        check_ptr(links, "links");
        check_ptr(mom, "mom");
        LQS_REQUIRE(mom != links, LQS_EINVAL, "mom must not overlap links");
        LQS_REQUIRE(std::isfinite(eps), LQS_EINVAL, "eps must be finite");
        LQS_HIP(hipSetDevice(ctx->device));
        launch_link_update(make_geom(dims), links, mom, eps, as_stream(stream));
    });
}

lqs_status kinetic_energy(lqs_ctx *ctx, const int32_t dims[4], const double *mom, double *K, void *stream)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr && K != nullptr, LQS_EINVAL, "ctx or K is NULL");
        check_dims(dims);
        check_ptr(mom, "mom");
        LQS_HIP(hipSetDevice(ctx->device));
        hipStream_t s = as_stream(stream);
        double *d = (double *)ctx->workspace("api.scalar", sizeof(double) * 2);
        launch_kinetic(*ctx, make_geom(dims), mom, d, 0, s);
        LQS_HIP(hipMemcpyAsync(K, d, sizeof(double), hipMemcpyDeviceToHost, s));
        LQS_HIP(hipStreamSynchronize(s));
    });
}

lqs_status hmc_trajectory(lqs_ctx *ctx, const int32_t dims[4], double *links, double *mom, const double *pf,
                          double u, const lqs_hmc_params *params, lqs_hmc_stats *stats, double *proposal,
                          double *phi_out, void *stream)
{
    lqs_status worst = LQS_OK;
    lqs_status st = guard([&] {
        LQS_REQUIRE(ctx != nullptr && params != nullptr && stats != nullptr, LQS_EINVAL,
                    "ctx, params or stats is NULL");
        check_dims(dims);
        check_ptr(links, "links");
        check_ptr(mom, "mom");
        LQS_REQUIRE(mom != links, LQS_EINVAL, "mom must not overlap links");
        const lqs_hmc_params &p = *params;
        LQS_REQUIRE(std::isfinite(p.beta) && p.beta >= 0, LQS_EINVAL, "beta must be finite and >= 0");
        LQS_REQUIRE(std::isfinite(p.tau) && p.tau > 0, LQS_EINVAL, "tau must be positive");
        LQS_REQUIRE(p.nsteps >= 1, LQS_EINVAL, "nsteps must be >= 1");
        LQS_REQUIRE(p.integrator == LQS_LEAPFROG || p.integrator == LQS_OMELYAN, LQS_EINVAL, "unknown integrator");
        LQS_REQUIRE(std::isfinite(p.lambda) && p.lambda >= 0 && p.lambda < 0.5, LQS_EINVAL,
                    "lambda must be in [0, 0.5)");
        LQS_REQUIRE(p.fermions >= 0 && p.fermions <= 2, LQS_EINVAL, "fermions must be 0, 1 or 2");
        LQS_REQUIRE(std::isfinite(p.force_tol) && p.force_tol >= 0, LQS_EINVAL, "force_tol must be finite and >= 0");
        LQS_REQUIRE(u >= 0 && u < 1, LQS_EINVAL, "u must be in [0, 1)");
        if (proposal) {
            check_ptr(proposal, "proposal");
            LQS_REQUIRE(proposal != links && proposal != mom, LQS_EINVAL, "proposal must not overlap links or mom");
        }
        if (p.fermions) {
            check_ptr(pf, "pf");
            LQS_REQUIRE(std::isfinite(p.mass) && p.mass > 0, LQS_EINVAL, "mass must be positive");
            const lqs_cg_params &c = p.cg;
            LQS_REQUIRE(c.tol > 0 && std::isfinite(c.tol), LQS_EINVAL, "cg.tol must be positive");
            LQS_REQUIRE(c.max_iter >= 1, LQS_EINVAL, "cg.max_iter must be >= 1");
            LQS_REQUIRE(c.inner_prec >= 0 && c.inner_prec <= 2, LQS_EINVAL, "bad cg.inner_prec");
            LQS_REQUIRE(c.inner_recon == 18 || c.inner_recon == 12, LQS_EINVAL, "cg.inner_recon must be 18 or 12");
            LQS_REQUIRE(c.reliable_interval >= 0 && c.reliable_delta >= 0 && c.reliable_delta < 1, LQS_EINVAL,
                        "bad reliable-update parameters");
            if (phi_out) check_ptr(phi_out, "phi_out");
        }
        LQS_HIP(hipSetDevice(ctx->device));
        lqs_hmc_params q = p;
        if (!q.fermions) {
            q.cg.inner_prec = LQS_F64;
            q.cg.inner_recon = 18;
        }
        *stats = lqs_hmc_stats{};
        hmc_trajectory_impl(*ctx, make_geom(dims), links, mom, pf, u, q, *stats, proposal,
                            q.fermions ? phi_out : nullptr, as_stream(stream));
        worst = stats->status;
    });
    return st != LQS_OK ? st : worst;
}

lqs_status lqs_profile_hops(lqs_ctx *ctx, int32_t enable)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        if (enable) {
            for (auto &row : ctx->prof)
                for (auto &p : row) p = Ctx::ProfSlot();
            ctx->prof_used = 0;
            ctx->profiling = true;
        } else {
            ctx->profiling = false;
        }
    });
}

lqs_status lqs_profile_hops_result(lqs_ctx *ctx, int32_t prec, int32_t recon, double min_ms, int64_t *launches,
                                   double *avg_ms, int64_t *sites_per_launch)
{
    return guard([&] {
        LQS_REQUIRE(ctx != nullptr, LQS_EINVAL, "ctx is NULL");
        LQS_REQUIRE(prec >= 0 && prec <= 2 && (recon == 18 || recon == 12), LQS_EINVAL, "bad format");
        // fold recorded events into the per-format sums (events must have completed)
        for (size_t i = 0; i < ctx->prof_used; ++i) {
            float ms = 0.f;
            LQS_HIP(hipEventSynchronize(ctx->prof_events[i].second));
            LQS_HIP(hipEventElapsedTime(&ms, ctx->prof_events[i].first, ctx->prof_events[i].second));
            if (ms < min_ms) continue;
            auto &slot = ctx->prof[ctx->prof_keys[i].first][ctx->prof_keys[i].second];
            slot.launches += 1;
            slot.ms += ms;
            slot.sites = ctx->prof_sites[i];
        }
        ctx->prof_used = 0;
        const auto &slot = ctx->prof[prec][recon == 12 ? 1 : 0];
        if (launches) *launches = slot.launches;
        if (avg_ms) *avg_ms = slot.launches ? slot.ms / slot.launches : 0.0;
        if (sites_per_launch) *sites_per_launch = slot.sites;
    });
}

}  // extern "C"
