// lqs_impl.hpp -- internal declarations shared by the host runtime and the
// kernel files: context and gauge objects, kernel argument blocks, the CG
// state kept in device memory, and the launch entry points of each kernel file.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lqs.h"
#include "dev.hpp"

namespace lqs {

// ---------------------------------------------------------------------------
// errors: internal code throws Error; the C ABI layer maps it to a status.

struct Error : std::runtime_error {
    lqs_status status;
    Error(lqs_status s, const std::string &msg) : std::runtime_error(msg), status(s) {}
};

#define LQS_HIP(call)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            throw ::lqs::Error(e_ == hipErrorOutOfMemory ? LQS_ENOMEM : LQS_EHIP,                        \
                               std::string(#call) + ": " + hipGetErrorString(e_));                       \
    } while (0)

#define LQS_REQUIRE(cond, status, msg)                                                                   \
    do {                                                                                                 \
        if (!(cond)) throw ::lqs::Error((status), (msg));                                                \
    } while (0)

// ---------------------------------------------------------------------------
// CG state of one right-hand side, in device memory.  Kernels of an
// iteration run only while state == RUNNING; the FP64 residual group runs
// only while reliable_pending is set.  Scalars never leave the device during
// the iteration; the host polls this record every few iterations.

enum CgPhase : int32_t {
    CG_RUNNING = 0,
    CG_INNER_DONE = 1,  // iterated residual below target, FP64 check pending
    CG_CONVERGED = 2,   // FP64 residual below target (final)
    CG_BREAKDOWN = 3,   // p.Mp <= 0 (final)
    CG_NONFINITE = 4,   // NaN / Inf in a scalar (final)
    CG_MAXITER = 5,     // iteration cap reached, residual checked (final)
};

struct CgState {
    double rho;        // |r|^2 of the iterated residual
    double rho_old;    // |r|^2 before the last update (for beta)
    double alpha, beta;
    double stop2;      // tol^2 |b|^2
    double max_rho;    // largest rho since the last FP64 residual update
    double delta2;     // reliable-update threshold delta^2
    double true_r2;    // last FP64 |b - M x|^2
    double b2;         // |b|^2
    double m2;         // mass^2 of this right-hand side's operator M = m^2 - D_eo D_oe
    int32_t phase;
    int32_t iters;
    int32_t since_rel;
    int32_t rel_interval;  // 0: FP64 solver (no periodic updates)
    int32_t reliable_pending;
    int32_t nreliable;
    int32_t restarts;
    int32_t max_iter;
};

// Default reliable-update threshold delta of a mixed solve (an update when
// ||r|| falls below delta * max ||r|| since the last one).  FP32 storage
// drifts less than FP16 and can go longer between updates: on 64^3 x 16,
// m = 0.01, delta 0.02 saved 1.5 % with FP32 inner at the same 213
// iterations, while FP16 inner needs 0.05 (0.02 cost 7 more iterations).
inline double default_reliable_delta(int inner_prec) { return inner_prec == F32 ? 0.02 : 0.05; }

// ---------------------------------------------------------------------------
// kernel argument blocks

struct LinkRef {
    const void *base;      // start of the 8 (mu, parity) blocks
    int64_t block_bytes;   // bytes of one block = bytes_per_site * pitch
    int32_t temporal;      // links in temporal gauge: U_t = 1 except leaving t = Nt - 1
    int32_t pitch;         // sites per word plane: vh, or vh + TEMPORAL_PAD in temporal gauge,
                           // where the two t-link blocks hold a unit link at index vh
};

// Extra sites per word plane of a temporal-gauge link format (keeps the
// planes 64-site aligned; index vh of the t-link blocks is the unit link).
constexpr int TEMPORAL_PAD = 64;

struct FieldRef {
    void *data;
    int64_t rhs_stride;    // bytes between consecutive right-hand sides
};

// ---------------------------------------------------------------------------
// library objects

struct Tuner;

struct Ctx {
    int device = 0;
    hipDeviceProp_t prop{};
    int num_cu = 0;
    bool tuning = false;
    bool graphs = true;  // capture CG iteration rounds into HIP graphs
    void *noalloc_scratch = nullptr;  // this device's scratch array (cg_solve_noalloc)
    std::unique_ptr<Tuner> tuner;
    // workspace buffers by slot, grown on demand, freed with the context
    std::map<std::string, std::pair<void *, size_t>> ws;
    // pinned host buffers by slot (CG state mirrors), freed with the context
    std::map<std::string, std::pair<void *, size_t>> pinned_ws;
    // side streams for concurrent solves (default priority, non-blocking)
    std::vector<hipStream_t> side_streams;
    // hop profiling: per (prec, recon) sums of event-timed launches
    bool profiling = false;
    struct ProfSlot {
        int64_t launches = 0;
        double ms = 0.0;
        int64_t sites = 0;
    } prof[3][2];
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    std::vector<std::pair<int, int>> prof_keys;
    std::vector<int64_t> prof_sites;
    size_t prof_used = 0;

    void *workspace(const std::string &slot, size_t bytes);
    void *pinned(const std::string &slot, size_t bytes);
    hipStream_t side_stream(int i);
    ~Ctx();
};

struct Gauge {
    Ctx *ctx = nullptr;
    Geom g{};
    int64_t vh = 0;
    void *fmt[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};  // [prec][recon==12]
    bool temporal = false;
    int64_t pitch = 0;  // sites per word plane of every format (LinkRef::pitch)
    LinkRef ref(int prec, int recon) const
    {
        const int rc = recon == 12 ? 1 : 0;
        const void *p = fmt[prec][rc];
        LQS_REQUIRE(p != nullptr, LQS_EUNSUPPORTED, "gauge does not hold the requested link format");
        return {p, (int64_t)link_block_bytes_per_site(prec, recon) * pitch, temporal ? 1 : 0, (int32_t)pitch};
    }
    ~Gauge();
};

Geom make_geom(const int32_t dims[4]);
int64_t field_bytes(const Geom &g, int prec, int nrhs);

// ---------------------------------------------------------------------------
// launch entry points (one kernel file each)

// pack.hip
void launch_pack_links(const Geom &g, const double *canon, int prec, int recon, int64_t pitch, void *out,
                       hipStream_t s);
// the unit link at index vh of the two t-link blocks of a temporal-gauge format
void launch_unit_link(const Geom &g, int prec, int recon, int64_t pitch, void *links, hipStream_t s);
void launch_field_pack(const Geom &g, const double *lex, const lqs_field &out, hipStream_t s);
void launch_field_unpack(const Geom &g, const lqs_field &in, double scale, double *lex, hipStream_t s);
void launch_convert(const Geom &g, int nrhs, int prec_in, const void *in, int prec_out, void *out, hipStream_t s);
void launch_gauge_fix_temporal(const Geom &g, const double *links, double *out, double *G, hipStream_t s);
double temporal_gauge_violation(Ctx &ctx, const Geom &g, const double *links, hipStream_t s);
struct Ctx;
void launch_field_dot(Ctx &ctx, const Geom &g, int nrhs, const void *a, const void *b, double *out, hipStream_t s);

// dslash.hip
struct LaunchShape {
    int block = 256;       // threads per block
    int rhs_per_thread = 1;
    int stream_links = 0;  // 1: link words fetched with streaming (nontemporal) loads
    int xcd_slab = -1;     // block -> tile map: 0 round robin, 1 one slab per XCD, 2 time-inner,
                           // 3 pencil, -1 by lattice shape
    int lds = 0;           // 1: x and y neighbours from an LDS window of the block's input sites
    int prefetch = 0;      // 1 (no LDS window): the words of a group of directions requested
                           // before their products (LF_PREFETCH)
    int trun = -1;         // time-inner and pencil maps: time slices per run (0: all, -1: time_run)
};
// Link footprint from which the hop streams its links by default: beyond
// about three quarters of the 256 MB last-level cache (MALL) the links of one
// application are no longer there at the next one.
constexpr int64_t STREAM_LINK_BYTES = 192ll << 20;
void launch_hop(Ctx &ctx, const Gauge &gauge, int prec, int recon, int dagger, int out_parity, int nrhs,
                const void *in, void *out, hipStream_t s, const CgState *gate);
LaunchShape default_hop_shape(const LinkRef &L, int nrhs);
void launch_hop_gated(const Geom &g, LinkRef L, int prec, int recon, int dagger, int parity, int nrhs,
                      const void *in, void *out, const CgState *gate, int gate_mode, LaunchShape sh, hipStream_t s);
void launch_hop_shape(const Geom &g, LinkRef links, int prec, int recon, int dagger, int out_parity, int nrhs,
                      const void *in, void *out, const CgState *gate, LaunchShape shape, hipStream_t s);

// blas.hip -- the CG kernels (fused hop + epilogue, vector updates)
struct CgVectors {
    int prec;               // inner precision of p, q, t
    int acc_prec;           // precision of x_lo and r (F64 in the plain solver)
    int recon;              // inner link format
    int nrhs;
    double mass;            // (the kernels read each right-hand side's m^2 from its CgState)
    void *p, *q, *t;        // p, q even; t odd
    void *r, *xlo;          // iterated residual and inner solution (even)
    double *x, *b, *rhi;    // FP64: solution, source, FP64 residual (even)
    void *t64;              // FP64 odd scratch (residual hop)
    CgState *state;         // nrhs records
    double *partials;       // nrhs * max_blocks (normal kernel, residual, init)
    double *partials2;      // nrhs * max_blocks (update kernel)
    int max_blocks;
};
void cg_init(Ctx &ctx, const Gauge &gauge, CgVectors &v, bool use_x0, hipStream_t s);
void cg_iteration(Ctx &ctx, const Gauge &gauge, CgVectors &v, hipStream_t s, bool with_reliable);
int cg_partials_needed(const Gauge &gauge, int nrhs);
// gflops and gbytes_per_s of one right-hand side's stats from its iterations
// and times (inner precision and link format of the iteration; nrhs
// right-hand sides share the link reads)
void cg_fill_rates(lqs_cg_stats &o, const Gauge &gauge, int prec, int recon, int nrhs);

// force.hip
void launch_force(const Geom &g, LinkRef links64, const double *X, const double *Y, const double *psx,
                  const double *psy, double coeff, int mode, double *out, hipStream_t s);

// persistent.hip
struct PersistentProblem {
    const Gauge *gauge;
    double mass;
    const double *b;
    double *x;
};
void persistent_solve(Ctx &ctx, const std::vector<PersistentProblem> &probs, const lqs_cg_params &prm,
                      lqs_cg_stats *stats, hipStream_t s);

// cg.hip: device workspace of one problem's solve
size_t cg_workspace_bytes(const Gauge &gauge, const lqs_cg_params &prm, int nrhs);
// cg.hip: the allocation-free solve and its per-device scratch array
constexpr size_t NOALLOC_SCRATCH_BYTES = LQS_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;
void *noalloc_scratch(int device);
void cg_solve_noalloc_impl(Ctx &ctx, const lqs_problem &pb, const lqs_cg_params &prm, lqs_cg_stats *stats,
                           hipStream_t s);
// cg.hip: one problem with the multi-kernel iteration (returns when done)
// masses: one per right-hand side (null: pb.mass for all)
void cg_solve_one(Ctx &ctx, const lqs_problem &pb, const lqs_cg_params &prm, lqs_cg_stats *stats, hipStream_t s,
                  const std::vector<double> *masses = nullptr);
// several problems, each on its own side stream, iterated concurrently
void cg_solve_concurrent(Ctx &ctx, int nprob, const lqs_problem *probs, const lqs_cg_params &prm,
                         lqs_cg_stats *stats, hipStream_t s);

// hmc.hip (canonical [4][V][3][3] complex128 links and momenta)
void launch_gauge_action(Ctx &ctx, const Geom &g, const double *U, double beta, double *out, int slot, hipStream_t s);
void launch_kinetic(Ctx &ctx, const Geom &g, const double *Q, double *out, int slot, hipStream_t s);
// packed: optional word-major FP64 18-real copy of U (read instead of U)
void launch_gauge_force(const Geom &g, const double *U, double beta, double coeff, int accumulate, double *out,
                        hipStream_t s, const LinkRef *packed = nullptr);
void launch_link_update(const Geom &g, double *U, const double *Q, double eps, hipStream_t s);
void hmc_trajectory_impl(Ctx &ctx, const Geom &g, double *links, double *mom, const double *pf, double u,
                         const lqs_hmc_params &prm, lqs_hmc_stats &st, double *proposal, double *phi_out,
                         hipStream_t s);

// multishift.hip
void multishift_solve(Ctx &ctx, const Gauge &gauge, int nmass, const double *masses, const double *b, double *const *x,
                      const lqs_cg_params &prm, lqs_cg_stats *stats, hipStream_t s);

// tune.cpp
struct Tuner {
    std::string path;
    std::map<std::string, std::string> cache;  // key -> "block,rhs_per_thread,stream_links,xcd_slab,lds"
    explicit Tuner(const char *p);
    bool lookup(const std::string &key, LaunchShape &out, int max_block = 512) const;
    void store(const std::string &key, const LaunchShape &v);
    void save() const;
};
std::string tune_key(const Ctx &ctx, const char *kernel, const Geom &g, int prec, int recon, int nrhs);

// profiling hooks around a hop launch (no-ops unless ctx.profiling)
void prof_begin(Ctx &ctx, hipStream_t s);
void prof_end(Ctx &ctx, int prec, int recon, int64_t sites, hipStream_t s);

}  // namespace lqs

// The opaque C handles are the library objects themselves.
struct lqs_ctx : lqs::Ctx {};
struct lqs_gauge : lqs::Gauge {};
