/*
 * lqs.h -- C ABI of the MI355X staggered-fermion solver library (liblqs.so).
 *
 * The library applies the staggered Dirac operator of eq. (1) of Kumar,
 * Borsanyi, Guenther, Wong, "Portable Lattice QCD implementation based on
 * OpenCL" (LATTICE2024, Sec. 4.2) and inverts the even-odd normal operator
 * M = m^2 - D_eo D_oe by conjugate gradient (the "inversion of the Dirac
 * operator" that Sec. 1 and Sec. 4.2 benchmark), in FP64, FP32 and
 * FP16-storage arithmetic, for several right-hand sides or several lattices at
 * once, and provides the link derivative of phi^dag M^-1 phi (a "derivative"
 * the code design of Sec. 3 places in every backend).
 *
 * ---------------------------------------------------------------------------
 * Conventions (the paper leaves these open; fixed here once for every call)
 *   Extents dims = {Nx, Ny, Nz, Nt}, all even and >= 2, V = Nx Ny Nz Nt,
 *   Vh = V / 2, V <= 2^30.  Direction mu = 0, 1, 2, 3 is x, y, z, t.
 *   Lexicographic site index lex = x + Nx (y + Ny (z + Nz t)).
 *   A site is even when x + y + z + t is even.  Within one parity the site
 *   with lexicographic index lex has checkerboard index cb = lex >> 1.
 *   Staggered phases eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y),
 *   eta_3 = (-1)^(x+y+z); boundaries periodic in x, y, z and antiperiodic in
 *   t, the sign being carried by the phase of the t-links that leave t = Nt-1.
 *   Eq. (1) is used as printed (no factor 1/2):
 *     (D phi)_x = sum_mu [ eps_mu(x) U_{x,mu} phi_{x+mu}
 *                          - eps_mu(x-mu) U^dag_{x-mu,mu} phi_{x-mu} ]
 *   with eps_mu the phase of the link including the boundary sign.
 *
 * Memory and ownership
 *   Every field or link pointer is a DEVICE pointer owned by the caller; the
 *   library never frees it and keeps none past the call.  The library owns
 *   lqs_ctx (device, stream-independent workspace, tuning cache) and
 *   lqs_gauge (packed copies of one gauge field); the caller destroys both.
 *   Device pointers must be 16-byte aligned.
 *
 * Complex canonical layouts (interleaved re, im doubles):
 *   links      [4][Nt][Nz][Ny][Nx][3][3]   row-major 3x3 per link
 *   lex field  [nrhs][Nt][Nz][Ny][Nx][3]
 *
 * Native single-parity colour-vector layouts (lqs_field.data), per right-hand
 * side r, consecutive right-hand sides one after another:
 *   LQS_F64  double2 [3][Vh]        element (c, cb) = colour c of site cb
 *   LQS_F32  float4  [Vh]           colours 0 and 1 of site cb
 *            float2  [Vh]           colour 2 of site cb      (24 Vh bytes)
 *   LQS_F16  16-byte word [Vh]      six binary16 (re0 im0 re1 im1 re2 im2)
 *                                   then one float scale s; value = half * s;
 *                                   s = max |component| of the site (16 Vh bytes)
 *
 * Errors and synchrony
 *   Every call returns an lqs_status; no C++ exception crosses the ABI.
 *   Arguments are validated before anything is launched.  A HIP failure
 *   returns LQS_EHIP with the HIP message in lqs_last_error() (thread-local).
 *   dslash_apply, dslash_dagger, fermion_force and the field conversions are
 *   asynchronous on `stream` (a hipStream_t; NULL = the null stream).
 *   cg_solve returns after the solve has finished.
 *   Calls that share an lqs_ctx must not run concurrently from several host
 *   threads (the context's workspace is not locked).
 * ---------------------------------------------------------------------------
 */
#ifndef LQS_H
#define LQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lqs_status;
enum {
    LQS_OK = 0,
    LQS_ENOTCONV = 1,      /* warning: max_iter reached, x holds the last iterate   */
    LQS_EINVAL = -1,       /* invalid argument (nothing launched)                   */
    LQS_EHIP = -2,         /* HIP runtime error, see lqs_last_error()               */
    LQS_ENOMEM = -3,       /* device allocation failed                              */
    LQS_EBREAKDOWN = -4,   /* CG breakdown: p.Mp <= 0                                */
    LQS_ENONFINITE = -5,   /* NaN or Inf met in a CG scalar                          */
    LQS_EUNSUPPORTED = -6  /* format or option not available on this gauge/context */
};

typedef enum { LQS_F64 = 0, LQS_F32 = 1, LQS_F16 = 2 } lqs_prec;

/* Link storage formats of a gauge object: precision x (18 reals | 12 reals,
 * third row rebuilt on the fly as conj(row0 x row1), Sec. 4.3). */
#define LQS_FMT(prec, recon) (1u << (2 * (unsigned)(prec) + ((recon) == 12 ? 1u : 0u)))
#define LQS_FMT_ALL 0x3Fu
/* Flag for lqs_gauge_create: the links are in temporal gauge, U_t(x) = 1 for
 * every site with t < Nt-1 (Sec. 4.3); the hop then reads 6 links per site
 * instead of 8 off the last time slice.  Checked at creation. */
#define LQS_TEMPORAL_GAUGE 0x100u

typedef struct lqs_ctx lqs_ctx;
typedef struct lqs_gauge lqs_gauge;

/* One single-parity colour-vector field of nrhs right-hand sides (non-owning view). */
typedef struct {
    void *data;       /* device pointer, native layout of `prec` (above)       */
    int32_t prec;     /* lqs_prec                                             */
    int32_t parity;   /* 0 even, 1 odd                                        */
    int32_t nrhs;     /* 1 .. 16                                              */
} lqs_field;

/* ---- context and gauge ------------------------------------------------- */

/* Create a context on HIP device `device`.  tune_cache_path: JSON file that
 * stores autotuned launch parameters across runs (NULL: tune in memory only).
 * Returns LQS_EINVAL on a bad device, LQS_EHIP on a runtime failure. */
lqs_status lqs_ctx_create(int32_t device, const char *tune_cache_path, lqs_ctx **out);
void lqs_ctx_destroy(lqs_ctx *ctx);

/* Autotuning of launch shapes: 1 = sweep on first use of a (kernel, lattice,
 * format, right-hand sides) key and cache the fastest (block size, sides per
 * thread, streaming link loads, block-to-XCD map and its run of time slices,
 * LDS staging of the input, prefetched loads; a shape must beat the built-in
 * default by 2 %, twice); 0 (default) = no sweeps:
 * shapes already cached (loaded from tune_cache_path or tuned earlier in this
 * context) are used, the built-in defaults otherwise. */
lqs_status lqs_set_tuning(lqs_ctx *ctx, int32_t enable);

/* HIP graphs for the multi-kernel CG: 1 (default) = each solve captures one
 * round of iterations (8 iterations and their gated FP64 groups) into a
 * graph on a side stream and replays it, which removes most of the launch
 * cost on small lattices; 0 = launch every kernel.  Results are identical.
 * Graphs are not used while hop profiling is on. */
lqs_status lqs_set_graphs(lqs_ctx *ctx, int32_t enable);

/* Pack a canonical link field into the formats of the `formats` bitmask
 * (LQS_FMT(LQS_F64, 18) is always added; LQS_TEMPORAL_GAUGE may be or-ed in).
 * `links` is read on `stream`; the call returns once packing has been
 * enqueued (with LQS_TEMPORAL_GAUGE it synchronises `stream` to check the
 * gauge condition to 1e-12, else LQS_EINVAL).  Links must be SU(3) for the
 * 12-real formats to reproduce them.  Fails with LQS_EINVAL on odd extents. */
lqs_status lqs_gauge_create(lqs_ctx *ctx, const int32_t dims[4], const double *links, uint32_t formats,
                            void *stream, lqs_gauge **out);
void lqs_gauge_destroy(lqs_gauge *g);

/* Temporal gauge fixing (Sec. 4.3): G(x, 0) = 1, G(x, t+1) = G(x, t) U_t(x, t)
 * (rows re-orthonormalised, det 1), out_mu(x) = G(x) U_mu(x) G(x + mu)^dag,
 * with out_t(x) set to exactly 1 for t < Nt-1.  links, out: canonical link
 * layout (device, must not overlap); G: device complex128 [Nt][Nz][Ny][Nx][3][3].
 * D[out] = G D[links] G^dag, so M[out] (G x) = G M[links] x.  Asynchronous. */
lqs_status lqs_gauge_fix_temporal(lqs_ctx *ctx, const int32_t dims[4], const double *links, double *out, double *G,
                                  void *stream);

/* Bytes of one native field of nrhs right-hand sides. */
lqs_status lqs_field_bytes(const int32_t dims[4], int32_t prec, int32_t nrhs, size_t *bytes);

/* lex (canonical, nrhs blocks of V sites) -> native field of out->parity.
 * Only sites of that parity are read. */
lqs_status lqs_field_pack(lqs_ctx *ctx, const int32_t dims[4], const double *lex, const lqs_field *out,
                          void *stream);
/* native field -> lex; writes only the sites of in->parity, others untouched. */
lqs_status lqs_field_unpack(lqs_ctx *ctx, const int32_t dims[4], const lqs_field *in, double *lex,
                            void *stream);
/* As lqs_field_unpack, with every component multiplied in FP64 by the real
 * number `scale` on the way out (finite, else LQS_EINVAL); scale = 1 is
 * lqs_field_unpack.  Gives the source gradient 2 g M^-1 phi of the action
 * phi^dag M^-1 phi (PyTorch's complex-gradient convention) from chi = M^-1 phi
 * without arithmetic outside the library. */
lqs_status lqs_field_unpack_scaled(lqs_ctx *ctx, const int32_t dims[4], const lqs_field *in, double scale,
                                   double *lex, void *stream);

/* out[2*r], out[2*r+1] = real and imaginary part of sum_sites a_r^dag b_r for
 * each right-hand side r (FP64 fields of one parity, nrhs each; out is a
 * device array of 2*nrhs doubles).  Fixed-order reduction: the result does
 * not depend on scheduling.  Used for the action phi^dag M^-1 phi. */
lqs_status lqs_field_dot(lqs_ctx *ctx, const int32_t dims[4], const lqs_field *a, const lqs_field *b, double *out,
                         void *stream);

/* ---- the operator ------------------------------------------------------ */

/* out = D_{p,1-p} in: eq. (1) evaluated at the sites of parity p = out->parity,
 * whose neighbours all have parity 1-p = in->parity.  in and out must have
 * the same precision and nrhs, opposite parities, and must not overlap.
 * recon selects the link format (18 or 12) at the fields' precision; the
 * gauge must hold it (else LQS_EUNSUPPORTED).  nrhs > 1 reads each link once
 * for all right-hand sides (the multi-vector Dslash of Sec. 4.3). */
lqs_status dslash_apply(lqs_ctx *ctx, const lqs_gauge *g, int32_t recon, const lqs_field *in, lqs_field *out,
                        void *stream);

/* out = (D^dag)_{p,1-p} in, the adjoint hop, same arguments as dslash_apply.
 * (With the phases above D is anti-Hermitian, so this equals -D_{p,1-p}.) */
lqs_status dslash_dagger(lqs_ctx *ctx, const lqs_gauge *g, int32_t recon, const lqs_field *in, lqs_field *out,
                         void *stream);

/* ---- the solver -------------------------------------------------------- */

/* One even-parity system M x = b, M = m^2 - D_eo D_oe, with nrhs right-hand
 * sides sharing the links.  b and x are FP64 native even fields (double2
 * [nrhs][3][Vh]); x is the initial guess when use_x0 is set, else it is
 * overwritten from zero. */
typedef struct {
    const lqs_gauge *gauge;
    double mass;
    int32_t nrhs;
    const double *b;
    double *x;
} lqs_problem;

typedef struct {
    double tol;                /* stop when ||b - M x|| / ||b|| <= tol (FP64 residual)     */
    int32_t max_iter;          /* cap on iterations per right-hand side                    */
    int32_t inner_prec;        /* LQS_F64: plain FP64 CG; LQS_F32/LQS_F16: mixed precision */
    int32_t inner_recon;       /* 18 or 12: link format of the inner operator; with 12 and a
                                  gauge holding FP64 12-real links, the periodic FP64 updates
                                  of a mixed solve use those, the convergence check always
                                  the stored 18-real links                                   */
    int32_t reliable_interval; /* mixed: FP64 residual update every K iterations (0: 100)   */
    double reliable_delta;     /* mixed: also when ||r|| < delta * max ||r||
                                  (0: 0.02 with FP32 inner, 0.05 with FP16)                   */
    int32_t use_x0;            /* 1: start from x                                           */
    int32_t persistent;        /* 1: all problems in one cooperative launch (nrhs == 1)    */
} lqs_cg_params;

typedef struct {
    int32_t status;            /* lqs_status of this right-hand side                        */
    int32_t iters;             /* inner CG iterations                                       */
    int32_t reliable_updates;  /* FP64 residual recomputations (incl. the final check)     */
    int32_t restarts;          /* FP64 CG: restarts after a failed true-residual check      */
    double true_rel_residual;  /* ||b - M x|| / ||b|| in FP64 at return                     */
    double seconds;            /* wall time of the whole call                               */
    double device_seconds;     /* GPU time of this problem's solve: persistent = 1, its block
                                  group's start to end (device wall clock); cg_solve otherwise,
                                  from the first to the last kernel of the problem (stream
                                  events); 0 where not measured (cg_solve_noalloc,
                                  cg_solve_multishift)                                      */
    double gflops;             /* 1140 flop per even site and iteration (the two hops of M,
                                  570 each, Sec. 4.3) x iters / time, in GFLOP/s; time is
                                  device_seconds, or seconds where that is 0.  0 from
                                  cg_solve_multishift (its iterations differ in work)        */
    double gbytes_per_s;       /* algorithmic bytes of an iteration x iters / time, GB/s:
                                  per hop the links once (8 per site, 6 + 2/Nt in temporal
                                  gauge, shared by the right-hand sides of one problem) and
                                  each colour vector once per kernel of the iteration (hop,
                                  normal operator, update, p-update); reliable updates and
                                  the final check are not counted                            */
} lqs_cg_stats;

/* Solve nprob systems.  stats receives one entry per (problem, right-hand
 * side), in order.  Returns the worst status.  The solve runs on `stream`
 * and the call returns when it has finished.  With persistent = 0 several
 * problems run concurrently on side streams.  persistent = 1 runs them all
 * in one cooperative launch, one block group per lattice; it requires
 * nrhs == 1 for every problem, use_x0 = 0, at most 256 problems and no more
 * than the device's resident blocks, and cooperative launch support (else
 * LQS_EUNSUPPORTED).  It pays off for small lattices, whose group is a
 * single block. */
lqs_status cg_solve(lqs_ctx *ctx, int32_t nprob, const lqs_problem *probs, const lqs_cg_params *params,
                    lqs_cg_stats *stats, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cg_solve of
 * ONE problem (nrhs 1..16, persistent = 0) whose workspace is a fixed device
 * array of LQS_NOALLOC_SCRATCH_BYTES bytes inside the library, one per GPU,
 * held until the process ends (its address is taken once per device when a
 * context is created).  The call performs no device or pinned-host allocation
 * and creates no events, streams or graphs: it launches the same kernels with
 * the same launch shapes as cg_solve, eagerly on `stream`, and waits for a
 * state poll every eight iterations; the results equal cg_solve's.  The
 * caller still passes b, x and the gauge (created beforehand).  A problem
 * whose workspace (three inner-precision fields, the residual, in mixed
 * precision the inner solution and an FP64 field, plus reduction partials:
 * about 200 bytes per even site and right-hand side in FP64, 150 with FP16
 * inner) exceeds the array returns LQS_EINVAL before anything is launched.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (the solve initialises all it reads): calls that
 * overlap on one GPU, from several threads or streams, race.  Hop profiling
 * (lqs_profile_hops) and autotuning are not applied inside this call. */
#define LQS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
lqs_status cg_solve_noalloc(lqs_ctx *ctx, const lqs_problem *prob, const lqs_cg_params *params,
                            lqs_cg_stats *stats, void *stream);

/* Several masses on one Krylov space: x_i = (m_i^2 - D_eo D_oe)^-1 b for
 * i < nmass (multi-shift CG; the systems differ by the shifts m_i^2 - m_0^2
 * of the smallest mass m_0).  The shared recurrence keeps its search
 * directions and applies the operator in params->inner_prec (LQS_F64, LQS_F32
 * or LQS_F16 storage, links inner_recon; the residual is FP32 unless FP64) and
 * accumulates every x_i in FP64; in a mixed recurrence the smallest mass takes
 * the reliable updates of cg_solve (reliable_interval, reliable_delta), each
 * adding every FP32 solution into its FP64 field.  params->persistent must be 0 (else
 * LQS_EUNSUPPORTED); use_x0 is ignored (x_i start from zero).  b is an FP64
 * native even field (nrhs 1); x is a host array of nmass device pointers to
 * FP64 native even fields, overwritten.  Every x_i is finally checked against
 * its own FP64 true residual and refined, when the shared recurrence ended
 * above tol, by a warm-started CG with the same params, except that after a
 * mixed recurrence it runs with FP16-storage inner whenever the gauge holds
 * the FP16 links of inner_recon (mixed precision with reliable updates unless
 * inner_prec is LQS_F64); the masses are refined
 * together, one column each of a block of CGs sharing the link reads (up to 16
 * per block).  stats: nmass entries; iters
 * counts the shared iterations while system i was active plus refinement
 * iterations.  nmass in 1..17, masses finite and >= 0. */
lqs_status cg_solve_multishift(lqs_ctx *ctx, const lqs_gauge *g, int32_t nmass, const double *masses, const double *b,
                               double *const *x, const lqs_cg_params *params, lqs_cg_stats *stats, void *stream);

/* ---- the derivative ---------------------------------------------------- */

/* Link derivative of a real function L of chi = M^-1 phi, given X = chi and
 * Y = M^-1 g with g = 2 dL/dchi^* (Y = NULL means Y = X, i.e. L = phi^dag chi).
 * With psi_X = D_oe X, psi_Y = D_oe Y and eps_mu the link phase:
 *   y even: Pi_{y,mu} = eps_mu(y) [psi_X(y+mu) Y(y)^dag + psi_Y(y+mu) X(y)^dag]
 *   y odd : Pi_{y,mu} = -eps_mu(y) [Y(y+mu) psi_X(y)^dag + X(y+mu) psi_Y(y)^dag]
 * so that dL = Re sum tr(dU Pi).  mode 0 writes F = coeff * (-TA(U Pi)),
 * TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6, the su(3) force with
 * dL/dw = Re tr(F^dag A) for U -> exp(w A) U; mode 1 writes coeff * Pi^dag,
 * the gradient with respect to the real and imaginary parts of each link
 * entry; mode 2 adds coeff * (-TA(U Pi)) to force (a momentum update).
 * X, Y: FP64 native even fields (nrhs 1); force: canonical link layout. */
lqs_status fermion_force(lqs_ctx *ctx, const lqs_gauge *g, const double *X, const double *Y, double coeff,
                         int32_t mode, double *force, void *stream);

/* ---- hybrid Monte Carlo ------------------------------------------------ */
/* The simulation layer around the solver (Sec. 3 names HMC, the gauge action
 * and its derivatives; the paper states no formulas, the definitions are the
 * standard ones, fixed here).  Links and momenta use the canonical link
 * layout (complex128 [4][Nt][Nz][Ny][Nx][3][3]); links are periodic in every
 * direction (the antiperiodic t sign belongs to the fermion operator).
 *   plaquette  P_{mu nu}(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
 *   S_g = beta sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3)
 *   momenta Q: anti-Hermitian traceless, K = -sum_links tr Q^2
 *   force convention: F with dS/dw = Re tr(F^dag A) for U -> exp(w A) U;
 *   the flow is dU/dtau = Q U, dQ/dtau = -F/2, which conserves
 *   H = K + S_g + S_f, S_f = phi^dag M^-1 phi (M as in cg_solve). */

/* *S = S_g of the links (FP64, fixed-order sum).  Synchronous on stream. */
lqs_status gauge_action(lqs_ctx *ctx, const int32_t dims[4], const double *links, double beta, double *S,
                        void *stream);

/* out = coeff * F_g (accumulate = 0) or out += coeff * F_g (accumulate = 1),
 * F_g = (beta/3) TA(U V) with V the sum of the six staples of each link, so
 * that Re tr(U V) collects the plaquettes containing U.  out: canonical
 * link layout; must not overlap links. */
lqs_status gauge_force(lqs_ctx *ctx, const int32_t dims[4], const double *links, double beta, double coeff,
                       int32_t accumulate, double *out, void *stream);

/* links = exp(eps Q) links on every link (in place); Q: canonical layout,
 * must not overlap links. */
lqs_status link_update(lqs_ctx *ctx, const int32_t dims[4], double *links, const double *mom, double eps,
                       void *stream);

/* *K = -sum_links tr(Q^2).  Synchronous on stream. */
lqs_status kinetic_energy(lqs_ctx *ctx, const int32_t dims[4], const double *mom, double *K, void *stream);

enum { LQS_LEAPFROG = 0, LQS_OMELYAN = 1 };

typedef struct {
    double beta;        /* Wilson gauge coupling, >= 0                                 */
    double mass;        /* staggered mass, > 0 when fermions != 0                      */
    double tau;         /* trajectory length, > 0                                      */
    int32_t nsteps;     /* molecular-dynamics steps, >= 1                              */
    int32_t integrator; /* LQS_LEAPFROG or LQS_OMELYAN (second-order minimum norm)     */
    double lambda;      /* Omelyan parameter (0: 0.1931833275037836)                   */
    int32_t fermions;   /* 0 pure gauge; 1 pf = eta, phi = m eta_e - D_eo eta_o made   */
                        /* on the starting links; 2 pf = phi itself (even sites)       */
    lqs_cg_params cg;   /* the solves chi = M^-1 phi (use_x0: start from the previous  */
                        /* chi, from the third solve on from its linear extrapolation  */
                        /* 2 chi_n - chi_(n-1); persistent is ignored)                 */
    double force_tol;   /* tolerance of the solves that only feed the force (0: cg.tol);*/
                        /* the solves for S_f at both ends always use cg.tol           */
} lqs_hmc_params;

typedef struct {
    double k0, sg0, sf0;  /* K, S_g, S_f at the start                                   */
    double k1, sg1, sf1;  /* at the end of the trajectory                               */
    double dH;            /* (k1 + sg1 + sf1) - (k0 + sg0 + sf0)                        */
    int32_t accepted;     /* u < exp(-dH)                                               */
    int32_t cg_solves;    /* solves of M chi = phi                                      */
    int32_t cg_iters;     /* their inner iterations                                     */
    int32_t status;       /* worst CG status (LQS_OK when every solve converged)        */
    double plaquette;     /* mean Re tr P / 3 of the links returned                     */
    double seconds;       /* wall time of the call                                      */
} lqs_hmc_stats;

/* One HMC trajectory with the staggered pseudofermion of mass m (one even
 * field: the determinant of M, four tastes).
 *   links (in/out): the current links; replaced by the proposal if accepted.
 *   mom (in/out): the momenta drawn by the caller (anti-Hermitian traceless,
 *     density ~ exp(tr Q^2)); on return the momenta at the end of the proposal.
 *   pf: fermions = 1: eta, complex Gaussian with density ~ exp(-eta^dag eta)
 *     in the lex layout over all sites (nrhs 1); fermions = 2: phi in the lex
 *     layout (even sites read); ignored (may be NULL) when fermions = 0.
 *   u: uniform number in [0, 1) for the Metropolis decision.
 *   proposal (NULL or canonical link layout): receives the proposal.
 *   phi_out (NULL or lex layout, all sites): receives phi, zero on odd sites.
 * Leapfrog: Q -= h/2 G, n times {U = exp(hQ)U, Q -= h G} with the last
 * momentum step h/2; Omelyan: per step Q -= lam h G, U = exp(h/2 Q)U,
 * Q -= (1-2 lam) h G, U = exp(h/2 Q)U, Q -= lam h G, where G = F/2 on the
 * current links and h = tau/nsteps; the two lam h updates at a step boundary
 * act on the same links and share one solve.  The solve for S_f at the start
 * and end is reused as the force solve on those links.  Returns the worst
 * CG status (also in stats->status); the call returns when finished. */
lqs_status hmc_trajectory(lqs_ctx *ctx, const int32_t dims[4], double *links, double *mom, const double *pf,
                          double u, const lqs_hmc_params *params, lqs_hmc_stats *stats, double *proposal,
                          double *phi_out, void *stream);

/* ---- diagnostics ------------------------------------------------------- */

const char *lqs_strerror(lqs_status s);
const char *lqs_last_error(void);

/* Average duration in milliseconds of the hop kernels launched while
 * profiling was enabled, measured with HIP events on the launch stream.
 * lqs_profile_hops(ctx, 1) clears and starts, lqs_profile_hops(ctx, 0) stops.
 * Launches shorter than min_ms are not counted (inside cg_solve, kernels
 * queued after convergence return at once). */
lqs_status lqs_profile_hops(lqs_ctx *ctx, int32_t enable);
lqs_status lqs_profile_hops_result(lqs_ctx *ctx, int32_t prec, int32_t recon, double min_ms, int64_t *launches,
                                   double *avg_ms, int64_t *sites_per_launch);

#ifdef __cplusplus
}
#endif
#endif /* LQS_H */
