/*
 * mrsdc.h -- C-ABI of the MI355X multi-rate spectral deferred correction
 * (MRSDC) heat-conduction stepper.
 *
 * The library advances the semi-discrete heat equation of a machine made of a
 * fixed stand and a moving stock (Naumann, Ruprecht, Wensch, arXiv 1707.03581,
 * §2, eq. coupledFEM and its splitting eq. ivp):
 *
 *     diag(m) dT/dt = f^I(T) + g + f^E(T, t)
 *     f^I(T) = -(K + h R) T          slow, implicit  (conduction + Robin)
 *     g      = h T_env r             slow source     (Robin load)
 *     f^E    = contact exchange alpha (T_other - T) and friction heat on the
 *              moving overlap Gamma_R(t) of two faces, or a moving heat-flux
 *              patch on one face                    (fast, explicit)
 *
 * with the MRSDC predictor (Alg. 1) followed by K correction sweeps (Alg. 2)
 * of §3: one implicit node solve (diag(m) + dtau_m (K + h R)) T* = rhs per
 * standard interval and P explicit Euler substeps of f^E at the embedded
 * nodes.  Every step of the sweep runs in HIP kernels on one gfx950 GPU.
 *
 * Conventions (all entry points):
 *  - Return an mrsdc_status; no exception crosses the ABI.  On error the
 *    context keeps its previous state and mrsdc_last_error(ctx) describes why.
 *  - All array arguments are HOST pointers unless the name says device; they
 *    are copied during the call and stay owned by the caller.
 *  - Device memory is owned by the context until mrsdc_destroy.
 *  - One thread at a time per context; distinct contexts are independent.
 *  - SI units, temperatures in degrees Celsius.
 *  - Bodies: 0 (stand / the only body) and 1 (stock).  Their nodes are
 *    concatenated in body order into one state vector (§2, eq. coupledFEM).
 */
#ifndef MRSDC_H
#define MRSDC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrsdc_ctx mrsdc_ctx;

typedef enum {
  MRSDC_OK = 0,
  MRSDC_EINVAL = -1,  /* bad argument: shape, CSR structure, NaN, scheme, horizon */
  MRSDC_ENOMEM = -2,  /* device or host allocation failed */
  MRSDC_EDEVICE = -3, /* HIP runtime error or no usable GPU */
  MRSDC_ENOCONV = -4, /* an implicit solve hit its iteration cap; state rolled back
                         to the last completed step */
  MRSDC_ESTATE = -5   /* call out of order (e.g. advance before bodies are set) */
} mrsdc_status;

enum { MRSDC_FP64 = 0, MRSDC_FP32_REFINE = 1 };
enum { MRSDC_LOBATTO = 0, MRSDC_EQUI_NOLEFT = 1 };
enum { MRSDC_MULTIRATE = 0, MRSDC_SINGLE_RATE = 1 };

/* Optional device allocator (for example a framework's caching allocator, so
 * that the framework owns and accounts the memory): alloc returns `bytes` of
 * device memory usable on `stream` (the context's hipStream_t) or NULL;
 * release takes back a pointer alloc returned.  The library calls them from
 * the thread that calls into the context; it copies this struct at
 * mrsdc_create. */
typedef struct {
  void *(*alloc)(size_t bytes, void *stream, void *user);
  void (*release)(void *ptr, void *stream, void *user);
  void *user;
} mrsdc_allocator;

typedef struct {
  int device;         /* HIP device ordinal */
  int precision;      /* MRSDC_FP64, or MRSDC_FP32_REFINE: FP32 inner CG with FP64
                         iterative refinement (FP64 residual, FP64 node states) */
  int M;              /* standard nodes, 2..8 (§3: tau_1 < ... < tau_M = t_{n+1});
                         1 is accepted for MRSDC_EQUI_NOLEFT (then the predictor
                         of the single-rate method is implicit Euler) */
  int node_family;    /* MRSDC_LOBATTO (tau_1 = t_n, first interval skipped) or
                         MRSDC_EQUI_NOLEFT (tau_m = t_n + m dt / M, §3) */
  int P;              /* embedded nodes per standard interval, 1..32 (equidistant,
                         no-left, §3) */
  int K;              /* correction sweeps after the predictor, 0..16 */
  double dt;          /* time step, > 0 */
  double pcg_rtol;    /* FP64 path: stop when ||r||_2 <= pcg_rtol ||b||_2 */
  int pcg_maxit;      /* iteration cap per solve (ENOCONV beyond it) */
  double refine_rtol; /* FP32_REFINE: outer FP64 tolerance on ||b - A x||_2 / ||b||_2 */
  int refine_maxit;   /* FP32_REFINE: outer refinement cap per solve */
  double inner_rtol;  /* FP32_REFINE: relative tolerance of each FP32 inner solve */
  int final_residual; /* nonzero: also evaluate the residual of the last sweep */
  int use_graph;      /* nonzero: after three steps run directly (which learn
                         the CG launch budgets), the time step is captured once
                         into a HIP graph and replayed (one launch per step
                         instead of hundreds); the learned budgets then only
                         grow, and the step is captured again when one does (a converged
                         solve's spare launches return at once:
                         FP64 results bit for bit those of use_graph = 0; in
                         FP32_REFINE an inner solve that a smaller budget would
                         have cut short runs on to its tolerance).  Needs a stream
                         that can be captured: with the legacy default stream
                         the context runs without graphs. */
  double sweep_tol;   /* > 0: residual control, a step stops sweeping once the
                         residual (eq. residual, max-norm) of its latest iterate
                         is <= sweep_tol (at most K sweeps; §3 states that each
                         sweep reduces it by a factor proportional to dt);
                         0: always K sweeps.  Per scenario in batched contexts */
  int method;         /* MRSDC_MULTIRATE: the method of §3 (f^E explicit on P
                         embedded substeps).  MRSDC_SINGLE_RATE: the single-rate
                         SDC used as comparison in §5, with the coupling f^E
                         taken into the implicit part (each node solve is
                         (diag(m) + dtau (K + h R + A_c(tau))) T = rhs, A_c the
                         linear exchange operator of f^E at the node time) and
                         no substeps; P is then unused.  FP64 only, single
                         (non-batched) contexts only */
  void *stream;       /* hipStream_t to run on, or NULL for a library-owned stream */
  int op_form;        /* storage of L = K + h R (§2, eq. femDiscr) read by the CG
                         product of single contexts.  Every form holds the same
                         entries in the same order, so every form gives the same
                         sums, bit for bit:
                           MRSDC_OP_AUTO     the most compact form that applies
                           MRSDC_OP_VALUES   value array (8 B per entry; FP32
                                             copy for the inner solves)
                           MRSDC_OP_DICT     1-byte index into the distinct
                                             values (at most 256 of them)
                           MRSDC_OP_PACKED   2-byte word: column offset and
                                             value index (at most 16 values,
                                             |col - row| <= 2047)
                           MRSDC_OP_PATTERNS 1-byte row form per row (at most
                                             128 distinct rows)
                         OR-ed with MRSDC_OP_COL32: int32 columns even where
                         16-bit offsets fit.  The first advance (or stationary
                         solve) returns EINVAL when the form does not apply.
                         Batched contexts take MRSDC_OP_AUTO (the column sweep,
                         which finds each entry from its stencil position, on
                         meshes whose bodies are boxes of the 27-point
                         pattern, else LDS tiles of the stored entries) or
                         MRSDC_OP_VALUES (the tiles on every mesh); the two
                         form each row's sums in the same order but reduce
                         p.q in a different order, so they agree to rounding */
  const mrsdc_allocator *alloc; /* NULL: hipMalloc / hipFree.  Otherwise every
                         device buffer of the context (and of its deformation
                         solve) comes from alloc and goes back through release;
                         both must be set */
  int autotune;       /* nonzero (batched contexts): before the first step,
                         time the launch variants of the CG kernels on this
                         mesh (stages in flight of the column sweep; in
                         FP32_REFINE also the row groups in flight of the two
                         CG updates) and keep the fastest.  Every variant
                         gives bit for bit the same results; the choice is
                         kept per process for the mesh, precision and
                         scenario count and reported in mrsdc_stats.  2 .. 9
                         pick a variant without timing (bits of autotune - 2:
                         1 one stage in flight, 2 two groups in (b), 4 eight
                         in (c)) */
} mrsdc_config;

enum {
  MRSDC_OP_AUTO = 0,
  MRSDC_OP_VALUES = 1,
  MRSDC_OP_DICT = 2,
  MRSDC_OP_PACKED = 3,
  MRSDC_OP_PATTERNS = 4,
  MRSDC_OP_COL32 = 0x100
};

typedef struct {
  int64_t steps;           /* completed time steps in the last advance */
  int64_t solves;          /* implicit node solves */
  int64_t pcg_iters;       /* CG iterations (FP32 inner iterations in FP32_REFINE) */
  int64_t refine_steps;    /* FP64 refinement residuals (FP32_REFINE) */
  int32_t max_iters;       /* largest iteration count of one solve */
  int32_t redone_steps;    /* steps repeated with a larger device iteration budget */
  double residual[17];     /* residual (eq. residual) of iterates k = 0..K of the
                              last step; k = K only with final_residual */
  double wall_s;           /* host wall time of the advance, to device completion */
  int64_t bytes_moved;     /* algorithmic device bytes of the advance (see docs) */
  int64_t sweeps;          /* correction sweeps run (over active scenarios) */
  int32_t op_form;         /* operator form the CG product read (MRSDC_OP_VALUES ..
                              MRSDC_OP_PATTERNS; 0 in batched contexts) */
  int32_t col_bytes;       /* bytes per stored column: 2 (offset) or 4 (int32) */
  int32_t graph_captures;  /* steps captured into a HIP graph in this call (use_graph) */
  int32_t graph_launches;  /* graph launches (steps replayed) in this call */
  int32_t col_depth;       /* batched: stages in flight of the column-sweep CG
                              product (0: the tiled product runs) */
  int32_t groups_b;        /* batched: row groups in flight of the CG updates */
  int32_t groups_c;
  int32_t autotuned;       /* 1 if the launch variants were chosen by timing */
} mrsdc_stats;

/* Fill *cfg with defaults: FP64, Lobatto M=3, P=2, K=2, dt=1, pcg_rtol 1e-13. */
void mrsdc_config_init(mrsdc_config *cfg);

/* Create a context on cfg->device.  EINVAL for a bad scheme, EDEVICE if the
 * GPU cannot be used.  *out is NULL on failure. */
mrsdc_status mrsdc_create(mrsdc_ctx **out, const mrsdc_config *cfg);

/* Finite element operators of one body (§2, eq. femDiscr):
 *  rowptr[n+1] (int64), col[nnz] (int32, 0-based, sorted, in [0,n)) describe
 *  the common sparsity pattern of K and R;
 *  K[nnz]  stiffness including conductivity (K = -A_X), symmetric;
 *  R[nnz]  unit-coefficient Robin boundary mass (B_X,env = -h R); may be NULL;
 *  mass[n] row-sum lumped mass (> 0);
 *  robin_load[n] = integral of phi_i over the Robin boundary; may be NULL.
 * EINVAL on a malformed CSR or non-finite values. */
mrsdc_status mrsdc_set_body(mrsdc_ctx *ctx, int body, int64_t n, int64_t nnz,
                            const int64_t *rowptr, const int32_t *col, const double *K,
                            const double *R, const double *mass, const double *robin_load);

/* Robin coefficient h >= 0 and environment temperature of one body
 * (§2, Robin conditions: f^I gets -h R, g = h T_env r). */
mrsdc_status mrsdc_set_robin(mrsdc_ctx *ctx, int body, double h, double T_env);

/* A tensor grid of face nodes of a body, registered under tag face (0..7):
 * u[nu], v[nv] strictly increasing coordinates in the face plane; node_ids
 * [nu*nv] body-local node of grid point (u[a], v[b]) at node_ids[a*nv+b].
 * Faces carry the coupling integrals of f^E (§2, eq. defCB). */
mrsdc_status mrsdc_set_face(mrsdc_ctx *ctx, int body, int face, int nu, int nv,
                            const double *u, const double *v, const int32_t *node_ids);

/* Motion of the moving part (§5): s(t) = s0 + a sin(2 pi t / period + phase),
 * period > 0.  The moving face (or patch) is shifted by s(t) along v. */
mrsdc_status mrsdc_set_motion(mrsdc_ctx *ctx, double s0, double a, double period,
                              double phase);

/* Contact coupling on Gamma_R(t) = overlap of the fixed face and the moving
 * face (§2, boundary conditions on Gamma_R and eqs. femContFix/femContMov).
 * The moving face's point (u, v) lies at (u + du, v + dv + s(t)) in the fixed
 * face's frame.  Row i of the fixed body receives
 *   int_{Gamma_R} phi_i (alpha (T_mov - T_fix) + split P_f / |Gamma_R(t)|),
 * row i of the moving body the same with the roles swapped and 1 - split.
 * The faces must be registered first. */
mrsdc_status mrsdc_set_contact(mrsdc_ctx *ctx, int fix_body, int fix_face, int mov_body,
                               int mov_face, double du, double dv, double alpha,
                               double friction_W, double split);

/* Rigid patch of width_u x width_v centred at (u_center, s(t)) on a face:
 * row i receives int_{patch(t)} phi_i (q0 + alpha (T_fixed - T)) (the moving
 * stock of the paper's 2D test, §4, with an added prescribed flux). */
mrsdc_status mrsdc_set_patch(mrsdc_ctx *ctx, int body, int face, double width_u,
                             double width_v, double u_center, double q0, double alpha,
                             double T_fixed);

/* Temperature of one body (n values, host array).  EINVAL on NaN/Inf. */
mrsdc_status mrsdc_set_temperature(mrsdc_ctx *ctx, int body, const double *T, int64_t n);

/* Current simulated time (resume: the state of the one-step method is (t, T)). */
mrsdc_status mrsdc_set_time(mrsdc_ctx *ctx, double t);
mrsdc_status mrsdc_get_time(const mrsdc_ctx *ctx, double *t);

/* Advance by horizon seconds (an integer multiple of dt, relative tolerance
 * 1e-9) and wait for the device.  stats may be NULL.  ENOCONV leaves the state
 * at the last completed step. */
mrsdc_status mrsdc_advance(mrsdc_ctx *ctx, double horizon, mrsdc_stats *stats);

/* Replace the field by the stationary one of the conduction and Robin part,
 * (K + h R) T = g with g = h T_env r (the initial data of the numerical
 * example, §5: the machine at rest, coupled only to its environment; the
 * mass term printed there is read as zero, since a stationary field has no
 * time derivative).  Jacobi-PCG warm-started from the current field (zero if
 * none was set) until ||r||_2 <= rtol ||g||_2, at most maxit iterations;
 * iters (nullable) receives the count.  Single contexts only (ESTATE for a
 * batched one).  EINVAL for rtol <= 0, maxit < 1, or a body without a
 * Robin term (singular problem); ENOCONV leaves the last iterate in place. */
mrsdc_status mrsdc_set_stationary(mrsdc_ctx *ctx, double rtol, int maxit, int *iters);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): mrsdc_set_stationary
 * without any allocation.  Its two work vectors (the Jacobi inverse of
 * K + h R and a zero mass vector) live in a fixed scratch array of
 * 2 * MRSDC_NOALLOC_MAX_ROWS doubles (64 MiB) that each device holds until
 * the process ends; the same kernels run, so the field and the iteration
 * count are those of mrsdc_set_stationary, bit for bit.  Requires a context
 * whose device state exists (an earlier advance or stationary solve; ESTATE
 * otherwise) and at most MRSDC_NOALLOC_MAX_ROWS rows (EINVAL otherwise).  All
 * calls on one device share the scratch: calls that overlap on one device
 * (from several host threads) race and must be serialised by the caller. */
#define MRSDC_NOALLOC_MAX_ROWS 4194304
mrsdc_status mrsdc_set_stationary_noalloc(mrsdc_ctx *ctx, double rtol, int maxit, int *iters);

/* Copy the temperature of one body to a host array of n values. */
mrsdc_status mrsdc_get_temperature(mrsdc_ctx *ctx, int body, double *out, int64_t n);

/* Copy the temperature of one body (n doubles) to DEVICE memory dptr on
 * stream (a hipStream_t, or NULL for the context's stream); asynchronous. */
mrsdc_status mrsdc_get_temperature_device(mrsdc_ctx *ctx, int body, void *dptr, int64_t n,
                                          void *stream);

/* Device bytes the context holds once prepared (operators, states, caches). */
mrsdc_status mrsdc_footprint_bytes(const mrsdc_ctx *ctx, int64_t *bytes);

/* Split of a prepared batched context's footprint for admission by HBM
 * footprint (a serving loop keeps each request's node states resident):
 * *per_scenario = device bytes that grow with the scenario count, per
 * scenario (node states T_m, F_j, I_m, CG vectors, interface caches and
 * coefficient tables, reduction partials); *shared = the rest (operators,
 * tiles, weights), held once.  footprint = shared + S * per_scenario, up to
 * the rounding of the division.  ESTATE for a single or unprepared context. */
mrsdc_status mrsdc_batch_slot_bytes(const mrsdc_ctx *ctx, int64_t *per_scenario,
                                    int64_t *shared);

/* Description of the last error of this context ("" if none). */
const char *mrsdc_last_error(const mrsdc_ctx *ctx);

/* Free the context and all its device memory.  NULL is accepted. */
mrsdc_status mrsdc_destroy(mrsdc_ctx *ctx);

/* Host-only: nodes and weights of one step (§3, weight definitions and Table
 * tab:weights), for inspection and tests.  Arrays use 1-based node indices:
 * tau[M+1]; s[(M+1)*(M+1)] at [m*(M+1)+j]; shat[(M+1)*(P+1)] at [m*(P+1)+q];
 * stil[(M+1)*(P+1)*(M+1)] at [(m*(P+1)+p)*(M+1)+j];
 * spq[(M+1)*(P+1)*(P+1)] at [(m*(P+1)+p)*(P+1)+q].  EINVAL on bad arguments. */
mrsdc_status mrsdc_quadrature(int M, int node_family, int P, double dt, double *tau,
                              double *s, double *shat, double *stil, double *spq);

/* ---- Batched ensembles: S scenarios of one machine advanced together ----
 * The scenarios share the operators, faces, motion law and scheme set with
 * the single-context calls above (mrsdc_set_body, _set_robin, _set_face,
 * _set_motion, _set_contact); each scenario has its own Robin coefficient h,
 * contact alpha, friction power, motion period, time and temperature field.
 * The operator is applied to all scenarios in one pass (multi-right-hand
 * side).  Both precisions: MRSDC_FP64, or MRSDC_FP32_REFINE (per scenario,
 * FP32 inner CG with FP32 operator values, vectors and row sums, inside FP64
 * iterative refinement; node states, quadrature and f^E stay FP64, as for a
 * single context).  Contact coupling (or none).  A scenario's result does not
 * depend on the other members of the batch. */

/* Create a batched context of S scenarios (1..64).  EINVAL for S out of
 * range. */
mrsdc_status mrsdc_batch_create(mrsdc_ctx **out, const mrsdc_config *cfg, int S);

/* Parameters of scenario s; unset scenarios use the context-wide values. */
mrsdc_status mrsdc_batch_set_scenario(mrsdc_ctx *ctx, int s, double h, double alpha,
                                      double friction_W, double period);

/* Temperature of scenario s over all nodes of both bodies (n = total nodes,
 * concatenated in body order); host array, copied. */
mrsdc_status mrsdc_batch_set_temperature(mrsdc_ctx *ctx, int s, const double *T, int64_t n);

/* Current time of scenario s (each scenario has its own clock). */
mrsdc_status mrsdc_batch_set_time(mrsdc_ctx *ctx, int s, double t);
mrsdc_status mrsdc_batch_get_time(const mrsdc_ctx *ctx, int s, double *t);

/* Include (active != 0) or leave out scenario s in the next steps; inactive
 * scenarios keep their state and clock. */
mrsdc_status mrsdc_batch_set_active(mrsdc_ctx *ctx, int s, int active);

/* Advance every active scenario by nsteps time steps of dt; waits for the
 * device.  Statistics add over the active scenarios.  ENOCONV leaves every
 * scenario at its last completed step. */
mrsdc_status mrsdc_batch_advance(mrsdc_ctx *ctx, int nsteps, mrsdc_stats *stats);

/* Temperature of scenario s over all nodes (n = total nodes) into a host array. */
mrsdc_status mrsdc_batch_get_temperature(mrsdc_ctx *ctx, int s, double *out, int64_t n);

/* Copy scenario s's temperature (n = N doubles, both bodies) to DEVICE memory
 * dptr on stream (a hipStream_t, or NULL for the context's stream);
 * asynchronous on that stream.  ESTATE before the first advance. */
mrsdc_status mrsdc_batch_get_temperature_device(mrsdc_ctx *ctx, int s, void *dptr, int64_t n,
                                                void *stream);

/* Advance every active scenario s by its own horizon[s] seconds (an integer
 * multiple of dt, relative tolerance 1e-9; inactive scenarios are skipped):
 * the batch steps until the longest horizon is reached, each scenario leaving
 * it once its own is, and every scenario that was active is active again on
 * return.  stats sum over the steps.  Errors as mrsdc_batch_advance (ENOCONV
 * leaves each scenario at its last committed step). */
mrsdc_status mrsdc_batch_advance_horizons(mrsdc_ctx *ctx, const double *horizon,
                                          mrsdc_stats *stats);

/* Per-kernel-class device time measured with HIP events on the context's
 * stream while profiling is on (mrsdc_profile).  cg_spmv: the operator
 * application q = (diag(m) + dtau L) p of every CG iteration within the
 * previous step's iteration count; cg_spmv_bytes: its algorithmic bytes per
 * launch (nnz (8 + index bytes) + slice offsets + 24 N). */
typedef struct {
  int64_t cg_spmv_launches;
  double cg_spmv_ms;
  int64_t cg_spmv_bytes;
  int64_t iface_launches;
  double iface_ms;
  int64_t nnz;
  int64_t n;
} mrsdc_kernel_times;

/* Turn event timing of the kernel classes on (nonzero) or off and reset it. */
mrsdc_status mrsdc_profile(mrsdc_ctx *ctx, int on);
mrsdc_status mrsdc_profile_read(const mrsdc_ctx *ctx, mrsdc_kernel_times *out);

/* Launch the CG operator application q = (diag(m) + dtau L) p (FP32 operator
 * for FP32_REFINE) reps times back to back between two HIP events on the
 * context's stream and report the average time per launch in microseconds and
 * the bytes its storage reads and writes once (single contexts: as
 * cg_spmv_bytes; batched: the stored operator form and the S right-hand sides
 * in and out).  Needs a prepared context (one advance); overwrites only CG
 * scratch vectors.  For roofline measurement. */
mrsdc_status mrsdc_time_operator(mrsdc_ctx *ctx, int reps, double *avg_us, int64_t *bytes);

/* ---- thermo-elastic deformation of one body (§5, deformation paragraphs) ----
 *
 * Linear elasticity driven by the temperature field: K_u u = G (T - T_ref),
 * with K_u the symmetric positive definite stiffness over the free
 * displacement DOFs (the caller assembles it and removes the Dirichlet DOFs)
 * and G the thermal load operator (n x nodes of the body).  As in §5 the
 * matrix is factorised once and every output is a forward and a backward
 * solve.  The factorisation is a block LU of K_u seen as block tridiagonal:
 * the rows are cut into blocks of the matrix half-bandwidth b (so only
 * neighbouring blocks couple), S_0 = A_00, S_k = A_kk - A_{k,k-1} S_{k-1}^{-1}
 * A_{k-1,k}, and the device keeps W_k = S_k^{-1} as dense FP64 blocks padded
 * to a multiple of 64 (about n (b + 64) 8 bytes; number DOFs so that b is
 * small, e.g. plane by plane).  Forward: w_k = W_k (f_k - A_{k,k-1} w_{k-1});
 * backward: u_k = w_k - W_k A_{k,k+1} u_{k+1}.  FP64 throughout. */
typedef struct {
  int64_t n;            /* free displacement DOFs */
  int64_t block;        /* block size b = half-bandwidth of K_u */
  int64_t padded_block; /* b rounded up to a multiple of 64 */
  int64_t nblocks;      /* ceil(n / b) */
  int64_t factor_bytes; /* device bytes of the W_k */
  double factor_ms;     /* wall time of the factorisation (device work included) */
  int64_t factor_launches; /* kernels the factorisation launched */
} mrsdc_deform_info;

/* Register the deformation problem of `body` and factorise it on the device
 * (synchronous).  rowptr[n+1] (int64), col (int32, sorted, in [0,n)) and Ku
 * give K_u in CSR (full symmetric pattern); growptr[n+1], gcol (int32, in
 * [0, nodes of the body)) and G give the thermal load operator.  Replaces an
 * earlier registration.  EINVAL: bad CSR, non-finite values, or a
 * non-positive pivot met during the factorisation (K_u not SPD); ENOMEM: the
 * blocks do not fit; ESTATE: the body is not set or the context is batched. */
mrsdc_status mrsdc_deform_setup(mrsdc_ctx *ctx, int body, int64_t n, int64_t nnz,
                                const int64_t *rowptr, const int32_t *col, const double *Ku,
                                int64_t gnnz, const int64_t *growptr, const int32_t *gcol,
                                const double *G, double T_ref);

/* Displacement u (n values, host array) of the registered body for the
 * context's current temperature.  ESTATE before mrsdc_deform_setup. */
mrsdc_status mrsdc_deform(mrsdc_ctx *ctx, double *u, int64_t n);

/* Same, written to device memory dptr (n doubles); the copy is ordered after
 * the solve on `stream` (hipStream_t, NULL: the context's stream). */
mrsdc_status mrsdc_deform_device(mrsdc_ctx *ctx, void *dptr, int64_t n, void *stream);

mrsdc_status mrsdc_deform_get_info(const mrsdc_ctx *ctx, mrsdc_deform_info *out);

/* Run reps forward/backward solves back to back between HIP events on the
 * context's stream: average microseconds per solve, and the average duration
 * of the block product u = W_k v (the solve's dominant step: the symmetric
 * product over the upper-triangle 64 x 64 tiles of W_k and the fixed-order
 * sum of its tile partials, timed as one with its own events) with its
 * algorithmic bytes per product (the upper-triangle tiles, the vectors, and
 * the partials written and read back).  For roofline measurement. */
mrsdc_status mrsdc_deform_time(mrsdc_ctx *ctx, int reps, double *solve_us, double *gemv_us,
                               int64_t *gemv_bytes);

/* Library version string. */
const char *mrsdc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MRSDC_H */
