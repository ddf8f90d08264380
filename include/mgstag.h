/*
 * mgstag: 4D staggered / HISQ Kahler-Dirac multigrid on one AMD MI355X (gfx950).
 *
 * The method is that of Ayyar, Brower, Clark, Wagner and Weinberg,
 * "Optimizing Staggered Multigrid for Exascale performance" (Lattice 2022,
 * arXiv:2212.12559): an outer flexible GCR on the full HISQ operator,
 * preconditioned by a K-cycle whose first level is the Kahler-Dirac (KD)
 * block-preconditioned operator (Sec. 2.2-2.3), followed by Galerkin
 * coarsenings with chirally split, block-orthonormal near-null vectors
 * (Sec. 2.1), CA-GCR post-smoothers and inner solves to 0.25 or 8 iterations
 * (Table 1).
 *
 * Conventions (all calls):
 *   - lattice extents dims = {X, Y, Z, T}, even, periodic in every direction
 *     (an antiperiodic time boundary is a sign the caller puts on the links);
 *   - complex numbers are interleaved (re, im);
 *   - fine vector:   [nrhs][T][Z][Y][X][3]
 *   - link field:    [4][T][Z][Y][X][3][3] complex128, mu = 0..3 is x,y,z,t,
 *                    row-major 3x3
 *   - coarse vector: [nrhs][Tc][Zc][Yc][Xc][2][Nvec], spin index 0 is the
 *                    chirality eps = +1 projection, Tc = T / block etc.
 *   - staggered phases eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y),
 *     eta_3 = (-1)^(x+y+z); eps(x) = (-1)^(x+y+z+t).
 *   - every pointer argument named "device" points to GPU memory of the
 *     current HIP device; the library reads inputs, writes outputs and keeps
 *     no reference to them after the call, except the two workspaces passed to
 *     mg_setup, which must stay allocated until mg_destroy.
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued on it.  mg_apply_*, mg_restrict and mg_prolong return
 *     without waiting; mg_setup and the solvers (mg_solve, mg_cg_solve,
 *     mg_msc_solve, mg_solve_backward) synchronise the stream before
 *     returning (they fill host-side results).
 *   - the library never allocates device memory; it carves everything it
 *     needs from the caller's workspaces (sizes from mg_workspace_bytes).
 *   - errors: every function returns an mg_status; MG_OK is 0.  Arguments are
 *     validated before any launch.  mg_last_error() gives a thread-local
 *     message for the last failure.  No C++ exception crosses this boundary.
 *   - one context is single-threaded; distinct contexts are independent.
 */
#ifndef MGSTAG_H
#define MGSTAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx_s* mg_ctx;

typedef enum {
  MG_OK = 0,
  MG_E_ARG = 1,        /* bad pointer, size or enum value */
  MG_E_CONFIG = 2,     /* inconsistent parameters (odd extents, block not dividing, ...) */
  MG_E_ALIGN = 3,      /* pointer not 16-byte aligned */
  MG_E_RANK = 4,       /* near-null vectors numerically rank deficient on some block */
  MG_E_NOCONV = 5,     /* solver hit its iteration cap; x holds the last iterate */
  MG_E_NONFINITE = 6,  /* NaN or Inf in a right-hand side or a residual */
  MG_E_HIP = 7,        /* a HIP runtime call failed */
  MG_E_STATE = 8,      /* call not valid in the context's current state */
  MG_E_WORKSPACE = 9   /* workspace smaller than mg_workspace_bytes asked for */
} mg_status;

/* element types of vectors and stored operators */
typedef enum { MG_C128 = 0, MG_C64 = 1, MG_CBF16 = 2, MG_CF16 = 3 } mg_dtype;

/* Multigrid parameters; defaults follow Table 1 of the paper where it gives
 * one (smoother CA-GCR(8), inner solves 0.25 or 8 iterations, setup CGNE to
 * 1e-6 or 2000 iterations).  mg_default_params fills every field. */
typedef struct {
  int32_t dims[4];           /* X, Y, Z, T: even, >= 4 */
  double c1, c3;             /* one-hop and three-hop coefficients: naive (1, 0), HISQ-style (9/8, -1/24) */
  int32_t kd_naik;           /* 1: keep the Naik term inside the KD level; 0: truncated KD operator (Sec. 3.1) */
  double mass0;              /* mass the hierarchy (KD inverse, null vectors, coarse operators) is built at */
  int32_t nagg;              /* aggregation levels after the KD level: 1 or 2 */
  int32_t block[2][4];       /* aggregation blocks per level (level 1: even extents) */
  int32_t nvec[2];           /* near-null vectors per level (<= 128) */
  int32_t setup_maxiter[2];  /* CGNE iteration cap per level */
  double setup_tol[2];       /* CGNE tolerance ||A phi|| / ||A phi0|| per level */
  int32_t smoother_s;        /* CA-GCR basis size (<= 8) */
  double inner_tol;          /* inner-level GCR: stop at ||r|| <= inner_tol ||r_in|| ... */
  int32_t inner_maxiter;     /* ... or after this many iterations (<= 16) */
  double coarsest_tol;       /* coarsest level GCR tolerance */
  int32_t coarsest_maxiter;  /* coarsest level GCR iteration cap (<= 16 per restart cycle) */
  int32_t coarsest_restarts; /* restart cycles on the coarsest level (>= 1) */
  int32_t outer_nkrylov;     /* outer GCR restart length (<= 16) */
  int32_t outer_maxiter;     /* outer GCR iteration cap */
  double reliable_delta;     /* outer GCR recomputes r = b - D x when ||r|| < delta * ||r at last recompute|| */
  int32_t fine_prec;         /* MG_C128 or MG_C64: precision of the K-cycle on levels 0 and 1 */
  int32_t coarse_prec;       /* stored coarse links: MG_C128 (needs fine_prec MG_C128), MG_C64, or 16-bit
                                MG_CBF16 / MG_CF16 applied on the matrix cores with FP32 accumulation
                                (nvec multiples of 8; FP16 links carry the power-of-two scale
                                2^-round(log2 max|L|)); coarse vectors
                                are kept in fine_prec */
  int32_t max_nrhs;          /* systems solved in lockstep (mass x rhs pairs) and largest nrhs of an apply */
  int32_t max_nmass;         /* KD inverse slots: masses in one lockstep batch (>= 1) */
  int32_t coarsest_deflate;  /* deflation of the coarsest solve (Table 1): 0 for none, else the number k of
                                low modes (multiple of 16, <= 64, <= max_nrhs), near-null vectors of the
                                coarsest operator from CGNE at set-up; each coarsest solve then starts from
                                the least-squares solution on their span */
  int32_t deflate_maxiter;   /* CGNE iterations for the deflation vectors */
  int32_t deflate_import;    /* 1: null_vectors of mg_setup holds nagg + 1 pointers and the last one gives the
                                coarsest_deflate deflation vectors (complex128 [k][coarsest vector]) in place of
                                the CGNE ones; 0: nagg pointers */
  int32_t coarse_op;         /* 0: Galerkin coarse levels A_l = P^dag A_{l-1} P; 1: block-preconditioned
                                A_l = X_l^{-1} P^dag A_{l-1} P with X_l the coarse-site diagonal block, each
                                coarser level built from the preconditioned one and every coarse level solve
                                run on A_l x = X_l^{-1} b (Sec. 2.3, Table 1); the near-null vectors of a
                                level come from its Galerkin operator */
  int32_t coarsest_solver;   /* 0: GCR (coarsest_maxiter directions per restart cycle, stop at coarsest_tol);
                                1: CA-GCR(s), s = coarsest_maxiter, in a Chebyshev basis on [0, lambda_max]
                                (lambda_max by power iteration at set-up), coarsest_restarts cycles or
                                coarsest_tol (Table 1: Chebyshev-basis CA-GCR(16)); 2: exact, x = A^{-1} b
                                with the dense inverse of the coarsest operator formed at set-up by
                                Gauss-Jordan elimination with partial pivoting in FP64 (coarsest levels of
                                at most 8192 dof; not with coarsest_deflate; MG_E_RANK if singular) */
  int32_t graph_coarsest;    /* 1: with coarsest_solver 1 and coarsest_restarts 1 the coarsest solve (a fixed
                                launch sequence) is captured once per system count into a HIP graph and
                                replayed (results identical to the eager launches); 0: always eager */
  int32_t compact_masses;    /* 1: in a multi-mass batch the K-cycle runs only on the masses with a system
                                still iterating (whole masses leave the preconditioner's batch once all their
                                right-hand sides have converged; results unchanged); 0: on every system */
  int32_t coarse_shadow;     /* 1 (16-bit coarse links): in the smoother's chain p_j = A p_{j-1} on a coarse
                                level the stencil also stores its output rounded to the link format, and the
                                next application reads those 16-bit inputs (results unchanged; half the
                                staging reads, one more write); 0 (default): off */
  int32_t cgne_start_import; /* 1: an imported level's null_vectors entry is the CGNE's starting vectors
                                instead of the near-null vectors themselves (the set-up still runs
                                setup_maxiter CGNE iterations on them); 0 (default): imported vectors are
                                used as they are */
  uint64_t seed;             /* seed of the GPU-generated null-vector starts */
} mg_params;

typedef struct {
  int32_t outer_iters;       /* outer GCR iterations (CG: iterations) */
  int32_t reliable_updates;  /* recomputations of the true residual */
  int32_t level_iters[4];    /* total inner iterations per level 1..3 (index 0: level 1) */
  double true_rel_residual;  /* ||b - D(m) x|| / ||b|| recomputed in FP64 at exit */
  double seconds;            /* wall time of this system's solve (shared by a batch) */
  int32_t status;            /* mg_status of this system */
} mg_solve_info;

/* Fill *p with defaults for the given extents: HISQ-style coefficients,
 * KD with Naik, two aggregations (4^4, Nvec 64 then 2^4, Nvec 96), FP32
 * fine and coarse levels, Table 1 solver settings. */
void mg_default_params(mg_params* p, const int32_t dims[4]);

/* Device bytes the library needs: `persistent` must outlive the context
 * (links, KD inverses, P, coarse operators, null vectors), `scratch` is
 * solver workspace.  Validates *p (MG_E_CONFIG on inconsistency). */
mg_status mg_workspace_bytes(const mg_params* p, size_t* persistent, size_t* scratch);

/* Build the hierarchy (Sec. 2.1, Sec. 2.3; setup is excluded from the
 * paper's time-to-solution, Sec. 3.2).
 *   fat, naik: device, complex128 link fields (naik ignored when c3 == 0)
 *   null_vectors: host array of nagg pointers (nagg + 1 with deflate_import)
 *     to device complex128 near-null vectors, level 1 as
 *     [nvec[0]][T][Z][Y][X][3], level 2 as [nvec[1]][Tc][Zc][Yc][Xc][2][nvec[0]],
 *     then the coarsest level's deflation vectors; pass NULL (or a NULL
 *     entry) to generate that level's vectors on the GPU by CGNE on the
 *     level's operator (Sec. 2.1, Table 1).  Imported vectors are copied.
 *   persistent_ws / scratch_ws: device, caller-owned, at least the sizes
 *     reported by mg_workspace_bytes (MG_E_WORKSPACE otherwise), 256-byte
 *     aligned.
 * Returns MG_E_RANK when block orthonormalisation finds a dependent set. */
mg_status mg_setup(const mg_params* p, const void* fat, const void* naik, const void* const* null_vectors,
                   void* persistent_ws, size_t persistent_bytes, void* scratch_ws, size_t scratch_bytes,
                   void* stream, mg_ctx* out);

/* Fine-level operator applications on a fine vector (device in/out,
 * distinct buffers), dtype MG_C128 or MG_C64:
 *   op 0: D(m) x                        (Sec. 2.2; HISQ stencil)
 *   op 1: A x = (B + m)^{-1} D x        (Sec. 2.2 Eq. 2, Sec. 3.1; Naik per kd_naik)
 *   op 2: (B + m)^{-1} x                (the KD block inverse alone, Sec. 3.1)
 *   op 3: D(m)^dag x = eps D eps x
 *   op 4: A^dag x = eps D (B + m)^{-1} eps x   (the adjoint used by the CGNE set-up)
 * For ops 1, 2 and 4 the KD inverse of mass is built on first use, in a free
 * mass slot or, when every slot is taken, in slot 0. */
mg_status mg_apply_dslash(mg_ctx ctx, int32_t op, double mass, int32_t dtype, const void* in, void* out,
                          int32_t nrhs, void* stream);

/* mg_apply_dslash for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operators, arguments and results, with the intermediate vector of
 * ops 1, 3 and 4 staged in a static device array of the library
 * (mg_noalloc_scratch_bytes() = 64 MiB, one per GPU, held until the process
 * ends) instead of the context's scratch workspace.  The call allocates
 * nothing; ops 1, 3 and 4 with nrhs fine vectors of the dtype larger than the
 * array return MG_E_ARG before any work.  Every call on one GPU shares that
 * array and leaves its last contents there: calls that overlap on one GPU
 * (concurrent streams or threads) race.  Device addresses of the array are
 * looked up per device at mg_setup or at the first call on a device. */
mg_status mg_apply_dslash_noalloc(mg_ctx ctx, int32_t op, double mass, int32_t dtype, const void* in, void* out,
                                  int32_t nrhs, void* stream);
size_t mg_noalloc_scratch_bytes(void);

/* Coarse operator of level 2 (P1^dag A P1) or 3 (P2^dag A2 P2) on a coarse
 * vector of that level (Sec. 2.1; 9-point stencil of dense blocks, Sec. 3.1).
 * dtype MG_C128 uses the FP64 operator; MG_C64 the coarse_prec operator
 * (FP32 links, or 16-bit links on the matrix cores). */
mg_status mg_apply_coarse(mg_ctx ctx, int32_t level, int32_t dtype, const void* in, void* out, int32_t nrhs,
                          void* stream);

/* Restriction R = P^dag from level `level` (1: fine, 2: first coarse) to the
 * next level (Sec. 2.1).  dtype MG_C128 or MG_C64. */
mg_status mg_restrict(mg_ctx ctx, int32_t level, int32_t dtype, const void* fine, void* coarse, int32_t nrhs,
                      void* stream);

/* Prolongation P from level `level` + 1 to `level` (Sec. 2.1: the coarse
 * correction is carried back to the finer level through the block-orthonormal,
 * chirally split near-null vectors, P the adjoint of the restriction):
 *   e[x,c] = sum_k P[(x,c),(a(x),sigma(x),k)] e_c[a(x),sigma(x),k]
 * with a(x) the aggregate of x and sigma(x) its chirality.
 *   coarse: device, [nrhs][Tc][Zc][Yc][Xc][2][Nvec] of level + 1 (input)
 *   fine:   device, [nrhs][T][Z][Y][X][3] (level 1) or the level-2 coarse
 *           layout (level 2); overwritten, or added into when accumulate = 1.
 * dtype MG_C128 or MG_C64, both buffers 16-byte aligned and distinct. */
mg_status mg_prolong(mg_ctx ctx, int32_t level, int32_t dtype, const void* coarse, void* fine,
                     int32_t accumulate, int32_t nrhs, void* stream);

/* Solve D(m_j) x = b for every mass m_j and right-hand side by the
 * MG-preconditioned GCR of Sec. 2.1 (K-cycle, Table 1), FP64 outer solver,
 * to ||b - D x|| / ||b|| <= tol (Sec. 3.2).  The hierarchy built at mass0 is
 * reused for every mass (Sec. 3.2-3.3); each mass gets its own exact KD
 * inverse.
 *   b: device complex128 [nrhs][T][Z][Y][X][3]
 *   x: device complex128 [nmass][nrhs][T][Z][Y][X][3] (overwritten)
 *   info: host array of nmass * nrhs entries (mass-major)
 * Systems are solved in lockstep batches of whole masses with at most
 * max_nrhs (mass, rhs) pairs each (nrhs <= max_nrhs; the masses of one batch
 * <= max_nmass).  Returns MG_OK when every system converged, MG_E_NOCONV
 * otherwise. */
mg_status mg_solve(mg_ctx ctx, const double* masses, int32_t nmass, const void* b, void* x, int32_t nrhs,
                   double tol, mg_solve_info* info, void* stream);

/* Baseline: single-parity (even) Schur CG in FP64 on the same stencil kernel
 * (Sec. 3.2): (m^2 - K_eo K_oe) x_e = m b_e - K_eo b_o, x_o = (b_o - K_oe x_e)/m,
 * iterated to ||r_e|| <= m tol ||b|| and confirmed on the true residual.
 * Same layouts and semantics as mg_solve; maxiter caps the CG iterations. */
mg_status mg_cg_solve(mg_ctx ctx, const double* masses, int32_t nmass, const void* b, void* x, int32_t nrhs,
                      double tol, int32_t maxiter, mg_solve_info* info, void* stream);

/* Multi-shift CG of the propagator workflow (Sec. 3.3: the masses a workflow
 * does not give to MG are solved together by multi-shift CG, one Krylov space
 * per parity).  D(m)^{-1} b = (m - K) y with (m^2 - K^2) y = b, which is
 * block-diagonal in parity; on each parity one CG on the smallest shift m_0^2
 * also solves (m_j^2 - K_pq K_qp) y_j = b_p through collinear residuals.  A
 * shift stops at |r_j| <= tol |b| / 2 on each parity; x_j = (m_j - K) y_j is
 * then checked on the true residual ||b - D(m_j) x_j|| / ||b|| <= tol, and a
 * system that misses it is finished by the Schur CG of mg_cg_solve started
 * from x_j (info.reliable_updates > 0 marks it).
 *   masses: host, 1..16 positive values (any order, repeats allowed)
 *   b: device complex128 [nrhs][T][Z][Y][X][3], nrhs <= max_nrhs
 *   x: device complex128 [nmass][nrhs][T][Z][Y][X][3] (overwritten)
 *   info: host, nmass * nrhs entries; outer_iters = iterations the system
 *     was updated (both parities), level_iters[0] = base iterations.
 * The search directions of all shifts live in the outer GCR work vectors:
 * MG_E_CONFIG when nmass blocks of nrhs half-lattice vectors do not fit in
 * (2 outer_nkrylov - 1) buffers of max_nrhs lattice vectors.  Synchronises
 * before returning; MG_E_NOCONV if a system still misses tol after maxiter. */
mg_status mg_msc_solve(mg_ctx ctx, const double* masses, int32_t nmass, const void* b, void* x, int32_t nrhs,
                       double tol, int32_t maxiter, mg_solve_info* info, void* stream);

/* Fermion force for HMC (the solver inside gauge generation, Sec. 4.2):
 * for S = sum_r phi_r^dag (D(m)^dag D(m))^{-1} phi_r computes
 *   X = (D^dag D)^{-1} phi and Y = D X  by two MG solves (D^dag = eps D eps),
 *   grad_fat[mu][x]  = -c1 eta_mu(x) sum_r [Y(x) X(x+mu)^dag  - X(x) Y(x+mu)^dag ]
 *   grad_naik[mu][x] = -c3 eta_mu(x) sum_r [Y(x) X(x+3mu)^dag - X(x) Y(x+3mu)^dag]
 * the gradients in PyTorch's convention (dS/dRe U + i dS/dIm U), canonical
 * link layout, complex128, overwritten.
 *   phi, X, Y: device complex128 [nrhs][T][Z][Y][X][3] (X, Y overwritten)
 *   action: host, nrhs doubles or NULL; receives S_r = Re <phi_r, X_r>
 *     (FP64 reduction on the device), so S = sum_r action[r]
 *   info: host, 2 * nrhs entries (the D^dag solves, then the D solves). */
mg_status mg_solve_backward(mg_ctx ctx, double mass, const void* phi, void* X, void* Y, void* grad_fat,
                            void* grad_naik, int32_t nrhs, double tol, double* action, mg_solve_info* info,
                            void* stream);

/* Replace the gauge links of an existing context (device, complex128): the
 * fine operator and the KD inverses follow the new links, the near-null
 * vectors, transfers and coarse operators stay those of the set-up (the
 * hierarchy then preconditions a nearby operator; solves stay exact).  As at
 * mg_setup, the long links are kept in 13-real form (two rows and det / scale,
 * Sec. 3.1) when every one is unitary to 1e-10, in full form otherwise; this
 * call synchronises the stream for that check. */
mg_status mg_update_links(mg_ctx ctx, const void* fat, const void* naik, void* stream);

/* Copy internal data to a caller buffer (device dst of at least `bytes`):
 *   what 0: fine index tables, int32 [V][22] (neighbours x+-mu, x+-3mu, eta
 *           bits, eps, hypercube, hypercube-local index, aggregate, chirality)
 *   what 1: near-null vectors of `level` (1 or 2), complex128, layout as the
 *           null_vectors argument of mg_setup; level nagg + 1: the coarsest
 *           level's deflation vectors [k][coarsest vector] (coarsest_deflate > 0)
 *   what 2: coarse links of `level` (2 or 3), complex128 [site][9][n][n]
 *           row-major blocks, n = 2 Nvec, d = 0 self, 1 + 2 mu: +mu, 2 + 2 mu: -mu
 * Returns the needed size in *bytes_needed when dst is NULL. */
mg_status mg_export(mg_ctx ctx, int32_t what, int32_t level, void* dst, size_t bytes, size_t* bytes_needed,
                    void* stream);

/* Coarse operators of several contexts in one persistent launch (the batch of
 * uneven problems): applies the level-`level` operator of ctxs[p] to in[p]
 * (device, MG_C64, nrhs[p] vectors of that context's level) into out[p], for
 * nprob <= 8 contexts whose level has 16-bit links of the same format and the
 * same 2 Nvec.  The workgroups walk one (problem, coarse site, 16-rhs tile)
 * work list with a grid-sized stride, so small lattices that could not fill
 * the device alone share it.  Results equal those of mg_apply_coarse with 16
 * rhs per workgroup.  Asynchronous on `stream`. */
mg_status mg_apply_coarse_multi(const mg_ctx* ctxs, int32_t nprob, int32_t level, const void* const* in,
                                void* const* out, const int32_t* nrhs, void* stream);

/* Tile-shape autotuner of the 16-bit coarse stencil (coarse_prec MG_CBF16 /
 * MG_CF16): for every coarse level, times each tile shape the kernel is
 * built for (16, 32 or 64 right-hand sides per workgroup x 1 or 2 16-row
 * m-tiles per wavefront) on nrhs (1..max_nrhs) random vectors of the
 * context's solver scratch, 2 untimed and 5 timed launches each with HIP
 * events on `stream`, and keeps the fastest for every later application with
 * a right-hand-side count in the same class (<= 16, 17..32, > 32).  info
 * (host, 2 entries, may be NULL) receives per level the shape chosen, its
 * time and that of the built-in choice.  Results are unchanged by the tile
 * shape up to FP32 summation order.  Synchronises the stream. */
typedef struct {
  int32_t level;             /* 2 or 3 (0: entry unused) */
  int32_t nrhs;
  int32_t rhs_per_workgroup, mtiles_per_wave;
  int32_t candidates;        /* shapes timed */
  double us_best, us_default;
} mg_tune_info;
mg_status mg_autotune(mg_ctx ctx, int32_t nrhs, mg_tune_info* info, void* stream);

/* Kernel timing (a measurement aid, not part of the method): between
 * mg_profile_start and mg_profile_stop every launch of one operator is
 * bracketed by a pair of HIP events recorded on the stream it runs on, so
 * the durations are those of the kernels inside a real solve.
 *   op    : an mg_prof_op.
 *   level : MG_PROF_COARSE: coarse level 2 or 3; MG_PROF_RESTRICT /
 *           MG_PROF_PROLONG: transfer level 1 or 2; MG_PROF_DSLASH: 0 for the
 *           stencil with the Naik term, 1 for the one-hop stencil of the KD
 *           level; MG_PROF_KD: 0.
 *   nrhs  : 0 times every launch; n > 0 only the launches over exactly n
 *           systems (a lockstep batch shrinks as its systems converge, and
 *           a measurement meant for the full batch must not mix in the
 *           smaller launches).  Negative: MG_E_ARG.
 * mg_profile_stop waits for the recorded events and returns the number of
 * launches and their summed duration in milliseconds, then stops recording.
 * Events are created on first use and kept until mg_destroy (host-side
 * runtime objects; no device workspace is used).  Starting again discards
 * any unread measurement. */
typedef enum {
  MG_PROF_COARSE = 0,
  MG_PROF_DSLASH = 1,
  MG_PROF_KD = 2,
  MG_PROF_RESTRICT = 3,
  MG_PROF_PROLONG = 4
} mg_prof_op;

mg_status mg_profile_start(mg_ctx ctx, int32_t op, int32_t level, int32_t nrhs);
mg_status mg_profile_stop(mg_ctx ctx, int32_t* launches, double* total_ms);

/* Measured ceilings of the device (measurement aids, not part of the
 * method; no context needed).  Each times its kernel with HIP events on
 * `stream` after one untimed launch.
 *   mg_peak_copy: a 16-byte-per-lane copy of `bytes` (multiple of 16) from
 *     src to dst (device, 16-byte aligned, distinct), reps timed launches;
 *     *gbs = 2 bytes / time (read + write) in GB/s.
 *   mg_peak_mfma: a loop of `iters` iterations of eight independent
 *     16x16x32 MFMA products per wavefront (fmt MG_CBF16 or MG_CF16, FP32
 *     accumulate) over 8 workgroups of four wavefronts per compute unit;
 *     sink: device, >= 8 KiB (receives per-workgroup sums that keep the
 *     products live); *tflops = dense 16-bit matrix-core rate in TFLOP/s. */
mg_status mg_peak_copy(const void* src, void* dst, size_t bytes, int32_t reps, void* stream, double* gbs);
mg_status mg_peak_mfma(int32_t fmt, int32_t iters, void* sink, void* stream, double* tflops);

mg_status mg_destroy(mg_ctx ctx);

const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGSTAG_H */
