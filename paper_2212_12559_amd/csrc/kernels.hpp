// Kernel argument blocks and host-side launchers of the mgstag HIP library.
#pragma once
#include "common.hpp"

namespace mg {

constexpr int kMaxPairs = 48;   // pair dot products per reduction launch
constexpr int kMaxTerms = 20;   // terms of one linear combination

// ---------------------------------------------------------------- Dslash
template <typename R>
struct DslashArgs {
  cplx<R>* out;
  const cplx<R>* in;
  const cplx<R>* xs;        // checkerboard mode: optional same-parity addend
  const cplx<R>* fat;       // [4][9][V], (c1/2) eta folded in
  const cplx<R>* lng;       // [4][9][V], (c3/2) eta folded in
  const float4* fat_pairs;  // optional FP32 one-hop links as element pairs [4][5][V] (last pair padded)
  const cplx<R>* lng_c;     // optional compressed Naik links [4][7][V]: rows 0, 1 and w, row 2 = w conj(row0 x row1)
  Geom g;
  int64_t in_stride, out_stride, xs_stride;   // per rhs, complex elements
  int nrhs;
  R mass;                   // full-lattice mode: out = mass * in + hops
  const R* mass_rhs;        // optional per-rhs mass (device)
  R a_coef, b_coef;         // checkerboard mode: out = a * xs + b * hops
  int parity;               // checkerboard mode: output parity
  int piece;                // Galerkin piece: 0 self, 1 + 2 mu (+mu face), 2 + 2 mu (-mu face)
  int blk[4];               // aggregation block of the piece decomposition
  int eps_out;              // multiply the result by epsilon(x)
  int off_cube;             // 1: only the hops that leave the site's 2^4 hypercube, no mass term (the rest of
                            //    D is B + m, which the KD inverse undoes: (B+m)^{-1} D = 1 + (B+m)^{-1} D_off)
};
template <typename R>
void launch_dslash(const DslashArgs<R>& a, bool naik, bool cb, bool piece, hipStream_t st);
// the one-hop FP32 stencil with the in-plane neighbours in LDS (the only one that implements off_cube):
// whether it takes this launch, and the launch itself (false: not applicable, nothing launched)
bool dslash_plane_ok(const DslashArgs<float>& a);
bool launch_dslash_plane(const DslashArgs<float>& a, hipStream_t st);
void launch_pack_links(const double2* src, double2* d64, float2* d32, float4* d32p, const Geom& g, double coef,
                       hipStream_t st);
void launch_export_fine_index(int32_t* out, const Geom& g, const Agg& A, hipStream_t st);
// Naik links in 13-real form (Sec. 3.1: long links are U(3) and compress to 13
// reals): with L = s N, s = (c3 / 2) eta_mu(x), store rows 0 and 1 of L and
// w = det(N) / s, so row 2 of L is w conj(row0 x row1).  dev_max receives the
// largest |N N^dag - 1| entry (as the bits of a non-negative double).
void launch_pack_naik_compressed(const double2* src, double2* d64, float2* d32, const Geom& g, double coef,
                                 unsigned long long* dev_max, hipStream_t st);
template <typename T>
void launch_eps(T* out, const T* in, const Geom& g, int nrhs, hipStream_t st);
void launch_cb_split(const double2* full, double2* ev, double2* od, const Geom& g, int nrhs, hipStream_t st);
void launch_cb_merge(double2* full, const double2* ev, const double2* od, const Geom& g, int nrhs, hipStream_t st);
void launch_force(const double2* X, const double2* Y, double2* gw, double2* gn, const Geom& g, int nrhs, double c1,
                  double c3, int accumulate, hipStream_t st);

// ---------------------------------------------------------------- KD
template <typename R>
struct KdArgs {
  cplx<R>* out;
  const cplx<R>* in;
  const cplx<R>* kinv;      // [slot][hc][48][48], column-major blocks
  Geom g;
  int64_t in_stride, out_stride;
  int nrhs;
  int rhs_per_slot;         // rhs r uses slot r / rhs_per_slot (0: slot 0 for all)
  int64_t slot_stride;
  int eps_in, eps_out;      // (B+m)^{-dag} = eps (B+m)^{-1} eps
  const cplx<R>* add;       // optional: out = (B+m)^{-1} in + add (add laid out as out)
};
void launch_kd_inverse(const double2* fat64, const Geom& g, double mass, double2* out64, float2* out32,
                       hipStream_t st);
template <typename R>
void launch_kd_apply(const KdArgs<R>& a, hipStream_t st);
// the FP32 KD kernel with LDS-staged 16-rhs tiles (the only one that implements `add`)
bool kd_lds_ok(const KdArgs<float>& a);

// ---------------------------------------------------------------- transfer
template <typename R>
struct RestrictArgs {
  cplx<R>* out;
  const cplx<R>* in;
  const cplx<R>* pr;        // [agg][2][nrows][nvec]
  Agg A;
  int64_t in_stride, out_stride;
  int64_t out_site_stride;  // complex elements between aggregates in the output (2 nvec normally)
  int nrhs;
};
template <typename R>
struct ProlongArgs {
  cplx<R>* out;
  const cplx<R>* in;        // coarse [nrhs][nagg][2][nvec]
  const cplx<R>* pp;        // [agg][2][nvec][nrows]
  Agg A;
  int64_t in_stride, out_stride;
  int nrhs;
  int accumulate;
  int unit_col;             // >= 0: prolong the unit coarse vector (sigma nvec + k == unit_col) on every aggregate
};
void launch_gather_null(const double2* nv, int64_t nflat, double2* pp, const Agg& A, hipStream_t st);
void launch_block_orth(double2* pp, const Agg& A, int* status, hipStream_t st);
void launch_p_layouts(const double2* pp64, double2* pr64, float2* pr32, float2* pp32, const Agg& A,
                      hipStream_t st);
template <typename R>
void launch_restrict(const RestrictArgs<R>& a, hipStream_t st);
template <typename R>
void launch_prolong(const ProlongArgs<R>& a, hipStream_t st);

// ---------------------------------------------------------------- coarse
template <typename R, typename LT>
struct CoarseArgs {
  cplx<R>* out;
  const cplx<R>* in;
  const LT* links;          // [site][9][n][n] (col-major blocks)
  Geom g;                   // coarse lattice
  int n;                    // 2 nvec
  int64_t in_stride, out_stride;
  int nrhs;
  int piece;
  int blk[4];
};
template <typename R, typename LT>
void launch_coarse(const CoarseArgs<R, LT>& a, bool piece, bool dag, hipStream_t st);
struct CoarseMfmaArgs {
  float2* out;
  const float2* in;
  const uint16_t* links;    // swizzled 16-bit fragments
  Geom g;
  int n;
  int64_t in_stride, out_stride;
  int nrhs;
  float inv_scale;
  int unit_self;            // the self block is the identity: skip its links, add the input instead (n % 32 == 0)
  int rt, mt;               // tile shape: 16 rt rhs per workgroup, mt m-tiles per wavefront (0, 0: by rhs count)
  const uint32_t* in16;     // optional: the input already in the link format, packed (re | im << 16)
  uint32_t* out16;          // optional: also store the output in that format (the next application's input)
};
// tile shapes the 16-bit coarse stencil is built for (rt, mt)
constexpr int kCoarseTiles[6][2] = {{1, 1}, {1, 2}, {2, 1}, {2, 2}, {4, 1}, {4, 2}};
void launch_coarse_mfma(const CoarseMfmaArgs& a, int fmt, hipStream_t st);   // fmt 0 bf16, 1 fp16
// several problems' 16-bit stencils (same n and format, 16 rhs per workgroup)
// in one persistent launch over their (problem, site, rhs tile) work list;
// start[p] is the first item of problem p, start[nprob] the total
constexpr int kMaxMulti = 8;
struct CoarseMultiArgs {
  CoarseMfmaArgs p[kMaxMulti];
  int64_t start[kMaxMulti + 1];
  int nprob;
};
void launch_coarse_mfma_multi(const CoarseMultiArgs& m, int fmt, hipStream_t st);
template <typename TI>
void launch_swizzle_links(const TI* cl, uint16_t* out, int64_t nsite, int n, int fmt, double scale,
                          hipStream_t st);
void launch_absmax(const double2* v, int64_t n, unsigned long long* out, hipStream_t st);
int64_t swizzled_link_elems(int64_t nsite, int n);
void launch_convert_links(const double2* in, float2* out, int64_t n, hipStream_t st);
template <typename T>
void launch_dagger_links(const T* in, T* out, const Geom& g, int n, hipStream_t st);
void launch_export_links(const double2* in, double2* out, int64_t nsite, int n, hipStream_t st);

// ---------------------------------------------------------------- block preconditioning
// C[b] = alpha A[b / a_div] B[b] + beta D[b]: batched complex products of
// column-major matrices (element (i, j) at j * ld + i); D optional
template <typename T>
struct BGemmArgs {
  const T* A; int64_t lda, sA; int a_div;
  const T* B; int64_t ldb, sB;
  T* C; int64_t ldc, sC;
  const T* D; int64_t ldd, sD;
  int m, n, k, batch;
  double alpha, beta;
};
template <typename T>
void launch_bgemm(const BGemmArgs<T>& a, hipStream_t st);
void launch_diag_block(const double2* L, double2* X, const Geom& g, int n, hipStream_t st);
void launch_unit_self(double2* L, const Geom& g, int n, hipStream_t st);
void launch_ns_init(const double2* X, double2* Y, int64_t nsite, int n, hipStream_t st);
void launch_ns_residual(const double2* T, int64_t nsite, int n, unsigned long long* out, hipStream_t st);
// dense inverse of the coarsest operator (links [site][9][col][row], ns dof per site) by Gauss-Jordan with
// partial pivoting: M scratch 2 n^2, f n, piv / pinv / status one word each; inverse column-major
constexpr int64_t kDirectMax = 8192;   // largest coarsest dof count solved directly
void dense_coarsest_inverse(const double2* links, const Geom& g, int ns, double2* M, double2* f, int* piv,
                            double2* pinv, int* status, double2* inv64, float2* inv32, hipStream_t st);

// ---------------------------------------------------------------- BLAS
template <typename T>
struct PairDotArgs {
  const T* x[kMaxPairs];
  const T* y[kMaxPairs];
  int np;
  int64_t n, stride;
  int nrhs;
};
template <typename T>
struct LinCombArgs {
  T* out;
  T* out2;                       // optional second output with the same coefficients over v2
  const T* v2[kMaxTerms];
  const T* v[kMaxTerms];
  const double2* c[kMaxTerms];   // per-rhs device coefficient, or null for cconst
  double2 cconst[kMaxTerms];
  int neg[kMaxTerms];
  int conj[kMaxTerms];
  int masked[kMaxTerms];
  const int* mask;
  int nt;
  int64_t n, stride;
  int nrhs;
};
// CA-GCR Gram data: u[0..s-1] = A p_0..A p_{s-1}, u[s] = t (s <= kMaxCA)
template <typename T>
struct GramArgs {
  const T* u[kMaxCA + 1];
  int s;
  int64_t n, stride;
  int nrhs;
};
// One reduction pass of a GCR direction: <q_i, q_k>, <q_i, r> (i < k), |q_k|^2, <q_k, r>
template <typename T>
struct GcrDotArgs {
  const T* q[kMaxNK];
  const T* qk;
  const T* r;
  int k;
  int64_t n, stride;
  int nrhs;
};
// q_k <- (q_k - sum_i beta_i q_i) inv, r <- r - alpha (q_k - sum_i beta_i q_i), znext <- r
template <typename T>
struct GcrUpdArgs {
  T* qk;
  const T* q[kMaxNK];
  const double2* beta[kMaxNK];
  T* r;
  T* znext;                      // optional copy of the new r (next direction of unpreconditioned GCR)
  const double2* alpha;
  const double2* inv;
  int k;
  int64_t n, stride;
  int nrhs;
};
// Deferred-update GCR scalars of one level, per system (ld = max systems):
// beta(i, k) at [i * kMaxNK + k], g_k at [kTriG + k], alpha'_k at [kTriA + k],
// gamma_k at [kTriC + k]
constexpr int kTriG = kMaxNK * kMaxNK;
constexpr int kTriA = kTriG + kMaxNK;
constexpr int kTriC = kTriA + kMaxNK;
constexpr int kTriSlots = kTriC + kMaxNK;
int reduce_blocks(int64_t n);
template <typename T>
void launch_pairdot(const PairDotArgs<T>& a, double2* part, double2* res, int ldr, hipStream_t st);
template <typename T>
void launch_lincomb(const LinCombArgs<T>& a, hipStream_t st);
template <typename TI, typename TO>
void launch_convert(TO* out, const TI* in, int64_t n, hipStream_t st);
void launch_gcr_scalars(const double2* qq, const double2* qr, const int* mask, int nrhs, double2* alpha,
                        double2* nalpha, double2* inv, hipStream_t st);
void launch_cagcr_solve(const double2* gram, int s, int nrhs, int ldr, const int* mask, double2* coef,
                        hipStream_t st);
void launch_cg_alpha(const double2* rr, const double2* pap, const int* mask, int nrhs, double2* alpha,
                     double2* nalpha, hipStream_t st);
void launch_cg_beta(double2* rr, const double2* rrnew, const int* mask, int nrhs, double2* beta, hipStream_t st);
template <typename T>
void launch_random_normal(T* out, int64_t n, uint64_t seed, hipStream_t st);
template <typename T>
void launch_gcr_update(T* x, T* r, T* q, T* z, const double2* alpha, const double2* inv, int64_t n, int nrhs,
                       double2* part, double2* res, int ldr, hipStream_t st);
void launch_cg_update(double2* x, double2* r, const double2* p, const double2* ap, const double2* alpha, int64_t n,
                      int nrhs, double2* part, double2* res, int ldr, hipStream_t st);
template <typename T>
void launch_gram(const GramArgs<T>& a, double2* part, double2* res, int ldr, hipStream_t st);
void launch_gcr_backsub(double2* tri, int nk, int nrhs, int ld, hipStream_t st);
template <typename T>
void launch_gcr_dots(const GcrDotArgs<T>& a, double2* part, double2* res, int ldr, hipStream_t st);
void launch_gcr_scalars_cgs(const double2* dots, int k, const int* mask, int nrhs, int ld, double2* tri,
                            double2* alpha, double2* inv, hipStream_t st);
template <typename T>
void launch_gcr_update_cgs(const GcrUpdArgs<T>& a, double2* part, double2* res, int ldr, hipStream_t st);
void launch_conv(int* mask, const double2* rn2, const double2* r0sq, double tol2, int nrhs, int init,
                 hipStream_t st);
// Per-system power-of-two scale s = 2^-e, e = round(log2 rms(b)), from |b|^2
// (r0sq, rescaled to |s b|^2 in place); fwd = s, inv = 1 / s.
void launch_rhs_scale(double2* r0sq, double2* fwd, double2* inv, int64_t n, int nrhs, hipStream_t st);

// Coarsest-level deflation (deflate.hip): at most kMaxDefl vectors.
constexpr int kMaxDefl = 64;
template <typename T>
void launch_ts_gram(const T* A, int64_t lda, int ka, const T* B, int64_t ldb, int kb, int64_t n, double2* part,
                    size_t part_elems, double2* C, hipStream_t st);
template <typename T>
void launch_ts_combine(T* out, int64_t ldo, const T* in, int64_t ldi, int ka, int kb, const double2* M, int64_t n,
                       int mode, hipStream_t st);
void launch_chol_rinv(const double2* G, int k, double2* R, double2* Rinv, int* status, hipStream_t st);

// Multi-shift CG (Sec. 3.3).  Device state of the shifted systems, slots of
// ld entries: per shift j at kMscPer * j + {zeta, previous zeta, alpha_j,
// zeta'_j, beta_j, update flag, on flag, iteration count}; per rhs at
// kMscPer * kMaxShift + {previous base alpha, previous base beta}.
constexpr int kMaxShift = 16;
constexpr int kMscPer = 8;
constexpr int kMscSlots = kMscPer * kMaxShift + 2;
struct MscScalArgs {
  double2* st;             // state slots [kMscSlots][ld]
  double2* rr;             // |r|^2 per rhs (replaced by the new value)
  const double2* rrnew;    // |r|^2 after the base step
  const double2* alpha;    // base alpha per rhs (0 when masked)
  const double2* target2;  // stopping |r_j|^2 per rhs
  int* mask;               // per rhs: 1 while any shift is on
  double delta[kMaxShift]; // sigma_j - sigma_base
  int nshift, base, nrhs, ld;
};
struct MscUpdArgs {
  double2* x[kMaxShift];   // solution of shift j, rhs r at x[j] + r * x_stride
  double2* p[kMaxShift];   // search direction of shift j at p[j] + r * p_stride
  const double2* r;        // base residual at r + rhs * r_stride
  const double2* st;
  int64_t n, x_stride, p_stride, r_stride;
  int nshift, nrhs, ld;
};
void launch_msc_init(double2* st, const double2* rr, const double2* target2, int* mask, int nshift, int nrhs, int ld,
                     hipStream_t st_);
void launch_msc_scalars(const MscScalArgs& a, hipStream_t st);
void launch_msc_update(const MscUpdArgs& a, hipStream_t st);

}  // namespace mg
