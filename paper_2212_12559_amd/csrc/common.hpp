// Shared device/host definitions of the mgstag HIP library (gfx950).
//
// Internal layouts (private; converted at the C-ABI boundary):
//   fine vector   [nrhs][V][3] complex, sites lexicographic (x fastest)
//   coarse vector [nrhs][Vc][2][Nvec] complex (spin/chirality major, +1 first)
//   fine links    [dir 0..3][entry 0..8][V] complex (structure of arrays), with
//                 the factor (c/2) * eta_mu(x) folded in
//   KD inverse    [hypercube][col 0..47][row 0..47] complex (column-major blocks)
//   P, restrict   [agg][chirality][row][k]   (lanes of a wave run over k)
//   P, prolong    [agg][chirality][k][row]   (lanes of a wave run over rows)
//   coarse links  [site][d 0..8][col][row], d = 0 self, 1 + 2 mu = +mu, 2 + 2 mu = -mu
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace mg {

// ------------------------------------------------------------------ complex
template <typename R> struct ctype;
template <> struct ctype<float> { using type = float2; };
template <> struct ctype<double> { using type = double2; };
template <typename R> using cplx = typename ctype<R>::type;

// acc += a * b
template <typename T>
__device__ __forceinline__ void cfma(T& acc, const T a, const T b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename T>
__device__ __forceinline__ void cfmac(T& acc, const T a, const T b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
template <typename T>
__device__ __forceinline__ T cmul(const T a, const T b) { T r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r; }

__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
template <typename T> __device__ __forceinline__ T from_d2(double2 a);
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }

// ------------------------------------------------------------------ geometry
struct Geom {
  int L[4];          // extents X, Y, Z, T
  int64_t V;         // volume
};

__host__ __device__ __forceinline__ void site_coords(int64_t s, const Geom& g, int c[4]) {
  c[0] = (int)(s % g.L[0]); s /= g.L[0];
  c[1] = (int)(s % g.L[1]); s /= g.L[1];
  c[2] = (int)(s % g.L[2]);
  c[3] = (int)(s / g.L[2]);
}
__host__ __device__ __forceinline__ int64_t site_index(const int c[4], const Geom& g) {
  return c[0] + (int64_t)g.L[0] * (c[1] + (int64_t)g.L[1] * (c[2] + (int64_t)g.L[2] * c[3]));
}
// site index of c shifted by h along mu (periodic), h in [-3, 3]
__host__ __device__ __forceinline__ int64_t site_shift(const int c[4], int mu, int h, const Geom& g) {
  int cc[4] = {c[0], c[1], c[2], c[3]};
  int v = cc[mu] + h;
  if (v >= g.L[mu]) v -= g.L[mu];
  if (v < 0) v += g.L[mu];
  cc[mu] = v;
  return site_index(cc, g);
}
__host__ __device__ __forceinline__ int site_parity(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

// Kahler-Dirac hypercubes: origin at even coordinates, local index
// s = sum_mu (x_mu mod 2) 2^mu, 48 x 48 block row 3 s + colour.
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumbering block b of nb so that XCD x runs one contiguous range of
// blocks keeps lattice neighbours, which share input data, in one L2 (blocks
// past the last multiple of 8 keep their number; the map is a bijection).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t per = nb >> 3;
  if (b >= per * 8) return b;
  return (b & 7) * per + (b >> 3);
}

__host__ __device__ __forceinline__ int64_t hc_site(int64_t hc, int sl, const Geom& g) {
  const int h0 = g.L[0] / 2, h1 = g.L[1] / 2, h2 = g.L[2] / 2;
  int c[4];
  c[0] = 2 * (int)(hc % h0) + (sl & 1); hc /= h0;
  c[1] = 2 * (int)(hc % h1) + ((sl >> 1) & 1); hc /= h1;
  c[2] = 2 * (int)(hc % h2) + ((sl >> 2) & 1);
  c[3] = 2 * (int)(hc / h2) + ((sl >> 3) & 1);
  return site_index(c, g);
}
__host__ __device__ __forceinline__ void hc_of_site(const int c[4], const Geom& g, int64_t* hc, int* sl) {
  const int h0 = g.L[0] / 2, h1 = g.L[1] / 2, h2 = g.L[2] / 2;
  *hc = (c[0] >> 1) + (int64_t)h0 * ((c[1] >> 1) + (int64_t)h1 * ((c[2] >> 1) + (int64_t)h2 * (c[3] >> 1)));
  *sl = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2) | ((c[3] & 1) << 3);
}
__host__ __device__ __forceinline__ int stag_eta(const int c[4], int mu) {
  // eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z)
  int e = 0;
  for (int nu = 0; nu < mu; ++nu) e += c[nu];
  return (e & 1) ? -1 : 1;
}

// Aggregation geometry of one transfer level.
//   level 1 (fine -> coarse): an aggregate is a block b of fine sites; its rows
//     of chirality sigma are (j, colour) with j enumerating the block sites of
//     parity sigma, 3 colours per site, so nrows = |b| / 2 * 3;
//   level 2 (coarse -> coarser): an aggregate is a block b of coarse sites; the
//     chirality is the spin index, rows (j, k) over all |b| sites and the Nvec
//     fine-level vectors, so nrows = |b| * nvec_in.
struct Agg {
  Geom fine;         // geometry of the level being aggregated
  int b[4];          // block
  int cd[4];         // coarse extents = fine.L / b
  int64_t nagg;      // number of aggregates
  int nrows;         // rows per (aggregate, chirality)
  int nvec;          // near-null vectors (coarse dof per chirality)
  int kind;          // 1: fine lattice (colour rows), 2: coarse lattice (spin x vec rows)
  int nvec_in;       // kind 2: Nvec of the level being aggregated
};

// flat index (into a single-rhs vector of the fine level) of row `row` of
// aggregate a, chirality sigma, as the aggregate's origin plus the row's
// offset from it: site_index is linear in the coordinates and an aggregate
// never wraps around the lattice, so
//   agg_row_index(A, a, sigma, row) = agg_base(A, a) + agg_row_rel(A, sigma, row)
// and a kernel that walks the rows of one aggregate takes agg_base once.
__host__ __device__ __forceinline__ int64_t agg_base(const Agg& A, int64_t a) {
  int c[4];
  int64_t t = a;
  c[0] = (int)(t % A.cd[0]) * A.b[0]; t /= A.cd[0];
  c[1] = (int)(t % A.cd[1]) * A.b[1]; t /= A.cd[1];
  c[2] = (int)(t % A.cd[2]) * A.b[2];
  c[3] = (int)(t / A.cd[2]) * A.b[3];
  const int64_t s = site_index(c, A.fine);
  return A.kind == 1 ? s * 3 : s * 2 * (int64_t)A.nvec_in;
}
__host__ __device__ __forceinline__ int64_t agg_row_rel(const Agg& A, int sigma, int row) {
  int u[4];
  if (A.kind == 1) {   // rows (site of chirality sigma, colour); x runs over the sites of that parity
    const int j = row / 3, col = row - 3 * j;
    const int hb0 = A.b[0] / 2;
    int rest = j / hb0;
    const int i = j - hb0 * rest;
    u[1] = rest % A.b[1]; rest /= A.b[1];
    u[2] = rest % A.b[2];
    u[3] = rest / A.b[2];
    u[0] = 2 * i + ((u[1] + u[2] + u[3] + sigma) & 1);
    return site_index(u, A.fine) * 3 + col;
  }
  const int j = row / A.nvec_in, k = row - A.nvec_in * j;   // rows (site, vector) of chirality sigma
  int rest = j;
  u[0] = rest % A.b[0]; rest /= A.b[0];
  u[1] = rest % A.b[1]; rest /= A.b[1];
  u[2] = rest % A.b[2];
  u[3] = rest / A.b[2];
  return (site_index(u, A.fine) * 2 + sigma) * (int64_t)A.nvec_in + k;
}
__host__ __device__ __forceinline__ int64_t agg_row_index(const Agg& A, int64_t a, int sigma, int row) {
  return agg_base(A, a) + agg_row_rel(A, sigma, row);
}

// ------------------------------------------------------------------ enums
enum Prec { P64 = 0, P32 = 1, PBF16 = 2, PF16 = 3 };
inline size_t csize(int p) { return p == P64 ? 16 : (p == P32 ? 8 : 4); }

// Per-level scalar slots (one double2 per system each):
//   0..47 dot products of one reduction (Gram matrix, projections)
//   48..53 GCR / CG scalars, 54..61 CA-GCR coefficients, 64.. norms
constexpr int kMaxSlots = 72;
constexpr int kSlotQQ = 48;          // GCR: <q,q>, <q,r>, alpha, -alpha, 1/|q|
constexpr int kSlotCoef = 54;        // CA-GCR coefficients (8)
constexpr int kSlotRN = 64;          // |r|^2 after a GCR step
constexpr int kSlotR0 = 65;          // |b|^2 of a level solve
constexpr int kSlotNorm = 66;        // norms read by the host
constexpr int kSlotScale = 67;       // power-of-two rhs scale of a coarse level solve, then its inverse (68)
constexpr int kMaxNK = 16;           // Krylov directions per GCR
constexpr int kMaxS = 8;             // CA-GCR basis size of the smoother
constexpr int kMaxCA = 16;           // CA-GCR basis size of the coarsest solver

}  // namespace mg
