// Coarse operator (Sec. 2.1 Galerkin A_c = R A P; Sec. 3.1 coarse stencil):
//   y(a) = X(a) x(a) + sum_mu [ Y_{+mu}(a) x(a+mu) + Y_{-mu}(a) x(a-mu) ]
// with dense (2 Nvec) x (2 Nvec) complex blocks, stored per site and direction
// as [d][col][row] so that the rows of one column are contiguous.  The +mu and
// -mu blocks are kept apart, so an extent-2 coarse direction (where
// a+mu = a-mu) is still exact.  The coarse lattices are small, so the
// matrix-vector product is split over the K dimension as well (the paper's
// "additional parallelism" for the coarse stencil, Sec. 3.1).
#include "kernels.hpp"

namespace mg {

template <typename R, typename LT>
__device__ __forceinline__ cplx<R> load_link(const LT* p);
template <>
__device__ __forceinline__ double2 load_link<double, double2>(const double2* p) { return *p; }
template <>
__device__ __forceinline__ float2 load_link<float, float2>(const float2* p) { return *p; }

// One workgroup per (coarse site, 64-row tile, rhs tile) whose wavefronts
// (16 for one or two right-hand sides, fewer for wider rhs tiles) split the
// K = 9 n columns of the site's block row evenly (lanes run over rows, so
// every link load is one coalesced segment); the partial sums are reduced in
// LDS.  This exposes far more parallelism than one thread per row, which the
// small coarse lattices need to keep enough loads in flight.
template <int NR>
struct CoarseWaves { static constexpr int value = NR <= 2 ? 16 : (NR <= 4 ? 8 : 4); };

template <typename R, typename LT, int NR, bool PIECE, bool DAG>
__global__ void __launch_bounds__(64 * CoarseWaves<NR>::value) coarse_kernel(const CoarseArgs<R, LT> a) {
  using T = cplx<R>;
  constexpr int kCoarseWaves = CoarseWaves<NR>::value;
  __shared__ T red[kCoarseWaves - 1][NR][64];
  const int n = a.n;
  const int64_t site = blockIdx.x;
  const int row0 = blockIdx.y * 64;
  const int r0 = blockIdx.z * NR;
  const int nr = (a.nrhs - r0) < NR ? (a.nrhs - r0) : NR;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = row0 + lane;
  const bool act = row < n;
  int c[4];
  site_coords(site, a.g, c);
  int64_t nb[9];
  int use[9];
  nb[0] = site;
  use[0] = PIECE ? (a.piece == 0) : 1;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    nb[1 + 2 * mu] = site_shift(c, mu, 1, a.g);
    nb[2 + 2 * mu] = site_shift(c, mu, -1, a.g);
    if (PIECE) {
      const int u = c[mu] % a.blk[mu];
      use[1 + 2 * mu] = ((u == a.blk[mu] - 1) ? 1 + 2 * mu : 0) == a.piece;
      use[2 + 2 * mu] = ((u == 0) ? 2 + 2 * mu : 0) == a.piece;
    } else {
      use[1 + 2 * mu] = 1;
      use[2 + 2 * mu] = 1;
    }
  }
  const int64_t nn = (int64_t)n * n;
  const int K = 9 * n;
  const int per = (K + kCoarseWaves - 1) / kCoarseWaves;
  const int k0 = wave * per;
  const int k1 = (k0 + per) < K ? (k0 + per) : K;
  T acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) { acc[r].x = 0; acc[r].y = 0; }
  const T* in = a.in + (int64_t)r0 * a.in_stride;
  int kk = k0;
  while (kk < k1) {
    const int d = kk / n;
    const int cbeg = kk - d * n;
    const int cend = (k1 - d * n) < n ? (k1 - d * n) : n;
    kk = d * n + cend;
    if (!use[d]) continue;
    const T* xv = in + nb[d] * n;
    if (!DAG) {
      const LT* L = a.links + (site * 9 + d) * nn + (act ? row : 0);
#pragma unroll 8
      for (int col = cbeg; col < cend; ++col) {
        T l;
        if (act) l = L[(int64_t)col * n];
        else { l.x = 0; l.y = 0; }
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) cfma(acc[r], l, xv[(int64_t)r * a.in_stride + col]);
      }
    } else {
      // (A^dag)_{a, nb} = (A_{nb, a})^dag: the opposite direction's block at the neighbour
      const int dd = d == 0 ? 0 : ((d & 1) ? d + 1 : d - 1);
      const LT* L = a.links + (nb[d] * 9 + dd) * nn + (int64_t)(act ? row : 0) * n;
#pragma unroll 4
      for (int col = cbeg; col < cend; ++col) {
        T l;
        if (act) l = L[col];
        else { l.x = 0; l.y = 0; }
#pragma unroll
        for (int r = 0; r < NR; ++r)
          if (r < nr) cfmac(acc[r], l, xv[(int64_t)r * a.in_stride + col]);
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) red[wave - 1][r][lane] = acc[r];
  }
  __syncthreads();
  if (wave == 0 && act) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nr) continue;
      T v = acc[r];
      for (int w = 0; w < kCoarseWaves - 1; ++w) { v.x += red[w][r][lane].x; v.y += red[w][r][lane].y; }
      a.out[(int64_t)(r0 + r) * a.out_stride + site * n + row] = v;
    }
  }
}

template <typename R, typename LT, int NR>
static void coarse_launch_nr(const CoarseArgs<R, LT>& a, bool piece, bool dag, hipStream_t st) {
  dim3 grid((unsigned)a.g.V, (unsigned)((a.n + 63) / 64), (unsigned)((a.nrhs + NR - 1) / NR));
  const int threads = 64 * CoarseWaves<NR>::value;
  if (piece) coarse_kernel<R, LT, NR, true, false><<<grid, threads, 0, st>>>(a);
  else if (dag) coarse_kernel<R, LT, NR, false, true><<<grid, threads, 0, st>>>(a);
  else coarse_kernel<R, LT, NR, false, false><<<grid, threads, 0, st>>>(a);
}

template <typename R, typename LT>
void launch_coarse(const CoarseArgs<R, LT>& a, bool piece, bool dag, hipStream_t st) {
  if (a.nrhs <= 0) return;
  // wider rhs tiles issue one broadcast load per rhs and link element and
  // become issue-bound (measured: 16 rhs per tile ran at a tenth of the
  // bandwidth of 4); many right-hand sides belong on the matrix cores
  if (a.nrhs >= 4) coarse_launch_nr<R, LT, 4>(a, piece, dag, st);
  else if (a.nrhs >= 2) coarse_launch_nr<R, LT, 2>(a, piece, dag, st);
  else coarse_launch_nr<R, LT, 1>(a, piece, dag, st);
}
template void launch_coarse<double, double2>(const CoarseArgs<double, double2>&, bool, bool, hipStream_t);
template void launch_coarse<float, float2>(const CoarseArgs<float, float2>&, bool, bool, hipStream_t);

// Adjoint stencil as explicit links: (A^dag)_{a, a+d} = (A_{a+d, a})^dag, i.e.
// out[a][d] = (in[nb_d(a)][opposite d])^dag, in the same [site][d][col][row]
// layout, so the adjoint apply is an ordinary coalesced apply.
template <typename T>
__global__ void dagger_links_kernel(const T* __restrict__ in, T* __restrict__ out, Geom g, int n) {
  const int64_t nn = (int64_t)n * n;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= g.V * 9 * nn) return;
  const int64_t sd = tid / nn;
  const int64_t e = tid - sd * nn;
  const int col = (int)(e / n), row = (int)(e - (int64_t)col * n);
  const int64_t site = sd / 9;
  const int d = (int)(sd - site * 9);
  int c[4];
  site_coords(site, g, c);
  int64_t nb = site;
  int dd = 0;
  if (d > 0) {
    const int mu = (d - 1) >> 1;
    nb = site_shift(c, mu, (d & 1) ? 1 : -1, g);
    dd = (d & 1) ? d + 1 : d - 1;
  }
  // element (row, col) of the adjoint block = conj(element (col, row) of the neighbour's block)
  T v = in[(nb * 9 + dd) * nn + (int64_t)row * n + col];
  v.y = -v.y;
  out[tid] = v;
}
template <typename T>
void launch_dagger_links(const T* in, T* out, const Geom& g, int n, hipStream_t st) {
  const int64_t tot = g.V * 9 * (int64_t)n * n;
  dagger_links_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(in, out, g, n);
}
template void launch_dagger_links<float2>(const float2*, float2*, const Geom&, int, hipStream_t);
template void launch_dagger_links<double2>(const double2*, double2*, const Geom&, int, hipStream_t);

__global__ void convert_c128_c64_kernel(const double2* __restrict__ in, float2* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}
void launch_convert_links(const double2* in, float2* out, int64_t n, hipStream_t st) {
  convert_c128_c64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(in, out, n);
}

// Coarse links to the canonical layout [site][d][row][col] (row-major blocks), FP64
__global__ void export_links_kernel(const double2* __restrict__ in, double2* __restrict__ out, int64_t nsite,
                                    int n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (i >= nsite * 9 * nn) return;
  const int64_t sd = i / nn;
  const int64_t rem = i - sd * nn;
  const int row = (int)(rem / n), col = (int)(rem - (int64_t)row * n);
  out[i] = in[sd * nn + (int64_t)col * n + row];
}
void launch_export_links(const double2* in, double2* out, int64_t nsite, int n, hipStream_t st) {
  const int64_t tot = nsite * 9 * (int64_t)n * n;
  export_links_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(in, out, nsite, n);
}

}  // namespace mg
