// Coarse operator (Sec. 2.1 Galerkin A_c = R A P; Sec. 3.1 coarse stencil):
//   y(a) = X(a) x(a) + sum_mu [ Y_{+mu}(a) x(a+mu) + Y_{-mu}(a) x(a-mu) ]
// with dense (2 Nvec) x (2 Nvec) complex blocks, stored per site and direction
// as [d][col][row] so that the rows of one column are contiguous: one thread
// per output row, a workgroup per coarse site, the nine neighbour vectors
// staged in LDS.  The +mu and -mu blocks are kept apart, so an extent-2
// coarse direction (where a+mu = a-mu) is still exact.
#include "kernels.hpp"

namespace mg {

template <typename R, typename LT>
__device__ __forceinline__ cplx<R> load_link(const LT* p);
template <>
__device__ __forceinline__ double2 load_link<double, double2>(const double2* p) { return *p; }
template <>
__device__ __forceinline__ float2 load_link<float, float2>(const float2* p) { return *p; }

template <typename R, typename LT, int NR, bool PIECE, bool DAG>
__global__ void __launch_bounds__(256) coarse_kernel(const CoarseArgs<R, LT> a) {
  using T = cplx<R>;
  extern __shared__ unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);   // [9][NR][n]
  const int n = a.n;
  const int64_t site = blockIdx.x;
  const int r0 = blockIdx.y * NR;
  const int nr = (a.nrhs - r0) < NR ? (a.nrhs - r0) : NR;
  const int tid = threadIdx.x;
  int c[4];
  site_coords(site, a.g, c);
  int64_t nb[9];
  int use[9];
  nb[0] = site;
  use[0] = 1;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    nb[1 + 2 * mu] = site_shift(c, mu, 1, a.g);
    nb[2 + 2 * mu] = site_shift(c, mu, -1, a.g);
    if (PIECE) {
      const int u = c[mu] % a.blk[mu];
      const int pf = (u == a.blk[mu] - 1) ? 1 + 2 * mu : 0;
      const int pb = (u == 0) ? 2 + 2 * mu : 0;
      use[1 + 2 * mu] = pf == a.piece;
      use[2 + 2 * mu] = pb == a.piece;
    } else {
      use[1 + 2 * mu] = 1;
      use[2 + 2 * mu] = 1;
    }
  }
  if (PIECE) use[0] = (a.piece == 0);
  for (int e = tid; e < 9 * NR * n; e += blockDim.x) {
    const int d = e / (NR * n);
    const int rem = e - d * NR * n;
    const int r = rem / n, col = rem - r * n;
    T v;
    v.x = 0; v.y = 0;
    if (r < nr && use[d]) v = a.in[(int64_t)(r0 + r) * a.in_stride + nb[d] * n + col];
    xs[e] = v;
  }
  __syncthreads();
  const int64_t nn = (int64_t)n * n;
  for (int row = tid; row < n; row += blockDim.x) {
    T acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) { acc[r].x = 0; acc[r].y = 0; }
    for (int d = 0; d < 9; ++d) {
      if (!use[d]) continue;
      const T* xd = xs + d * NR * n;
      if (!DAG) {
        const LT* L = a.links + (site * 9 + d) * nn + row;
#pragma unroll 8
        for (int col = 0; col < n; ++col) {
          const T l = load_link<R, LT>(L + (int64_t)col * n);
#pragma unroll
          for (int r = 0; r < NR; ++r) cfma(acc[r], l, xd[r * n + col]);
        }
      } else {
        // (A^dag)_{a, nb} = (A_{nb, a})^dag: the opposite direction's block at the neighbour
        const int dd = d == 0 ? 0 : ((d & 1) ? d + 1 : d - 1);
        const LT* L = a.links + (nb[d] * 9 + dd) * nn + (int64_t)row * n;
#pragma unroll 8
        for (int col = 0; col < n; ++col) {
          const T l = load_link<R, LT>(L + col);
#pragma unroll
          for (int r = 0; r < NR; ++r) cfmac(acc[r], l, xd[r * n + col]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nr) continue;
      a.out[(int64_t)(r0 + r) * a.out_stride + site * n + row] = acc[r];
    }
  }
}

template <typename R, typename LT, int NR>
static void coarse_launch_nr(const CoarseArgs<R, LT>& a, bool piece, bool dag, hipStream_t st) {
  const int threads = ((a.n + 63) / 64) * 64 > 256 ? 256 : ((a.n + 63) / 64) * 64;
  dim3 grid((unsigned)a.g.V, (unsigned)((a.nrhs + NR - 1) / NR));
  const size_t lds = (size_t)9 * NR * a.n * sizeof(cplx<R>);
  if (piece) coarse_kernel<R, LT, NR, true, false><<<grid, threads, lds, st>>>(a);
  else if (dag) coarse_kernel<R, LT, NR, false, true><<<grid, threads, lds, st>>>(a);
  else coarse_kernel<R, LT, NR, false, false><<<grid, threads, lds, st>>>(a);
}

template <typename R, typename LT>
void launch_coarse(const CoarseArgs<R, LT>& a, bool piece, bool dag, hipStream_t st) {
  if (a.nrhs <= 0) return;
  // keep the staged neighbour vectors within 64 KiB of LDS
  const size_t per = (size_t)9 * a.n * sizeof(cplx<R>);
  if (a.nrhs >= 4 && 4 * per <= 65536) coarse_launch_nr<R, LT, 4>(a, piece, dag, st);
  else if (a.nrhs >= 2 && 2 * per <= 65536) coarse_launch_nr<R, LT, 2>(a, piece, dag, st);
  else coarse_launch_nr<R, LT, 1>(a, piece, dag, st);
}
template void launch_coarse<double, double2>(const CoarseArgs<double, double2>&, bool, bool, hipStream_t);
template void launch_coarse<float, float2>(const CoarseArgs<float, float2>&, bool, bool, hipStream_t);

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
