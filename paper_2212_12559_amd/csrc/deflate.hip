// Deflation of the coarsest solve (Table 1: the coarsest level is deflated
// with low modes of its operator).  With W the deflation vectors and Z = A W,
// a Cholesky QR  Z^H Z = R^H R  gives Q = Z R^{-1} and W' = W R^{-1}; the
// deflated start of a coarsest solve is the least-squares one,
//   c = Q^H b,  x0 = W' c,  r0 = b - Q c.
// Vectors are stored system-major ([vector][n], stride ld), k <= 64.
#include <algorithm>
#include <stdexcept>

#include "kernels.hpp"

namespace mg {

__device__ __forceinline__ double2 ld_d2(const float2* p) { const float2 v = *p; return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 ld_d2(const double2* p) { return *p; }
template <typename T> __device__ __forceinline__ T st_t(double2 v);
template <> __device__ __forceinline__ float2 st_t<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ __forceinline__ double2 st_t<double2>(double2 v) { return v; }

constexpr int kTsE = 16;     // elements per LDS stage
constexpr int kTsBlocks = 128;

// Partial C[i][s] = sum_e conj(A[i][e]) B[s][e] over one chunk of e per
// block: both 64 x 16 tiles staged in LDS, a 4 x 4 register tile of FP64
// accumulators per thread (rows ti + 16 a, columns ts + 16 b).
template <typename T>
__global__ void __launch_bounds__(256) ts_gram_kernel(const T* __restrict__ A, int64_t lda, int ka,
                                                      const T* __restrict__ B, int64_t ldb, int kb, int64_t n,
                                                      int64_t chunk, double2* __restrict__ part) {
  __shared__ double2 As[kMaxDefl][kTsE + 1];
  __shared__ double2 Bs[kMaxDefl][kTsE + 1];
  const int tid = threadIdx.x, ti = tid >> 4, ts = tid & 15;
  const int64_t e_lo = (int64_t)blockIdx.x * chunk, e_hi = std::min<int64_t>(n, e_lo + chunk);
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
  for (int64_t e0 = e_lo; e0 < e_hi; e0 += kTsE) {
    __syncthreads();
    for (int q = tid; q < kMaxDefl * kTsE; q += 256) {
      const int i = q / kTsE, e = q - i * kTsE;
      const int64_t ee = e0 + e;
      const bool in = ee < e_hi;
      As[i][e] = (in && i < ka) ? ld_d2(A + i * lda + ee) : make_double2(0.0, 0.0);
      Bs[i][e] = (in && i < kb) ? ld_d2(B + i * ldb + ee) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int e = 0; e < kTsE; ++e) {
      double2 av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[ti + 16 * a][e];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[ts + 16 * b][e];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b].x = fma(av[a].x, bv[b].x, fma(av[a].y, bv[b].y, acc[a][b].x));
          acc[a][b].y = fma(av[a].x, bv[b].y, fma(-av[a].y, bv[b].x, acc[a][b].y));
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      part[((int64_t)blockIdx.x * kMaxDefl + ti + 16 * a) * kMaxDefl + ts + 16 * b] = acc[a][b];
}

// C[i * kb + s] = sum over blocks, in block order
__global__ void ts_gram_reduce_kernel(const double2* __restrict__ part, int nblk, int ka, int kb,
                                      double2* __restrict__ C) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ka * kb) return;
  const int i = q / kb, s = q - i * kb;
  double2 v = make_double2(0.0, 0.0);
  for (int b = 0; b < nblk; ++b) {
    const double2 p = part[((int64_t)b * kMaxDefl + i) * kMaxDefl + s];
    v.x += p.x;
    v.y += p.y;
  }
  C[q] = v;
}

template <typename T>
void launch_ts_gram(const T* A, int64_t lda, int ka, const T* B, int64_t ldb, int kb, int64_t n, double2* part,
                    size_t part_elems, double2* C, hipStream_t st) {
  if (ka < 1 || kb < 1 || ka > kMaxDefl || kb > kMaxDefl) throw std::runtime_error("ts_gram: 1..64 vectors");
  int64_t chunk = (n + kTsBlocks - 1) / kTsBlocks;
  chunk = (chunk + kTsE - 1) / kTsE * kTsE;
  const int nblk = (int)((n + chunk - 1) / chunk);
  if ((size_t)nblk * kMaxDefl * kMaxDefl > part_elems) throw std::runtime_error("ts_gram: partial buffer too small");
  ts_gram_kernel<T><<<nblk, 256, 0, st>>>(A, lda, ka, B, ldb, kb, n, chunk, part);
  ts_gram_reduce_kernel<<<(ka * kb + 255) / 256, 256, 0, st>>>(part, nblk, ka, kb, C);
}
template void launch_ts_gram<float2>(const float2*, int64_t, int, const float2*, int64_t, int, int64_t, double2*,
                                     size_t, double2*, hipStream_t);
template void launch_ts_gram<double2>(const double2*, int64_t, int, const double2*, int64_t, int, int64_t, double2*,
                                      size_t, double2*, hipStream_t);

// out[j][e] = sign * out[j][e] (mode 1 / -1: keep and add / subtract; mode 0:
// overwrite) + sum_i in[i][e] M[i * kb + j].  A wavefront owns 64 elements
// and 16 columns j, so its M reads are uniform.
template <typename T>
__global__ void __launch_bounds__(256) ts_combine_kernel(T* __restrict__ out, int64_t ldo, const T* __restrict__ in,
                                                         int64_t ldi, int ka, int kb, const double2* __restrict__ M,
                                                         int64_t n, int mode) {
  const int64_t e = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int j0 = (threadIdx.x >> 6) * 16;
  if (j0 >= kb) return;
  double2 acc[16];
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) acc[jj] = make_double2(0.0, 0.0);
  if (e < n) {
    for (int i = 0; i < ka; ++i) {
      const double2 v = ld_d2(in + i * ldi + e);
      const double2* m = M + (int64_t)i * kb + j0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        if (j0 + jj < kb) {
          const double2 c = m[jj];
          acc[jj].x = fma(v.x, c.x, fma(-v.y, c.y, acc[jj].x));
          acc[jj].y = fma(v.x, c.y, fma(v.y, c.x, acc[jj].y));
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      if (j0 + jj >= kb) break;
      T* o = out + (int64_t)(j0 + jj) * ldo + e;
      double2 r = acc[jj];
      if (mode != 0) {
        const double2 old = ld_d2(o);
        r = mode > 0 ? make_double2(old.x + r.x, old.y + r.y) : make_double2(old.x - r.x, old.y - r.y);
      }
      *o = st_t<T>(r);
    }
  }
}

template <typename T>
void launch_ts_combine(T* out, int64_t ldo, const T* in, int64_t ldi, int ka, int kb, const double2* M, int64_t n,
                       int mode, hipStream_t st) {
  if (ka < 1 || kb < 1 || ka > kMaxDefl || kb > kMaxDefl) throw std::runtime_error("ts_combine: 1..64 vectors");
  ts_combine_kernel<T><<<(unsigned)((n + 63) / 64), 256, 0, st>>>(out, ldo, in, ldi, ka, kb, M, n, mode);
}
template void launch_ts_combine<float2>(float2*, int64_t, const float2*, int64_t, int, int, const double2*, int64_t,
                                        int, hipStream_t);
template void launch_ts_combine<double2>(double2*, int64_t, const double2*, int64_t, int, int, const double2*,
                                         int64_t, int, hipStream_t);

// Cholesky G = R^H R (R upper, G Hermitian positive definite, k x k row-major)
// and the inverse of R, in FP64 by one workgroup; R is built in place of its
// work copy.  status = 1 when a pivot is not positive against the diagonal
// (the deflation vectors are numerically dependent).
__global__ void __launch_bounds__(64) chol_rinv_kernel(const double2* __restrict__ G, int k, double2* __restrict__ R,
                                                       double2* __restrict__ Rinv, int* status) {
  const int t = threadIdx.x;
  for (int q = t; q < k * k; q += 64) R[q] = G[q];
  __syncthreads();
  __shared__ int bad;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    // diagonal (one thread), then row j to the right of it
    if (t == 0) {
      double d = R[j * k + j].x;
      for (int p = 0; p < j; ++p) d -= R[p * k + j].x * R[p * k + j].x + R[p * k + j].y * R[p * k + j].y;
      const double g = G[j * k + j].x;
      if (!(d > 1e-13 * g) || !(g > 0.0)) { bad = 1; d = 1.0; }
      R[j * k + j] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    const double rjj = R[j * k + j].x;
    for (int i = j + 1 + t; i < k; i += 64) {
      double2 v = R[j * k + i];
      for (int p = 0; p < j; ++p) {
        const double2 a = R[p * k + j], b = R[p * k + i];   // conj(a) * b
        v.x -= a.x * b.x + a.y * b.y;
        v.y -= a.x * b.y - a.y * b.x;
      }
      R[j * k + i] = make_double2(v.x / rjj, v.y / rjj);
    }
    __syncthreads();
  }
  // zero below the diagonal, then column j of R^{-1} by back substitution
  for (int q = t; q < k * k; q += 64)
    if (q / k > q % k) R[q] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int j = t; j < k; j += 64) {
    for (int i = k - 1; i >= 0; --i) {
      double2 v = make_double2(i == j ? 1.0 : 0.0, 0.0);
      if (i < j) {
        for (int p = i + 1; p <= j; ++p) {
          const double2 a = R[i * k + p], b = Rinv[p * k + j];
          v.x -= a.x * b.x - a.y * b.y;
          v.y -= a.x * b.y + a.y * b.x;
        }
      }
      // divide by the real diagonal; entries below the diagonal stay zero
      Rinv[i * k + j] = i > j ? make_double2(0.0, 0.0) : make_double2(v.x / R[i * k + i].x, v.y / R[i * k + i].x);
    }
  }
  __syncthreads();
  if (t == 0 && bad) *status = 1;
}

void launch_chol_rinv(const double2* G, int k, double2* R, double2* Rinv, int* status, hipStream_t st) {
  if (k < 1 || k > kMaxDefl) throw std::runtime_error("chol_rinv: 1..64");
  chol_rinv_kernel<<<1, 64, 0, st>>>(G, k, R, Rinv, status);
}

}  // namespace mg
