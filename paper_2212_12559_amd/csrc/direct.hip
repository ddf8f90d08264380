// Exact coarsest solve for small coarsest levels (coarsest_solver 2): the
// dense matrix of the coarsest operator is assembled from its FP64 links and
// inverted once at set-up by Gauss-Jordan elimination with partial pivoting
// (FP64); every coarsest solve is then the product x = A^{-1} b (the batched
// complex GEMM of blockprec.hip with one batch, n x nsys right-hand sides).
//
// The elimination works on the row-major augmented matrix M = [A | 1]
// (n x 2n).  Step k: pivot p = argmax_{i >= k} |M[i][k]|, swap rows k and p,
// scale row k by 1 / M[k][k], then subtract M[i][k] times row k from every
// other row i.  Left columns below k are unit vectors by then (row k is zero
// there), so a step touches columns k .. 2n - 1 only.  At the end the right
// half holds A^{-1}.
#include "kernels.hpp"

namespace mg {

// M = [0 | 1]
__global__ void gj_init_kernel(double2* __restrict__ M, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * n * n) return;
  const int64_t i = t / (2 * n), j = t - i * 2 * n;
  M[t] = make_double2(j - n == i ? 1.0 : 0.0, 0.0);
}

// M[site ns + row][nb(site, d) ns + col] += L[site][d][col][row] for one
// direction d (for a fixed d, site -> nb(site, d) is a bijection, so the
// blocks of one launch never overlap; the nine launches run in order, which
// sums the blocks that land on one position when a coarse extent is 1 or 2)
__global__ void gj_assemble_kernel(const double2* __restrict__ L, double2* __restrict__ M, Geom g, int ns, int d) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)ns * ns;
  if (t >= g.V * nn) return;
  const int64_t site = t / nn;
  const int e = (int)(t - site * nn);
  const int col = e / ns, row = e - col * ns;
  int c[4];
  site_coords(site, g, c);
  const int64_t nb = d == 0 ? site : site_shift(c, (d - 1) >> 1, (d & 1) ? 1 : -1, g);
  const int64_t n = g.V * ns;
  double2* m = M + (site * ns + row) * 2 * n + nb * ns + col;
  const double2 v = L[(site * 9 + d) * nn + e];
  m->x += v.x;
  m->y += v.y;
}

// one workgroup: pivot row of column k, its inverse; a zero column sets the
// status word
__global__ void __launch_bounds__(256) gj_pivot_kernel(const double2* __restrict__ M, int64_t n, int k,
                                                       int* __restrict__ piv, double2* __restrict__ pinv,
                                                       int* __restrict__ status) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  double best = -1.0;
  int bidx = k;
  for (int64_t i = k + threadIdx.x; i < n; i += 256) {
    const double2 v = M[i * 2 * n + k];
    const double a = v.x * v.x + v.y * v.y;
    if (a > best) { best = a; bidx = (int)i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const int oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int p = bi[0];
    const double2 v = M[(int64_t)p * 2 * n + k];
    const double a = v.x * v.x + v.y * v.y;
    piv[0] = p;
    if (!(a > 0.0)) {
      status[0] = 1;
      pinv[0] = make_double2(0.0, 0.0);
    } else {
      pinv[0] = make_double2(v.x / a, -v.y / a);   // 1 / v
    }
  }
}

// swap rows k and p and scale the new row k, columns k .. 2n - 1
__global__ void gj_swap_scale_kernel(double2* __restrict__ M, int64_t n, int k, const int* __restrict__ piv,
                                     const double2* __restrict__ pinv) {
  const int64_t j = k + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 2 * n) return;
  const int64_t p = piv[0];
  const double2 s = pinv[0];
  double2* rk = M + (int64_t)k * 2 * n;
  double2* rp = M + p * 2 * n;
  const double2 a = rp[j], b = rk[j];
  if (p != k) rp[j] = b;
  rk[j] = make_double2(a.x * s.x - a.y * s.y, a.x * s.y + a.y * s.x);
}

// f[i] = M[i][k] (the elimination factors, read before column k changes)
__global__ void gj_column_kernel(const double2* __restrict__ M, int64_t n, int k, double2* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = M[i * 2 * n + k];
}

// M[i][j] -= f[i] M[k][j] for i != k, j in k .. 2n - 1 (one row per blockIdx.y)
__global__ void gj_eliminate_kernel(double2* __restrict__ M, int64_t n, int k, const double2* __restrict__ f) {
  const int64_t i = blockIdx.y;
  const int64_t j = k + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == k || j >= 2 * n) return;
  const double2 a = f[i];
  if (a.x == 0.0 && a.y == 0.0) return;
  const double2 b = M[(int64_t)k * 2 * n + j];
  double2* m = M + i * 2 * n + j;
  double2 v = *m;
  v.x -= a.x * b.x - a.y * b.y;
  v.y -= a.x * b.y + a.y * b.x;
  *m = v;
}

// right half of M -> column-major A^{-1} (FP64 and FP32 copies)
__global__ void gj_extract_kernel(const double2* __restrict__ M, int64_t n, double2* __restrict__ inv64,
                                  float2* __restrict__ inv32) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int64_t col = t / n, row = t - col * n;
  const double2 v = M[row * 2 * n + n + col];
  inv64[t] = v;
  inv32[t] = make_float2((float)v.x, (float)v.y);
}

void dense_coarsest_inverse(const double2* links, const Geom& g, int ns, double2* M, double2* f, int* piv,
                            double2* pinv, int* status, double2* inv64, float2* inv32, hipStream_t st) {
  const int64_t n = g.V * ns;
  gj_init_kernel<<<(unsigned)((2 * n * n + 255) / 256), 256, 0, st>>>(M, n);
  for (int d = 0; d < 9; ++d)
    gj_assemble_kernel<<<(unsigned)((g.V * ns * ns + 255) / 256), 256, 0, st>>>(links, M, g, ns, d);
  for (int k = 0; k < n; ++k) {
    gj_pivot_kernel<<<1, 256, 0, st>>>(M, n, k, piv, pinv, status);
    const unsigned gx = (unsigned)((2 * n - k + 255) / 256);
    gj_swap_scale_kernel<<<gx, 256, 0, st>>>(M, n, k, piv, pinv);
    gj_column_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(M, n, k, f);
    gj_eliminate_kernel<<<dim3(gx, (unsigned)n), 256, 0, st>>>(M, n, k, f);
  }
  gj_extract_kernel<<<(unsigned)((n * n + 255) / 256), 256, 0, st>>>(M, n, inv64, inv32);
}

}  // namespace mg
