// Block-preconditioned coarse levels (Sec. 2.3: the block-preconditioned
// version of each coarse operator is what is coarsened; Table 1 runs levels 2
// and 3 preconditioned): A_l = X_l^{-1} P^dag A_{l-1} P, X_l(a) the
// coarse-site diagonal block.  Kernels:
//   * a batched complex GEMM (column-major, one 32 x 32 tile of C per
//     workgroup, LDS-staged 16-deep k panels), used for the Newton-Schulz
//     inverse, for the preconditioned links X^{-1} L_d and for the right-hand
//     side X^{-1} b of a level solve;
//   * the diagonal block, the Newton-Schulz start and its residual.
// X^{-1} comes from the Newton-Schulz iteration Y <- Y (2 - X Y), which only
// needs products (quadratic convergence from Y_0 = X^H / (|X|_1 |X|_inf)).
#include "kernels.hpp"

namespace mg {

template <typename T>
__global__ void __launch_bounds__(256) bgemm_kernel(const BGemmArgs<T> a) {
  using R = decltype(T{}.x);
  __shared__ T As[16][32];
  __shared__ T Bs[32][17];
  const int b = blockIdx.z;
  const T* A = a.A + (int64_t)(b / a.a_div) * a.sA;
  const T* B = a.B + (int64_t)b * a.sB;
  T* C = a.C + (int64_t)b * a.sC;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int t = threadIdx.x;
  const int ii = t & 31, jg = t >> 5;   // row of C, group of 4 columns
  T acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) { acc[c].x = 0; acc[c].y = 0; }
  for (int k0 = 0; k0 < a.k; k0 += 16) {
    for (int e = t; e < 512; e += 256) {
      const int r = e & 31, kk = e >> 5;          // A tile: 16 k x 32 rows
      T v; v.x = 0; v.y = 0;
      if (i0 + r < a.m && k0 + kk < a.k) v = A[(int64_t)(k0 + kk) * a.lda + i0 + r];
      As[kk][r] = v;
      const int kb = e & 15, jj = e >> 4;         // B tile: 32 cols x 16 k
      T w; w.x = 0; w.y = 0;
      if (j0 + jj < a.n && k0 + kb < a.k) w = B[(int64_t)(j0 + jj) * a.ldb + k0 + kb];
      Bs[jj][kb] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const T av = As[kk][ii];
#pragma unroll
      for (int c = 0; c < 4; ++c) cfma(acc[c], av, Bs[jg * 4 + c][kk]);
    }
    __syncthreads();
  }
  if (i0 + ii >= a.m) return;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = j0 + jg * 4 + c;
    if (j >= a.n) continue;
    T r;
    r.x = (R)a.alpha * acc[c].x;
    r.y = (R)a.alpha * acc[c].y;
    if (a.D) {
      const T d = a.D[(int64_t)b * a.sD + (int64_t)j * a.ldd + i0 + ii];
      r.x += (R)a.beta * d.x;
      r.y += (R)a.beta * d.y;
    }
    C[(int64_t)j * a.ldc + i0 + ii] = r;
  }
}

template <typename T>
void launch_bgemm(const BGemmArgs<T>& a, hipStream_t st) {
  if (a.m <= 0 || a.n <= 0 || a.batch <= 0) return;
  dim3 grid((unsigned)((a.m + 31) / 32), (unsigned)((a.n + 31) / 32), (unsigned)a.batch);
  bgemm_kernel<T><<<grid, 256, 0, st>>>(a);
}
template void launch_bgemm<double2>(const BGemmArgs<double2>&, hipStream_t);
template void launch_bgemm<float2>(const BGemmArgs<float2>&, hipStream_t);

// X(a) = L_0(a) + sum of the +-mu pieces whose neighbour is a itself (coarse
// extent 1 along mu); links [site][9][col][row]
__global__ void diag_block_kernel(const double2* __restrict__ L, double2* __restrict__ X, Geom g, int n) {
  const int64_t site = blockIdx.y;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const double2* Ls = L + site * 9 * nn + e;
    double2 v = Ls[0];
    for (int mu = 0; mu < 4; ++mu) {
      if (g.L[mu] != 1) continue;
      const double2 p = Ls[(1 + 2 * mu) * nn], q = Ls[(2 + 2 * mu) * nn];
      v.x += p.x + q.x;
      v.y += p.y + q.y;
    }
    X[site * nn + e] = v;
  }
}

// Y_0 = X^H / (|X|_1 |X|_inf) per site (one workgroup per site, n <= 1024)
__global__ void __launch_bounds__(256) ns_init_kernel(const double2* __restrict__ X, double2* __restrict__ Y,
                                                      int n) {
  __shared__ double red[2][256];
  const int64_t site = blockIdx.x;
  const double2* Xs = X + site * (int64_t)n * n;
  double c1 = 0.0, ci = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double cs = 0.0, rs = 0.0;
    for (int i = 0; i < n; ++i) {
      const double2 v = Xs[(int64_t)j * n + i];   // column j
      cs += hypot(v.x, v.y);
      const double2 w = Xs[(int64_t)i * n + j];   // row j
      rs += hypot(w.x, w.y);
    }
    c1 = fmax(c1, cs);
    ci = fmax(ci, rs);
  }
  red[0][threadIdx.x] = c1;
  red[1][threadIdx.x] = ci;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + o]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + o]);
    }
    __syncthreads();
  }
  const double s = red[0][0] * red[1][0];
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  double2* Ys = Y + site * (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double2 v = Xs[(int64_t)i * n + j];     // X(j, i)
    Ys[e] = make_double2(v.x * inv, -v.y * inv);  // Y(i, j) = conj X(j, i) / s
  }
}

// max over sites and entries of |T - 1| (T = X Y), as the bits of a
// non-negative double (atomicMax on the integer order)
__global__ void ns_residual_kernel(const double2* __restrict__ T, int64_t nsite, int n,
                                   unsigned long long* out) {
  const int64_t nn = (int64_t)n * n;
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nsite * nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e % nn;
    const int i = (int)(q % n), j = (int)(q / n);
    const double2 v = T[e];
    m = fmax(m, fmax(fabs(v.x - (i == j ? 1.0 : 0.0)), fabs(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// self block d = 0 of every site set to the identity (links [site][9][n][n])
__global__ void unit_self_kernel(double2* __restrict__ L, int n) {
  const int64_t site = blockIdx.y;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x)
    L[site * 9 * nn + e] = make_double2((e % n) == (e / n) ? 1.0 : 0.0, 0.0);
}
void launch_unit_self(double2* L, const Geom& g, int n, hipStream_t st) {
  const int64_t nn = (int64_t)n * n;
  dim3 grid((unsigned)((nn + 255) / 256), (unsigned)g.V);
  unit_self_kernel<<<grid, 256, 0, st>>>(L, n);
}

void launch_diag_block(const double2* L, double2* X, const Geom& g, int n, hipStream_t st) {
  const int64_t nn = (int64_t)n * n;
  dim3 grid((unsigned)((nn + 255) / 256), (unsigned)g.V);
  diag_block_kernel<<<grid, 256, 0, st>>>(L, X, g, n);
}
void launch_ns_init(const double2* X, double2* Y, int64_t nsite, int n, hipStream_t st) {
  ns_init_kernel<<<(unsigned)nsite, 256, 0, st>>>(X, Y, n);
}
void launch_ns_residual(const double2* T, int64_t nsite, int n, unsigned long long* out, hipStream_t st) {
  ns_residual_kernel<<<480, 256, 0, st>>>(T, nsite, n, out);
}

}  // namespace mg
