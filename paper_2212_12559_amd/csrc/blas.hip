// Krylov BLAS for the GCR / CA-GCR / CG drivers.  Vectors are batches of
// nrhs independent systems, [nrhs][n] complex; every scalar lives on the
// device as one double2 per (slot, rhs), so the drivers never wait on the host
// except for their convergence tests.  All reductions accumulate in FP64 and
// combine their per-block partial sums in a fixed order (bit-reproducible).
#include <algorithm>
#include <stdexcept>

#include "kernels.hpp"

namespace mg {

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Elements e and e + 1 (e even) of a vector: one 16-byte access for FP32
// complex (vectors and per-system offsets are even and 16-byte aligned).
__device__ __forceinline__ void ld2(const float2* p, int64_t e, double2& a, double2& b) {
  const float4 v = *reinterpret_cast<const float4*>(p + e);
  a = make_double2(v.x, v.y);
  b = make_double2(v.z, v.w);
}
__device__ __forceinline__ void ld2(const double2* p, int64_t e, double2& a, double2& b) {
  a = p[e];
  b = p[e + 1];
}
__device__ __forceinline__ void st2(float2* p, int64_t e, double2 a, double2 b) {
  *reinterpret_cast<float4*>(p + e) = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
}
__device__ __forceinline__ void st2(double2* p, int64_t e, double2 a, double2 b) {
  p[e] = a;
  p[e + 1] = b;
}

// partial sums of <x_p, y_p> (conjugate on x) for p < np
template <typename T, int MAXP>
__global__ void __launch_bounds__(256) pairdot_kernel(const PairDotArgs<T> a, double2* __restrict__ part,
                                                      int nblk) {
  __shared__ double2 red[4][MAXP];
  const int r = blockIdx.y;
  const int64_t off = (int64_t)r * a.stride;
  double2 acc[MAXP];
#pragma unroll
  for (int p = 0; p < MAXP; ++p) acc[p] = make_double2(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < a.n; e += (int64_t)nblk * 256) {
#pragma unroll
    for (int p = 0; p < MAXP; ++p) {
      if (p < a.np) {
        const double2 x = to_d2(a.x[p][off + e]);
        const double2 y = to_d2(a.y[p][off + e]);
        cfmac(acc[p], x, y);
      }
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int p = 0; p < MAXP; ++p) {
    if (p < a.np) {
      const double sx = wsum(acc[p].x), sy = wsum(acc[p].y);
      if (lane == 0) red[wave][p] = make_double2(sx, sy);
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < a.np; p += 256) {
    double2 s = red[0][p];
    for (int w = 1; w < 4; ++w) { s.x += red[w][p].x; s.y += red[w][p].y; }
    part[((int64_t)p * a.nrhs + r) * nblk + blockIdx.x] = s;
  }
}

// res[p][r] = sum of the nblk partials of product p, system r: one
// wavefront per (p, r), lanes over the partials, then a shuffle tree (a fixed
// order for a given nblk)
__global__ void __launch_bounds__(256) finalize_kernel(const double2* __restrict__ part, int nblk, int np, int nrhs,
                                                       double2* __restrict__ res, int ldr) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= (int64_t)np * nrhs) return;
  const int lane = threadIdx.x & 63;
  const int p = (int)(q / nrhs), r = (int)(q - (int64_t)p * nrhs);
  const double2* s = part + ((int64_t)p * nrhs + r) * nblk;
  double2 acc = make_double2(0.0, 0.0);
  for (int b = lane; b < nblk; b += 64) { acc.x += s[b].x; acc.y += s[b].y; }
  const double sx = wsum(acc.x), sy = wsum(acc.y);
  if (lane == 0) res[(int64_t)p * ldr + r] = make_double2(sx, sy);
}
static void launch_finalize(const double2* part, int nblk, int np, int nrhs, double2* res, int ldr, hipStream_t st) {
  const int64_t nq = (int64_t)np * nrhs;
  finalize_kernel<<<(unsigned)((nq + 3) / 4), 256, 0, st>>>(part, nblk, np, nrhs, res, ldr);
}

int reduce_blocks(int64_t n) {
  int64_t b = (n + 511) / 512;
  if (b < 1) b = 1;
  if (b > 480) b = 480;
  return (int)b;
}

template <typename T>
void launch_pairdot(const PairDotArgs<T>& a, double2* part, double2* res, int ldr, hipStream_t st) {
  const int nblk = reduce_blocks(a.n);
  dim3 grid(nblk, a.nrhs);
  if (a.np <= 4) pairdot_kernel<T, 4><<<grid, 256, 0, st>>>(a, part, nblk);
  else if (a.np <= 18) pairdot_kernel<T, 18><<<grid, 256, 0, st>>>(a, part, nblk);
  else pairdot_kernel<T, kMaxPairs><<<grid, 256, 0, st>>>(a, part, nblk);
  launch_finalize(part, nblk, a.np, a.nrhs, res, ldr, st);
}
template void launch_pairdot<float2>(const PairDotArgs<float2>&, double2*, double2*, int, hipStream_t);
template void launch_pairdot<double2>(const PairDotArgs<double2>&, double2*, double2*, int, hipStream_t);

// out = sum_t coef_t(r) v_t  (out may alias one of the v_t); MAXT bounds the
// term count (registers), TWO adds the second output over v2.  A thread
// handles element pairs (n is even).
template <typename T, int MAXT, bool TWO>
__global__ void __launch_bounds__(256) lincomb_kernel(const LinCombArgs<T> a) {
  const int r = blockIdx.y;
  const int64_t off = (int64_t)r * a.stride;
  double2 cf[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    cf[t] = make_double2(0.0, 0.0);
    if (t < a.nt) {
      double2 c = a.c[t] ? a.c[t][r] : a.cconst[t];
      if (a.conj[t]) c.y = -c.y;
      if (a.neg[t]) { c.x = -c.x; c.y = -c.y; }
      if (a.mask && a.mask[r] == 0 && a.masked[t]) { c.x = 0.0; c.y = 0.0; }
      cf[t] = c;
    }
  }
  const int64_t npair = a.n / 2;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < npair; q += (int64_t)gridDim.x * 256) {
    const int64_t e = off + 2 * q;
    double2 acc0 = make_double2(0.0, 0.0), acc1 = acc0, bcc0 = acc0, bcc1 = acc0;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < a.nt) {
        double2 v0, v1;
        ld2(a.v[t], e, v0, v1);
        cfma(acc0, cf[t], v0);
        cfma(acc1, cf[t], v1);
        if (TWO) {
          ld2(a.v2[t], e, v0, v1);
          cfma(bcc0, cf[t], v0);
          cfma(bcc1, cf[t], v1);
        }
      }
    }
    st2(a.out, e, acc0, acc1);
    if (TWO) st2(a.out2, e, bcc0, bcc1);
  }
}

template <typename T, int MAXT>
static void lincomb_launch(const LinCombArgs<T>& a, dim3 grid, hipStream_t st) {
  if (a.out2) lincomb_kernel<T, MAXT, true><<<grid, 256, 0, st>>>(a);
  else lincomb_kernel<T, MAXT, false><<<grid, 256, 0, st>>>(a);
}

template <typename T>
void launch_lincomb(const LinCombArgs<T>& a, hipStream_t st) {
  if (a.n % 2 || a.stride % 2) throw std::runtime_error("lincomb: vector lengths must be even");
  int64_t b = (a.n / 2 + 255) / 256;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  dim3 grid((unsigned)b, a.nrhs);
  if (a.nt <= 4) lincomb_launch<T, 4>(a, grid, st);
  else if (a.nt <= 10) lincomb_launch<T, 10>(a, grid, st);
  else lincomb_launch<T, kMaxTerms>(a, grid, st);
}
template void launch_lincomb<float2>(const LinCombArgs<float2>&, hipStream_t);
template void launch_lincomb<double2>(const LinCombArgs<double2>&, hipStream_t);

template <typename TI, typename TO>
__global__ void convert_kernel(TO* __restrict__ out, const TI* __restrict__ in, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = from_d2<TO>(to_d2(in[i]));
}
template <typename TI, typename TO>
void launch_convert(TO* out, const TI* in, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  convert_kernel<TI, TO><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, in, n);
}
template void launch_convert<double2, float2>(float2*, const double2*, int64_t, hipStream_t);
template void launch_convert<float2, double2>(double2*, const float2*, int64_t, hipStream_t);
template void launch_convert<double2, double2>(double2*, const double2*, int64_t, hipStream_t);
template void launch_convert<float2, float2>(float2*, const float2*, int64_t, hipStream_t);

// GCR update after orthogonalisation, one pass over the four vectors:
//   x += alpha z, r -= alpha q, q *= inv, z *= inv, and partial sums of |r|^2
template <typename T>
__global__ void __launch_bounds__(256) gcr_update_kernel(T* __restrict__ x, T* __restrict__ r, T* __restrict__ q,
                                                         T* __restrict__ z, const double2* __restrict__ alpha,
                                                         const double2* __restrict__ inv, int64_t n,
                                                         double2* __restrict__ part, int nblk, int nrhs) {
  __shared__ double red[4];
  const int rr = blockIdx.y;
  const int64_t off = (int64_t)rr * n;
  const double2 al = alpha[rr];
  const double iv = inv[rr].x;
  double s = 0.0;
  for (int64_t e = off + (int64_t)blockIdx.x * 256 + threadIdx.x; e < off + n; e += (int64_t)nblk * 256) {
    const double2 zv = to_d2(z[e]), qv = to_d2(q[e]);
    double2 xv = to_d2(x[e]), rv = to_d2(r[e]);
    cfma(xv, al, zv);
    cfma(rv, make_double2(-al.x, -al.y), qv);
    const T rt = from_d2<T>(rv);
    x[e] = from_d2<T>(xv);
    r[e] = rt;
    q[e] = from_d2<T>(make_double2(qv.x * iv, qv.y * iv));
    z[e] = from_d2<T>(make_double2(zv.x * iv, zv.y * iv));
    const double2 rs = to_d2(rt);
    s += rs.x * rs.x + rs.y * rs.y;
  }
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)rr * nblk + blockIdx.x] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
}
template <typename T>
void launch_gcr_update(T* x, T* r, T* q, T* z, const double2* alpha, const double2* inv, int64_t n, int nrhs,
                       double2* part, double2* res, int ldr, hipStream_t st) {
  const int nblk = reduce_blocks(n);
  dim3 grid(nblk, nrhs);
  gcr_update_kernel<T><<<grid, 256, 0, st>>>(x, r, q, z, alpha, inv, n, part, nblk, nrhs);
  launch_finalize(part, nblk, 1, nrhs, res, ldr, st);
}
template void launch_gcr_update<float2>(float2*, float2*, float2*, float2*, const double2*, const double2*, int64_t,
                                        int, double2*, double2*, int, hipStream_t);
template void launch_gcr_update<double2>(double2*, double2*, double2*, double2*, const double2*, const double2*,
                                         int64_t, int, double2*, double2*, int, hipStream_t);

// CG update in one pass: x += alpha p (x may be null), r -= alpha Ap, partial sums of |r|^2
__global__ void __launch_bounds__(256) cg_update_kernel(double2* __restrict__ x, double2* __restrict__ r,
                                                       const double2* __restrict__ p, const double2* __restrict__ ap,
                                                       const double2* __restrict__ alpha, int64_t n,
                                                       double2* __restrict__ part, int nblk) {
  __shared__ double red[4];
  const int rr = blockIdx.y;
  const int64_t off = (int64_t)rr * n;
  const double al = alpha[rr].x;
  double s = 0.0;
  for (int64_t e = off + (int64_t)blockIdx.x * 256 + threadIdx.x; e < off + n; e += (int64_t)nblk * 256) {
    const double2 av = ap[e];
    if (x) {
      const double2 pv = p[e];
      double2 xv = x[e];
      xv.x = fma(al, pv.x, xv.x);
      xv.y = fma(al, pv.y, xv.y);
      x[e] = xv;
    }
    double2 rv = r[e];
    rv.x = fma(-al, av.x, rv.x);
    rv.y = fma(-al, av.y, rv.y);
    r[e] = rv;
    s += rv.x * rv.x + rv.y * rv.y;
  }
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)rr * nblk + blockIdx.x] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
}
void launch_cg_update(double2* x, double2* r, const double2* p, const double2* ap, const double2* alpha, int64_t n,
                      int nrhs, double2* part, double2* res, int ldr, hipStream_t st) {
  const int nblk = reduce_blocks(n);
  dim3 grid(nblk, nrhs);
  cg_update_kernel<<<grid, 256, 0, st>>>(x, r, p, ap, alpha, n, part, nblk);
  launch_finalize(part, nblk, 1, nrhs, res, ldr, st);
}

// ------------------------------------------------------------ CA-GCR Gram
// The smoother's Gram data in one pass over its s + 1 vectors (u_i = A p_i
// for i < s, u_s = t): G(i, j) = <u_i, u_j> for i <= j < s, then
// c_i = <u_i, t>, in the slot order of the Cholesky solve.  A block stages
// 256 elements of every vector in LDS (each element fetched once); its four
// wavefronts then take the pairs of the largest basis round-robin, so each
// holds at most 11 FP64 accumulators.
__device__ __forceinline__ void ldraw(const float2* p, int64_t e, float2& a, float2& b) {
  const float4 v = *reinterpret_cast<const float4*>(p + e);
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void ldraw(const double2* p, int64_t e, double2& a, double2& b) {
  a = p[e];
  b = p[e + 1];
}

template <typename T, int S, int NW>
__global__ void __launch_bounds__(64 * NW) gram_kernel(const GramArgs<T> a, double2* __restrict__ part, int nblk) {
  constexpr int NPF = S * (S + 1) / 2 + S;
  constexpr int PW = (NPF + NW - 1) / NW;
  __shared__ T us[S + 1][256];
  const int r = blockIdx.y;
  const int64_t off = (int64_t)r * a.stride;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int s = a.s;
  double2 acc[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q) acc[q] = make_double2(0.0, 0.0);
  // the loads of the next pass are issued before the products of this one
  T pa[S + 1], pb[S + 1];
  auto fetch = [&](int64_t e0) {
    if (threadIdx.x < 128) {   // element pairs, one 16-byte load each for FP32
      const int64_t e = e0 + 2 * threadIdx.x;
#pragma unroll
      for (int i = 0; i <= S; ++i) {
        const int src = i < S ? i : s;
        if ((i < s || i == S) && e < a.n) ldraw(a.u[src], off + e, pa[i], pb[i]);
        else { pa[i] = from_d2<T>(make_double2(0.0, 0.0)); pb[i] = pa[i]; }
      }
    }
  };
  const int64_t step = (int64_t)nblk * 256;
  if ((int64_t)blockIdx.x * 256 < a.n) fetch((int64_t)blockIdx.x * 256);
  for (int64_t e0 = (int64_t)blockIdx.x * 256; e0 < a.n; e0 += step) {
    __syncthreads();
    if (threadIdx.x < 128) {
      const int el = 2 * threadIdx.x;
#pragma unroll
      for (int i = 0; i <= S; ++i) {
        us[i][el] = pa[i];
        us[i][el + 1] = pb[i];
      }
    }
    __syncthreads();
    if (e0 + step < a.n) fetch(e0 + step);
#pragma unroll 1
    for (int q4 = 0; q4 < 4; ++q4) {
      const int el = lane + 64 * q4;
      double2 v[S + 1];
#pragma unroll
      for (int i = 0; i <= S; ++i) v[i] = (i < s || i == S) ? to_d2(us[i][el]) : make_double2(0.0, 0.0);
      int f = 0;
#pragma unroll
      for (int i = 0; i < S; ++i) {
#pragma unroll
        for (int j = i; j <= S; ++j) {
          if ((f % NW) == wave && i < s && (j < s || j == S)) cfmac(acc[f / NW], v[i], v[j]);
          ++f;
        }
      }
    }
  }
  int f = 0;
#pragma unroll
  for (int i = 0; i < S; ++i) {
#pragma unroll
    for (int j = i; j <= S; ++j) {
      if ((f % NW) == wave && i < s && (j < s || j == S)) {
        const double sx = wsum(acc[f / NW].x), sy = wsum(acc[f / NW].y);
        const int p = j < S ? i * s - i * (i - 1) / 2 + (j - i) : s * (s + 1) / 2 + i;
        if (lane == 0) part[((int64_t)p * a.nrhs + r) * nblk + blockIdx.x] = make_double2(sx, sy);
      }
      ++f;
    }
  }
}

// Gram data of a CA-GCR(s) cycle with s up to 16 (the coarsest solver): the
// same products and output order as gram_kernel, 16 wavefronts each owning
// ten of the 152 products (pair indices in registers, operands read from
// the LDS stage), so no per-element register copy of all 17 vectors.
template <typename T>
__global__ void __launch_bounds__(1024) gram16_kernel(const GramArgs<T> a, double2* __restrict__ part, int nblk) {
  constexpr int S = kMaxCA, NW = 16;
  constexpr int NPF = S * (S + 1) / 2 + S;
  constexpr int PW = (NPF + NW - 1) / NW;
  __shared__ T us[S + 1][256];
  const int r = blockIdx.y;
  const int64_t off = (int64_t)r * a.stride;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int s = a.s;
  int pi[PW], pj[PW], po[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q) { pi[q] = -1; pj[q] = 0; po[q] = 0; }
  {
    int f = 0;
    for (int i = 0; i < S; ++i)
      for (int j = i; j <= S; ++j, ++f) {
        if (f % NW != wave || !(i < s && (j < s || j == S))) continue;
        const int q = f / NW;
#pragma unroll
        for (int qq = 0; qq < PW; ++qq)
          if (qq == q) {
            pi[qq] = i;
            pj[qq] = j;
            po[qq] = j < S ? i * s - i * (i - 1) / 2 + (j - i) : s * (s + 1) / 2 + i;
          }
      }
  }
  double2 acc[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q) acc[q] = make_double2(0.0, 0.0);
  const int64_t step = (int64_t)nblk * 256;
  for (int64_t e0 = (int64_t)blockIdx.x * 256; e0 < a.n; e0 += step) {
    __syncthreads();
    // every thread stages: (vector, element pair) pieces, 16 bytes each for FP32
    for (int q = threadIdx.x; q < (S + 1) * 128; q += 64 * NW) {
      const int i = q >> 7, el = 2 * (q & 127);
      const int64_t e = e0 + el;
      const int src = i < S ? i : s;
      T va = from_d2<T>(make_double2(0.0, 0.0)), vb = va;
      if ((i < s || i == S) && e < a.n) ldraw(a.u[src], off + e, va, vb);
      us[i][el] = va;
      us[i][el + 1] = vb;
    }
    __syncthreads();
#pragma unroll 1
    for (int q4 = 0; q4 < 4; ++q4) {
      const int el = lane + 64 * q4;
#pragma unroll
      for (int q = 0; q < PW; ++q)
        if (pi[q] >= 0) cfmac(acc[q], to_d2(us[pi[q]][el]), to_d2(us[pj[q]][el]));
    }
  }
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    if (pi[q] < 0) continue;
    const double sx = wsum(acc[q].x), sy = wsum(acc[q].y);
    if (lane == 0) part[((int64_t)po[q] * a.nrhs + r) * nblk + blockIdx.x] = make_double2(sx, sy);
  }
}

template <typename T>
void launch_gram(const GramArgs<T>& a, double2* part, double2* res, int ldr, hipStream_t st) {
  if (a.n % 2 || a.stride % 2) throw std::runtime_error("gram: vector lengths must be even");
  const int nblk = reduce_blocks(a.n);
  if (a.s <= kMaxS) gram_kernel<T, kMaxS, 4><<<dim3(nblk, a.nrhs), 256, 0, st>>>(a, part, nblk);
  else if (a.s <= kMaxCA) gram16_kernel<T><<<dim3(nblk, a.nrhs), 1024, 0, st>>>(a, part, nblk);
  else throw std::runtime_error("gram: at most 16 basis vectors");
  launch_finalize(part, nblk, a.s * (a.s + 1) / 2 + a.s, a.nrhs, res, ldr, st);
}
template void launch_gram<float2>(const GramArgs<float2>&, double2*, double2*, int, hipStream_t);
template void launch_gram<double2>(const GramArgs<double2>&, double2*, double2*, int, hipStream_t);

// Coefficients of the deferred solution update x += sum_k gamma_k z_k: the
// raw directions satisfy z_k = g_k zt_k + sum_{i<k} beta(i, k) zt_i with
// A zt_k the normalised q_k, so gamma solves the upper-triangular system
// U gamma = alpha' (U(i, k) = beta(i, k), U(k, k) = g_k) by back substitution.
__global__ void gcr_backsub_kernel(double2* tri, int nk, int nrhs, int ld) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double2 gm[kMaxNK];
  for (int i = nk - 1; i >= 0; --i) {
    double2 v = tri[(int64_t)(kTriA + i) * ld + r];
    for (int k = i + 1; k < nk; ++k) {   // v -= beta(i, k) gamma_k
      const double2 b = tri[(int64_t)(i * kMaxNK + k) * ld + r];
      v.x -= b.x * gm[k].x - b.y * gm[k].y;
      v.y -= b.x * gm[k].y + b.y * gm[k].x;
    }
    const double g = tri[(int64_t)(kTriG + i) * ld + r].x;
    gm[i] = make_double2(v.x / g, v.y / g);
    tri[(int64_t)(kTriC + i) * ld + r] = gm[i];
  }
}
void launch_gcr_backsub(double2* tri, int nk, int nrhs, int ld, hipStream_t st) {
  if (nk <= 0) return;
  gcr_backsub_kernel<<<(nrhs + 63) / 64, 64, 0, st>>>(tri, nk, nrhs, ld);
}

// ------------------------------------------- single-reduction GCR direction
// Pass 1: <q_i, q_k>, <q_i, r> for i < k, |q_k|^2 and <q_k, r> (results
// p = i, k + i, 2k, 2k + 1).  A block stages CH elements of each of the k + 2
// vectors in LDS (every element fetched once); its four wavefronts take the
// 2k + 2 products round-robin, at most nine accumulators each.
template <typename T, int CH>
__global__ void __launch_bounds__(256) gcr_dots_kernel(const GcrDotArgs<T> a, double2* __restrict__ part,
                                                       int nblk) {
  constexpr int PW = (2 * kMaxNK + 2 + 3) / 4;
  __shared__ T vs[kMaxNK + 2][CH];
  const int rr = blockIdx.y;
  const int64_t off = (int64_t)rr * a.stride;
  const int k = a.k, nv = k + 2, np = 2 * k + 2;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  double2 acc[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int64_t e0 = (int64_t)blockIdx.x * CH; e0 < a.n; e0 += (int64_t)nblk * CH) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < nv * (CH / 2); idx += 256) {   // element pairs
      const int v = idx / (CH / 2), el = 2 * (idx - v * (CH / 2));
      const T* src = v < k ? a.q[v] : (v == k ? a.qk : a.r);
      const int64_t e = e0 + el;
      double2 x0 = make_double2(0.0, 0.0), x1 = x0;
      if (e < a.n) ld2(src, off + e, x0, x1);
      vs[v][el] = from_d2<T>(x0);
      vs[v][el + 1] = from_d2<T>(x1);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      const int p = wave + 4 * q;
      if (p < np) {
        const int xi = p < k ? p : (p < 2 * k ? p - k : k);
        const int yi = p < k ? k : (p < 2 * k ? k + 1 : (p == 2 * k ? k : k + 1));
        for (int el = lane; el < CH; el += 64) cfmac(acc[q], to_d2(vs[xi][el]), to_d2(vs[yi][el]));
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    const int p = wave + 4 * q;
    if (p < np) {
      const double sx = wsum(acc[q].x), sy = wsum(acc[q].y);
      if (lane == 0) part[((int64_t)p * a.nrhs + rr) * nblk + blockIdx.x] = make_double2(sx, sy);
    }
  }
}

template <typename T>
void launch_gcr_dots(const GcrDotArgs<T>& a, double2* part, double2* res, int ldr, hipStream_t st) {
  constexpr int CH = sizeof(T) == 8 ? 256 : 128;   // 36 KiB of LDS either way
  if (a.n % 2 || a.stride % 2) throw std::runtime_error("gcr_dots: vector lengths must be even");
  int64_t b = (a.n + 4 * CH - 1) / (4 * CH);
  if (b < 1) b = 1;
  if (b > 480) b = 480;
  const int nblk = (int)b;
  gcr_dots_kernel<T, CH><<<dim3(nblk, a.nrhs), 256, 0, st>>>(a, part, nblk);
  launch_finalize(part, nblk, 2 * a.k + 2, a.nrhs, res, ldr, st);
}
template void launch_gcr_dots<float2>(const GcrDotArgs<float2>&, double2*, double2*, int, hipStream_t);
template void launch_gcr_dots<double2>(const GcrDotArgs<double2>&, double2*, double2*, int, hipStream_t);

// Scalars of direction k from pass 1 (q_0..q_{k-1} orthonormal): the
// projection coefficients beta_i = <q_i, q_k>, |q'|^2 = |q_k|^2 - sum |beta_i|^2
// and <q', r> = <q_k, r> - sum conj(beta_i) <q_i, r> for q' = q_k - sum beta_i q_i.
// g_k = |q'|, alpha'_k = <q', r> / g_k, alpha = <q', r> / g_k^2, inv = 1 / g_k.
// A masked system, or a direction whose projection keeps less than 1e-10 of
// |q_k|^2 (within the rounding of the sums), contributes nothing (g_k = 1,
// alpha'_k = alpha = inv = 0).
__global__ void gcr_scalars_cgs_kernel(const double2* dots, int k, const int* mask, int nrhs, int ld, double2* tri,
                                       double2* alpha, double2* inv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double qq = dots[(int64_t)(2 * k) * ld + r].x;
  double g2 = qq;
  double2 qr = dots[(int64_t)(2 * k + 1) * ld + r];
  for (int i = 0; i < k; ++i) {
    const double2 b = dots[(int64_t)i * ld + r];
    const double2 c = dots[(int64_t)(k + i) * ld + r];
    tri[(int64_t)(i * kMaxNK + k) * ld + r] = b;
    g2 -= b.x * b.x + b.y * b.y;
    qr.x -= b.x * c.x + b.y * c.y;   // conj(b) c
    qr.y -= b.x * c.y - b.y * c.x;
  }
  const bool on = (mask == nullptr || mask[r] != 0) && qq > 0.0 && qq < 1e300 && g2 > 1e-10 * qq;
  const double g = on ? sqrt(g2) : 1.0;
  tri[(int64_t)(kTriG + k) * ld + r] = make_double2(g, 0.0);
  tri[(int64_t)(kTriA + k) * ld + r] = on ? make_double2(qr.x / g, qr.y / g) : make_double2(0.0, 0.0);
  alpha[r] = on ? make_double2(qr.x / g2, qr.y / g2) : make_double2(0.0, 0.0);
  inv[r] = make_double2(on ? 1.0 / g : 0.0, 0.0);
}
void launch_gcr_scalars_cgs(const double2* dots, int k, const int* mask, int nrhs, int ld, double2* tri,
                            double2* alpha, double2* inv, hipStream_t st) {
  gcr_scalars_cgs_kernel<<<(nrhs + 63) / 64, 64, 0, st>>>(dots, k, mask, nrhs, ld, tri, alpha, inv);
}

// Pass 2: q' = q_k - sum_i beta_i q_i, r -= alpha q', q_k <- inv q', the new r
// optionally copied to znext, and partial sums of |r|^2
template <typename T, int MAXV>
__global__ void __launch_bounds__(256) gcr_update_cgs_kernel(const GcrUpdArgs<T> a, double2* __restrict__ part,
                                                             int nblk) {
  __shared__ double red[4];
  const int rr = blockIdx.y;
  const int64_t off = (int64_t)rr * a.stride;
  double2 b[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) b[i] = i < a.k ? a.beta[i][rr] : make_double2(0.0, 0.0);
  const double2 al = a.alpha[rr];
  const double iv = a.inv[rr].x;
  double s = 0.0;
  const int64_t npair = a.n / 2;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < npair; q += (int64_t)nblk * 256) {
    const int64_t e = off + 2 * q;
    double2 qv[2], rv[2], x[2];
    ld2(a.qk, e, qv[0], qv[1]);
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
      if (i < a.k) {
        ld2(a.q[i], e, x[0], x[1]);
        cfma(qv[0], make_double2(-b[i].x, -b[i].y), x[0]);
        cfma(qv[1], make_double2(-b[i].x, -b[i].y), x[1]);
      }
    }
    ld2(a.r, e, rv[0], rv[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      cfma(rv[h], make_double2(-al.x, -al.y), qv[h]);
      rv[h] = to_d2(from_d2<T>(rv[h]));   // the stored value
      s += rv[h].x * rv[h].x + rv[h].y * rv[h].y;
    }
    st2(a.r, e, rv[0], rv[1]);
    if (a.znext) st2(a.znext, e, rv[0], rv[1]);
    st2(a.qk, e, make_double2(qv[0].x * iv, qv[0].y * iv), make_double2(qv[1].x * iv, qv[1].y * iv));
  }
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)rr * nblk + blockIdx.x] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
}

template <typename T>
void launch_gcr_update_cgs(const GcrUpdArgs<T>& a, double2* part, double2* res, int ldr, hipStream_t st) {
  if (a.n % 2 || a.stride % 2) throw std::runtime_error("gcr_update: vector lengths must be even");
  const int nblk = reduce_blocks(a.n / 2);
  dim3 grid(nblk, a.nrhs);
  if (a.k <= 4) gcr_update_cgs_kernel<T, 4><<<grid, 256, 0, st>>>(a, part, nblk);
  else gcr_update_cgs_kernel<T, kMaxNK><<<grid, 256, 0, st>>>(a, part, nblk);
  launch_finalize(part, nblk, 1, a.nrhs, res, ldr, st);
}
template void launch_gcr_update_cgs<float2>(const GcrUpdArgs<float2>&, double2*, double2*, int, hipStream_t);
template void launch_gcr_update_cgs<double2>(const GcrUpdArgs<double2>&, double2*, double2*, int, hipStream_t);

// Convergence on the device: mask[r] stays 1 while |r|^2 > tol^2 |r0|^2
// (and both are finite); init sets mask from |r0|^2 > 0.
__global__ void conv_kernel(int* mask, const double2* rn2, const double2* r0sq, double tol2, int nrhs, int init) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double a = rn2[r].x, b = r0sq[r].x;
  if (init) mask[r] = (b > 0.0 && b < 1e300) ? 1 : 0;
  else if (mask[r]) mask[r] = (a > tol2 * b && a < 1e300) ? 1 : 0;
}
void launch_conv(int* mask, const double2* rn2, const double2* r0sq, double tol2, int nrhs, int init,
                 hipStream_t st) {
  conv_kernel<<<(nrhs + 63) / 64, 64, 0, st>>>(mask, rn2, r0sq, tol2, nrhs, init);
}

// A power of two brings each system's right-hand side to entries of order
// one: exact in every format with the range, and it keeps the inputs of the
// 16-bit coarse stencil clear of FP16's subnormal range however far the
// outer residual has fallen.
__global__ void rhs_scale_kernel(double2* r0sq, double2* fwd, double2* inv, int64_t n, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double b2 = r0sq[r].x;
  int e = 0;
  if (b2 > 0.0 && b2 < 1e300) e = (int)rint(0.5 * log2(b2 / (double)n));
  fwd[r] = make_double2(ldexp(1.0, -e), 0.0);
  inv[r] = make_double2(ldexp(1.0, e), 0.0);
  r0sq[r].x = ldexp(b2, -2 * e);
}
void launch_rhs_scale(double2* r0sq, double2* fwd, double2* inv, int64_t n, int nrhs, hipStream_t st) {
  rhs_scale_kernel<<<(nrhs + 63) / 64, 64, 0, st>>>(r0sq, fwd, inv, n, nrhs);
}

// ---------------------------------------------------------------- scalars
// GCR: after orthogonalisation, qq = <q, q>, qr = <q, r>.
//   alpha = qr / qq (0 for masked systems), inv = 1 / sqrt(qq)
// out slots: alpha, -alpha, inv
__global__ void gcr_scalars_kernel(const double2* qq, const double2* qr, const int* mask, int nrhs,
                                   double2* alpha, double2* nalpha, double2* inv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double q = qq[r].x;
  const bool on = (mask == nullptr || mask[r] != 0) && q > 0.0;
  double2 al = on ? make_double2(qr[r].x / q, qr[r].y / q) : make_double2(0.0, 0.0);
  alpha[r] = al;
  nalpha[r] = make_double2(-al.x, -al.y);
  inv[r] = make_double2(q > 0.0 ? 1.0 / sqrt(q) : 0.0, 0.0);
}
void launch_gcr_scalars(const double2* qq, const double2* qr, const int* mask, int nrhs, double2* alpha,
                        double2* nalpha, double2* inv, hipStream_t st) {
  gcr_scalars_kernel<<<(nrhs + 63) / 64, 64, 0, st>>>(qq, qr, mask, nrhs, alpha, nalpha, inv);
}

// CA-GCR: solve the s x s normal equations G a = c per system by Cholesky
// (FP64).  G[i][j] = <q_i, q_j> given for i <= j in slot order
// (0,0),(0,1)..(0,s-1),(1,1),...; c_i = <q_i, r> in slots after them.
// A pivot below 1e-13 of the largest diagonal truncates the basis there.
// One wavefront per system with G in LDS: lane i owns row i, so each column
// of the factor, and each step of the two triangular solves, is one parallel
// update (a thread-per-system version kept G in scratch memory and took
// 0.23 ms per launch at s = 16).
template <int S>
__global__ void __launch_bounds__(64) cagcr_solve_kernel(const double2* gram, int s, int nrhs, int ldr,
                                                         const int* mask, double2* coef) {
  __shared__ double2 G[S][S + 1];
  __shared__ double2 c[S];
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  const int np = s * (s + 1) / 2;
  for (int p = lane; p < np + s; p += 64) {
    const double2 g = gram[(int64_t)p * ldr + r];
    if (p < np) {   // packed upper triangle: row i starts at i s - i (i - 1) / 2
      int i = 0, off = 0;
      while (off + (s - i) <= p) { off += s - i; ++i; }
      const int j = i + (p - off);
      G[i][j] = g;
      G[j][i] = make_double2(g.x, -g.y);
    } else {
      c[p - np] = g;
    }
  }
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < s; ++i) dmax = fmax(dmax, G[i][i].x);
  int k = s;   // the same on every lane
  // Cholesky G = L L^dag, L in G's lower triangle
  for (int j = 0; j < s; ++j) {
    double d = G[j][j].x;
    for (int q = 0; q < j; ++q) d -= G[j][q].x * G[j][q].x + G[j][q].y * G[j][q].y;
    if (!(d > 1e-13 * dmax)) { k = j; break; }
    const double ljj = sqrt(d);
    if (lane > j && lane < s) {
      double2 v = G[lane][j];
      for (int q = 0; q < j; ++q) {   // v -= L[i][q] conj(L[j][q])
        const double2 a = G[lane][q], b = G[j][q];
        v.x -= a.x * b.x + a.y * b.y;
        v.y -= a.y * b.x - a.x * b.y;
      }
      G[lane][j] = make_double2(v.x / ljj, v.y / ljj);
    }
    __syncthreads();   // column j complete; everyone has read G[j][j]
    if (lane == 0) G[j][j] = make_double2(ljj, 0.0);
    __syncthreads();
  }
  // L y = c, column by column (y overwrites c)
  for (int i = 0; i < k; ++i) {
    const double li = G[i][i].x;
    const double2 yi = make_double2(c[i].x / li, c[i].y / li);
    __syncthreads();
    if (lane == i) c[i] = yi;
    if (lane > i && lane < k) {
      const double2 a = G[lane][i];
      c[lane].x -= a.x * yi.x - a.y * yi.y;
      c[lane].y -= a.x * yi.y + a.y * yi.x;
    }
    __syncthreads();
  }
  // L^dag a = y: once a_i is known, rows q < i drop conj(L[i][q]) a_i
  for (int i = k - 1; i >= 0; --i) {
    const double li = G[i][i].x;
    const double2 ai = make_double2(c[i].x / li, c[i].y / li);
    __syncthreads();
    if (lane == i) c[i] = ai;
    if (lane < i) {
      const double2 a = G[i][lane];
      c[lane].x -= a.x * ai.x + a.y * ai.y;
      c[lane].y -= a.x * ai.y - a.y * ai.x;
    }
    __syncthreads();
  }
  const bool on = mask == nullptr || mask[r] != 0;
  if (lane < s) coef[(int64_t)lane * ldr + r] = (on && lane < k) ? c[lane] : make_double2(0.0, 0.0);
}
void launch_cagcr_solve(const double2* gram, int s, int nrhs, int ldr, const int* mask, double2* coef,
                        hipStream_t st) {
  if (nrhs <= 0) return;
  if (s <= kMaxS) cagcr_solve_kernel<kMaxS><<<nrhs, 64, 0, st>>>(gram, s, nrhs, ldr, mask, coef);
  else cagcr_solve_kernel<kMaxCA><<<nrhs, 64, 0, st>>>(gram, s, nrhs, ldr, mask, coef);
}

// CG scalars: alpha = rr / pAp, -alpha; beta = rr_new / rr (rr updated in place)
__global__ void cg_alpha_kernel(const double2* rr, const double2* pap, const int* mask, int nrhs, double2* alpha,
                                double2* nalpha) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const bool on = (mask == nullptr || mask[r] != 0) && pap[r].x > 0.0;
  const double a = on ? rr[r].x / pap[r].x : 0.0;
  alpha[r] = make_double2(a, 0.0);
  nalpha[r] = make_double2(-a, 0.0);
}
__global__ void cg_beta_kernel(double2* rr, const double2* rrnew, const int* mask, int nrhs, double2* beta) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const bool on = (mask == nullptr || mask[r] != 0) && rr[r].x > 0.0;
  beta[r] = make_double2(on ? rrnew[r].x / rr[r].x : 0.0, 0.0);
  if (on) rr[r] = rrnew[r];
}
void launch_cg_alpha(const double2* rr, const double2* pap, const int* mask, int nrhs, double2* alpha,
                     double2* nalpha, hipStream_t st) {
  cg_alpha_kernel<<<(nrhs + 63) / 64, 64, 0, st>>>(rr, pap, mask, nrhs, alpha, nalpha);
}
void launch_cg_beta(double2* rr, const double2* rrnew, const int* mask, int nrhs, double2* beta, hipStream_t st) {
  cg_beta_kernel<<<(nrhs + 63) / 64, 64, 0, st>>>(rr, rrnew, mask, nrhs, beta);
}

// ------------------------------------------------------ multi-shift CG
// Shifted systems (sigma_base + d_j + A) y_j = b share the base CG's Krylov
// space; their residuals are zeta_j r (Sec. 3.3 workflow).  One thread per
// right-hand side walks the shifts.
__global__ void msc_init_kernel(double2* st, const double2* rr, const double2* target2, int* mask, int nshift,
                                int nrhs, int ld) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  auto S = [&](int s) -> double2& { return st[(int64_t)s * ld + r]; };
  const bool on = rr[r].x > target2[r].x && rr[r].x < 1e300;
  for (int j = 0; j < nshift; ++j) {
    S(kMscPer * j + 0) = make_double2(1.0, 0.0);
    S(kMscPer * j + 1) = make_double2(1.0, 0.0);
    S(kMscPer * j + 5) = make_double2(0.0, 0.0);
    S(kMscPer * j + 6) = make_double2(on ? 1.0 : 0.0, 0.0);
    S(kMscPer * j + 7) = make_double2(0.0, 0.0);
  }
  S(kMscPer * kMaxShift + 0) = make_double2(1.0, 0.0);
  S(kMscPer * kMaxShift + 1) = make_double2(0.0, 0.0);
  mask[r] = on ? 1 : 0;
}
void launch_msc_init(double2* st, const double2* rr, const double2* target2, int* mask, int nshift, int nrhs, int ld,
                     hipStream_t st_) {
  msc_init_kernel<<<(nrhs + 63) / 64, 64, 0, st_>>>(st, rr, target2, mask, nshift, nrhs, ld);
}

// After the base step (alpha, |r'|^2): beta, then for every shift still on
// zeta'_j, alpha_j = alpha zeta'_j / zeta_j and beta_j = beta (zeta'_j /
// zeta_j)^2 (the base keeps zeta = 1).  A shift whose |zeta'_j| |r'| reaches
// the target is updated this once more and then frozen.
__global__ void msc_scalars_kernel(const MscScalArgs a) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.nrhs) return;
  auto S = [&](int s) -> double2& { return a.st[(int64_t)s * a.ld + r]; };
  if (!a.mask[r]) {
    for (int j = 0; j < a.nshift; ++j) S(kMscPer * j + 5) = make_double2(0.0, 0.0);
    return;
  }
  const double al = a.alpha[r].x, rro = a.rr[r].x, rrn = a.rrnew[r].x;
  const double be = rro > 0.0 ? rrn / rro : 0.0;
  const double ap = S(kMscPer * kMaxShift + 0).x, bp = S(kMscPer * kMaxShift + 1).x;
  const double t2 = a.target2[r].x;
  int any = 0;
  for (int j = 0; j < a.nshift; ++j) {
    // the base direction drives every shift: it steps while any shift is on
    if (j != a.base && S(kMscPer * j + 6).x == 0.0) {
      S(kMscPer * j + 5) = make_double2(0.0, 0.0);
      continue;
    }
    const double z = S(kMscPer * j + 0).x, zo = S(kMscPer * j + 1).x;
    double zn = 1.0;
    if (j != a.base) zn = z * zo * ap / (al * bp * (zo - z) + zo * ap * (1.0 + al * a.delta[j]));
    const double q = zn / z;
    S(kMscPer * j + 2) = make_double2(al * q, 0.0);
    S(kMscPer * j + 3) = make_double2(zn, 0.0);
    S(kMscPer * j + 4) = make_double2(be * q * q, 0.0);
    S(kMscPer * j + 5) = make_double2(1.0, 0.0);
    S(kMscPer * j + 7).x += 1.0;
    S(kMscPer * j + 1) = make_double2(z, 0.0);
    S(kMscPer * j + 0) = make_double2(zn, 0.0);
    const bool on = zn * zn * rrn > t2 && rrn < 1e300 && zn == zn;
    S(kMscPer * j + 6) = make_double2(on ? 1.0 : 0.0, 0.0);
    any |= on;
  }
  S(kMscPer * kMaxShift + 0) = make_double2(al, 0.0);
  S(kMscPer * kMaxShift + 1) = make_double2(be, 0.0);
  a.rr[r] = make_double2(rrn, 0.0);
  a.mask[r] = any;
}
void launch_msc_scalars(const MscScalArgs& a, hipStream_t st) {
  msc_scalars_kernel<<<(a.nrhs + 63) / 64, 64, 0, st>>>(a);
}

// x_j += alpha_j p_j, p_j = zeta'_j r + beta_j p_j for every shift flagged
// for update; r is read once per element for all shifts.
__global__ void __launch_bounds__(256) msc_update_kernel(const MscUpdArgs a) {
  const int rr = blockIdx.y;
  double ax[kMaxShift], pz[kMaxShift], pb[kMaxShift];
  bool up[kMaxShift];
#pragma unroll
  for (int j = 0; j < kMaxShift; ++j) {
    up[j] = false;
    ax[j] = pz[j] = pb[j] = 0.0;
    if (j < a.nshift) {
      const int64_t o = (int64_t)kMscPer * j * a.ld + rr;
      up[j] = a.st[o + 5 * (int64_t)a.ld].x != 0.0;
      ax[j] = a.st[o + 2 * (int64_t)a.ld].x;
      pz[j] = a.st[o + 3 * (int64_t)a.ld].x;
      pb[j] = a.st[o + 4 * (int64_t)a.ld].x;
    }
  }
  const double2* rv_ = a.r + (int64_t)rr * a.r_stride;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < a.n; e += (int64_t)gridDim.x * 256) {
    const double2 rv = rv_[e];
#pragma unroll
    for (int j = 0; j < kMaxShift; ++j) {
      if (!up[j]) continue;
      double2* pp = a.p[j] + (int64_t)rr * a.p_stride + e;
      const double2 pv = *pp;
      if (ax[j] != 0.0) {
        double2* xp = a.x[j] + (int64_t)rr * a.x_stride + e;
        double2 xv = *xp;
        xv.x = fma(ax[j], pv.x, xv.x);
        xv.y = fma(ax[j], pv.y, xv.y);
        *xp = xv;
      }
      *pp = make_double2(fma(pz[j], rv.x, pb[j] * pv.x), fma(pz[j], rv.y, pb[j] * pv.y));
    }
  }
}
void launch_msc_update(const MscUpdArgs& a, hipStream_t st) {
  if (a.nshift < 1 || a.nshift > kMaxShift) throw std::runtime_error("multi-shift: 1..16 shifts");
  dim3 grid((unsigned)std::min<int64_t>((a.n + 255) / 256, 1024), (unsigned)a.nrhs);
  msc_update_kernel<<<grid, 256, 0, st>>>(a);
}

}  // namespace mg

namespace mg {

// Seeded standard complex normal numbers (E|z|^2 = 1): a splitmix64 hash of
// (seed, index) gives two uniforms, Box-Muller gives the pair.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
template <typename T>
__global__ void random_normal_kernel(T* out, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t h1 = splitmix64(seed ^ splitmix64((uint64_t)i * 2 + 1));
  const uint64_t h2 = splitmix64(h1 + 0x632BE59BD9B4E019ull);
  const double u1 = ((h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((h2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double rad = sqrt(-log(u1));          // sqrt(-2 log u1) / sqrt(2)
  const double ang = 6.283185307179586 * u2;
  out[i] = from_d2<T>(make_double2(rad * cos(ang), rad * sin(ang)));
}
template <typename T>
void launch_random_normal(T* out, int64_t n, uint64_t seed, hipStream_t st) {
  random_normal_kernel<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, n, seed);
}
template void launch_random_normal<float2>(float2*, int64_t, uint64_t, hipStream_t);
template void launch_random_normal<double2>(double2*, int64_t, uint64_t, hipStream_t);

}  // namespace mg
