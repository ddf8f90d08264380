// Transfer operators (Sec. 2.1, Sec. 2.3): near-null vectors are split by
// the chiral projectors (1 +- eps)/2, block-orthonormalised per aggregate and
// chirality (FP64), and define P and R = P^dag.
//
//   restrict  r_c[a, sigma, k] = sum_{rows of (a, sigma)} conj(P[row, k]) r[row]
//             one workgroup per (a, sigma); lanes run over k (Nvec <= 128),
//             eight wavefronts over interleaved rows, reduced in LDS.
//   prolong   e[row] = sum_k P[row, k] e_c[a, sigma, k] (optionally += e)
//             one workgroup per (a, sigma); threads over rows, P read in its
//             second, row-contiguous copy, e_c staged in LDS.
// Workgroup numbers go through xcd_block, so that the (a, +) and (a, -)
// workgroups, which read or write the same cache lines of the fine vector
// (the two parities of each row of sites), run on one XCD and share its L2.
#include "kernels.hpp"

namespace mg {

// Null vectors (canonical single-level layout, nv[k][flat]) -> P in the
// prolong layout PP[a][sigma][k][row], FP64, before orthonormalisation.
__global__ void gather_null_kernel(const double2* __restrict__ nv, int64_t nflat, double2* __restrict__ pp,
                                   Agg A) {
  const int64_t per = (int64_t)A.nvec * A.nrows;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= A.nagg * 2 * per) return;
  const int64_t as = tid / per;
  const int rem = (int)(tid - as * per);
  const int k = rem / A.nrows, row = rem - k * A.nrows;
  const int64_t a = as >> 1;
  const int sigma = (int)(as & 1);
  pp[tid] = nv[(int64_t)k * nflat + agg_row_index(A, a, sigma, row)];
}

void launch_gather_null(const double2* nv, int64_t nflat, double2* pp, const Agg& A, hipStream_t st) {
  const int64_t n = A.nagg * 2 * (int64_t)A.nvec * A.nrows;
  gather_null_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(nv, nflat, pp, A);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block orthonormalisation in place (FP64): for every (a, sigma) the columns
// of PP become the Q factor of the thin QR with positive real diag(R), by
// classical Gram-Schmidt applied twice per column.  status[0] is set to 1 when
// a column loses more than 1 - 1e-12 of its norm (numerically rank deficient).
__global__ void __launch_bounds__(256) block_orth_kernel(double2* __restrict__ pp, Agg A,
                                                         int* __restrict__ status) {
  __shared__ double2 d[128];
  __shared__ double red[4];
  const int nrows = A.nrows, nvec = A.nvec;
  double2* Q = pp + (int64_t)blockIdx.x * nvec * nrows;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int k = 0; k < nvec; ++k) {
    double2* v = Q + (int64_t)k * nrows;
    // initial norm
    double s = 0.0;
    for (int row = tid; row < nrows; row += 256) s += v[row].x * v[row].x + v[row].y * v[row].y;
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    const double n0 = sqrt(red[0] + red[1] + red[2] + red[3]);
    __syncthreads();
    for (int pass = 0; pass < 2 && k > 0; ++pass) {
      for (int j = wave; j < k; j += 4) {
        const double2* q = Q + (int64_t)j * nrows;
        double2 acc = make_double2(0.0, 0.0);
        for (int row = lane; row < nrows; row += 64) cfmac(acc, q[row], v[row]);
        acc.x = wave_sum(acc.x);
        acc.y = wave_sum(acc.y);
        if (lane == 0) d[j] = acc;
      }
      __syncthreads();
      for (int row = tid; row < nrows; row += 256) {
        double2 w = v[row];
        for (int j = 0; j < k; ++j) {
          const double2 q = Q[(int64_t)j * nrows + row];
          const double2 dj = d[j];
          w.x -= q.x * dj.x - q.y * dj.y;
          w.y -= q.x * dj.y + q.y * dj.x;
        }
        v[row] = w;
      }
      __syncthreads();
    }
    s = 0.0;
    for (int row = tid; row < nrows; row += 256) s += v[row].x * v[row].x + v[row].y * v[row].y;
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    const double n1 = sqrt(red[0] + red[1] + red[2] + red[3]);
    __syncthreads();
    if (!(n1 > 1e-12 * n0) || !(n0 > 0.0)) {
      if (tid == 0) atomicOr(status, 1);
    }
    const double inv = n1 > 0.0 ? 1.0 / n1 : 0.0;
    for (int row = tid; row < nrows; row += 256) {
      double2 w = v[row];
      v[row] = make_double2(w.x * inv, w.y * inv);
    }
    __syncthreads();
  }
}

void launch_block_orth(double2* pp, const Agg& A, int* status, hipStream_t st) {
  block_orth_kernel<<<(unsigned)(A.nagg * 2), 256, 0, st>>>(pp, A, status);
}

// PP64 -> PR64 (restrict layout), PR32, PP32
__global__ void p_layouts_kernel(const double2* __restrict__ pp64, double2* __restrict__ pr64,
                                 float2* __restrict__ pr32, float2* __restrict__ pp32, Agg A) {
  const int64_t per = (int64_t)A.nvec * A.nrows;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= A.nagg * 2 * per) return;
  const int64_t as = tid / per;
  const int rem = (int)(tid - as * per);
  const int row = rem / A.nvec, k = rem - row * A.nvec;   // restrict-layout position
  const int64_t src = as * per + (int64_t)k * A.nrows + row;
  const double2 v = pp64[src];
  pr64[tid] = v;
  if (pr32) pr32[tid] = make_float2((float)v.x, (float)v.y);
  if (pp32) pp32[src] = make_float2((float)v.x, (float)v.y);
}

void launch_p_layouts(const double2* pp64, double2* pr64, float2* pr32, float2* pp32, const Agg& A,
                      hipStream_t st) {
  const int64_t n = A.nagg * 2 * (int64_t)A.nvec * A.nrows;
  p_layouts_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(pp64, pr64, pr32, pp32, A);
}

constexpr int kRestrictWaves = 8;

template <typename R, int NR, int KPL>
__global__ void __launch_bounds__(64 * kRestrictWaves) restrict_kernel(const RestrictArgs<R> a) {
  using T = cplx<R>;
  __shared__ T red[kRestrictWaves - 1][NR][KPL * 64];
  extern __shared__ unsigned char xs_raw[];   // [NR][nrows] input values of this (a, sigma)
  T* xs = reinterpret_cast<T*>(xs_raw);
  const int64_t as = xcd_block(blockIdx.x, gridDim.x);
  const int64_t agg = as >> 1;
  const int sigma = (int)(as & 1);
  const int r0 = blockIdx.y * NR;
  const int nr = (a.nrhs - r0) < NR ? (a.nrhs - r0) : NR;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nvec = a.A.nvec, nrows = a.A.nrows;
  const T* P = a.pr + as * (int64_t)nrows * nvec;
  // gather the tile's inputs once (rows are spread over the fine lattice)
  for (int row = tid; row < nrows; row += 64 * kRestrictWaves) {
    const int64_t fi = agg_row_index(a.A, agg, sigma, row);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T v;
      v.x = 0; v.y = 0;
      if (r < nr) v = a.in[(int64_t)(r0 + r) * a.in_stride + fi];
      xs[r * nrows + row] = v;
    }
  }
  __syncthreads();
  T acc[NR][KPL];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int q = 0; q < KPL; ++q) { acc[r][q].x = 0; acc[r][q].y = 0; }
#pragma unroll 2
  for (int row = wave; row < nrows; row += kRestrictWaves) {
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int k = lane + 64 * q;
      if (k < nvec) {
        const T p = P[(int64_t)row * nvec + k];
#pragma unroll
        for (int r = 0; r < NR; ++r) cfmac(acc[r][q], p, xs[r * nrows + row]);
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < KPL; ++q) red[wave - 1][r][lane + 64 * q] = acc[r][q];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int k = lane + 64 * q;
      if (k >= nvec) continue;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r >= nr) continue;
        T v = acc[r][q];
        for (int w = 0; w < kRestrictWaves - 1; ++w) { v.x += red[w][r][k].x; v.y += red[w][r][k].y; }
        a.out[(int64_t)(r0 + r) * a.out_stride + agg * a.out_site_stride + sigma * nvec + k] = v;
      }
    }
  }
}

template <typename R, int NR, int KPL>
static void restrict_launch(const RestrictArgs<R>& a, hipStream_t st) {
  dim3 grid((unsigned)(a.A.nagg * 2), (unsigned)((a.nrhs + NR - 1) / NR));
  const size_t lds = (size_t)NR * a.A.nrows * sizeof(cplx<R>);
  restrict_kernel<R, NR, KPL><<<grid, 64 * kRestrictWaves, lds, st>>>(a);
}

// ------------------------------------------------- FP32 matrix-core transfer
// Per (aggregate, chirality) block the transfers are small complex GEMMs:
// restriction C[nvec x N] = P^dag X[nrows x N], prolongation
// Y[nrows x N] = P C[nvec x N], with N right-hand sides.  They run on
// v_mfma_f32_16x16x4f32 as four real products per step; a workgroup takes one
// block and 16 RT right-hand sides (RT = 4, or 1 for 16 or fewer), so P is
// read once per 16 RT of them.
typedef __attribute__((ext_vector_type(4))) float f32x4;
constexpr int kXferChunk = 32;    // fine rows staged per pass (restriction)

__device__ __forceinline__ void cmfma(f32x4& yr, f32x4& yi, float ar, float ai, float br, float bi) {
  yr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, yr, 0, 0, 0);
  yr = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, yr, 0, 0, 0);
  yi = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, yi, 0, 0, 0);
  yi = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, yi, 0, 0, 0);
}

// one wavefront per 16 coarse rows k; lane l: A = conj P(row 4 s + l / 16,
// k 16 kt + l % 16), B = X(row 4 s + l / 16, rhs l % 16), D rows k = 16 kt +
// 4 (l / 16) + t of rhs l % 16
template <int RT>
__global__ void __launch_bounds__(512) restrict_mfma_kernel(const RestrictArgs<float> a) {
  __shared__ float2 xs[kXferChunk][16 * RT + 1];
  // block -> ((aggregate, chirality), rhs tile), tile fastest: the tiles of a
  // block of P and the two chiralities of an aggregate (which share cache
  // lines of the fine vector) run back to back on one XCD
  const int ntile = (a.nrhs + 16 * RT - 1) / (16 * RT);
  const int64_t bl = xcd_block(blockIdx.x, gridDim.x);
  const int64_t as = bl / ntile;
  const int64_t agg = as >> 1;
  const int sigma = (int)(as & 1);
  const int r0 = (int)(bl - as * ntile) * 16 * RT;
  const int tid = threadIdx.x, kt = tid >> 6, lane = tid & 63;
  const int nthreads = blockDim.x;
  const int nvec = a.A.nvec, nrows = a.A.nrows;
  const float2* P = a.pr + as * (int64_t)nrows * nvec;
  const int kk = lane >> 4, jl = lane & 15;
  const int kcol = 16 * kt + jl;
  f32x4 yr[RT], yi[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    yr[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
    yi[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // staging: element e = tid + u nthreads of a pass is fine row
  // row0 + e % kXferChunk of rhs r0 + e / kXferChunk; nthreads is a multiple
  // of kXferChunk, so a thread's row is the same for every u and its flat
  // index is formed once per pass (the aggregate's origin once per block).
  // The gathers are unconditional (an element outside the input reads
  // element 0 and is zeroed afterwards), so a thread has kQ in flight.
  const int64_t abase = agg_base(a.A, agg);
  const int q = tid % kXferChunk, rq = tid / kXferChunk, rstep = nthreads / kXferChunk;
  const int upt = (16 * RT + rstep - 1) / rstep;
  constexpr int kQ = RT == 1 ? 2 : 8;   // gathered values a thread has in flight before it waits
  for (int row0 = 0; row0 < nrows; row0 += kXferChunk) {
    __syncthreads();
    const bool rok = row0 + q < nrows;
    const int64_t fi = rok ? abase + agg_row_rel(a.A, sigma, row0 + q) : 0;
#pragma unroll 1
    for (int u0 = 0; u0 < upt; u0 += kQ) {
      float2 v[kQ];
      bool ok[kQ];
#pragma unroll
      for (int u = 0; u < kQ; ++u) {
        const int rr = rq + (u0 + u) * rstep;
        ok[u] = u0 + u < upt && rr < 16 * RT && rok && r0 + rr < a.nrhs;
        v[u] = a.in[ok[u] ? (int64_t)(r0 + rr) * a.in_stride + fi : 0];
      }
#pragma unroll
      for (int u = 0; u < kQ; ++u) {
        const int rr = rq + (u0 + u) * rstep;
        if (u0 + u < upt && rr < 16 * RT) xs[q][rr] = ok[u] ? v[u] : make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < kXferChunk / 4; ++s) {
      const int row = row0 + 4 * s + kk;
      float2 p = make_float2(0.f, 0.f);
      if (row < nrows && kcol < nvec) p = P[(int64_t)row * nvec + kcol];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const float2 x = xs[4 * s + kk][16 * rt + jl];
        cmfma(yr[rt], yi[rt], p.x, -p.y, x.x, x.y);
      }
    }
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int r = r0 + 16 * rt + jl;
    if (r >= a.nrhs) continue;
    float2* o = a.out + (int64_t)r * a.out_stride + agg * a.out_site_stride + sigma * nvec;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = 16 * kt + 4 * kk + t;
      if (k < nvec) o[k] = make_float2(yr[rt][t], yi[rt][t]);
    }
  }
}

// eight wavefronts walk the 16-row tiles of the block; the coarse block
// C[nvec x 16 RT] sits in LDS.  The product is formed transposed,
// Y^T = C^T P^T, so that a lane's results are one fine row for four
// right-hand sides and the 16 lanes of a group store 16 consecutive rows:
// lane l: A = C(k 4 s + l / 16, rhs l % 16), B = P(row 16 mt + l % 16,
// k 4 s + l / 16), D = Y(row 16 mt + l % 16, rhs 4 (l / 16) + t).
template <int RT>
__global__ void __launch_bounds__(512) prolong_mfma_kernel(const ProlongArgs<float> a) {
  __shared__ float2 cs[128][16 * RT + 1];
  // numbered as in the restriction: both chiralities' stores merge in one L2
  const int ntile = (a.nrhs + 16 * RT - 1) / (16 * RT);
  const int64_t bl = xcd_block(blockIdx.x, gridDim.x);
  const int64_t as = bl / ntile;
  const int64_t agg = as >> 1;
  const int sigma = (int)(as & 1);
  const int r0 = (int)(bl - as * ntile) * 16 * RT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nvec = a.A.nvec, nrows = a.A.nrows;
  const float2* P = a.pp + as * (int64_t)nrows * nvec;
  const int ksteps = (nvec + 3) / 4;
  constexpr int kQ = 8;   // staged values a thread has in flight before it waits
  for (int e0 = tid; e0 < 4 * ksteps * 16 * RT; e0 += kQ * 512) {
    float2 v[kQ];
#pragma unroll
    for (int u = 0; u < kQ; ++u) {
      const int e = e0 + u * 512;
      const int k = e / (16 * RT), rr = e - k * (16 * RT);
      v[u] = make_float2(0.f, 0.f);
      if (e < 4 * ksteps * 16 * RT && k < nvec && r0 + rr < a.nrhs)
        v[u] = a.in[(int64_t)(r0 + rr) * a.in_stride + agg * 2 * nvec + sigma * nvec + k];
    }
#pragma unroll
    for (int u = 0; u < kQ; ++u) {
      const int e = e0 + u * 512;
      const int k = e / (16 * RT), rr = e - k * (16 * RT);
      if (e < 4 * ksteps * 16 * RT) cs[k][rr] = v[u];
    }
  }
  __syncthreads();
  const int kk = lane >> 4, il = lane & 15;
  const int mt_n = (nrows + 15) / 16;
  const int64_t abase = agg_base(a.A, agg);
  for (int mt = wave; mt < mt_n; mt += 8) {
    const int row = 16 * mt + il;
    f32x4 yr[RT], yi[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      yr[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
      yi[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll 2
    for (int s = 0; s < ksteps; ++s) {
      const int k = 4 * s + kk;
      float2 p = make_float2(0.f, 0.f);
      if (row < nrows && k < nvec) p = P[(int64_t)k * nrows + row];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const float2 c = cs[k][16 * rt + il];
        cmfma(yr[rt], yi[rt], c.x, c.y, p.x, p.y);
      }
    }
    if (row >= nrows) continue;
    const int64_t fi = abase + agg_row_rel(a.A, sigma, row);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = r0 + 16 * rt + 4 * kk + t;
        if (r >= a.nrhs) continue;
        float2* o = a.out + (int64_t)r * a.out_stride + fi;
        float2 v = make_float2(yr[rt][t], yi[rt][t]);
        if (a.accumulate) { const float2 old = *o; v.x += old.x; v.y += old.y; }
        *o = v;
      }
    }
  }
}

template <typename R>
void launch_restrict(const RestrictArgs<R>& a, hipStream_t st) {
  if (a.nrhs <= 0) return;
  if constexpr (sizeof(R) == 4) {
    if (a.nrhs >= 4) {
      const unsigned gx = (unsigned)(a.A.nagg * 2), nt = 64 * ((a.A.nvec + 15) / 16);
      static_assert(64 % kXferChunk == 0, "restrict_mfma: a thread's staged row must not change with u");
      if (a.nrhs <= 16) restrict_mfma_kernel<1><<<dim3(gx), nt, 0, st>>>(a);
      else restrict_mfma_kernel<4><<<dim3(gx * (unsigned)((a.nrhs + 63) / 64)), nt, 0, st>>>(a);
      return;
    }
  }
  const bool big = a.A.nvec > 64;
  // the staged inputs must fit next to the reduction buffer (64 KiB budget)
  const size_t row_bytes = (size_t)a.A.nrows * sizeof(cplx<R>);
  if (a.nrhs >= 8 && sizeof(R) == 4 && 8 * row_bytes <= 65536) {
    if (big) restrict_launch<R, 8, 2>(a, st);
    else restrict_launch<R, 8, 1>(a, st);
  } else if (a.nrhs >= 4 && 4 * row_bytes <= 65536) {
    if (big) restrict_launch<R, 4, 2>(a, st);
    else restrict_launch<R, 4, 1>(a, st);
  } else {
    if (big) restrict_launch<R, 1, 2>(a, st);
    else restrict_launch<R, 1, 1>(a, st);
  }
}
template void launch_restrict<float>(const RestrictArgs<float>&, hipStream_t);
template void launch_restrict<double>(const RestrictArgs<double>&, hipStream_t);

template <typename R, int NR>
__global__ void __launch_bounds__(512) prolong_kernel(const ProlongArgs<R> a) {
  using T = cplx<R>;
  __shared__ T ec[NR][128];
  const int64_t as = xcd_block(blockIdx.x, gridDim.x);
  const int64_t agg = as >> 1;
  const int sigma = (int)(as & 1);
  const int r0 = blockIdx.y * NR;
  const int nr = (a.nrhs - r0) < NR ? (a.nrhs - r0) : NR;
  const int tid = threadIdx.x;
  const int nvec = a.A.nvec, nrows = a.A.nrows;
  const T* P = a.pp + as * (int64_t)nrows * nvec;
  for (int e = tid; e < NR * nvec; e += 512) {
    const int r = e / nvec, k = e - r * nvec;
    T v;
    v.x = 0; v.y = 0;
    if (r < nr) {
      if (a.unit_col >= 0) {
        if (sigma * nvec + k == a.unit_col) v.x = 1;
      } else {
        v = a.in[(int64_t)(r0 + r) * a.in_stride + agg * 2 * nvec + sigma * nvec + k];
      }
    }
    ec[r][k] = v;
  }
  __syncthreads();
  for (int row = tid; row < nrows; row += 512) {
    T acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) { acc[r].x = 0; acc[r].y = 0; }
    for (int k = 0; k < nvec; ++k) {
      const T p = P[(int64_t)k * nrows + row];
#pragma unroll
      for (int r = 0; r < NR; ++r) cfma(acc[r], p, ec[r][k]);
    }
    const int64_t fi = agg_row_index(a.A, agg, sigma, row);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r >= nr) continue;
      T* o = a.out + (int64_t)(r0 + r) * a.out_stride + fi;
      T v = acc[r];
      if (a.accumulate) { const T old = *o; v.x += old.x; v.y += old.y; }
      *o = v;
    }
  }
}

template <typename R>
void launch_prolong(const ProlongArgs<R>& a, hipStream_t st) {
  if (a.nrhs <= 0) return;
  const unsigned gx = (unsigned)(a.A.nagg * 2);
  if constexpr (sizeof(R) == 4) {
    if (a.nrhs >= 4 && a.unit_col < 0) {
      if (a.nrhs <= 16) prolong_mfma_kernel<1><<<dim3(gx), 512, 0, st>>>(a);
      else prolong_mfma_kernel<4><<<dim3(gx * (unsigned)((a.nrhs + 63) / 64)), 512, 0, st>>>(a);
      return;
    }
  }
  if (a.nrhs >= 8 && sizeof(R) == 4) {
    dim3 grid(gx, (unsigned)((a.nrhs + 7) / 8));
    prolong_kernel<R, 8><<<grid, 512, 0, st>>>(a);
  } else if (a.nrhs >= 4) {
    dim3 grid(gx, (unsigned)((a.nrhs + 3) / 4));
    prolong_kernel<R, 4><<<grid, 512, 0, st>>>(a);
  } else {
    dim3 grid(gx, (unsigned)a.nrhs);
    prolong_kernel<R, 1><<<grid, 512, 0, st>>>(a);
  }
}
template void launch_prolong<float>(const ProlongArgs<float>&, hipStream_t);
template void launch_prolong<double>(const ProlongArgs<double>&, hipStream_t);

}  // namespace mg
