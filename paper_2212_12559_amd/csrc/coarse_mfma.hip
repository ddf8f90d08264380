// Coarse stencil with 16-bit links on the matrix cores (Sec. 3.1: the coarse
// links are stored in 16 bits).  For a coarse site the stencil is one complex
// GEMM  Y[n x N] = L[n x 9n] X[9n x N]  over the nine neighbour vectors and N
// right-hand sides; it runs as four real GEMMs on
// v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation:
//   Re Y += Re L Re X - Im L Im X,   Im Y += Re L Im X + Im L Re X.
//
// Links are pre-swizzled into MFMA A-fragments at set-up:
//   [site][m-tile (16 rows)][k-chunk (32)][re/im][lane 0..63][8 x 16-bit]
// lane l holds row 16 mt + (l % 16), k = 32 kc + 8 (l / 16) + t, t = 0..7, so
// every fragment is one contiguous 1 KiB load of a wavefront.  The B operand
// (the site's 16 right-hand-side columns, converted to 16 bits with
// round-to-nearest-even) is staged once per workgroup in LDS as [rhs][k]
// planes, read with the same k mapping.  FP16 links carry a power-of-two scale
// (2^-round(log2 max|L|)) undone on the FP32 result.
#include "kernels.hpp"

namespace mg {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// FP32 -> 16-bit bit patterns, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) {
  _Float16 h = (_Float16)f;   // IEEE conversion, round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}
template <int FMT>
__device__ __forceinline__ uint16_t to16(float f) { return FMT == 0 ? f32_to_bf16_rne(f) : f32_to_f16_rne(f); }


template <int FMT>
__device__ __forceinline__ f32x4 mfma16(uint4 a, uint4 b, f32x4 c) {
  if constexpr (FMT == 0) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                  0, 0, 0);
  }
}

// links [site][d][col][row] (FP64 or FP32) -> swizzled 16-bit fragments (scaled)
template <int FMT, typename TI>
__global__ void swizzle_links_kernel(const TI* __restrict__ cl, uint16_t* __restrict__ out, int64_t nsite,
                                     int n, int kc_n, double scale) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int mt_n = n / 16;
  const int64_t per_site = (int64_t)mt_n * kc_n * 2 * 64 * 8;
  if (tid >= nsite * per_site) return;
  const int64_t site = tid / per_site;
  int64_t rem = tid - site * per_site;
  const int t = (int)(rem & 7); rem >>= 3;
  const int lane = (int)(rem & 63); rem >>= 6;
  const int plane = (int)(rem & 1); rem >>= 1;
  const int kc = (int)(rem % kc_n);
  const int mt = (int)(rem / kc_n);
  const int row = mt * 16 + (lane & 15);
  const int k = kc * 32 + 8 * (lane >> 4) + t;
  float v = 0.0f;
  if (k < 9 * n) {
    const int d = k / n, col = k - d * n;
    const TI l = cl[((site * 9 + d) * n + col) * (int64_t)n + row];
    v = (float)((double)(plane ? l.y : l.x) * scale);
  }
  out[tid] = to16<FMT>(v);
}

template <typename TI>
void launch_swizzle_links(const TI* cl, uint16_t* out, int64_t nsite, int n, int fmt, double scale,
                          hipStream_t st) {
  const int kc_n = (9 * n + 31) / 32;
  const int64_t tot = nsite * (n / 16) * kc_n * 2 * 64 * 8;
  const unsigned g = (unsigned)((tot + 255) / 256);
  if (fmt == 0) swizzle_links_kernel<0, TI><<<g, 256, 0, st>>>(cl, out, nsite, n, kc_n, scale);
  else swizzle_links_kernel<1, TI><<<g, 256, 0, st>>>(cl, out, nsite, n, kc_n, scale);
}
template void launch_swizzle_links<double2>(const double2*, uint16_t*, int64_t, int, int, double, hipStream_t);
template void launch_swizzle_links<float2>(const float2*, uint16_t*, int64_t, int, int, double, hipStream_t);

__global__ void absmax_kernel(const double2* __restrict__ v, int64_t n, unsigned long long* out) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fmax(fabs(v[i].x), fabs(v[i].y)));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  // non-negative doubles order like their bit patterns
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}
void launch_absmax(const double2* v, int64_t n, unsigned long long* out, hipStream_t st) {
  absmax_kernel<<<480, 256, 0, st>>>(v, n, out);
}

constexpr int kMfmaWaves = 8;

template <int FMT>
__global__ void __launch_bounds__(64 * kMfmaWaves) coarse_mfma_kernel(const CoarseMfmaArgs a) {
  extern __shared__ uint16_t bsm[];              // [2 planes][16 rhs][KP]
  const int n = a.n;
  const int K = 9 * n;
  const int kc_n = (K + 31) / 32;
  const int KP = kc_n * 32 + 8;                  // padded row: staggers LDS banks between rhs rows
  uint16_t* Bre = bsm;
  uint16_t* Bim = bsm + 16 * KP;
  const int64_t site = blockIdx.x;
  const int r0 = blockIdx.y * 16;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  int c[4];
  site_coords(site, a.g, c);
  int64_t nb[9];
  nb[0] = site;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    nb[1 + 2 * mu] = site_shift(c, mu, 1, a.g);
    nb[2 + 2 * mu] = site_shift(c, mu, -1, a.g);
  }
  // stage B: column j = rhs r0 + j, row k = d n + col; each thread converts two
  // consecutive k (same direction, n is even) per step: one 16-byte load, two
  // 4-byte LDS stores; the direction / column walk is incremental
  const int KC = kc_n * 32;
  constexpr int NT = 64 * kMfmaWaves;
  for (int j = 0; j < 16; ++j) {
    const bool live = r0 + j < a.nrhs;
    const float2* xj = a.in + (int64_t)(live ? r0 + j : 0) * a.in_stride;
    int k = 2 * tid;
    int d = k / n, col = k - (k / n) * n;
    for (; k < KC; k += 2 * NT) {
      uint32_t pre = 0, pim = 0;
      if (live && k < K) {
        const float4 v = *reinterpret_cast<const float4*>(xj + nb[d] * n + col);
        pre = (uint32_t)to16<FMT>(v.x) | ((uint32_t)to16<FMT>(v.z) << 16);
        pim = (uint32_t)to16<FMT>(v.y) | ((uint32_t)to16<FMT>(v.w) << 16);
      }
      *reinterpret_cast<uint32_t*>(Bre + j * KP + k) = pre;
      *reinterpret_cast<uint32_t*>(Bim + j * KP + k) = pim;
      col += 2 * NT;
      while (col >= n) { col -= n; ++d; }
    }
  }
  __syncthreads();
  const int mt_n = n / 16;
  const uint4* L = reinterpret_cast<const uint4*>(a.links) + site * (int64_t)mt_n * kc_n * 2 * 64;
  const int j = lane & 15, g = lane >> 4;
  for (int mt = wave; mt < mt_n; mt += kMfmaWaves) {
    f32x4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
    const uint4* Lm = L + (int64_t)mt * kc_n * 2 * 64;
#pragma unroll 4
    for (int kc = 0; kc < kc_n; ++kc) {
      const uint4 are = Lm[(kc * 2 + 0) * 64 + lane];
      const uint4 aim = Lm[(kc * 2 + 1) * 64 + lane];
      const int kb = kc * 32 + 8 * g;
      const uint4 bre = *reinterpret_cast<const uint4*>(Bre + j * KP + kb);
      const uint4 bim = *reinterpret_cast<const uint4*>(Bim + j * KP + kb);
      const uint4 bimn = make_uint4(bim.x ^ 0x80008000u, bim.y ^ 0x80008000u, bim.z ^ 0x80008000u,
                                    bim.w ^ 0x80008000u);
      yr = mfma16<FMT>(are, bre, yr);
      yr = mfma16<FMT>(aim, bimn, yr);
      yi = mfma16<FMT>(are, bim, yi);
      yi = mfma16<FMT>(aim, bre, yi);
    }
    // D fragment: column j (rhs), rows 4 g + t
    if (r0 + j < a.nrhs) {
      float2* o = a.out + (int64_t)(r0 + j) * a.out_stride + site * n + mt * 16 + 4 * g;
#pragma unroll
      for (int t = 0; t < 4; ++t) o[t] = make_float2(yr[t] * a.inv_scale, yi[t] * a.inv_scale);
    }
  }
}

void launch_coarse_mfma(const CoarseMfmaArgs& a, int fmt, hipStream_t st) {
  if (a.nrhs <= 0) return;
  const int kc_n = (9 * a.n + 31) / 32;
  const int KP = kc_n * 32 + 8;
  const size_t lds = (size_t)2 * 16 * KP * sizeof(uint16_t);
  dim3 grid((unsigned)a.g.V, (unsigned)((a.nrhs + 15) / 16));
  if (fmt == 0) coarse_mfma_kernel<0><<<grid, 64 * kMfmaWaves, lds, st>>>(a);
  else coarse_mfma_kernel<1><<<grid, 64 * kMfmaWaves, lds, st>>>(a);
}

int64_t swizzled_link_elems(int64_t nsite, int n) {
  const int kc_n = (9 * n + 31) / 32;
  return nsite * (int64_t)(n / 16) * kc_n * 2 * 64 * 8;
}

}  // namespace mg
