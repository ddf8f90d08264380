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
// (the site's right-hand-side columns, converted to 16 bits with
// round-to-nearest-even) is staged in LDS as [rhs][k] planes, read with the
// same k mapping.  FP16 links carry a power-of-two scale
// (2^-round(log2 max|L|)) undone on the FP32 result.
#include <algorithm>
#include <stdexcept>
#include <type_traits>

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


typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;

// Streaming (non-temporal) accesses for the links, each read by one workgroup
// only, and for the result: they leave the L2 to the neighbour inputs, which
// nine workgroups read.
__device__ __forceinline__ uint4 load_stream(const uint4* p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void store_stream(float2* p, float re, float im) {
  __builtin_nontemporal_store(f32x2{re, im}, reinterpret_cast<f32x2*>(p));
}

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

// One workgroup per (coarse site, group of 16 RT right-hand sides); each
// wavefront takes MT m-tiles (n <= 256: at most 16 m-tiles).  The B operand is
// staged through LDS in passes of kMfmaCK k-chunks; a B fragment read from LDS
// feeds 4 MT products and an A fragment streamed from HBM feeds 4 RT, so the
// links, which dominate the traffic, are read once per 16 RT right-hand sides
// and the LDS reads per product fall as 1 / MT.  A thread has the loads of
// kStageQ staging quads in flight before it waits (more cost occupancy, which
// hides the latency of the link loads better).
constexpr int kMfmaCK = 4;
constexpr int kMfmaMaxWaves = 16;
constexpr int kStageQ = 4;        // staging quads whose loads a thread has in flight at once

// The work of one workgroup: coarse site `site`, right-hand sides r0 ..
// r0 + 16 RT - 1 (bsm: the B staging area, nbs: the neighbour table, both in
// LDS).
template <int FMT, int RT, int MT>
__device__ __forceinline__ void coarse_mfma_site(const CoarseMfmaArgs& a, const int64_t site, const int r0,
                                                 uint16_t* bsm, int64_t* nbs) {
  constexpr int NR = 16 * RT;          // right-hand sides per workgroup
  constexpr int KCH = kMfmaCK * 32;    // k per staging pass
  constexpr int KPC = KCH + 8;         // padded LDS row: staggers banks between rhs rows
  uint16_t* Bre = bsm;
  uint16_t* Bim = bsm + NR * KPC;
  const int n = a.n;
  const int K = 9 * n;
  const int kc_n = (K + 31) / 32;
  const int mt_n = n / 16;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nthreads = blockDim.x;
  const int nw = mt_n / MT;            // wavefronts; this one owns m-tiles wave + nw m
  if (tid < 9) {
    int c[4];
    site_coords(site, a.g, c);
    nbs[tid] = tid == 0 ? site : site_shift(c, (tid - 1) >> 1, (tid & 1) ? 1 : -1, a.g);
  }
  f32x4 yr[MT][RT], yi[MT][RT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      yr[m][rt] = f32x4{0.f, 0.f, 0.f, 0.f};
      yi[m][rt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  const uint4* Lm[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
    Lm[m] = reinterpret_cast<const uint4*>(a.links) + (site * mt_n + wave + nw * m) * (int64_t)kc_n * 2 * 64;
  const int j = lane & 15, g = lane >> 4;
  // With an identity self block (unit_self) the k range starts at direction 1.
  // Where a staging pass is exactly one direction (n = KCH), neighbouring
  // workgroups read the same input vector in the same pass: a site with odd x
  // takes -x, self, +x in its first three passes (its -x is the self of the
  // site before it, its self the +x of that site), and rows y = 2, 3 mod 4
  // (z likewise) take -y before +y (reading the row that y - 2 reads with +y).
  const int kc_begin = a.unit_self ? n / 32 : 0;
  const bool perm = n == KCH && kc_n == 9 * kMfmaCK;
  const int64_t sx = site % a.g.L[0], sy = (site / a.g.L[0]) % a.g.L[1],
                sz = (site / ((int64_t)a.g.L[0] * a.g.L[1])) % a.g.L[2];
  const bool xodd = perm && (sx & 1), yswap = perm && ((sy >> 1) & 1), zswap = perm && ((sz >> 1) & 1);
  const int npass = (kc_n - kc_begin + kMfmaCK - 1) / kMfmaCK;
  // quads of the staging pass: quad e = tid + q nthreads holds rhs row
  // e / (KCH / 4) at k offset 4 (e mod KCH / 4); nthreads is a multiple of 64,
  // so every quad of a thread has the same k offset (and direction) and its
  // rows step by nthreads / (KCH / 4).  A thread issues the loads of kStageQ
  // quads before the first is waited for.
  const int nq = NR * (KCH / 4);
  const int qpt = (nq + nthreads - 1) / nthreads;
  const int kq = 4 * (tid % (KCH / 4)), jq = tid / (KCH / 4), jstep = nthreads / (KCH / 4);
  // A fragments (Re, Im) of a k-chunk
  auto load_a = [&](uint4 (&dst)[MT][2], int kc) {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      dst[m][0] = load_stream(Lm[m] + (kc * 2 + 0) * 64 + lane);
      dst[m][1] = load_stream(Lm[m] + (kc * 2 + 1) * 64 + lane);
    }
  };
  for (int pi = 0; pi < npass; ++pi) {
    // direction-ordered passes: d = pi (+1 without the self block), reordered as above
    int pd = pi + (a.unit_self && perm ? 1 : 0);
    if (xodd) {
      if (a.unit_self) { if (pd <= 2) pd = 3 - pd; }
      else if (pd <= 2) pd = pd == 0 ? 2 : pd - 1;
    }
    if (yswap && (pd == 3 || pd == 4)) pd = 7 - pd;
    if (zswap && (pd == 5 || pd == 6)) pd = 11 - pd;
    const int kc0 = perm ? pd * kMfmaCK : kc_begin + pi * kMfmaCK;
    __syncthreads();   // neighbour table ready / previous pass consumed
    // stage k in [32 kc0, 32 kc0 + KCH): quads (k .. k + 3) lie in one
    // direction (n is a multiple of 16) and are two 16-byte loads (one for
    // 16-bit inputs; inputs are 16-byte aligned) and one 8-byte LDS store per
    // plane
    const int k = kc0 * 32 + kq;
    const int d = min(k / n, 8);
    const int64_t cb = nbs[d] * n + (k - d * n);   // offset of this thread's k in an input row
    // The loads are unconditional (a quad outside the input reads element 0
    // and is zeroed afterwards) and the input format is a compile-time branch:
    // loads under per-lane branches let the compiler move the conversion into
    // the branch and wait there, which left one quad in flight per thread.
    auto stage = [&](auto in16_tag) {
      constexpr bool I16 = decltype(in16_tag)::value;
#pragma unroll 1
      for (int q0 = 0; q0 < qpt; q0 += kStageQ) {
        uint4 raw0[kStageQ], raw1[kStageQ];
        bool ok[kStageQ];
#pragma unroll
        for (int q = 0; q < kStageQ; ++q) {
          const int jj = jq + (q0 + q) * jstep;
          ok[q] = q0 + q < qpt && jj < NR && r0 + jj < a.nrhs && k < K;
          const int rr = ok[q] ? r0 + jj : 0;
          const int64_t off = (int64_t)rr * a.in_stride + (ok[q] ? cb : 0);
          if constexpr (I16) {
            raw0[q] = *reinterpret_cast<const uint4*>(a.in16 + off);
          } else {
            const uint4* src = reinterpret_cast<const uint4*>(a.in + off);
            raw0[q] = src[0];
            raw1[q] = src[1];
          }
        }
#pragma unroll
        for (int q = 0; q < kStageQ; ++q) {
          const int jj = jq + (q0 + q) * jstep;
          if (q0 + q < qpt && jj < NR) {
            uint2 pre, pim;
            const uint4 z = make_uint4(0u, 0u, 0u, 0u);
            const uint4 c = ok[q] ? raw0[q] : z;
            if constexpr (I16) {   // four packed 16-bit complex numbers, split into the two planes
              pre.x = (c.x & 0xFFFFu) | (c.y << 16);
              pre.y = (c.z & 0xFFFFu) | (c.w << 16);
              pim.x = (c.x >> 16) | (c.y & 0xFFFF0000u);
              pim.y = (c.z >> 16) | (c.w & 0xFFFF0000u);
            } else {
              const float4 v0 = make_float4(__uint_as_float(c.x), __uint_as_float(c.y), __uint_as_float(c.z),
                                            __uint_as_float(c.w));
              const uint4 c1 = ok[q] ? raw1[q] : z;
              const float4 v1 = make_float4(__uint_as_float(c1.x), __uint_as_float(c1.y), __uint_as_float(c1.z),
                                            __uint_as_float(c1.w));
              pre.x = (uint32_t)to16<FMT>(v0.x) | ((uint32_t)to16<FMT>(v0.z) << 16);
              pre.y = (uint32_t)to16<FMT>(v1.x) | ((uint32_t)to16<FMT>(v1.z) << 16);
              pim.x = (uint32_t)to16<FMT>(v0.y) | ((uint32_t)to16<FMT>(v0.w) << 16);
              pim.y = (uint32_t)to16<FMT>(v1.y) | ((uint32_t)to16<FMT>(v1.w) << 16);
            }
            *reinterpret_cast<uint2*>(Bre + jj * KPC + kq) = pre;
            *reinterpret_cast<uint2*>(Bim + jj * KPC + kq) = pim;
          }
        }
      }
    };
    if (a.in16) stage(std::true_type{});
    else stage(std::false_type{});
    __syncthreads();
#pragma unroll
    for (int kcl = 0; kcl < kMfmaCK; ++kcl) {
      const int kc = kc0 + kcl;
      if (kc < kc_n) {
        uint4 acur[MT][2], aimn[MT];   // Re A, Im A and -Im A (sign bits flipped)
        load_a(acur, kc);
#pragma unroll
        for (int m = 0; m < MT; ++m)
          aimn[m] = make_uint4(acur[m][1].x ^ 0x80008000u, acur[m][1].y ^ 0x80008000u,
                               acur[m][1].z ^ 0x80008000u, acur[m][1].w ^ 0x80008000u);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const int off = (rt * 16 + j) * KPC + kcl * 32 + 8 * g;
          const uint4 bre = *reinterpret_cast<const uint4*>(Bre + off);
          const uint4 bim = *reinterpret_cast<const uint4*>(Bim + off);
#pragma unroll
          for (int m = 0; m < MT; ++m) {
            yr[m][rt] = mfma16<FMT>(acur[m][0], bre, yr[m][rt]);
            yr[m][rt] = mfma16<FMT>(aimn[m], bim, yr[m][rt]);
            yi[m][rt] = mfma16<FMT>(acur[m][0], bim, yi[m][rt]);
            yi[m][rt] = mfma16<FMT>(acur[m][1], bre, yi[m][rt]);
          }
        }
      }
    }
  }
  // D fragment: column j (rhs), rows 4 g + t of each m-tile
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int mt = wave + nw * m;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int r = r0 + rt * 16 + j;
      if (r < a.nrhs) {
        float2* o = a.out + (int64_t)r * a.out_stride + site * n + mt * 16 + 4 * g;
        float2 xs[4] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
        if (a.unit_self) {
          const float2* xi = a.in + (int64_t)r * a.in_stride + site * n + mt * 16 + 4 * g;
#pragma unroll
          for (int t = 0; t < 4; ++t) xs[t] = xi[t];
        }
        float vr[4], vi[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          vr[t] = fmaf(yr[m][rt][t], a.inv_scale, xs[t].x);
          vi[t] = fmaf(yi[m][rt][t], a.inv_scale, xs[t].y);
          store_stream(o + t, vr[t], vi[t]);
        }
        if (a.out16) {   // the same values rounded as the next application would round them
          uint4 c;
          c.x = (uint32_t)to16<FMT>(vr[0]) | ((uint32_t)to16<FMT>(vi[0]) << 16);
          c.y = (uint32_t)to16<FMT>(vr[1]) | ((uint32_t)to16<FMT>(vi[1]) << 16);
          c.z = (uint32_t)to16<FMT>(vr[2]) | ((uint32_t)to16<FMT>(vi[2]) << 16);
          c.w = (uint32_t)to16<FMT>(vr[3]) | ((uint32_t)to16<FMT>(vi[3]) << 16);
          *reinterpret_cast<uint4*>(a.out16 + (int64_t)r * a.out_stride + site * n + mt * 16 + 4 * g) = c;
        }
      }
    }
  }
}

template <int FMT, int RT, int MT>
__global__ void __launch_bounds__(64 * kMfmaMaxWaves) coarse_mfma_kernel(const CoarseMfmaArgs a) {
  extern __shared__ uint16_t bsm[];    // [2 planes][16 RT][KCH + 8]
  __shared__ int64_t nbs[9];
  // block -> (site, rhs tile) with the rhs tile fastest, after the XCD
  // renumbering: the tiles of a site run back to back on one XCD and read its
  // links once from HBM, the other times from that XCD's L2
  const int ntile = (a.nrhs + 16 * RT - 1) / (16 * RT);
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int64_t site = b / ntile;
  coarse_mfma_site<FMT, RT, MT>(a, site, (int)(b - site * ntile) * 16 * RT, bsm, nbs);
}

// One persistent launch over the (problem, site, rhs tile) work list of up to
// kMaxMulti problems of the same n and link format: each workgroup walks the
// list with a grid-sized stride.
template <int FMT, int RT, int MT>
__global__ void __launch_bounds__(64 * kMfmaMaxWaves) coarse_mfma_multi_kernel(const CoarseMultiArgs m) {
  extern __shared__ uint16_t bsm[];
  __shared__ int64_t nbs[9];
  for (int64_t item = blockIdx.x; item < m.start[m.nprob]; item += gridDim.x) {
    int p = 0;
    while (item >= m.start[p + 1]) ++p;
    const int64_t li = item - m.start[p];
    const int ntile = (m.p[p].nrhs + 16 * RT - 1) / (16 * RT);
    __syncthreads();   // the previous item is done with the LDS
    coarse_mfma_site<FMT, RT, MT>(m.p[p], li / ntile, (int)(li % ntile) * 16 * RT, bsm, nbs);
  }
}

void launch_coarse_mfma_multi(const CoarseMultiArgs& m, int fmt, hipStream_t st) {
  if (m.nprob < 1 || m.nprob > kMaxMulti) throw std::runtime_error("coarse_mfma_multi: 1..8 problems");
  const int n = m.p[0].n;
  for (int p = 0; p < m.nprob; ++p) {
    if (m.p[p].n != n) throw std::runtime_error("coarse_mfma_multi: problems must share n");
    if (reinterpret_cast<uintptr_t>(m.p[p].in) % 16 || m.p[p].in_stride % 2)
      throw std::runtime_error("coarse_mfma_multi: inputs must be 16-byte aligned");
    if (m.p[p].unit_self && n % 32) throw std::runtime_error("coarse_mfma_multi: implicit identity needs n % 32 == 0");
  }
  if (n % 16 || n < 16 || n > 16 * kMfmaMaxWaves) throw std::runtime_error("coarse_mfma_multi: n in 16..256");
  const int64_t total = m.start[m.nprob];
  if (total <= 0) return;
  const size_t lds = (size_t)2 * 16 * (kMfmaCK * 32 + 8) * sizeof(uint16_t);
  const unsigned grid = (unsigned)std::min<int64_t>(total, 1024);
  if (fmt == 0) coarse_mfma_multi_kernel<0, 1, 1><<<grid, 64 * (n / 16), lds, st>>>(m);
  else coarse_mfma_multi_kernel<1, 1, 1><<<grid, 64 * (n / 16), lds, st>>>(m);
}

template <int FMT, int RT, int MT>
static void coarse_mfma_launch(const CoarseMfmaArgs& a, hipStream_t st) {
  const int mt_n = a.n / 16;
  const size_t lds = (size_t)2 * 16 * RT * (kMfmaCK * 32 + 8) * sizeof(uint16_t);
  const int64_t nb = a.g.V * ((a.nrhs + 16 * RT - 1) / (16 * RT));
  if (nb > 0x7fffffff) throw std::runtime_error("coarse_mfma: too many (site, rhs tile) blocks");
  coarse_mfma_kernel<FMT, RT, MT><<<dim3((unsigned)nb), 64 * (mt_n / MT), lds, st>>>(a);
}

template <int FMT>
static void coarse_mfma_dispatch(const CoarseMfmaArgs& a, hipStream_t st) {
  if (a.rt > 0) {   // an explicit tile shape (autotuned)
    const int mt_n = a.n / 16;
    if (a.mt < 1 || mt_n % a.mt) throw std::runtime_error("coarse_mfma: m-tiles per wavefront must divide n / 16");
    const int key = a.rt * 8 + a.mt;
    switch (key) {
      case 9: coarse_mfma_launch<FMT, 1, 1>(a, st); return;
      case 10: coarse_mfma_launch<FMT, 1, 2>(a, st); return;
      case 17: coarse_mfma_launch<FMT, 2, 1>(a, st); return;
      case 18: coarse_mfma_launch<FMT, 2, 2>(a, st); return;
      case 33: coarse_mfma_launch<FMT, 4, 1>(a, st); return;
      case 34: coarse_mfma_launch<FMT, 4, 2>(a, st); return;
      default: throw std::runtime_error("coarse_mfma: no such tile shape");
    }
  }
  // two m-tiles per wavefront once several rhs tiles share the B reads
  const bool mt2 = a.nrhs > 16 && (a.n / 16) % 2 == 0;
  if (a.nrhs <= 16) coarse_mfma_launch<FMT, 1, 1>(a, st);
  else if (a.nrhs <= 32) {
    if (mt2) coarse_mfma_launch<FMT, 2, 2>(a, st);
    else coarse_mfma_launch<FMT, 2, 1>(a, st);
  } else {
    if (mt2) coarse_mfma_launch<FMT, 4, 2>(a, st);
    else coarse_mfma_launch<FMT, 4, 1>(a, st);
  }
}

void launch_coarse_mfma(const CoarseMfmaArgs& a, int fmt, hipStream_t st) {
  if (a.nrhs <= 0) return;
  if (a.n % 16 || a.n < 16 || a.n > 16 * kMfmaMaxWaves)
    throw std::runtime_error("coarse_mfma: n must be a multiple of 16 in 16..256");
  if (reinterpret_cast<uintptr_t>(a.in) % 16 || a.in_stride % 2)
    throw std::runtime_error("coarse_mfma: input must be 16-byte aligned");
  if (a.unit_self && a.n % 32)
    throw std::runtime_error("coarse_mfma: an implicit identity self block needs n to be a multiple of 32");
  if (fmt == 0) coarse_mfma_dispatch<0>(a, st);
  else coarse_mfma_dispatch<1>(a, st);
}

int64_t swizzled_link_elems(int64_t nsite, int n) {
  const int kc_n = (9 * n + 31) / 32;
  return nsite * (int64_t)(n / 16) * kc_n * 2 * 64 * 8;
}

}  // namespace mg
