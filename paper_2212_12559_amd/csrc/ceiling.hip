// Measured ceilings of the chip (measurement aids, not part of the method):
// a streaming copy kernel for the HBM bandwidth a kernel can reach, and a
// loop of independent 16-bit MFMA products for the matrix-core rate.  Both
// are timed with HIP events on the caller's stream.
#include <cstring>

#include "mg.hpp"

namespace {

// out[i] = in[i] over 16-byte elements, grid-stride, blocks numbered so that
// consecutive blocks of one XCD walk one contiguous range
__global__ void __launch_bounds__(256) copy16_kernel(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                     int64_t n) {
  const int64_t b = mg::xcd_block(blockIdx.x, gridDim.x);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = b * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kChains = 8;   // independent accumulators per wavefront (covers the MFMA latency)

template <int FMT>
__global__ void __launch_bounds__(256) mfma_loop_kernel(int iters, float* sink) {
  const uint32_t seed = 0x3c003c00u ^ (threadIdx.x * 0x00010001u);
  const uint4 ab = make_uint4(seed, seed ^ 0x00400040u, seed ^ 0x00200020u, seed ^ 0x00100010u);
  f32x4 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (FMT == 0)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ab), __builtin_bit_cast(bf16x8, ab),
                                                         acc[c], 0, 0, 0);
      else
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, ab), __builtin_bit_cast(f16x8, ab),
                                                        acc[c], 0, 0, 0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (threadIdx.x == 0) sink[blockIdx.x] = s;   // keeps the products live
}

mg_status fail(mg_status s, const char* m) { return mg::set_last_error(s, m); }

// Time `launch` reps times between two events on stream st; returns ms per launch.
template <typename F>
mg_status time_launches(F&& launch, int reps, hipStream_t st, double* ms_per) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(MG_E_HIP, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MG_E_HIP, "hipEventCreate");
  }
  launch();   // warm-up
  mg_status s = MG_OK;
  float ms = 0.f;
  if (hipEventRecord(e0, st) != hipSuccess) s = fail(MG_E_HIP, "hipEventRecord");
  for (int r = 0; r < reps && s == MG_OK; ++r) launch();
  if (s == MG_OK && hipGetLastError() != hipSuccess) s = fail(MG_E_HIP, "kernel launch");
  if (s == MG_OK && hipEventRecord(e1, st) != hipSuccess) s = fail(MG_E_HIP, "hipEventRecord");
  if (s == MG_OK && hipEventSynchronize(e1) != hipSuccess) s = fail(MG_E_HIP, "hipEventSynchronize");
  if (s == MG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = fail(MG_E_HIP, "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s == MG_OK) *ms_per = (double)ms / reps;
  return s;
}

}  // namespace

extern "C" {

mg_status mg_peak_copy(const void* src, void* dst, size_t bytes, int32_t reps, void* stream, double* gbs) {
  if (!src || !dst || !gbs || reps < 1) return fail(MG_E_ARG, "null argument or reps < 1");
  if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15) || (bytes & 15)) return fail(MG_E_ALIGN, "16-byte alignment");
  const int64_t n = (int64_t)(bytes / 16);
  const unsigned grid = 256u * 16u;   // 16 workgroups of 256 per compute unit
  hipStream_t st = (hipStream_t)stream;
  double ms = 0.0;
  mg_status s = time_launches(
      [&] { copy16_kernel<<<grid, 256, 0, st>>>((const uint4*)src, (uint4*)dst, n); }, reps, st, &ms);
  if (s == MG_OK) *gbs = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
  return s;
}

mg_status mg_peak_mfma(int32_t fmt, int32_t iters, void* sink, void* stream, double* tflops) {
  if (!sink || !tflops || iters < 1 || (fmt != MG_CBF16 && fmt != MG_CF16)) return fail(MG_E_ARG, "bad argument");
  const unsigned grid = 256u * 8u;    // eight workgroups of four wavefronts per compute unit
  hipStream_t st = (hipStream_t)stream;
  double ms = 0.0;
  mg_status s = time_launches(
      [&] {
        if (fmt == MG_CBF16) mfma_loop_kernel<0><<<grid, 256, 0, st>>>(iters, (float*)sink);
        else mfma_loop_kernel<1><<<grid, 256, 0, st>>>(iters, (float*)sink);
      },
      3, st, &ms);
  // 2 * 16 * 16 * 32 flops per product, kChains products per iteration and wavefront
  if (s == MG_OK) *tflops = (double)grid * 4 * iters * kChains * 16384.0 / (ms * 1e-3) / 1e12;
  return s;
}

}  // extern "C"
