// Kahler-Dirac block preconditioner (Sec. 2.2 Eq. 1-2, Sec. 3.1).
//
// B holds the one-hop terms of D inside each 2^4 hypercube; the paper stores
// the explicit (B + m)^{-1}, one 48 x 48 complex matrix per hypercube, and
// applies it in a kernel of its own after the stencil.
//
// Set-up (FP64): B is anti-Hermitian, so (B + m)(m - B) = m^2 + B^dag B = M,
// a Hermitian positive definite matrix; (B + m)^{-1} = (m - B) M^{-1}.
// M is inverted by Gauss-Jordan without pivoting (safe for HPD), all in LDS,
// one workgroup per hypercube.  This avoids pivoting; the oracle uses plain LU.
//
// Apply: one wavefront per hypercube, lane = row (48 of 64 lanes), the
// matrix stored column-major so each column is one coalesced segment; the
// hypercube's 48 input components are exchanged between lanes with
// cross-lane shuffles.
#include <stdexcept>

#include "kernels.hpp"

namespace mg {

__global__ void __launch_bounds__(256) kd_inverse_kernel(const double2* __restrict__ fat, Geom g,
                                                         double mass, double2* __restrict__ out64,
                                                         float2* __restrict__ out32) {
  // Bs[u][mu][3 i + j]: the 3x3 block of B at block row u, block column u ^ (1 << mu)
  __shared__ double2 Bs[16][4][9];
  __shared__ double2 M[48][48];
  const int64_t hc = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t V = g.V;
  for (int e = tid; e < 16 * 4 * 9; e += 256) {
    const int u = e / 36, mu = (e / 9) % 4, k = e % 9;
    const int i = k / 3, j = k % 3;
    double2 v;
    if (((u >> mu) & 1) == 0) {
      // forward hop x -> x + mu inside the cube: W'_mu(x)[i][j]
      const int64_t x = hc_site(hc, u, g);
      v = fat[((int64_t)mu * 9 + 3 * i + j) * V + x];
    } else {
      // backward hop x -> x - mu: -(W'_mu(x - mu)^dag)[i][j] = -conj(W'_mu(x - mu)[j][i])
      const int64_t xm = hc_site(hc, u ^ (1 << mu), g);
      const double2 w = fat[((int64_t)mu * 9 + 3 * j + i) * V + xm];
      v = make_double2(-w.x, w.y);
    }
    Bs[u][mu][k] = v;
  }
  __syncthreads();
  // M = m^2 + B^dag B; (B^dag B)[(s,i),(t,j)] = sum over block rows u adjacent to both s and t
  for (int e = tid; e < 48 * 48; e += 256) {
    const int a = e / 48, b = e % 48;
    const int sa = a / 3, ia = a % 3, sb = b / 3, ib = b % 3;
    double2 acc = make_double2(a == b ? mass * mass : 0.0, 0.0);
    for (int mu = 0; mu < 4; ++mu) {
      const int u = sa ^ (1 << mu);
      const int d = u ^ sb;
      if (__popc(d) != 1) continue;
      const int nu = __ffs(d) - 1;
      for (int k = 0; k < 3; ++k) cfmac(acc, Bs[u][mu][3 * k + ia], Bs[u][nu][3 * k + ib]);
    }
    M[a][b] = acc;
  }
  __syncthreads();
  // Gauss-Jordan inversion in place, no pivoting
  for (int k = 0; k < 48; ++k) {
    const double2 p = M[k][k];
    const double pn = p.x * p.x + p.y * p.y;
    const double2 pinv = make_double2(p.x / pn, -p.y / pn);
    __syncthreads();
    if (tid < 48 && tid != k) M[k][tid] = cmul(M[k][tid], pinv);
    __syncthreads();
    for (int e = tid; e < 48 * 48; e += 256) {
      const int i = e / 48, j = e % 48;
      if (i != k && j != k) {
        const double2 f = M[i][k];
        const double2 t = M[k][j];
        double2 v = M[i][j];
        v.x -= f.x * t.x - f.y * t.y;
        v.y -= f.x * t.y + f.y * t.x;
        M[i][j] = v;
      }
    }
    __syncthreads();
    if (tid < 48 && tid != k) {
      const double2 q = cmul(M[tid][k], pinv);
      M[tid][k] = make_double2(-q.x, -q.y);
    }
    if (tid == 0) M[k][k] = pinv;
    __syncthreads();
  }
  // (B + m)^{-1} = (m - B) M^{-1}, stored column-major: out[hc][col][row]
  for (int e = tid; e < 48 * 48; e += 256) {
    const int j = e / 48, i = e % 48;   // column j, row i
    const int si = i / 3, ci = i % 3;
    double2 acc = make_double2(mass * M[i][j].x, mass * M[i][j].y);
    for (int mu = 0; mu < 4; ++mu) {
      const int sn = si ^ (1 << mu);
      for (int k = 0; k < 3; ++k) {
        const double2 b = Bs[si][mu][3 * ci + k];
        const double2 m = M[3 * sn + k][j];
        acc.x -= b.x * m.x - b.y * m.y;
        acc.y -= b.x * m.y + b.y * m.x;
      }
    }
    const int64_t o = hc * 2304 + (int64_t)j * 48 + i;
    out64[o] = acc;
    if (out32) out32[o] = make_float2((float)acc.x, (float)acc.y);
  }
}

void launch_kd_inverse(const double2* fat64, const Geom& g, double mass, double2* out64, float2* out32,
                       hipStream_t st) {
  const int64_t nhc = g.V / 16;
  kd_inverse_kernel<<<(unsigned)nhc, 256, 0, st>>>(fat64, g, mass, out64, out32);
}

template <typename R, int NR>
__global__ void __launch_bounds__(256) kd_apply_kernel(const KdArgs<R> a) {
  using T = cplx<R>;
  const int lane = threadIdx.x & 63;
  const int64_t hc = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nhc = a.g.V / 16;
  if (hc >= nhc) return;
  const int r0 = blockIdx.y * NR;
  const int nr = (a.nrhs - r0) < NR ? (a.nrhs - r0) : NR;
  const bool act = lane < 48;
  const int sl = act ? lane / 3 : 0;
  const int col = act ? lane - 3 * (lane / 3) : 0;
  const int64_t site = hc_site(hc, sl, a.g);
  const int64_t vi = site * 3 + col;
  const bool odd = (__popc(sl) & 1) != 0;
  const int slot = a.rhs_per_slot > 0 ? r0 / a.rhs_per_slot : 0;
  const T* K = a.kinv + (int64_t)slot * a.slot_stride + hc * 2304;

  T xr[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    T v;
    v.x = 0; v.y = 0;
    if (act && r < nr) {
      v = a.in[(int64_t)(r0 + r) * a.in_stride + vi];
      if (a.eps_in && odd) { v.x = -v.x; v.y = -v.y; }
    }
    xr[r] = v;
  }
  T acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) { acc[r].x = 0; acc[r].y = 0; }
#pragma unroll 4
  for (int j = 0; j < 48; ++j) {
    T k;
    if (act) k = K[j * 48 + lane];
    else { k.x = 0; k.y = 0; }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T xj;
      xj.x = __shfl(xr[r].x, j, 64);
      xj.y = __shfl(xr[r].y, j, 64);
      cfma(acc[r], k, xj);
    }
  }
  if (!act) return;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) continue;
    T v = acc[r];
    if (a.eps_out && odd) { v.x = -v.x; v.y = -v.y; }
    a.out[(int64_t)(r0 + r) * a.out_stride + vi] = v;
  }
}

typedef __attribute__((ext_vector_type(4))) float f32x4;

// (B + m)^{-1} on 16 right-hand sides per wavefront on the FP32 matrix cores:
// per hypercube Y[48 x 16] = K[48 x 48] X[48 x 16] as four real products per
// 16x16x4 step (Re Y = Re K Re X - Im K Im X, Im Y = Re K Im X + Im K Re X).
// A fragments come straight from the column-major inverse (lane l: row
// 16 mt + l % 16, column 4 ks + l / 16); B fragments are the inputs of rhs
// l % 16 at row 4 ks + l / 16; lane l ends with rows 16 mt + 4 (l / 16) + t of
// rhs l % 16.
__global__ void __launch_bounds__(256) kd_apply_mfma_kernel(const KdArgs<float> a) {
  const int lane = threadIdx.x & 63;
  const int64_t hc = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  const int64_t nhc = a.g.V / 16;
  if (hc >= nhc) return;
  const int r0 = blockIdx.y * 16;
  const int rl = lane & 15, kq = lane >> 4;
  const int r = r0 + rl;
  const bool live = r < a.nrhs;
  const int slot = a.rhs_per_slot > 0 ? r0 / a.rhs_per_slot : 0;
  const float2* K = a.kinv + (int64_t)slot * a.slot_stride + hc * 2304;
  const float2* xin = a.in + (int64_t)(live ? r : 0) * a.in_stride;
  // site of local index sl: the hypercube's origin (even coordinates, so the
  // 2^4 cube never wraps) plus the unit offsets selected by the bits of sl
  const int64_t s0 = hc_site(hc, 0, a.g);
  const int64_t L0 = a.g.L[0], L01 = L0 * a.g.L[1], L012 = L01 * a.g.L[2];
  auto site_of = [&](int sl) -> int64_t {
    return s0 + (sl & 1) + ((sl >> 1) & 1) * L0 + ((sl >> 2) & 1) * L01 + (int64_t)(sl >> 3) * L012;
  };
  float bre[12], bim[12];
#pragma unroll
  for (int ks = 0; ks < 12; ++ks) {
    const int j = 4 * ks + kq;
    const int sl = j / 3, col = j - 3 * (j / 3);
    float2 v = make_float2(0.f, 0.f);
    if (live) {
      v = xin[site_of(sl) * 3 + col];
      if (a.eps_in && (__popc(sl) & 1)) { v.x = -v.x; v.y = -v.y; }
    }
    bre[ks] = v.x;
    bim[ks] = v.y;
  }
  float2* yout = a.out + (int64_t)(live ? r : 0) * a.out_stride;
#pragma unroll
  for (int mt = 0; mt < 3; ++mt) {
    f32x4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 12; ++ks) {
      const float2 k = K[(4 * ks + kq) * 48 + 16 * mt + rl];
      yr = __builtin_amdgcn_mfma_f32_16x16x4f32(k.x, bre[ks], yr, 0, 0, 0);
      yr = __builtin_amdgcn_mfma_f32_16x16x4f32(-k.y, bim[ks], yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_16x16x4f32(k.x, bim[ks], yi, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_16x16x4f32(k.y, bre[ks], yi, 0, 0, 0);
    }
    if (live) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = 16 * mt + 4 * kq + t;
        const int sl = i / 3, col = i - 3 * (i / 3);
        float2 v = make_float2(yr[t], yi[t]);
        if (a.eps_out && (__popc(sl) & 1)) { v.x = -v.x; v.y = -v.y; }
        yout[site_of(sl) * 3 + col] = v;
      }
    }
  }
}

// Blocks of four x-adjacent hypercubes: the 16-rhs input tile (per rhs, eight
// 192-byte rows of 8 sites) is loaded with 16-byte coalesced loads into LDS,
// the matrix-core product runs as above, and the result leaves through LDS
// with the same coalesced stores.  Needs (L0 / 2) % 4 == 0.
__global__ void __launch_bounds__(256) kd_apply_mfma_lds_kernel(const KdArgs<float> a) {
  __shared__ float2 xs[16][4][49];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t hc0 = xcd_block(blockIdx.x, gridDim.x) * 4;
  const int64_t hc = hc0 + wave;
  const int r0 = blockIdx.y * 16;
  const int slot = a.rhs_per_slot > 0 ? r0 / a.rhs_per_slot : 0;
  const int64_t L0 = a.g.L[0], L01 = L0 * a.g.L[1], L012 = L01 * a.g.L[2];
  const int64_t s0 = hc_site(hc0, 0, a.g);
  // the six 16-byte pieces of a thread are loaded before the first is used
  float4 vin[6];
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int it = tid + 256 * u;
    const int q = it % 12, rho = (it / 12) % 8, rr = it / 96;
    const int64_t rs = s0 + ((rho & 1) ? L0 : 0) + ((rho & 2) ? L01 : 0) + ((rho & 4) ? L012 : 0);
    vin[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r0 + rr < a.nrhs) vin[u] = *reinterpret_cast<const float4*>(a.in + (int64_t)(r0 + rr) * a.in_stride + rs * 3 + 2 * q);
  }
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int it = tid + 256 * u;
    const int q = it % 12, rho = (it / 12) % 8, rr = it / 96;
    const float4 v = vin[u];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int fl = 2 * q + e, xo = fl / 3, col = fl - 3 * (fl / 3);
      const int sl = (xo & 1) | (rho << 1);
      float2 c = e ? make_float2(v.z, v.w) : make_float2(v.x, v.y);
      if (a.eps_in && (__popc(sl) & 1)) { c.x = -c.x; c.y = -c.y; }
      xs[rr][xo >> 1][sl * 3 + col] = c;
    }
  }
  __syncthreads();
  const int rl = lane & 15, kq = lane >> 4;
  const float2* K = a.kinv + (int64_t)slot * a.slot_stride + hc * 2304;
  float bre[12], bim[12];
#pragma unroll
  for (int ks = 0; ks < 12; ++ks) {
    const float2 v = xs[rl][wave][4 * ks + kq];
    bre[ks] = v.x;
    bim[ks] = v.y;
  }
  f32x4 yr[3], yi[3];
  // A fragments of an m-tile are loaded together, the next m-tile's while
  // this one's products run
  float2 kf[2][12];
#pragma unroll
  for (int ks = 0; ks < 12; ++ks) kf[0][ks] = K[(4 * ks + kq) * 48 + rl];
#pragma unroll
  for (int mt = 0; mt < 3; ++mt) {
    if (mt + 1 < 3) {
#pragma unroll
      for (int ks = 0; ks < 12; ++ks) kf[(mt + 1) & 1][ks] = K[(4 * ks + kq) * 48 + 16 * (mt + 1) + rl];
    }
    yr[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    yi[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 12; ++ks) {
      const float2 k = kf[mt & 1][ks];
      yr[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(k.x, bre[ks], yr[mt], 0, 0, 0);
      yr[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(-k.y, bim[ks], yr[mt], 0, 0, 0);
      yi[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(k.x, bim[ks], yi[mt], 0, 0, 0);
      yi[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(k.y, bre[ks], yi[mt], 0, 0, 0);
    }
  }
  __syncthreads();   // every wavefront has read its inputs
#pragma unroll
  for (int mt = 0; mt < 3; ++mt)
#pragma unroll
    for (int t = 0; t < 4; ++t) xs[rl][wave][16 * mt + 4 * kq + t] = make_float2(yr[mt][t], yi[mt][t]);
  __syncthreads();
  for (int it = tid; it < 16 * 8 * 12; it += 256) {
    const int q = it % 12, rho = (it / 12) % 8, rr = it / 96;
    if (r0 + rr >= a.nrhs) continue;
    const int64_t rs = s0 + ((rho & 1) ? L0 : 0) + ((rho & 2) ? L01 : 0) + ((rho & 4) ? L012 : 0);
    float2 c[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int fl = 2 * q + e, xo = fl / 3, col = fl - 3 * (fl / 3);
      const int sl = (xo & 1) | (rho << 1);
      c[e] = xs[rr][xo >> 1][sl * 3 + col];
      if (a.eps_out && (__popc(sl) & 1)) { c[e].x = -c[e].x; c[e].y = -c[e].y; }
    }
    float4 o4 = make_float4(c[0].x, c[0].y, c[1].x, c[1].y);
    if (a.add) {   // out = (B+m)^{-1} in + add, add laid out as out
      const float4 ad = *reinterpret_cast<const float4*>(a.add + (int64_t)(r0 + rr) * a.out_stride + rs * 3 + 2 * q);
      o4.x += ad.x; o4.y += ad.y; o4.z += ad.z; o4.w += ad.w;
    }
    *reinterpret_cast<float4*>(a.out + (int64_t)(r0 + rr) * a.out_stride + rs * 3 + 2 * q) = o4;
  }
}

bool kd_lds_ok(const KdArgs<float>& a) {
  const int64_t nhc = a.g.V / 16;
  return a.nrhs >= 16 && (a.rhs_per_slot <= 0 || a.rhs_per_slot % 16 == 0) && (a.g.L[0] / 2) % 4 == 0 &&
         nhc % 4 == 0 && (uintptr_t)a.in % 16 == 0 && (uintptr_t)a.out % 16 == 0 &&
         (a.add == nullptr || (uintptr_t)a.add % 16 == 0) && a.in_stride % 2 == 0 && a.out_stride % 2 == 0;
}

template <typename R>
void launch_kd_apply(const KdArgs<R>& a, hipStream_t st) {
  if (a.nrhs <= 0) return;
  if (a.add != nullptr) {   // only the LDS-staged FP32 kernel adds
    if constexpr (sizeof(R) == 4) {
      if (!kd_lds_ok(a)) throw std::runtime_error("kd_apply: add needs the LDS-staged FP32 kernel's shapes");
    } else {
      throw std::runtime_error("kd_apply: add is FP32 only");
    }
  }
  const int64_t nhc = a.g.V / 16;
  const unsigned gx = (unsigned)((nhc + 3) / 4);
  const bool tile16 = sizeof(R) == 4 && a.nrhs >= 16 && (a.rhs_per_slot <= 0 || a.rhs_per_slot % 16 == 0);
  const bool tile8 = a.nrhs >= 8 && (a.rhs_per_slot <= 0 || a.rhs_per_slot % 8 == 0);
  const bool tile4 = a.nrhs >= 4 && (a.rhs_per_slot <= 0 || a.rhs_per_slot % 4 == 0);
  if (tile16) {
    dim3 grid(gx, (unsigned)((a.nrhs + 15) / 16));
    if constexpr (sizeof(R) == 4) {
      if ((a.g.L[0] / 2) % 4 == 0 && nhc % 4 == 0) kd_apply_mfma_lds_kernel<<<grid, 256, 0, st>>>(a);
      else kd_apply_mfma_kernel<<<grid, 256, 0, st>>>(a);
    }
    else kd_apply_kernel<R, 16><<<grid, 256, 0, st>>>(a);
  } else if (tile8) {
    dim3 grid(gx, (unsigned)((a.nrhs + 7) / 8));
    kd_apply_kernel<R, 8><<<grid, 256, 0, st>>>(a);
  } else if (tile4) {
    dim3 grid(gx, (unsigned)((a.nrhs + 3) / 4));
    kd_apply_kernel<R, 4><<<grid, 256, 0, st>>>(a);
  } else {
    dim3 grid(gx, (unsigned)a.nrhs);
    kd_apply_kernel<R, 1><<<grid, 256, 0, st>>>(a);
  }
}
template void launch_kd_apply<float>(const KdArgs<float>&, hipStream_t);
template void launch_kd_apply<double>(const KdArgs<double>&, hipStream_t);

}  // namespace mg
