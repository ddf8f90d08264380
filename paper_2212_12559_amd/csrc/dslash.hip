// Fine staggered / HISQ operator (Sec. 2.2, Sec. 3.1):
//   (D x)(x) = m x(x) + sum_mu [ W'_mu(x) x(x+mu) - W'_mu(x-mu)^dag x(x-mu)
//                              + N'_mu(x) x(x+3mu) - N'_mu(x-3mu)^dag x(x-3mu) ]
// with W' = (c1/2) eta_mu W and N' = (c3/2) eta_mu N folded in at set-up.
//
// One thread per output site; the links of a direction are stored as nine
// site-contiguous arrays so every load of a wavefront is one contiguous
// 512 B (FP32) or 1 KiB (FP64) segment; the backward links W'(x-mu) are the
// same arrays read at the neighbour, served from L2 / Infinity Cache.  A tile
// of NR right-hand sides shares every link load.
#include <stdexcept>

#include "kernels.hpp"

namespace mg {

template <typename R, int NR, bool NAIK, bool CB, bool PIECE>
__global__ void __launch_bounds__(256) dslash_kernel(const DslashArgs<R> a) {
  using T = cplx<R>;
  const int64_t V = a.g.V;
  const int64_t nout = CB ? V / 2 : V;
  // block b -> (site block, rhs tile) with the rhs tile fastest, after the
  // XCD renumbering: the tiles of a site block run back to back on one XCD
  // and share its links (and neighbour spinors) through that L2
  const int ntile = (a.nrhs + NR - 1) / NR;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int64_t sb = b / ntile;
  const int64_t tid = sb * blockDim.x + threadIdx.x;
  if (tid >= nout) return;
  const int r0 = (int)(b - sb * ntile) * NR;
  const int nr = (a.nrhs - r0) < NR ? (a.nrhs - r0) : NR;
  int c[4];
  int64_t s;
  if (CB) {
    const int hx = a.g.L[0] / 2;
    int64_t rest = tid / hx;
    c[1] = (int)(rest % a.g.L[1]); rest /= a.g.L[1];
    c[2] = (int)(rest % a.g.L[2]);
    c[3] = (int)(rest / a.g.L[2]);
    c[0] = 2 * (int)(tid % hx) + ((c[1] + c[2] + c[3] + a.parity) & 1);
    s = site_index(c, a.g);
  } else {
    s = tid;
    site_coords(s, a.g, c);
  }
  T acc[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < 3; ++i) { acc[r][i].x = 0; acc[r][i].y = 0; }

  const T* in = a.in + (int64_t)r0 * a.in_stride;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
    for (int h = 0; h < (NAIK ? 2 : 1); ++h) {
      const int hop = h ? 3 : 1;
      const T* L = (h ? a.lng : a.fat) + (int64_t)mu * 9 * V;
      // compressed long links: rows 0 and 1 and w; row 2 = w conj(row0 x row1)
      const bool cmp = h && a.lng_c != nullptr;
      const T* Lc = cmp ? a.lng_c + (int64_t)mu * 7 * V : nullptr;
      auto load_link = [&](T (&U)[9], int64_t q) {
        if (cmp) {
#pragma unroll
          for (int k = 0; k < 6; ++k) U[k] = Lc[k * V + q];
          const T w = Lc[6 * V + q];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const T p = cmul(U[j1], U[3 + j2]), m = cmul(U[j2], U[3 + j1]);
            T cc;
            cc.x = p.x - m.x;
            cc.y = m.y - p.y;   // conj of the cross product's component j
            U[6 + j] = cmul(w, cc);
          }
        } else {
#pragma unroll
          for (int k = 0; k < 9; ++k) U[k] = L[k * V + q];
        }
      };
      bool use_f = true, use_b = true;
      if (PIECE) {
        const int u = c[mu] % a.blk[mu];
        const int pf = (u + hop >= a.blk[mu]) ? 1 + 2 * mu : 0;
        const int pb = (u - hop < 0) ? 2 + 2 * mu : 0;
        use_f = (pf == a.piece);
        use_b = (pb == a.piece);
      }
      if (use_f) {
        const int64_t sf = site_shift(c, mu, hop, a.g);
        const int64_t vi = CB ? (sf >> 1) * 3 : sf * 3;
        T U[9];
        load_link(U, s);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r < nr) {
            const T* v = in + r * a.in_stride + vi;
            const T v0 = v[0], v1 = v[1], v2 = v[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              cfma(acc[r][i], U[3 * i + 0], v0);
              cfma(acc[r][i], U[3 * i + 1], v1);
              cfma(acc[r][i], U[3 * i + 2], v2);
            }
          }
        }
      }
      if (use_b) {
        const int64_t sb = site_shift(c, mu, -hop, a.g);
        const int64_t vi = CB ? (sb >> 1) * 3 : sb * 3;
        T U[9];
        load_link(U, sb);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r < nr) {
            const T* v = in + r * a.in_stride + vi;
            const T v0 = v[0], v1 = v[1], v2 = v[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              T t; t.x = 0; t.y = 0;
              cfmac(t, U[0 + i], v0);
              cfmac(t, U[3 + i], v1);
              cfmac(t, U[6 + i], v2);
              acc[r][i].x -= t.x;
              acc[r][i].y -= t.y;
            }
          }
        }
      }
    }
  }

#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) continue;
    if (CB) {
      const int64_t o = (int64_t)(r0 + r) * a.out_stride + (s >> 1) * 3;
      const R bc = a.b_coef;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T res;
        res.x = bc * acc[r][i].x;
        res.y = bc * acc[r][i].y;
        if (a.xs) {
          const T xv = a.xs[(int64_t)(r0 + r) * a.xs_stride + (s >> 1) * 3 + i];
          res.x = fma(a.a_coef, xv.x, res.x);
          res.y = fma(a.a_coef, xv.y, res.y);
        }
        a.out[o + i] = res;
      }
    } else {
      const R m = a.mass_rhs ? a.mass_rhs[r0 + r] : a.mass;
      const bool with_mass = !PIECE || a.piece == 0;
      const R sg = (a.eps_out && site_parity(c)) ? R(-1) : R(1);
      const T* xin = in + r * a.in_stride + s * 3;
      const int64_t o = (int64_t)(r0 + r) * a.out_stride + s * 3;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T res = acc[r][i];
        if (with_mass) {
          const T xv = xin[i];
          res.x = fma(m, xv.x, res.x);
          res.y = fma(m, xv.y, res.y);
        }
        res.x *= sg;
        res.y *= sg;
        a.out[o + i] = res;
      }
    }
  }
}

// One-hop full-lattice stencil with the in-plane neighbours taken from LDS: a
// workgroup owns RB = 256 / L0 consecutive x-rows (a y range at fixed z, t)
// and NR right-hand sides.  The rows y0 - 1 .. y0 + RB of every right-hand side
// are staged with 16-byte loads, so the own, +-x and +-y spinors come from LDS
// and only the +-z, +-t neighbours and the links are read per site (the
// per-site reads are what bound the plain kernel: address processing, not
// bytes).
// OFF: only the hops that leave the site's 2^4 hypercube (forward where x_mu
// is odd, backward where it is even) and no mass term; in z and t the choice
// is uniform over a workgroup's plane, so half of the per-site gathers go.
template <int NR, bool PAIRS, bool OFF>
__global__ void __launch_bounds__(256) dslash_plane_kernel(const DslashArgs<float> a) {
  using T = float2;
  extern __shared__ float4 lds4[];
  T* xs = reinterpret_cast<T*>(lds4);   // [NR][RB + 2][L0 * 3]
  const int L0 = a.g.L[0], L1 = a.g.L[1], L2 = a.g.L[2];
  const int RB = 256 / L0, rowc = 3 * L0;
  const int64_t V = a.g.V;
  const int ntile = (a.nrhs + NR - 1) / NR;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int64_t pb = b / ntile;
  const int r0 = (int)(b - pb * ntile) * NR;
  const int nr = (a.nrhs - r0) < NR ? (a.nrhs - r0) : NR;
  const int nyb = L1 / RB;
  const int yb = (int)(pb % nyb);
  const int64_t zt = pb / nyb;
  const int z = (int)(zt % L2), t = (int)(zt / L2);
  const int y0 = yb * RB;
  const int nq = rowc / 2;   // 16-byte pieces per row (L0 even)
  // a thread has the loads of up to kPlaneQ pieces in flight before it waits
  constexpr int kPlaneQ = 8;
  const int npiece = NR * (RB + 2) * nq;
  for (int it0 = threadIdx.x; it0 < npiece; it0 += kPlaneQ * 256) {
    float4 v[kPlaneQ];
#pragma unroll
    for (int u = 0; u < kPlaneQ; ++u) {
      const int it = it0 + u * 256;
      const int q = it % nq, rw = (it / nq) % (RB + 2), rr = it / (nq * (RB + 2));
      const int y = (y0 - 1 + rw + L1) % L1;
      const int64_t rs = (((int64_t)t * L2 + z) * L1 + y) * L0;
      v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (it < npiece && rr < nr)
        v[u] = *reinterpret_cast<const float4*>(a.in + (int64_t)(r0 + rr) * a.in_stride + rs * 3 + 2 * q);
    }
#pragma unroll
    for (int u = 0; u < kPlaneQ; ++u) {
      const int it = it0 + u * 256;
      if (it < npiece) {
        const int q = it % nq, rw = (it / nq) % (RB + 2), rr = it / (nq * (RB + 2));
        T* d = xs + ((int64_t)rr * (RB + 2) + rw) * rowc + 2 * q;
        d[0] = make_float2(v[u].x, v[u].y);
        d[1] = make_float2(v[u].z, v[u].w);
      }
    }
  }
  __syncthreads();
  const int x = threadIdx.x % L0, yr = threadIdx.x / L0;
  int c[4] = {x, y0 + yr, z, t};
  const int64_t s = site_index(c, a.g);
  // LDS position of a spinor in the staged rows
  auto at = [&](int r, int row, int col) -> const T* { return xs + ((int64_t)r * (RB + 2) + row) * rowc + col * 3; };
  T acc[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < 3; ++i) { acc[r][i].x = 0; acc[r][i].y = 0; }
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const T* L = a.fat + (int64_t)mu * 9 * V;
    const float4* Lp = a.fat_pairs + (int64_t)mu * 5 * V;
    // the nine link elements at site q: nine 8-byte loads, or five 16-byte ones
    auto load_link = [&](T (&U)[9], int64_t q) {
      if constexpr (PAIRS) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const float4 w = Lp[k * V + q];
          U[2 * k] = make_float2(w.x, w.y);
          if (2 * k + 1 < 9) U[2 * k + 1] = make_float2(w.z, w.w);
        }
      } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) U[k] = L[k * V + q];
      }
    };
    const bool odd = (c[mu] & 1) != 0;
    if (!OFF || odd) {   // forward hop: W'(x) x(x + mu)
      const int64_t sf = mu >= 2 ? site_shift(c, mu, 1, a.g) : 0;
      T U[9];
      load_link(U, s);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nr) {
          T v0, v1, v2;
          if (mu < 2) {
            const T* p = mu == 0 ? at(r, yr + 1, (x + 1) % L0) : at(r, yr + 2, x);
            v0 = p[0]; v1 = p[1]; v2 = p[2];
          } else {
            const T* p = a.in + (int64_t)(r0 + r) * a.in_stride + sf * 3;
            v0 = p[0]; v1 = p[1]; v2 = p[2];
          }
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            cfma(acc[r][i], U[3 * i + 0], v0);
            cfma(acc[r][i], U[3 * i + 1], v1);
            cfma(acc[r][i], U[3 * i + 2], v2);
          }
        }
      }
    }
    if (!OFF || !odd) {   // backward hop: -W'(x - mu)^dag x(x - mu)
      const int64_t sb = site_shift(c, mu, -1, a.g);
      T U[9];
      load_link(U, sb);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nr) {
          T v0, v1, v2;
          if (mu < 2) {
            const T* p = mu == 0 ? at(r, yr + 1, (x + L0 - 1) % L0) : at(r, yr, x);
            v0 = p[0]; v1 = p[1]; v2 = p[2];
          } else {
            const T* p = a.in + (int64_t)(r0 + r) * a.in_stride + sb * 3;
            v0 = p[0]; v1 = p[1]; v2 = p[2];
          }
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            T tt; tt.x = 0; tt.y = 0;
            cfmac(tt, U[0 + i], v0);
            cfmac(tt, U[3 + i], v1);
            cfmac(tt, U[6 + i], v2);
            acc[r][i].x -= tt.x;
            acc[r][i].y -= tt.y;
          }
        }
      }
    }
  }
  const float sg = (a.eps_out && site_parity(c)) ? -1.f : 1.f;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) continue;
    const float m = a.mass_rhs ? a.mass_rhs[r0 + r] : a.mass;
    const T* xin = at(r, yr + 1, x);
    const int64_t o = (int64_t)(r0 + r) * a.out_stride + s * 3;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T res = acc[r][i];
      if (!OFF) {
        res.x = fmaf(m, xin[i].x, res.x);
        res.y = fmaf(m, xin[i].y, res.y);
      }
      res.x *= sg;
      res.y *= sg;
      a.out[o + i] = res;
    }
  }
}

template <int NR>
static bool plane_fits(const DslashArgs<float>& a) {
  const int L0 = a.g.L[0];
  if (L0 > 256 || 256 % L0 || a.g.L[1] % (256 / L0)) return false;
  return (size_t)NR * (256 / L0 + 2) * 3 * L0 * sizeof(float2) <= 65536;
}

template <int NR>
static bool launch_plane(const DslashArgs<float>& a, hipStream_t st) {
  if (!plane_fits<NR>(a)) return false;
  const int L0 = a.g.L[0];
  const int RB = 256 / L0;
  const size_t lds = (size_t)NR * (RB + 2) * 3 * L0 * sizeof(float2);
  const int64_t nplane = a.g.V / 256;
  dim3 grid((unsigned)(nplane * ((a.nrhs + NR - 1) / NR)));
  if (a.off_cube) {
    if (a.fat_pairs) dslash_plane_kernel<NR, true, true><<<grid, 256, lds, st>>>(a);
    else dslash_plane_kernel<NR, false, true><<<grid, 256, lds, st>>>(a);
  } else {
    if (a.fat_pairs) dslash_plane_kernel<NR, true, false><<<grid, 256, lds, st>>>(a);
    else dslash_plane_kernel<NR, false, false><<<grid, 256, lds, st>>>(a);
  }
  return true;
}

bool dslash_plane_ok(const DslashArgs<float>& a) {
  if (a.nrhs <= 0 || a.g.V <= 0 || (uintptr_t)a.in % 16 != 0 || a.in_stride % 2 != 0) return false;
  return a.nrhs == 1 ? plane_fits<1>(a) : plane_fits<4>(a);
}

bool launch_dslash_plane(const DslashArgs<float>& a, hipStream_t st) {
  if (!dslash_plane_ok(a)) return false;
  return a.nrhs == 1 ? launch_plane<1>(a, st) : launch_plane<4>(a, st);
}

template <typename R, int NR>
static void launch_nr(const DslashArgs<R>& a, bool naik, bool cb, bool piece, hipStream_t st) {
  const int64_t nout = cb ? a.g.V / 2 : a.g.V;
  dim3 grid((unsigned)((nout + 255) / 256 * ((a.nrhs + NR - 1) / NR)));
  dim3 block(256);
  if (piece) {
    if (naik) dslash_kernel<R, NR, true, false, true><<<grid, block, 0, st>>>(a);
    else dslash_kernel<R, NR, false, false, true><<<grid, block, 0, st>>>(a);
  } else if (cb) {
    if (naik) dslash_kernel<R, NR, true, true, false><<<grid, block, 0, st>>>(a);
    else dslash_kernel<R, NR, false, true, false><<<grid, block, 0, st>>>(a);
  } else {
    if (naik) dslash_kernel<R, NR, true, false, false><<<grid, block, 0, st>>>(a);
    else dslash_kernel<R, NR, false, false, false><<<grid, block, 0, st>>>(a);
  }
}

template <typename R>
void launch_dslash(const DslashArgs<R>& a, bool naik, bool cb, bool piece, hipStream_t st) {
  if (a.nrhs <= 0 || a.g.V <= 0) return;
  if (a.off_cube) throw std::runtime_error("dslash: the off-cube form is the plane kernel's (launch_dslash_plane)");
  if constexpr (sizeof(R) == 4) {
    // one-hop FP32 full-lattice stencil: in-plane neighbours through LDS
    if (!naik && !cb && !piece && (uintptr_t)a.in % 16 == 0 && a.in_stride % 2 == 0) {
      bool done;
      // 4-rhs tiles: at 8 the LDS tile (61 KB) leaves two workgroups per CU
      if (a.nrhs == 1) done = launch_plane<1>(a, st);
      else done = launch_plane<4>(a, st);
      if (done) return;
    }
  }
  if (a.nrhs == 1) launch_nr<R, 1>(a, naik, cb, piece, st);
  else if (a.nrhs < 8) launch_nr<R, 4>(a, naik, cb, piece, st);
  else launch_nr<R, 8>(a, naik, cb, piece, st);
}
template void launch_dslash<float>(const DslashArgs<float>&, bool, bool, bool, hipStream_t);
template void launch_dslash<double>(const DslashArgs<double>&, bool, bool, bool, hipStream_t);

// Canonical links [4][T][Z][Y][X][3][3] (complex128) -> internal structure of
// arrays with (c/2) eta_mu(x) folded in; FP64 and FP32 copies, and optionally
// the FP32 elements in pairs (one 16-byte load for two of them).
__global__ void pack_links_kernel(const double2* __restrict__ src, double2* __restrict__ d64,
                                  float2* __restrict__ d32, float4* __restrict__ d32p, Geom g, double coef) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 4 * g.V) return;
  const int mu = (int)(tid / g.V);
  const int64_t s = tid - (int64_t)mu * g.V;
  int c[4];
  site_coords(s, g, c);
  const double f = coef * stag_eta(c, mu);
  for (int k = 0; k < 9; ++k) {
    const double2 v = src[tid * 9 + k];
    const double2 w = make_double2(f * v.x, f * v.y);
    d64[((int64_t)mu * 9 + k) * g.V + s] = w;
    if (d32) d32[((int64_t)mu * 9 + k) * g.V + s] = make_float2((float)w.x, (float)w.y);
  }
  if (d32p) {
    for (int q = 0; q < 5; ++q) {
      const double2 v0 = src[tid * 9 + 2 * q];
      const double2 v1 = 2 * q + 1 < 9 ? src[tid * 9 + 2 * q + 1] : make_double2(0.0, 0.0);
      d32p[((int64_t)mu * 5 + q) * g.V + s] =
          make_float4((float)(f * v0.x), (float)(f * v0.y), (float)(f * v1.x), (float)(f * v1.y));
    }
  }
}

__global__ void pack_naik_compressed_kernel(const double2* __restrict__ src, double2* __restrict__ d64,
                                            float2* __restrict__ d32, Geom g, double coef,
                                            unsigned long long* dev_max) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dev = 0.0;
  if (tid < 4 * g.V) {
    const int mu = (int)(tid / g.V);
    const int64_t s = tid - (int64_t)mu * g.V;
    int c[4];
    site_coords(s, g, c);
    const double f = coef * stag_eta(c, mu);
    double2 N[9];
    for (int k = 0; k < 9; ++k) N[k] = src[tid * 9 + k];
    // unitarity: |(N N^dag)_ij - delta_ij|
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double2 t = make_double2(i == j ? -1.0 : 0.0, 0.0);
        for (int k = 0; k < 3; ++k) cfmac(t, N[3 * j + k], N[3 * i + k]);   // N_ik conj(N_jk)
        dev = fmax(dev, fmax(fabs(t.x), fabs(t.y)));
      }
    // det N along the first row: sum_j N_0j (N_1,j+1 N_2,j+2 - N_1,j+2 N_2,j+1)
    double2 det = make_double2(0.0, 0.0);
    for (int j = 0; j < 3; ++j) {
      const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      const double2 p = cmul(N[3 + j1], N[6 + j2]), m = cmul(N[3 + j2], N[6 + j1]);
      cfma(det, N[j], make_double2(p.x - m.x, p.y - m.y));
    }
    const double2 w = make_double2(det.x / f, det.y / f);
    for (int k = 0; k < 7; ++k) {
      const double2 v = k < 6 ? make_double2(f * N[k].x, f * N[k].y) : w;
      d64[((int64_t)mu * 7 + k) * g.V + s] = v;
      d32[((int64_t)mu * 7 + k) * g.V + s] = make_float2((float)v.x, (float)v.y);
    }
  }
  for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o, 64));
  if ((threadIdx.x & 63) == 0 && dev > 0.0) atomicMax(dev_max, (unsigned long long)__double_as_longlong(dev));
}

void launch_pack_naik_compressed(const double2* src, double2* d64, float2* d32, const Geom& g, double coef,
                                 unsigned long long* dev_max, hipStream_t st) {
  const int64_t n = 4 * g.V;
  pack_naik_compressed_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, d64, d32, g, coef, dev_max);
}

void launch_pack_links(const double2* src, double2* d64, float2* d32, float4* d32p, const Geom& g, double coef,
                       hipStream_t st) {
  const int64_t n = 4 * g.V;
  pack_links_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, d64, d32, d32p, g, coef);
}

// Index tables of the fine lattice exactly as the kernels compute them, for
// the bit-exact comparison with the oracle's definitions.  Per site, int32:
//   [0..3] x+mu  [4..7] x-mu  [8..11] x+3mu  [12..15] x-3mu
//   [16] eta bits (bit mu set when eta_mu = -1)  [17] epsilon (+1/-1)
//   [18] hypercube  [19] hypercube-local index  [20] aggregate  [21] chirality
__global__ void export_fine_index_kernel(int32_t* __restrict__ out, Geom g, Agg A) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  int c[4];
  site_coords(s, g, c);
  int32_t* o = out + s * 22;
  for (int mu = 0; mu < 4; ++mu) {
    o[mu] = (int32_t)site_shift(c, mu, 1, g);
    o[4 + mu] = (int32_t)site_shift(c, mu, -1, g);
    o[8 + mu] = (int32_t)site_shift(c, mu, 3, g);
    o[12 + mu] = (int32_t)site_shift(c, mu, -3, g);
  }
  int bits = 0;
  for (int mu = 0; mu < 4; ++mu) bits |= (stag_eta(c, mu) < 0 ? 1 : 0) << mu;
  o[16] = bits;
  o[17] = site_parity(c) ? -1 : 1;
  int64_t hc;
  int sl;
  hc_of_site(c, g, &hc, &sl);
  o[18] = (int32_t)hc;
  o[19] = sl;
  int ac[4];
  for (int mu = 0; mu < 4; ++mu) ac[mu] = c[mu] / A.b[mu];
  o[20] = (int32_t)(ac[0] + A.cd[0] * (ac[1] + A.cd[1] * (ac[2] + A.cd[2] * ac[3])));
  o[21] = site_parity(c);
}

void launch_export_fine_index(int32_t* out, const Geom& g, const Agg& A, hipStream_t st) {
  export_fine_index_kernel<<<(unsigned)((g.V + 255) / 256), 256, 0, st>>>(out, g, A);
}

// Multiply by epsilon(x) (per site sign), in place or out of place.
template <typename T>
__global__ void eps_kernel(T* out, const T* in, Geom g, int64_t nrhs) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= g.V * 3 * nrhs) return;
  const int64_t s = (tid / 3) % g.V;
  int c[4];
  site_coords(s, g, c);
  T v = in[tid];
  if (site_parity(c)) { v.x = -v.x; v.y = -v.y; }
  out[tid] = v;
}
template <typename T>
void launch_eps(T* out, const T* in, const Geom& g, int nrhs, hipStream_t st) {
  const int64_t n = g.V * 3 * nrhs;
  eps_kernel<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(out, in, g, nrhs);
}
template void launch_eps<float2>(float2*, const float2*, const Geom&, int, hipStream_t);
template void launch_eps<double2>(double2*, const double2*, const Geom&, int, hipStream_t);

}  // namespace mg

namespace mg {

// Full-lattice batch [nrhs][V][3] <-> checkerboard halves [nrhs][V/2][3]
// (index site >> 1 within each parity).
__global__ void cb_split_kernel(const double2* __restrict__ full, double2* __restrict__ ev,
                                double2* __restrict__ od, Geom g, int nrhs) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= g.V * 3 * nrhs) return;
  const int64_t r = tid / (g.V * 3);
  const int64_t e = tid - r * g.V * 3;
  const int64_t s = e / 3;
  const int col = (int)(e - s * 3);
  int c[4];
  site_coords(s, g, c);
  double2* dst = site_parity(c) ? od : ev;
  dst[r * (g.V / 2) * 3 + (s >> 1) * 3 + col] = full[tid];
}
__global__ void cb_merge_kernel(double2* __restrict__ full, const double2* __restrict__ ev,
                                const double2* __restrict__ od, Geom g, int nrhs) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= g.V * 3 * nrhs) return;
  const int64_t r = tid / (g.V * 3);
  const int64_t e = tid - r * g.V * 3;
  const int64_t s = e / 3;
  const int col = (int)(e - s * 3);
  int c[4];
  site_coords(s, g, c);
  const double2* src = site_parity(c) ? od : ev;
  full[tid] = src[r * (g.V / 2) * 3 + (s >> 1) * 3 + col];
}
void launch_cb_split(const double2* full, double2* ev, double2* od, const Geom& g, int nrhs, hipStream_t st) {
  const int64_t n = g.V * 3 * nrhs;
  cb_split_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(full, ev, od, g, nrhs);
}
void launch_cb_merge(double2* full, const double2* ev, const double2* od, const Geom& g, int nrhs, hipStream_t st) {
  const int64_t n = g.V * 3 * nrhs;
  cb_merge_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(full, ev, od, g, nrhs);
}

}  // namespace mg

namespace mg {

// Fermion force outer products, summed over right-hand sides (HMC use of the
// solver, Sec. 4.2): for S = sum_r phi_r^dag (D^dag D)^{-1} phi_r with
// X = (D^dag D)^{-1} phi, Y = D X,
//   G^W_mu(x) = -c1 eta_mu(x) sum_r [ Y(x) X(x+mu)^dag  - X(x) Y(x+mu)^dag  ]
//   G^N_mu(x) = -c3 eta_mu(x) sum_r [ Y(x) X(x+3mu)^dag - X(x) Y(x+3mu)^dag ]
// in PyTorch's gradient convention, written in the canonical link layout
// [mu][site][3][3]; accumulate adds into the output.
__global__ void __launch_bounds__(256) force_kernel(const double2* __restrict__ X, const double2* __restrict__ Y,
                                                    double2* __restrict__ gw, double2* __restrict__ gn, Geom g,
                                                    int nrhs, double c1, double c3, int accumulate) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 4 * g.V) return;
  const int mu = (int)(tid / g.V);
  const int64_t s = tid - (int64_t)mu * g.V;
  int c[4];
  site_coords(s, g, c);
  const double eta = (double)stag_eta(c, mu);
  for (int h = 0; h < 2; ++h) {
    double2* out = h ? gn : gw;
    if (!out) continue;
    const double coef = -(h ? c3 : c1) * eta;
    const int64_t sn = site_shift(c, mu, h ? 3 : 1, g);
    double2 acc[9];
    for (int k = 0; k < 9; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int r = 0; r < nrhs; ++r) {
      const double2* xr = X + (int64_t)r * g.V * 3;
      const double2* yr = Y + (int64_t)r * g.V * 3;
      double2 xa[3], ya[3], xb[3], yb[3];
      for (int i = 0; i < 3; ++i) {
        xa[i] = xr[s * 3 + i]; ya[i] = yr[s * 3 + i];
        xb[i] = xr[sn * 3 + i]; yb[i] = yr[sn * 3 + i];
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          // Y_i(x) conj(X_j(x+h)) - X_i(x) conj(Y_j(x+h))
          double2 t = make_double2(0.0, 0.0);
          cfmac(t, xb[j], ya[i]);
          double2 u = make_double2(0.0, 0.0);
          cfmac(u, yb[j], xa[i]);
          acc[3 * i + j].x += t.x - u.x;
          acc[3 * i + j].y += t.y - u.y;
        }
    }
    double2* o = out + tid * 9;
    for (int k = 0; k < 9; ++k) {
      double2 v = make_double2(coef * acc[k].x, coef * acc[k].y);
      if (accumulate) { v.x += o[k].x; v.y += o[k].y; }
      o[k] = v;
    }
  }
}

void launch_force(const double2* X, const double2* Y, double2* gw, double2* gn, const Geom& g, int nrhs, double c1,
                  double c3, int accumulate, hipStream_t st) {
  const int64_t n = 4 * g.V;
  force_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(X, Y, gw, gn, g, nrhs, c1, c3, accumulate);
}

}  // namespace mg
