// Hierarchy set-up (Sec. 2.1, Sec. 2.3, Table 1): links to the internal
// layout, the KD block inverse at mass0, near-null vectors (imported, or CGNE
// on the level's own operator), chiral doubling + FP64 block
// orthonormalisation, and the Galerkin coarse operators.
#include <cmath>
#include <cstring>

#include "mg.hpp"

namespace mg {

#define HIPCHK(x)                                                                 \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) throw Error{MG_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

static void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{MG_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e)};
}

void Ctx::setup(const void* fat, const void* naik, const void* const* nvs) {
  launch_pack_links((const double2*)fat, fat64, fat32, fat32p, g0, 0.5 * P.c1, st);
  check_launch();
  if (P.c3 != 0.0) {
    pack_naik(naik);
    check_launch();
  }
  ensure_kd({P.mass0});
  rhs_per_slot = 0;
  setup_phase = true;
  for (int l = 0; l < P.nagg; ++l) {
    build_level(l, nvs ? nvs[l] : nullptr);   // near-null vectors from the Galerkin operator of level l + 1
    if (P.coarse_op == 1 && l > 0) {
      // the previous level is preconditioned only now (its Galerkin operator
      // gave this level's near-null vectors); rebuild this level's links from it
      precondition_links(l - 1);
      finish_links(l - 1);
      galerkin(l);
    }
    if (P.coarse_op == 1 && l == P.nagg - 1) precondition_links(l);
    finish_links(l);
  }
  if (defl_k > 0) build_deflation(nvs && P.deflate_import ? nvs[P.nagg] : nullptr);
  if (P.coarsest_solver == 1) estimate_lambda_max();
  if (P.coarsest_solver == 2) build_direct();
  setup_phase = false;
  HIPCHK(hipStreamSynchronize(st));
}

// Exact coarsest solve (coarsest_solver 2): the dense matrix of the coarsest
// operator, assembled from its FP64 links (block-preconditioned ones when
// coarse_op is 1, matching the X^{-1} b of the level solve), inverted by
// Gauss-Jordan with partial pivoting in FP64.
void Ctx::build_direct() {
  const int lc = P.nagg - 1;
  const int ns = ncoarse[lc];
  const int64_t n = gc[lc].V * ns;
  const size_t mb = ((size_t)2 * n * n * 16 + 255) & ~(size_t)255;
  const size_t fb = ((size_t)n * 16 + 255) & ~(size_t)255;
  double2* M = (double2*)scratch_base;
  double2* f = (double2*)(scratch_base + mb);
  int* piv = (int*)(scratch_base + mb + fb);
  double2* pinv = (double2*)(scratch_base + mb + fb + 256);
  int* flag = (int*)((char*)status_dev + 160);
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), st));
  dense_coarsest_inverse(cl64[lc], gc[lc], ns, M, f, piv, pinv, flag, dinv64, dinv32, st);
  check_launch();
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bad) throw Error{MG_E_RANK, "the coarsest operator is singular: no direct coarsest solve"};
}

// Largest eigenvalue modulus of the coarsest operator by 30 power iterations
// from a seeded random vector; the Chebyshev basis of the CA-GCR coarsest
// solver then maps [0, 1.05 lambda_max] onto [-1, 1].
void Ctx::estimate_lambda_max() {
  const int lc = nlev - 1;
  LevelBufs& B = L[lc];
  const int64_t n = B.n;
  const Vec &v = B.z[0], &w = B.q[0];
  if (B.prec == P64) launch_random_normal<double2>((double2*)v.p, n, P.seed + 4242ull, st);
  else launch_random_normal<float2>((float2*)v.p, n, P.seed + 4242ull, st);
  check_launch();
  std::vector<double> nv, nw;
  double lam = 1.0;
  for (int it = 0; it < 30; ++it) {
    norms_host(B.prec, n, 1, v.p, slot(lc, kSlotNorm), nv);
    apply_level(lc, w, v, 1);
    norms_host(B.prec, n, 1, w.p, slot(lc, kSlotNorm), nw);
    if (!(nv[0] > 0.0) || !(nw[0] > 0.0) || !std::isfinite(nw[0])) break;
    lam = nw[0] / nv[0];
    lincomb(B.prec, n, 1, v.p, {{w.p, nullptr}}, {}, {make_double2(1.0 / nw[0], 0.0)});
  }
  cheb_c = cheb_d = 0.5 * 1.05 * lam;
  // Per-step growth of the Chebyshev basis on this operator, from the same
  // recurrence run on a random vector (every eigencomponent present, so an
  // upper estimate for the residuals of the solves): for a non-Hermitian
  // operator the spectrum leaves the real interval and T_j grows there.  The
  // solver divides basis vector j by gamma^j, which spans the same Krylov
  // space and keeps the vectors of order one (16-bit stencil inputs in range).
  // The pair (z_j, z_{j-1}) is renormalised every step; gamma is the
  // geometric mean of the normalisations.
  cheb_g = 1.0;
  const int s = P.coarsest_maxiter;
  if (s > 2) {
    const Vec* zm = &B.z[0];
    const Vec* zc = &B.z[1];
    const Vec* zn = &B.z[2];
    const double c = cheb_c, d = cheb_d;
    if (B.prec == P64) launch_random_normal<double2>((double2*)zm->p, n, P.seed + 4343ull, st);
    else launch_random_normal<float2>((float2*)zm->p, n, P.seed + 4343ull, st);
    check_launch();
    norms_host(B.prec, n, 1, zm->p, slot(lc, kSlotNorm), nv);
    if (!(nv[0] > 0.0)) return;
    lincomb(B.prec, n, 1, zm->p, {{zm->p, nullptr}}, {}, {make_double2(1.0 / nv[0], 0.0)});
    apply_level(lc, w, *zm, 1);
    lincomb(B.prec, n, 1, zc->p, {{w.p, nullptr}, {zm->p, nullptr}}, {},
            {make_double2(1.0 / d, 0.0), make_double2(-c / d, 0.0)});
    double lg = 0.0;
    for (int j = 1; j < s - 1; ++j) {
      norms_host(B.prec, n, 1, zc->p, slot(lc, kSlotNorm), nv);
      if (!(nv[0] > 0.0) || !std::isfinite(nv[0])) return;
      lg += std::log(nv[0]);
      lincomb(B.prec, n, 1, zc->p, {{zc->p, nullptr}}, {}, {make_double2(1.0 / nv[0], 0.0)});
      lincomb(B.prec, n, 1, zm->p, {{zm->p, nullptr}}, {}, {make_double2(1.0 / nv[0], 0.0)});
      apply_level(lc, w, *zc, 1);
      lincomb(B.prec, n, 1, zn->p, {{w.p, nullptr}, {zc->p, nullptr}, {zm->p, nullptr}}, {},
              {make_double2(2.0 / d, 0.0), make_double2(-2.0 * c / d, 0.0), make_double2(-1.0, 0.0)});
      std::swap(zm, zc);
      std::swap(zc, zn);
    }
    norms_host(B.prec, n, 1, zc->p, slot(lc, kSlotNorm), nv);
    if (!(nv[0] > 0.0) || !std::isfinite(nv[0])) return;
    lg += std::log(nv[0]);
    cheb_g = std::max(1.0, std::exp(lg / (s - 1)));
  }
}

// Naik links: the full FP64 / FP32 copies, and the 13-real form (Sec. 3.1)
// that the stencil uses when every link is unitary to 1e-10.
void Ctx::pack_naik(const void* naik) {
  launch_pack_links((const double2*)naik, lng64, lng32, nullptr, g0, 0.5 * P.c3, st);
  unsigned long long* dmax = (unsigned long long*)((char*)status_dev + 128);
  HIPCHK(hipMemsetAsync(dmax, 0, sizeof(unsigned long long), st));
  launch_pack_naik_compressed((const double2*)naik, lng64c, lng32c, g0, 0.5 * P.c3, dmax, st);
  check_launch();
  unsigned long long bits = 0;
  HIPCHK(hipMemcpyAsync(&bits, dmax, sizeof(bits), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double dev;
  std::memcpy(&dev, &bits, sizeof(dev));
  naik_compressed = dev <= 1e-10;
}

void Ctx::build_level(int l, const void* imp) {
  const Agg& a = A[l];
  const int64_t nflat = a.nagg * 2 * a.nrows;
  if (imp && !P.cgne_start_import) {
    HIPCHK(hipMemcpyAsync(nv[l], imp, (size_t)a.nvec * nflat * 16, hipMemcpyDeviceToDevice, st));
  } else {
    cgne_null(l, a.nvec, nflat, P.setup_maxiter[l], P.setup_tol[l], nv[l], (const double2*)imp);
  }
  launch_gather_null(nv[l], nflat, pp64[l], a, st);
  check_launch();
  HIPCHK(hipMemsetAsync(status_dev, 0, sizeof(int), st));
  launch_block_orth(pp64[l], a, status_dev, st);
  check_launch();
  int status = 0;
  HIPCHK(hipMemcpyAsync(&status, status_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (status) throw Error{MG_E_RANK, "block orthonormalisation: near-null vectors are rank deficient on a block"};
  launch_p_layouts(pp64[l], pr64[l], pr32[l], pp32[l], a, st);
  check_launch();
  galerkin(l);
}

// Near-null vectors by CGNE on A phi = 0 from seeded random starts (or the
// caller's starting vectors, FP64), all nvec
// vectors as one batch (Sec. 2.1, Table 1: CGNE to tol or maxiter):
//   t = A^dag p, alpha = |r|^2 / |t|^2, phi += alpha t, r -= alpha A t, ...
// l = 0: A = (B + m0)^{-1} D, A^dag = eps D (B + m0)^{-1} eps.
// l >= 1: the coarse operator of level l + 1 and its adjoint stencil.
// nvec vectors of n entries; the result goes to `out` (FP64) and stays in
// the first scratch block in the level's precision.
void Ctx::cgne_null(int l, int nvec, int64_t n, int maxiter, double tol, double2* out, const double2* start) {
  const int nv_ = nvec;
  const int prec = L[l + 1].prec;
  const int lc = l - 1;   // coarse-level index of the operator for l >= 1
  const size_t vb = ((size_t)nv_ * n * csize(prec) + 255) & ~(size_t)255;
  char* base = scratch_base;
  void* phi = base;
  void* r = base + vb;
  void* p = base + 2 * vb;
  void* t = base + 3 * vb;
  void* At = base + 4 * vb;
  void* tmp = base + 5 * vb;
  // past the six CGNE vectors and the three Galerkin vectors
  void* dagl = nullptr;
  uint16_t* dag16 = nullptr;
  if (l >= 1) {
    const size_t gb = ((size_t)n * 16 + 255) & ~(size_t)255;
    dagl = base + 6 * vb + 3 * gb;
    const int nc = ncoarse[lc];
    if (prec == P64) launch_dagger_links<double2>(cl64[lc], (double2*)dagl, gc[lc], nc, st);
    else launch_dagger_links<float2>(cl32[lc], (float2*)dagl, gc[lc], nc, st);
    check_launch();
    if (fmt16 >= 0) {
      // 16-bit operator: the set-up iterates with the links the solver applies
      dag16 = (uint16_t*)((char*)dagl + (((size_t)gc[lc].V * 9 * nc * nc * csize(prec) + 255) & ~(size_t)255));
      launch_swizzle_links<float2>((const float2*)dagl, dag16, gc[lc].V, nc, fmt16, 1.0 / cl16_inv_scale[lc], st);
      check_launch();
    }
  }
  auto A_apply = [&](void* out, const void* in, bool dag) {
    if (l == 0) {
      const bool nk = P.kd_naik != 0;
      if (!dag) {
        apply_kd_operator(prec, out, in, tmp, nv_, nullptr, P.mass0, 0);
      } else {
        apply_KD(prec, tmp, in, nv_, true, false, 0);
        apply_D(prec, out, tmp, nv_, nk, nullptr, P.mass0, true);
      }
    } else if (fmt16 >= 0 && prec == P32) {
      setup_phase = false;   // the 16-bit matrix-core stencil, forward or adjoint links
      if (!dag) {
        apply_coarse(l + 1, prec, out, in, nv_, false);
      } else {
        CoarseMfmaArgs c{};
        c.out = (float2*)out; c.in = (const float2*)in; c.links = dag16;
        c.g = gc[lc]; c.n = ncoarse[lc]; c.in_stride = c.out_stride = gc[lc].V * ncoarse[lc]; c.nrhs = nv_;
        c.inv_scale = cl16_inv_scale[lc];
        launch_coarse_mfma(c, fmt16, st);
        check_launch();
      }
      setup_phase = true;
    } else if (!dag) {
      apply_coarse(l + 1, prec, out, in, nv_, false);
    } else {
      // the adjoint stencil through its explicit links (coalesced)
      const int nc = ncoarse[lc];
      if (prec == P64) {
        CoarseArgs<double, double2> c{};
        c.out = (double2*)out; c.in = (const double2*)in; c.links = (const double2*)dagl;
        c.g = gc[lc]; c.n = nc; c.in_stride = c.out_stride = gc[lc].V * nc; c.nrhs = nv_;
        launch_coarse(c, false, false, st);
      } else {
        CoarseArgs<float, float2> c{};
        c.out = (float2*)out; c.in = (const float2*)in; c.links = (const float2*)dagl;
        c.g = gc[lc]; c.n = nc; c.in_stride = c.out_stride = gc[lc].V * nc; c.nrhs = nv_;
        launch_coarse(c, false, false, st);
      }
      check_launch();
    }
  };
  if (start) {   // caller's starting vectors (FP64), in the level's precision
    if (prec == P64) launch_convert<double2, double2>((double2*)phi, start, (int64_t)nv_ * n, st);
    else launch_convert<double2, float2>((float2*)phi, start, (int64_t)nv_ * n, st);
  } else if (prec == P64) {
    launch_random_normal<double2>((double2*)phi, (int64_t)nv_ * n, P.seed + 7919ull * l, st);
  } else {
    launch_random_normal<float2>((float2*)phi, (int64_t)nv_ * n, P.seed + 7919ull * l, st);
  }
  check_launch();
  A_apply(r, phi, false);
  lincomb(prec, n, nv_, r, {{r, nullptr}}, {1}, {});
  std::vector<double> r0, rn;
  double2* rr = slot(3, kSlotQQ);
  double2* rrn = slot(3, kSlotQQ + 1);
  double2* al = slot(3, kSlotQQ + 2);
  double2* nal = slot(3, kSlotQQ + 3);
  double2* be = slot(3, kSlotQQ + 4);
  double2* tt = slot(3, kSlotQQ + 5);
  norms_host(prec, n, nv_, r, rr, r0);
  HIPCHK(hipMemcpyAsync(p, r, (size_t)nv_ * n * csize(prec), hipMemcpyDeviceToDevice, st));
  std::vector<int> act(nv_, 1);
  int* mk = lmask(3);
  HIPCHK(hipMemcpyAsync(mk, act.data(), nv_ * sizeof(int), hipMemcpyHostToDevice, st));
  int nact = nv_;
  for (int it = 0; it < maxiter && nact > 0; ++it) {
    A_apply(t, p, true);
    A_apply(At, t, false);
    dots(prec, n, nv_, {{t, t}}, tt);
    launch_cg_alpha(rr, tt, mk, nv_, al, nal, st);
    check_launch();
    lincomb(prec, n, nv_, phi, {{phi, nullptr}, {t, al}}, {}, {});
    lincomb(prec, n, nv_, r, {{r, nullptr}, {At, nal}}, {}, {});
    norms_host(prec, n, nv_, r, rrn, rn);
    launch_cg_beta(rr, rrn, mk, nv_, be, st);
    check_launch();
    lincomb(prec, n, nv_, p, {{r, nullptr}, {p, be}}, {}, {});
    bool changed = false;
    for (int s = 0; s < nv_; ++s)
      if (act[s] && !(rn[s] > tol * r0[s])) { act[s] = 0; --nact; changed = true; }
    if (changed) HIPCHK(hipMemcpyAsync(mk, act.data(), nv_ * sizeof(int), hipMemcpyHostToDevice, st));
  }
  if (prec == P64) launch_convert<double2, double2>(out, (const double2*)phi, (int64_t)nv_ * n, st);
  else launch_convert<float2, double2>(out, (const float2*)phi, (int64_t)nv_ * n, st);
  check_launch();
}

// Deflation space of the coarsest solve (Table 1 deflates it with low modes of
// its operator): k near-null vectors W of the coarsest operator A by CGNE,
// Z = A W with the stencil the solver applies, Z^H Z = R^H R (Cholesky, FP64),
// Q = Z R^{-1} and W' = W R^{-1}.
void Ctx::build_deflation(const void* imp) {
  const int lv = nlev - 1;
  const int k = defl_k;
  const int64_t n = defl_n;
  const int prec = L[lv].prec;
  if (imp) {   // imported vectors: kept in FP64, W in the level's precision
    HIPCHK(hipMemcpyAsync(nv[P.nagg], imp, (size_t)k * n * 16, hipMemcpyDeviceToDevice, st));
    if (prec == P64) launch_convert<double2, double2>((double2*)scratch_base, nv[P.nagg], (int64_t)k * n, st);
    else launch_convert<double2, float2>((float2*)scratch_base, nv[P.nagg], (int64_t)k * n, st);
    check_launch();
  } else {
    cgne_null(P.nagg, k, n, P.deflate_maxiter, 1e-6, nv[P.nagg]);
  }
  const size_t vb = ((size_t)k * n * csize(prec) + 255) & ~(size_t)255;
  void* W = scratch_base;        // CGNE result, level precision
  void* Z = scratch_base + vb;
  setup_phase = false;
  apply_coarse(lv, prec, Z, W, k, false);
  setup_phase = true;
  HIPCHK(hipMemsetAsync(status_dev, 0, sizeof(int), st));
  if (prec == P64) {
    launch_ts_gram<double2>((const double2*)Z, n, k, (const double2*)Z, n, k, n, part, part_elems, defl_g, st);
    launch_chol_rinv(defl_g, k, defl_rm, defl_rinv, status_dev, st);
    launch_ts_combine<double2>((double2*)defl_q, n, (const double2*)Z, n, k, k, defl_rinv, n, 0, st);
    launch_ts_combine<double2>((double2*)defl_w, n, (const double2*)W, n, k, k, defl_rinv, n, 0, st);
  } else {
    launch_ts_gram<float2>((const float2*)Z, n, k, (const float2*)Z, n, k, n, part, part_elems, defl_g, st);
    launch_chol_rinv(defl_g, k, defl_rm, defl_rinv, status_dev, st);
    launch_ts_combine<float2>((float2*)defl_q, n, (const float2*)Z, n, k, k, defl_rinv, n, 0, st);
    launch_ts_combine<float2>((float2*)defl_w, n, (const float2*)W, n, k, k, defl_rinv, n, 0, st);
  }
  check_launch();
  int status = 0;
  HIPCHK(hipMemcpyAsync(&status, status_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (status) throw Error{MG_E_RANK, "coarsest deflation vectors are numerically dependent"};
}

// Galerkin coarse operator (Sec. 2.1: A_c = R A P), built column by column
// in FP64: for coarse dof j, v = P e_j on every aggregate at once; each of the
// nine stencil pieces of the level operator (hops staying inside the
// aggregate, or crossing its +mu / -mu face) is applied to v and restricted,
// which yields column j of X(a) and of Y_{+-mu}(a) for every aggregate a.
void Ctx::galerkin(int l) {
  const Agg& a = A[l];
  const int n = 2 * a.nvec;
  const int64_t nflat = a.nagg * 2 * a.nrows;
  const size_t vb = ((size_t)nflat * 16 + 255) & ~(size_t)255;
  // past the CGNE buffers of this level
  const size_t cg = (((size_t)a.nvec * nflat * csize(L[l + 1].prec) + 255) & ~(size_t)255) * 6;
  double2* v = (double2*)(scratch_base + cg);
  double2* w = (double2*)(scratch_base + cg + vb);
  double2* u = (double2*)(scratch_base + cg + 2 * vb);
  for (int j = 0; j < n; ++j) {
    ProlongArgs<double> pa{};
    pa.out = v; pa.in = nullptr; pa.pp = pp64[l]; pa.A = a;
    pa.in_stride = a.nagg * n; pa.out_stride = nflat; pa.nrhs = 1; pa.accumulate = 0; pa.unit_col = j;
    launch_prolong(pa, st);
    check_launch();
    for (int piece = 0; piece < 9; ++piece) {
      const double2* src;
      if (l == 0) {
        DslashArgs<double> d{};
        d.out = w; d.in = v; d.fat = fat64; d.lng = lng64; d.lng_c = naik_compressed ? lng64c : nullptr; d.g = g0;
        d.in_stride = d.out_stride = g0.V * 3; d.nrhs = 1; d.mass = P.mass0; d.b_coef = 1;
        d.piece = piece;
        for (int mu = 0; mu < 4; ++mu) d.blk[mu] = a.b[mu];
        launch_dslash(d, P.c3 != 0.0 && P.kd_naik, false, true, st);
        check_launch();
        apply_KD(P64, u, w, 1, false, false, 0);
        src = u;
      } else {
        CoarseArgs<double, double2> c{};
        c.out = w; c.in = v; c.links = cl64[0]; c.g = gc[0]; c.n = ncoarse[0];
        c.in_stride = c.out_stride = gc[0].V * ncoarse[0]; c.nrhs = 1; c.piece = piece;
        for (int mu = 0; mu < 4; ++mu) c.blk[mu] = a.b[mu];
        launch_coarse(c, true, false, st);
        check_launch();
        src = w;
      }
      RestrictArgs<double> ra{};
      ra.out = cl64[l] + ((int64_t)piece * n + j) * n;
      ra.in = src; ra.pr = pr64[l]; ra.A = a;
      ra.in_stride = nflat; ra.out_stride = 0; ra.out_site_stride = (int64_t)9 * n * n; ra.nrhs = 1;
      launch_restrict(ra, st);
      check_launch();
    }
  }
}


// FP32 copy and 16-bit fragments of the FP64 links of level l
void Ctx::finish_links(int l) {
  const int n = ncoarse[l];
  launch_convert_links(cl64[l], cl32[l], gc[l].V * 9 * (int64_t)n * n, st);
  check_launch();
  if (fmt16 >= 0) {
    // 16-bit fragments; FP16 links get the power-of-two scale 2^-round(log2 max|L|),
    // which puts max |L| in [2^-1/2, 2^1/2] (far from the FP16 range limits, and
    // with no tie at the exact powers of two a Galerkin identity block produces)
    double scale = 1.0;
    if (fmt16 == 1) {
      unsigned long long* mx = (unsigned long long*)(status_dev + 16);
      HIPCHK(hipMemsetAsync(mx, 0, sizeof(unsigned long long), st));
      launch_absmax(cl64[l], gc[l].V * 9 * (int64_t)n * n, mx, st);
      check_launch();
      unsigned long long bits = 0;
      HIPCHK(hipMemcpyAsync(&bits, mx, sizeof(bits), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      double amax;
      memcpy(&amax, &bits, sizeof(amax));
      if (amax > 0.0) scale = std::ldexp(1.0, -(int)std::lround(std::log2(amax)));
    }
    cl16_inv_scale[l] = (float)(1.0 / scale);
    launch_swizzle_links<double2>(cl64[l], cl16[l], gc[l].V, n, fmt16, scale, st);
    check_launch();
  }
}

// Block preconditioning of coarse level l + 2 (Sec. 2.3, Table 1): X = the
// coarse-site diagonal block of the FP64 links, X^{-1} by Newton-Schulz
// (Y <- Y (2 - X Y) from Y_0 = X^H / (|X|_1 |X|_inf), to max |1 - X Y| <= 1e-13),
// then every link block L_d <- X^{-1} L_d.
void Ctx::precondition_links(int l) {
  const int n = ncoarse[l];
  const int64_t Vc = gc[l].V, nn = (int64_t)n * n;
  const size_t bb = ((size_t)Vc * nn * 16 + 255) & ~(size_t)255;
  double2* X = (double2*)scratch_base;
  double2* Y = (double2*)(scratch_base + bb);
  double2* T = (double2*)(scratch_base + 2 * bb);
  double2* Y2 = (double2*)(scratch_base + 3 * bb);
  launch_diag_block(cl64[l], X, gc[l], n, st);
  launch_ns_init(X, Y, Vc, n, st);
  check_launch();
  auto gemm = [&](double2* C, const double2* A, int a_div, const double2* B, int64_t sB, const double2* D,
                  double alpha, double beta, int batch) {
    BGemmArgs<double2> g{};
    g.A = A; g.lda = n; g.sA = nn; g.a_div = a_div;
    g.B = B; g.ldb = n; g.sB = sB;
    g.C = C; g.ldc = n; g.sC = nn;
    g.D = D; g.ldd = n; g.sD = nn;
    g.m = n; g.n = n; g.k = n; g.batch = batch;
    g.alpha = alpha; g.beta = beta;
    launch_bgemm(g, st);
    check_launch();
  };
  unsigned long long* dmax = (unsigned long long*)((char*)status_dev + 136);
  double res = 1.0;
  for (int it = 0; it < 100 && res > 1e-13; ++it) {
    gemm(T, X, 1, Y, nn, nullptr, 1.0, 0.0, (int)Vc);          // T = X Y
    if (it % 4 == 3) {
      HIPCHK(hipMemsetAsync(dmax, 0, sizeof(unsigned long long), st));
      launch_ns_residual(T, Vc, n, dmax, st);
      check_launch();
      unsigned long long bits = 0;
      HIPCHK(hipMemcpyAsync(&bits, dmax, sizeof(bits), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      std::memcpy(&res, &bits, sizeof(res));
      if (res <= 1e-13) break;
    }
    gemm(Y2, Y, 1, T, nn, Y, -1.0, 2.0, (int)Vc);             // Y' = 2 Y - Y T
    std::swap(Y, Y2);
  }
  if (!(res <= 1e-13))
    throw Error{MG_E_RANK, "coarse-site diagonal block is singular or too ill-conditioned to invert"};
  HIPCHK(hipMemcpyAsync(xinv64[l], Y, (size_t)Vc * nn * 16, hipMemcpyDeviceToDevice, st));
  launch_convert<double2, float2>(xinv32[l], Y, Vc * nn, st);
  check_launch();
  for (int d = 0; d < 9; ++d) {
    // T = X^{-1} L_d for every site, then back into the links
    BGemmArgs<double2> g{};
    g.A = xinv64[l]; g.lda = n; g.sA = nn; g.a_div = 1;
    g.B = cl64[l] + d * nn; g.ldb = n; g.sB = 9 * nn;
    g.C = T; g.ldc = n; g.sC = nn;
    g.m = n; g.n = n; g.k = n; g.batch = (int)Vc;
    g.alpha = 1.0;
    launch_bgemm(g, st);
    check_launch();
    HIPCHK(hipMemcpy2DAsync(cl64[l] + d * nn, (size_t)9 * nn * 16, T, (size_t)nn * 16, (size_t)nn * 16, (size_t)Vc,
                            hipMemcpyDeviceToDevice, st));
  }
  // with no coarse extent 1 the self piece is the whole diagonal block, so
  // X^{-1} L_0 is the identity: stored exactly, and the 16-bit stencil adds
  // the input instead of reading that block
  bool ext1 = false;
  for (int mu = 0; mu < 4; ++mu) ext1 = ext1 || gc[l].L[mu] == 1;
  if (!ext1) {
    launch_unit_self(cl64[l], gc[l], n, st);
    check_launch();
  }
  unit_self[l] = !ext1 && n % 32 == 0;
}

// out = X^{-1} in for the systems of a coarse level (coarse_op 1), site by site
void Ctx::apply_xinv(int lvl, int prec, void* out, const void* in, int nsys) {
  const int l = lvl - 2;
  const int n = ncoarse[l];
  const int64_t nn = (int64_t)n * n, stride = gc[l].V * n;
  if (prec == P64) {
    BGemmArgs<double2> g{};
    g.A = xinv64[l]; g.lda = n; g.sA = nn; g.a_div = 1;
    g.B = (const double2*)in; g.ldb = stride; g.sB = n;
    g.C = (double2*)out; g.ldc = stride; g.sC = n;
    g.m = n; g.n = nsys; g.k = n; g.batch = (int)gc[l].V; g.alpha = 1.0;
    launch_bgemm(g, st);
  } else {
    BGemmArgs<float2> g{};
    g.A = xinv32[l]; g.lda = n; g.sA = nn; g.a_div = 1;
    g.B = (const float2*)in; g.ldb = stride; g.sB = n;
    g.C = (float2*)out; g.ldc = stride; g.sC = n;
    g.m = n; g.n = nsys; g.k = n; g.batch = (int)gc[l].V; g.alpha = 1.0;
    launch_bgemm(g, st);
  }
  check_launch();
}

}  // namespace mg
