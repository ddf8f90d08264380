// Host driver of the staggered KD multigrid: workspace plan, hierarchy
// set-up (Sec. 2.1, Sec. 2.3, Table 1), operator dispatch and the Krylov
// drivers.  Every vector operation is a kernel on the context's stream; the
// host only reads one norm per system and iteration for convergence tests.
#include "mg.hpp"

#include <cmath>
#include <cstring>
#include <type_traits>

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

// ======================================================================= plan
bool Ctx::plan(const mg_params& p, Ctx* c, Arena& pers, Arena& scr, std::string* why) {
  auto fail = [&](const std::string& s) { *why = s; return false; };
  for (int mu = 0; mu < 4; ++mu)
    if (p.dims[mu] < 4 || (p.dims[mu] & 1)) return fail("lattice extents must be even and >= 4");
  if (p.nagg < 1 || p.nagg > 2) return fail("nagg must be 1 or 2");
  if (p.fine_prec != MG_C128 && p.fine_prec != MG_C64) return fail("fine_prec must be MG_C128 or MG_C64");
  if (p.coarse_prec < MG_C128 || p.coarse_prec > MG_CF16) return fail("coarse_prec must be an mg_dtype");
  if (p.fine_prec == MG_C128 && p.coarse_prec != MG_C128)
    return fail("coarse_prec must be MG_C128 when fine_prec is MG_C128");
  if (p.fine_prec == MG_C64 && p.coarse_prec == MG_C128)
    return fail("coarse_prec MG_C128 needs fine_prec MG_C128 (coarse vectors share the level-1 precision)");
  if (p.smoother_s < 1 || p.smoother_s > kMaxS) return fail("smoother_s must be in 1..8");
  if (p.inner_maxiter < 1 || p.inner_maxiter > kMaxNK) return fail("inner_maxiter must be in 1..16");
  if (p.coarsest_maxiter < 1 || p.coarsest_maxiter > kMaxNK) return fail("coarsest_maxiter must be in 1..16");
  if (p.coarsest_restarts < 1) return fail("coarsest_restarts must be >= 1");
  if (p.outer_nkrylov < 1 || p.outer_nkrylov > kMaxNK) return fail("outer_nkrylov must be in 1..16");
  if (p.outer_maxiter < 1) return fail("outer_maxiter must be >= 1");
  if (p.max_nrhs < 1 || p.max_nmass < 1) return fail("max_nrhs and max_nmass must be >= 1");
  if (!(p.mass0 > 0.0)) return fail("mass0 must be positive");
  if (p.coarsest_deflate < 0 || p.coarsest_deflate > kMaxDefl || p.coarsest_deflate % 16)
    return fail("coarsest_deflate must be 0, 16, 32, 48 or 64");
  if (p.coarsest_deflate > 0 && p.deflate_maxiter < 1) return fail("deflate_maxiter must be >= 1");
  if (p.deflate_import != 0 && p.deflate_import != 1) return fail("deflate_import must be 0 or 1");
  if (p.coarse_op != 0 && p.coarse_op != 1) return fail("coarse_op must be 0 (Galerkin) or 1 (block-preconditioned)");
  if (p.coarsest_solver < 0 || p.coarsest_solver > 2)
    return fail("coarsest_solver must be 0 (GCR), 1 (CA-GCR) or 2 (direct)");
  if (p.coarsest_solver == 2 && p.coarsest_deflate > 0)
    return fail("coarsest_deflate needs an iterative coarsest solver (coarsest_solver 0 or 1), not the direct one");
  if (p.graph_coarsest != 0 && p.graph_coarsest != 1) return fail("graph_coarsest must be 0 or 1");
  if (p.compact_masses != 0 && p.compact_masses != 1) return fail("compact_masses must be 0 or 1");
  if (p.coarse_shadow != 0 && p.coarse_shadow != 1) return fail("coarse_shadow must be 0 or 1");
  if (p.cgne_start_import != 0 && p.cgne_start_import != 1) return fail("cgne_start_import must be 0 or 1");
  const bool naik_kd = p.c3 != 0.0 && p.kd_naik;
  Geom g0{};
  g0.V = 1;
  for (int mu = 0; mu < 4; ++mu) { g0.L[mu] = p.dims[mu]; g0.V *= p.dims[mu]; }
  Geom gcur = g0;
  Agg A[2]{};
  Geom gc[2]{};
  int nin = 0;
  for (int l = 0; l < p.nagg; ++l) {
    Agg& a = A[l];
    a.fine = gcur;
    a.kind = l == 0 ? 1 : 2;
    a.nvec = p.nvec[l];
    a.nvec_in = nin;
    int bs = 1;
    Geom g{};
    g.V = 1;
    for (int mu = 0; mu < 4; ++mu) {
      const int b = p.block[l][mu];
      if (b < 1 || gcur.L[mu] % b) return fail("aggregation block must divide the lattice");
      if (l == 0 && (b & 1)) return fail("first aggregation block must have even extents");
      if (l == 0 && naik_kd && b < 3) return fail("Naik term with a first block below 3 reaches beyond neighbouring aggregates");
      a.b[mu] = b;
      a.cd[mu] = gcur.L[mu] / b;
      g.L[mu] = a.cd[mu];
      g.V *= a.cd[mu];
      bs *= b;
    }
    a.nagg = g.V;
    a.nrows = l == 0 ? bs / 2 * 3 : bs * nin;
    if (a.nvec < 1 || a.nvec > 128) return fail("nvec must be in 1..128");
    if ((p.coarse_prec == MG_CBF16 || p.coarse_prec == MG_CF16) && (a.nvec % 8))
      return fail("nvec must be a multiple of 8 for 16-bit coarse links (16-row MFMA tiles)");
    if (a.nvec > a.nrows) return fail("nvec exceeds the rows of an aggregate and chirality");
    if (a.nrows > 4096) return fail("more than 4096 rows per aggregate and chirality");
    gc[l] = g;
    gcur = g;
    nin = a.nvec;
  }
  const int kd = p.coarsest_deflate;
  const int64_t ncl = gc[p.nagg - 1].V * 2 * A[p.nagg - 1].nvec;   // coarsest-level dof
  if (kd > ncl) return fail("coarsest_deflate exceeds the coarsest level's dimension");
  if (p.coarsest_solver == 2 && ncl > kDirectMax)
    return fail("coarsest_solver 2 (direct) needs a coarsest level of at most 8192 dof");
  if (c) {
    c->P = p;
    c->g0 = g0;
    c->nlev = 2 + p.nagg;
    for (int l = 0; l < 2; ++l) { c->A[l] = A[l]; c->gc[l] = gc[l]; c->ncoarse[l] = 2 * A[l].nvec; }
  }
  const int64_t V = g0.V;
  auto P = [&](size_t n) { return pers.take(n); };
  // ---- persistent
  void* fat64 = P(36 * V * 16);
  void* fat32 = P(36 * V * 8);
  void* fat32p = P(20 * V * 16);   // FP32 one-hop links in element pairs
  void* lng64 = p.c3 != 0.0 ? P(36 * V * 16) : nullptr;
  void* lng32 = p.c3 != 0.0 ? P(36 * V * 8) : nullptr;
  void* lng64c = p.c3 != 0.0 ? P(28 * V * 16) : nullptr;   // compressed Naik links (7 per link)
  void* lng32c = p.c3 != 0.0 ? P(28 * V * 8) : nullptr;
  const int64_t kslot = V / 16 * 2304;
  void* kinv64 = P((size_t)p.max_nmass * kslot * 16);
  void* kinv32 = P((size_t)p.max_nmass * kslot * 8);
  void *nvp[2]{}, *pp64[2]{}, *pr64[2]{}, *pp32[2]{}, *pr32[2]{}, *cl64[2]{}, *cl32[2]{}, *cl16[2]{};
  void *xi64[2]{}, *xi32[2]{};
  const bool c16 = p.coarse_prec == MG_CBF16 || p.coarse_prec == MG_CF16;
  for (int l = 0; l < p.nagg; ++l) {
    const int64_t nflat = A[l].nagg * 2 * A[l].nrows;   // dof of the aggregated level
    const int64_t pel = nflat * A[l].nvec;
    nvp[l] = P(pel * 16);
    pp64[l] = P(pel * 16);
    pr64[l] = P(pel * 16);
    pp32[l] = P(pel * 8);
    pr32[l] = P(pel * 8);
    const int64_t n = 2 * A[l].nvec;
    cl64[l] = P(gc[l].V * 9 * n * n * 16);
    cl32[l] = P(gc[l].V * 9 * n * n * 8);
    if (c16) cl16[l] = P(swizzled_link_elems(gc[l].V, (int)n) * 2);
    if (p.coarse_op == 1) {   // X^{-1} per coarse site
      xi64[l] = P(gc[l].V * n * n * 16);
      xi32[l] = P(gc[l].V * n * n * 8);
    }
  }
  const int cprec_ = p.coarse_prec == MG_C128 ? P64 : P32;
  void *nvd = nullptr, *dq = nullptr, *dw = nullptr, *dg = nullptr, *drm = nullptr, *dri = nullptr;
  if (kd > 0) {
    nvd = P((size_t)kd * ncl * 16);
    dq = P((size_t)kd * ncl * csize(cprec_));
    dw = P((size_t)kd * ncl * csize(cprec_));
    dg = P((size_t)kd * kd * 16);
    drm = P((size_t)kd * kd * 16);
    dri = P((size_t)kd * kd * 16);
  }
  void *dinv64 = nullptr, *dinv32 = nullptr;
  if (p.coarsest_solver == 2) {   // dense inverse of the coarsest operator (column-major)
    dinv64 = P((size_t)ncl * ncl * 16);
    dinv32 = P((size_t)ncl * ncl * 8);
  }
  void* status = P(256);
  // ---- scratch
  const int ms = std::max({p.max_nrhs, p.nvec[0], p.nagg > 1 ? p.nvec[1] : 1, kd});
  auto S = [&](size_t n) { return scr.take(n); };
  const int npart = p.coarsest_solver == 1 ? kMaxCA * (kMaxCA + 1) / 2 + kMaxCA : kMaxPairs;   // products per reduction
  const size_t part_elems = std::max((size_t)npart * ms * 480, kd > 0 ? (size_t)128 * kMaxDefl * kMaxDefl : 0);
  void* part = S(part_elems * 16);
  void* scal = S((size_t)4 * kMaxSlots * ms * 16);
  void* tri = S((size_t)4 * kTriSlots * ms * 16);
  void* m64 = S((size_t)2 * ms * 8);    // per-system masses of the batch, then of the K-cycle's systems
  void* m32 = S((size_t)2 * ms * 4);
  void* mask = S((size_t)5 * ms * 4);   // levels 0..3, then level 0 of a compacted K-cycle
  void* dcoef = kd > 0 ? S((size_t)kd * ms * 16) : nullptr;
  // 16-bit copies of the smoother chain's stencil outputs, two per coarse level that has a smoother
  void* sh16[2][2]{};
  if (c16 && p.coarse_shadow && p.fine_prec == MG_C64)
    for (int l = 0; l + 1 < p.nagg; ++l)
      for (int q = 0; q < 2; ++q) sh16[l][q] = S((size_t)p.max_nrhs * gc[l].V * 2 * A[l].nvec * 4);
  const size_t solver_base = scr.off;
  // solver buffers
  LevelBufs L[4];
  const int64_t nlv[4] = {V * 3, V * 3, p.nagg >= 1 ? gc[0].V * 2 * A[0].nvec : 0,
                          p.nagg >= 2 ? gc[1].V * 2 * A[1].nvec : 0};
  const int fp = p.fine_prec == MG_C128 ? P64 : P32;
  const int cp = p.coarse_prec == MG_C128 ? P64 : P32;
  const int precs[4] = {P64, fp, cp, cp};
  const int nks[4] = {p.outer_nkrylov, p.inner_maxiter, p.inner_maxiter, p.inner_maxiter};
  const int nlev = 2 + p.nagg;
  Vec r0s, e0s;
  for (int l = 0; l < nlev; ++l) {
    LevelBufs& B = L[l];
    B.prec = precs[l];
    B.n = nlv[l];
    const bool coarsest = l == nlev - 1;
    B.nk = coarsest ? p.coarsest_maxiter : nks[l];
    auto mk = [&](Vec& v, int prec) { v.prec = prec; v.n = B.n; v.p = S((size_t)p.max_nrhs * B.n * csize(prec)); };
    mk(B.b, B.prec);
    if (l > 0) mk(B.x, B.prec);
    mk(B.r, B.prec);
    for (int k = 0; k < B.nk; ++k) { mk(B.z[k], B.prec); mk(B.q[k], B.prec); }
    if (!coarsest) {
      // K-cycle / smoother work vectors, in the level's smoothing precision
      const int sp = l == 0 ? fp : B.prec;
      mk(B.t, sp);
      mk(B.tmp, sp);
      for (int j = 0; j < p.smoother_s; ++j) mk(B.sm[j], sp);
    } else if (l == 1) {
      mk(B.tmp, B.prec);
    }
    if (l == 0) {
      r0s.prec = fp; r0s.n = B.n; r0s.p = S((size_t)p.max_nrhs * B.n * csize(fp));
      e0s.prec = fp; e0s.n = B.n; e0s.p = S((size_t)p.max_nrhs * B.n * csize(fp));
    }
  }
  const size_t solver_end = scr.off;
  // set-up scratch aliases the solver buffers
  scr.off = solver_base;
  for (int l = 0; l < p.nagg; ++l) {
    const int64_t n = l == 0 ? V * 3 : gc[0].V * 2 * A[0].nvec;
    const int prec = l == 0 ? fp : cp;
    for (int v = 0; v < 6; ++v) S((size_t)p.nvec[l] * n * csize(prec));   // CGNE
    for (int v = 0; v < 3; ++v) S((size_t)n * 16);                          // Galerkin
    scr.off = solver_base;
  }
  size_t setup_end = solver_base;
  for (int l = 0; l < p.nagg; ++l) {
    const int64_t n = l == 0 ? V * 3 : gc[0].V * 2 * A[0].nvec;
    const int prec = l == 0 ? fp : cp;
    size_t e = solver_base + 6 * (((size_t)p.nvec[l] * n * csize(prec) + 255) & ~(size_t)255) +
               3 * (((size_t)n * 16 + 255) & ~(size_t)255) + 256;
    if (l == 1) {   // explicit adjoint links of the level-2 stencil (+ their 16-bit fragments)
      const int64_t nc = 2 * A[0].nvec;
      e += (size_t)gc[0].V * 9 * nc * nc * csize(prec) + 256;
      if (c16) e += (size_t)swizzled_link_elems(gc[0].V, (int)nc) * 2 + 256;
    }
    setup_end = std::max(setup_end, e);
  }
  if (p.coarse_op == 1) {   // Newton-Schulz inverse and preconditioned links: X, Y, T, Y' blocks (FP64)
    for (int l = 0; l < p.nagg; ++l) {
      const int64_t n = 2 * A[l].nvec;
      setup_end = std::max(setup_end, solver_base + 4 * (((size_t)gc[l].V * n * n * 16 + 255) & ~(size_t)255) + 256);
    }
  }
  if (kd > 0) {   // CGNE on the coarsest operator: six k-vector blocks, its adjoint links (+ 16-bit fragments)
    const int lc = p.nagg - 1;
    const int64_t nc = 2 * A[lc].nvec;
    size_t e = solver_base + 6 * (((size_t)kd * ncl * csize(cprec_) + 255) & ~(size_t)255) +
               3 * (((size_t)ncl * 16 + 255) & ~(size_t)255) + 256;
    e += (size_t)gc[lc].V * 9 * nc * nc * csize(cprec_) + 256;
    if (c16) e += (size_t)swizzled_link_elems(gc[lc].V, (int)nc) * 2 + 256;
    setup_end = std::max(setup_end, e);
  }
  if (p.coarsest_solver == 2)   // Gauss-Jordan: [A | 1] (FP64, n x 2n), the factor column, pivot words
    setup_end = std::max(setup_end, solver_base + (((size_t)2 * ncl * ncl * 16 + 255) & ~(size_t)255) +
                                        (((size_t)ncl * 16 + 255) & ~(size_t)255) + 512);
  scr.off = std::max(solver_end, setup_end);
  if (c) {
    c->fat64 = (double2*)fat64; c->fat32 = (float2*)fat32; c->fat32p = (float4*)fat32p;
    c->lng64 = (double2*)lng64; c->lng32 = (float2*)lng32;
    c->lng64c = (double2*)lng64c; c->lng32c = (float2*)lng32c;
    c->kinv64 = (double2*)kinv64; c->kinv32 = (float2*)kinv32;
    c->kinv_slot = kslot;
    c->kd_mass.assign(p.max_nmass, NAN);
    for (int l = 0; l < 2; ++l) {
      c->nv[l] = (double2*)nvp[l];
      c->pp64[l] = (double2*)pp64[l]; c->pr64[l] = (double2*)pr64[l];
      c->pp32[l] = (float2*)pp32[l]; c->pr32[l] = (float2*)pr32[l];
      c->cl64[l] = (double2*)cl64[l]; c->cl32[l] = (float2*)cl32[l];
      c->cl16[l] = (uint16_t*)cl16[l];
      c->xinv64[l] = (double2*)xi64[l];
      c->xinv32[l] = (float2*)xi32[l];
    }
    c->fmt16 = p.coarse_prec == MG_CBF16 ? 0 : (p.coarse_prec == MG_CF16 ? 1 : -1);
    c->status_dev = (int*)status;
    c->max_sys = ms;
    c->part = (double2*)part;
    c->part_elems = part_elems;
    c->defl_k = kd;
    c->defl_n = ncl;
    c->nv[p.nagg] = (double2*)nvd;
    c->defl_q = dq;
    c->defl_w = dw;
    c->defl_g = (double2*)dg;
    c->defl_rm = (double2*)drm;
    c->defl_rinv = (double2*)dri;
    c->defl_c = (double2*)dcoef;
    c->dinv64 = (double2*)dinv64;
    c->dinv32 = (float2*)dinv32;
    for (int l = 0; l < 2; ++l)
      for (int q = 0; q < 2; ++q) c->shadow16[l][q] = (uint32_t*)sh16[l][q];
    c->scal = (double2*)scal;
    c->tri = (double2*)tri;
    c->mass64 = (double*)m64;
    c->mass32 = (float*)m32;
    c->mask = (int*)mask;
    for (int l = 0; l < 4; ++l) c->L[l] = L[l];
    c->r0s = r0s;
    c->e0s = e0s;
    c->scratch_base = scr.base ? scr.base + solver_base : nullptr;
    c->scratch_cap = scr.off - solver_base;
  }
  return true;
}

// ================================================================ profiling
void Ctx::prof_mark(int op, int level, int nsys) {
  if (op != prof_op || level != prof_level || (prof_nrhs > 0 && nsys != prof_nrhs)) return;
  if (prof_used == prof_events.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    prof_events.push_back(e);
  }
  HIPCHK(hipEventRecord(prof_events[prof_used++], st));
}

Ctx::~Ctx() {
  for (hipEvent_t e : prof_events) (void)hipEventDestroy(e);
  for (auto& g : coarsest_graphs) (void)hipGraphExecDestroy(g.second);
  if (capture_st) (void)hipStreamDestroy(capture_st);
}

// ================================================================== operators
template <typename R>
static DslashArgs<R> dslash_args(const Ctx& c, void* out, const void* in, int nsys) {
  DslashArgs<R> a{};
  a.out = (cplx<R>*)out;
  a.in = (const cplx<R>*)in;
  const bool d = sizeof(R) == 8;
  a.fat = d ? (const cplx<R>*)c.fat64 : (const cplx<R>*)c.fat32;
  a.lng = d ? (const cplx<R>*)c.lng64 : (const cplx<R>*)c.lng32;
  a.fat_pairs = d ? nullptr : c.fat32p;
  a.lng_c = c.naik_compressed ? (d ? (const cplx<R>*)c.lng64c : (const cplx<R>*)c.lng32c) : nullptr;
  a.g = c.g0;
  a.in_stride = a.out_stride = a.xs_stride = c.g0.V * 3;
  a.nrhs = nsys;
  a.b_coef = 1;
  return a;
}

void Ctx::apply_D(int prec, void* out, const void* in, int nsys, bool naik, const void* mass_rhs, double mass,
                  bool eps_out) {
  prof_mark(MG_PROF_DSLASH, naik && P.c3 != 0.0 ? 0 : 1, nsys);
  naik = naik && P.c3 != 0.0;
  if (prec == P64) {
    auto a = dslash_args<double>(*this, out, in, nsys);
    a.mass = mass;
    a.mass_rhs = (const double*)mass_rhs;
    a.eps_out = eps_out;
    launch_dslash(a, naik, false, false, st);
  } else {
    auto a = dslash_args<float>(*this, out, in, nsys);
    a.mass = (float)mass;
    a.mass_rhs = (const float*)mass_rhs;
    a.eps_out = eps_out;
    launch_dslash(a, naik, false, false, st);
  }
  prof_mark(MG_PROF_DSLASH, naik && P.c3 != 0.0 ? 0 : 1, nsys);
  check_launch();
}

void Ctx::apply_KD(int prec, void* out, const void* in, int nsys, bool eps_in, bool eps_out, int rps) {
  prof_mark(MG_PROF_KD, 0, nsys);
  if (prec == P64) {
    KdArgs<double> a{};
    a.out = (double2*)out; a.in = (const double2*)in; a.kinv = kinv64 + (int64_t)kd_base * kinv_slot;
    a.g = g0; a.in_stride = a.out_stride = g0.V * 3; a.nrhs = nsys;
    a.rhs_per_slot = rps; a.slot_stride = kinv_slot; a.eps_in = eps_in; a.eps_out = eps_out;
    launch_kd_apply(a, st);
  } else {
    KdArgs<float> a{};
    a.out = (float2*)out; a.in = (const float2*)in; a.kinv = kinv32 + (int64_t)kd_base * kinv_slot;
    a.g = g0; a.in_stride = a.out_stride = g0.V * 3; a.nrhs = nsys;
    a.rhs_per_slot = rps; a.slot_stride = kinv_slot; a.eps_in = eps_in; a.eps_out = eps_out;
    launch_kd_apply(a, st);
  }
  prof_mark(MG_PROF_KD, 0, nsys);
  check_launch();
}

// The KD-level operator A = (B+m)^{-1} D.  D = B + m + D_off with D_off the
// hops that leave a site's 2^4 hypercube (every Naik hop does), so
// A = 1 + (B+m)^{-1} D_off: where the one-hop plane stencil and the LDS-staged
// KD kernel take the launch (FP32, truncated KD, 16-rhs tiles), the stencil
// computes D_off (half the per-site hops) and the KD kernel adds x; otherwise
// D then (B+m)^{-1}.  tmp: one level-1 vector block for the intermediate.
void Ctx::apply_kd_operator(int prec, void* out, const void* in, void* tmp, int nsys, const void* mass_rhs,
                            double mass, int rps) {
  const bool naik = P.kd_naik != 0 && P.c3 != 0.0;
  if (prec == P32 && !naik) {
    DslashArgs<float> d = dslash_args<float>(*this, tmp, in, nsys);
    d.off_cube = 1;
    KdArgs<float> k{};
    k.out = (float2*)out; k.in = (const float2*)tmp; k.add = (const float2*)in;
    k.kinv = kinv32 + (int64_t)kd_base * kinv_slot;
    k.g = g0; k.in_stride = k.out_stride = g0.V * 3; k.nrhs = nsys;
    k.rhs_per_slot = rps; k.slot_stride = kinv_slot;
    if (dslash_plane_ok(d) && kd_lds_ok(k)) {
      prof_mark(MG_PROF_DSLASH, 1, nsys);
      launch_dslash_plane(d, st);
      prof_mark(MG_PROF_DSLASH, 1, nsys);
      check_launch();
      prof_mark(MG_PROF_KD, 0, nsys);
      launch_kd_apply(k, st);
      prof_mark(MG_PROF_KD, 0, nsys);
      check_launch();
      return;
    }
  }
  apply_D(prec, tmp, in, nsys, naik, mass_rhs, mass);
  apply_KD(prec, out, tmp, nsys, false, false, rps);
}

void Ctx::apply_coarse(int lvl, int prec, void* out, const void* in, int nsys, bool dag, const uint32_t* in16,
                       uint32_t* out16) {
  prof_mark(MG_PROF_COARSE, lvl, nsys);
  const int l = lvl - 2;
  const int n = ncoarse[l];
  if (prec == P64) {
    CoarseArgs<double, double2> a{};
    a.out = (double2*)out; a.in = (const double2*)in; a.links = cl64[l];
    a.g = gc[l]; a.n = n; a.in_stride = a.out_stride = gc[l].V * n; a.nrhs = nsys;
    launch_coarse(a, false, dag, st);
  } else if (fmt16 >= 0 && !dag && !setup_phase) {
    CoarseMfmaArgs a{};
    a.out = (float2*)out; a.in = (const float2*)in; a.links = cl16[l];
    a.g = gc[l]; a.n = n; a.in_stride = a.out_stride = gc[l].V * n; a.nrhs = nsys;
    a.inv_scale = cl16_inv_scale[l];
    a.unit_self = unit_self[l] ? 1 : 0;
    a.rt = tune[l][rhs_class(nsys)][0];
    a.mt = tune[l][rhs_class(nsys)][1];
    a.in16 = in16;
    a.out16 = out16;
    launch_coarse_mfma(a, fmt16, st);
  } else {
    CoarseArgs<float, float2> a{};
    a.out = (float2*)out; a.in = (const float2*)in; a.links = cl32[l];
    a.g = gc[l]; a.n = n; a.in_stride = a.out_stride = gc[l].V * n; a.nrhs = nsys;
    launch_coarse(a, false, dag, st);
  }
  prof_mark(MG_PROF_COARSE, lvl, nsys);
  check_launch();
}

void Ctx::restrict_(int lvl, int prec, void* out, const void* in, int nsys) {
  prof_mark(MG_PROF_RESTRICT, lvl, nsys);
  const int l = lvl - 1;   // lvl 1: fine -> level 2, lvl 2: level 2 -> level 3
  const Agg& a = A[l];
  const int64_t nin = a.nagg * 2 * a.nrows, nout = a.nagg * 2 * a.nvec;
  if (prec == P64) {
    RestrictArgs<double> r{};
    r.out = (double2*)out; r.in = (const double2*)in; r.pr = pr64[l]; r.A = a;
    r.in_stride = nin; r.out_stride = nout; r.out_site_stride = 2 * a.nvec; r.nrhs = nsys;
    launch_restrict(r, st);
  } else {
    RestrictArgs<float> r{};
    r.out = (float2*)out; r.in = (const float2*)in; r.pr = pr32[l]; r.A = a;
    r.in_stride = nin; r.out_stride = nout; r.out_site_stride = 2 * a.nvec; r.nrhs = nsys;
    launch_restrict(r, st);
  }
  prof_mark(MG_PROF_RESTRICT, lvl, nsys);
  check_launch();
}

void Ctx::prolong_(int lvl, int prec, void* out, const void* in, int nsys, bool acc) {
  prof_mark(MG_PROF_PROLONG, lvl, nsys);
  const int l = lvl - 1;
  const Agg& a = A[l];
  const int64_t nfine = a.nagg * 2 * a.nrows, ncrs = a.nagg * 2 * a.nvec;
  if (prec == P64) {
    ProlongArgs<double> r{};
    r.out = (double2*)out; r.in = (const double2*)in; r.pp = pp64[l]; r.A = a;
    r.in_stride = ncrs; r.out_stride = nfine; r.nrhs = nsys; r.accumulate = acc; r.unit_col = -1;
    launch_prolong(r, st);
  } else {
    ProlongArgs<float> r{};
    r.out = (float2*)out; r.in = (const float2*)in; r.pp = pp32[l]; r.A = a;
    r.in_stride = ncrs; r.out_stride = nfine; r.nrhs = nsys; r.accumulate = acc; r.unit_col = -1;
    launch_prolong(r, st);
  }
  prof_mark(MG_PROF_PROLONG, lvl, nsys);
  check_launch();
}

// A_lvl on a batch: level 0 D(m_s), level 1 (B + m_s)^{-1} D(m_s), coarse levels
void Ctx::apply_level(int lvl, const Vec& out, const Vec& in, int nsys) {
  // inside a compacted K-cycle the systems are those of the active masses
  const int64_t mo = kc_compact ? max_sys : 0;
  const void* m = in.prec == P64 ? (const void*)(mass64 + mo) : (const void*)(mass32 + mo);
  if (lvl == 0) {
    apply_D(in.prec, out.p, in.p, nsys, true, m, 0.0);
  } else if (lvl == 1) {
    apply_kd_operator(in.prec, out.p, in.p, L[1].tmp.p, nsys, m, 0.0, rhs_per_slot);
  } else {
    apply_coarse(lvl, in.prec, out.p, in.p, nsys, false);
  }
}

// ======================================================================= BLAS
void Ctx::dots(int prec, int64_t n, int nsys, const std::vector<std::pair<const void*, const void*>>& pairs,
               double2* res) {
  if (pairs.empty()) return;
  if ((int)pairs.size() > kMaxPairs) throw Error{MG_E_ARG, "too many dot products in one reduction"};
  if (prec == P64) {
    PairDotArgs<double2> a{};
    for (size_t i = 0; i < pairs.size(); ++i) { a.x[i] = (const double2*)pairs[i].first; a.y[i] = (const double2*)pairs[i].second; }
    a.np = (int)pairs.size(); a.n = n; a.stride = n; a.nrhs = nsys;
    launch_pairdot(a, part, res, max_sys, st);
  } else {
    PairDotArgs<float2> a{};
    for (size_t i = 0; i < pairs.size(); ++i) { a.x[i] = (const float2*)pairs[i].first; a.y[i] = (const float2*)pairs[i].second; }
    a.np = (int)pairs.size(); a.n = n; a.stride = n; a.nrhs = nsys;
    launch_pairdot(a, part, res, max_sys, st);
  }
  check_launch();
}

// out = sum_t c_t v_t; c_t from a device per-system array when given, else consts[t]; neg flips sign
void Ctx::lincomb(int prec, int64_t n, int nsys, void* out,
                  const std::vector<std::pair<const void*, const double2*>>& terms, const std::vector<int>& neg,
                  const std::vector<double2>& consts) {
  if ((int)terms.size() > kMaxTerms) throw Error{MG_E_ARG, "too many terms in a linear combination"};
  auto fill = [&](auto& a) {
    for (size_t t = 0; t < terms.size(); ++t) {
      a.v[t] = (decltype(a.v[0]))terms[t].first;
      a.c[t] = terms[t].second;
      a.cconst[t] = t < consts.size() ? consts[t] : make_double2(1.0, 0.0);
      a.neg[t] = t < neg.size() ? neg[t] : 0;
    }
    a.nt = (int)terms.size(); a.n = n; a.stride = n; a.nrhs = nsys;
  };
  if (prec == P64) {
    LinCombArgs<double2> a{};
    a.out = (double2*)out;
    fill(a);
    launch_lincomb(a, st);
  } else {
    LinCombArgs<float2> a{};
    a.out = (float2*)out;
    fill(a);
    launch_lincomb(a, st);
  }
  check_launch();
}

void Ctx::copy(const Vec& dst, const Vec& src, int nsys) {
  const int64_t n = src.n * nsys;
  // copies are kernels (no copy nodes in a captured coarsest solve)
  if (dst.prec == src.prec && src.prec == P64) {
    launch_convert<double2, double2>((double2*)dst.p, (const double2*)src.p, n, st);
  } else if (dst.prec == src.prec) {
    launch_convert<float2, float2>((float2*)dst.p, (const float2*)src.p, n, st);
  } else if (src.prec == P64) {
    launch_convert<double2, float2>((float2*)dst.p, (const double2*)src.p, n, st);
  } else {
    launch_convert<float2, double2>((double2*)dst.p, (const float2*)src.p, n, st);
  }
  check_launch();
}

void Ctx::zero(const Vec& v, int nsys) {
  HIPCHK(hipMemsetAsync(v.p, 0, (size_t)v.n * nsys * csize(v.prec), st));
}

void Ctx::norms_host(int prec, int64_t n, int nsys, const void* v, double2* res_dev, std::vector<double>& out) {
  dots(prec, n, nsys, {{v, v}}, res_dev);
  std::vector<double2> h(nsys);
  HIPCHK(hipMemcpyAsync(h.data(), res_dev, nsys * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  out.resize(nsys);
  // NaN propagates (a non-finite input must be reported, not read as zero)
  for (int s = 0; s < nsys; ++s) out[s] = h[s].x >= 0.0 ? std::sqrt(h[s].x) : (h[s].x < 0.0 ? 0.0 : h[s].x);
}

// ==================================================================== solvers
// CA-GCR(s) smoother: e += argmin_{v in K_s(A, t)} ||t - A v|| via the power
// basis p_0 = t, p_j = A p_{j-1}, one Gram reduction and an s x s Cholesky
// solve in FP64 (the basis-free definition of the smoother's result).
void Ctx::smoother(int lvl, const Vec& e, const Vec& t, int nsys) {
  LevelBufs& B = L[lvl];
  const int s = P.smoother_s;
  const int prec = t.prec;
  // on a coarse level with 16-bit links each basis vector is also kept in
  // that format for the next application (two alternating copies)
  const bool sh = lvl >= 2 && shadow16[lvl - 2][0] && fmt16 >= 0 && prec == P32 && !setup_phase;
  for (int j = 0; j < s; ++j) {
    const Vec& src = j == 0 ? t : B.sm[j - 1];
    if (sh) {
      apply_coarse(lvl, prec, B.sm[j].p, src.p, nsys, false, j > 0 ? shadow16[lvl - 2][(j - 1) & 1] : nullptr,
                   j + 1 < s ? shadow16[lvl - 2][j & 1] : nullptr);
    } else {
      apply_level(lvl, B.sm[j], src, nsys);
    }
  }
  // Gram data <A p_i, A p_j> (i <= j) and <A p_i, t> in one pass over the basis
  double2* gram = slot(lvl, 0);
  auto fill = [&](auto& a) {
    using TP = decltype(a.u[0]);
    for (int j = 0; j < s; ++j) a.u[j] = (TP)B.sm[j].p;
    a.u[s] = (TP)t.p;
    a.s = s; a.n = t.n; a.stride = t.n; a.nrhs = nsys;
  };
  if (prec == P64) {
    GramArgs<double2> a{};
    fill(a);
    launch_gram(a, part, gram, max_sys, st);
  } else {
    GramArgs<float2> a{};
    fill(a);
    launch_gram(a, part, gram, max_sys, st);
  }
  check_launch();
  double2* a = slot(lvl, kSlotCoef);
  launch_cagcr_solve(gram, s, nsys, max_sys, lmask(lvl), a, st);
  check_launch();
  std::vector<std::pair<const void*, const double2*>> terms;
  terms.push_back({e.p, nullptr});
  terms.push_back({t.p, a});
  for (int j = 1; j < s; ++j) terms.push_back({B.sm[j - 1].p, a + (int64_t)j * max_sys});
  lincomb(prec, t.n, nsys, e.p, terms, {}, {});
}

// K_lvl(r) -> e (Sec. 2.1 K-cycle: no pre-smoothing, restrict, solve the next
// level to its tolerance, prolong, post-smooth)
void Ctx::kcycle(int lvl, const Vec& r, const Vec& e, int nsys, SolveStats& stats) {
  if (lvl == 0) {
    // only the masses with a system still iterating (kc_groups, nrhs systems
    // each) enter the K-cycle; their residuals are gathered, the result
    // scattered back and the other systems' directions left zero
    const bool compact = !kc_groups.empty();
    const int nall = nsys;
    if (compact) {
      const int64_t per = (int64_t)kc_nrhs * r.n;
      for (size_t ci = 0; ci < kc_groups.size(); ++ci) {
        Vec src{(char*)r.p + (size_t)kc_groups[ci] * per * csize(r.prec), r.prec, r.n};
        Vec dst{(char*)r0s.p + (size_t)ci * per * csize(r0s.prec), r0s.prec, r0s.n};
        copy(dst, src, kc_nrhs);
      }
      nsys = (int)kc_groups.size() * kc_nrhs;
      kc_compact = true;
    } else {
      copy(r0s, r, nsys);
    }
    // level 0 -> 1: r1 = (B + m)^{-1} r (in the fine precision), e0 = e1
    apply_KD(r0s.prec, L[1].b.p, r0s.p, nsys, false, false, rhs_per_slot);
    level_solve(1, nsys, stats);
    copy(e0s, L[1].x, nsys);
    // t = r - D e0
    apply_level(0, L[0].t, e0s, nsys);
    lincomb(r0s.prec, r0s.n, nsys, L[0].t.p, {{r0s.p, nullptr}, {L[0].t.p, nullptr}}, {0, 1}, {});
    smoother(0, e0s, L[0].t, nsys);
    if (compact) {
      kc_compact = false;
      zero(e, nall);
      const int64_t per = (int64_t)kc_nrhs * e.n;
      for (size_t ci = 0; ci < kc_groups.size(); ++ci) {
        Vec dst{(char*)e.p + (size_t)kc_groups[ci] * per * csize(e.prec), e.prec, e.n};
        Vec src{(char*)e0s.p + (size_t)ci * per * csize(e0s.prec), e0s.prec, e0s.n};
        copy(dst, src, kc_nrhs);
      }
    } else {
      copy(e, e0s, nsys);
    }
    return;
  }
  LevelBufs& B = L[lvl];
  LevelBufs& C = L[lvl + 1];
  restrict_(lvl, r.prec, C.b.p, r.p, nsys);
  level_solve(lvl + 1, nsys, stats);
  prolong_(lvl, r.prec, e.p, C.x.p, nsys, false);
  apply_level(lvl, B.t, e, nsys);
  lincomb(r.prec, r.n, nsys, B.t.p, {{r.p, nullptr}, {B.t.p, nullptr}}, {0, 1}, {});
  smoother(lvl, e, B.t, nsys);
}

// One flexible-GCR direction on level lvl: z_k already holds K(r).
// q_k = A z_k; classical Gram-Schmidt twice against q_0..q_{k-1} (the same
// combination applied to z_k); then x += alpha z_k, r -= alpha q_k with
// alpha = <q_k, r> / |q_k|^2 and q_k, z_k normalised, in one fused pass that
// also leaves |r|^2 per system in slot(lvl, kSlotRN).
void Ctx::gcr_step(int lvl, LevelBufs& B, const Vec& X, int k, int nsys) {
  const int prec = B.prec;
  const int64_t n = B.n;
  apply_level(lvl, B.q[k], B.z[k], nsys);
  for (int pass = 0; pass < 2 && k > 0; ++pass) {
    std::vector<std::pair<const void*, const void*>> pr;
    for (int i = 0; i < k; ++i) pr.push_back({B.q[i].p, B.q[k].p});
    double2* beta = slot(lvl, 0);
    dots(prec, n, nsys, pr, beta);
    project(prec, n, nsys, B, k, beta);
  }
  double2* qq = slot(lvl, kSlotQQ);
  dots(prec, n, nsys, {{B.q[k].p, B.q[k].p}, {B.q[k].p, B.r.p}}, qq);
  double2 *al = slot(lvl, kSlotQQ + 2), *nal = slot(lvl, kSlotQQ + 3), *inv = slot(lvl, kSlotQQ + 4);
  launch_gcr_scalars(qq, qq + max_sys, lmask(lvl), nsys, al, nal, inv, st);
  check_launch();
  if (prec == P64)
    launch_gcr_update<double2>((double2*)X.p, (double2*)B.r.p, (double2*)B.q[k].p, (double2*)B.z[k].p, al, inv, n,
                               nsys, part, slot(lvl, kSlotRN), max_sys, st);
  else
    launch_gcr_update<float2>((float2*)X.p, (float2*)B.r.p, (float2*)B.q[k].p, (float2*)B.z[k].p, al, inv, n, nsys,
                              part, slot(lvl, kSlotRN), max_sys, st);
  check_launch();
}

// q_k -= sum_i beta_i q_i and z_k -= sum_i beta_i z_i in one pass
void Ctx::project(int prec, int64_t n, int nsys, LevelBufs& B, int k, const double2* beta) {
  auto fill = [&](auto& a) {
    using TP = decltype(a.out);
    a.out = (TP)B.q[k].p;
    a.out2 = (TP)B.z[k].p;
    a.v[0] = (TP)B.q[k].p;
    a.v2[0] = (TP)B.z[k].p;
    a.cconst[0] = make_double2(1.0, 0.0);
    for (int i = 0; i < k; ++i) {
      a.v[i + 1] = (TP)B.q[i].p;
      a.v2[i + 1] = (TP)B.z[i].p;
      a.c[i + 1] = beta + (int64_t)i * max_sys;
      a.neg[i + 1] = 1;
    }
    a.nt = k + 1; a.n = n; a.stride = n; a.nrhs = nsys;
  };
  if (prec == P64) {
    LinCombArgs<double2> a{};
    fill(a);
    launch_lincomb(a, st);
  } else {
    LinCombArgs<float2> a{};
    fill(a);
    launch_lincomb(a, st);
  }
  check_launch();
}

std::vector<double> Ctx::read_norms(const double2* dev, int nsys) {
  std::vector<double2> h(nsys);
  HIPCHK(hipMemcpyAsync(h.data(), dev, nsys * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> out(nsys);
  for (int s = 0; s < nsys; ++s) out[s] = h[s].x >= 0.0 ? std::sqrt(h[s].x) : (h[s].x < 0.0 ? 0.0 : h[s].x);
  return out;
}

bool Ctx::any_active(int lvl, int nsys) {
  std::vector<int> h(nsys);
  HIPCHK(hipMemcpyAsync(h.data(), lmask(lvl), nsys * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int s = 0; s < nsys; ++s)
    if (h[s]) return true;
  return false;
}

// Flexible GCR on level lvl (>= 1) from x = 0 for L[lvl].b, preconditioned by
// the K-cycle except on the coarsest level; stops per system at
// ||r|| <= tol ||b|| or after the iteration cap (Table 1: 0.25 or 8).
// Convergence is tracked on the device (a converged system's updates become
// no-ops); the host reads the flags after every iteration, or every fourth
// on the coarsest level, whose iterations are short.
//
// The iterates are those of the flexible GCR with an orthonormal q basis, but
// the directions z_k are never orthogonalised: each step stores the
// projection coefficients beta(i, k) = <q_i, A z_k>, the norm g_k and
// alpha'_k = <q_k, r>, and the solution x = sum_k gamma_k z_k is formed once
// at the end of a cycle from the triangular system they define.  Per step the
// vector passes are: q_k = A z_k; one reduction pass (classical Gram-Schmidt
// coefficients with |q'|^2 from Pythagoras); one update pass.
void Ctx::level_solve(int lvl, int nsys, SolveStats& stats) {
  LevelBufs& B = L[lvl];
  const bool coarsest = lvl == nlev - 1;
  // A single CA-GCR cycle makes the coarsest solve a fixed sequence of
  // launches with no host decision: it is captured once per system count
  // (on a private stream) and replayed as one graph launch.
  if (coarsest && P.coarsest_solver == 1 && P.coarsest_restarts == 1 && P.graph_coarsest && !capturing &&
      !(prof_op >= 0 && prof_level == lvl)) {
    auto it = coarsest_graphs.find(nsys);
    if (it == coarsest_graphs.end()) {
      if (!capture_st) HIPCHK(hipStreamCreateWithFlags(&capture_st, hipStreamNonBlocking));
      hipStream_t user = st;
      st = capture_st;
      capturing = true;
      SolveStats dummy;
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        level_solve(lvl, nsys, dummy);
      } catch (...) {
        (void)hipStreamEndCapture(st, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        capturing = false;
        st = user;
        throw;
      }
      HIPCHK(hipStreamEndCapture(st, &graph));
      capturing = false;
      st = user;
      hipGraphExec_t exec = nullptr;
      const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) throw Error{MG_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
      it = coarsest_graphs.emplace(nsys, exec).first;
    }
    HIPCHK(hipGraphLaunch(it->second, st));
    stats.level[lvl - 1] += P.coarsest_maxiter;
    return;
  }
  const double tol = coarsest ? P.coarsest_tol : P.inner_tol;
  const int maxit = coarsest ? P.coarsest_maxiter : P.inner_maxiter;
  const int cycles = coarsest ? P.coarsest_restarts : 1;
  const int every = coarsest ? 4 : 1;
  const int prec = B.prec;
  const int64_t n = B.n;
  double2* r0 = slot(lvl, kSlotR0);
  // block-preconditioned coarse levels solve X^{-1} A x = X^{-1} b
  const bool blk = lvl >= 2 && P.coarse_op == 1;
  if (blk) apply_xinv(lvl, prec, B.r.p, B.b.p, nsys);
  const Vec& src = blk ? B.r : B.b;
  dots(prec, n, nsys, {{src.p, src.p}}, r0);
  // coarse levels solve for s b with a per-system power of two s (entries of
  // b of order one) and return x / s: the iterates are those of b scaled
  // exactly, and 16-bit stencil inputs stay in range at any residual size
  const bool scaled = lvl >= 2;
  if (scaled) {
    launch_rhs_scale(r0, slot(lvl, kSlotScale), slot(lvl, kSlotScale + 1), n, nsys, st);
    check_launch();
    auto fill = [&](auto& a) {
      using TP = decltype(a.out);
      a.out = (TP)B.b.p;
      a.out2 = (TP)B.r.p;
      a.v[0] = (TP)src.p;
      a.v2[0] = (TP)src.p;
      a.c[0] = slot(lvl, kSlotScale);
      a.nt = 1; a.n = n; a.stride = n; a.nrhs = nsys;
    };
    if (prec == P64) {
      LinCombArgs<double2> a{};
      fill(a);
      launch_lincomb(a, st);
    } else {
      LinCombArgs<float2> a{};
      fill(a);
      launch_lincomb(a, st);
    }
    check_launch();
  } else {
    copy(B.r, B.b, nsys);
  }
  launch_conv(lmask(lvl), nullptr, r0, tol * tol, nsys, 1, st);
  check_launch();
  if (coarsest && P.coarsest_solver == 2) {   // exact: x = A^{-1} b (one product)
    stats.level[lvl - 1] += 1;
    direct_apply(lvl, prec, B.x.p, B.b.p, nsys);
    if (scaled) lincomb(prec, n, nsys, B.x.p, {{B.x.p, slot(lvl, kSlotScale + 1)}}, {}, {});
    return;
  }
  const bool deflated = coarsest && defl_k > 0;
  if (deflated) deflate_start(lvl, nsys);   // x = W' Q^H b, r = b - Q Q^H b
  if (coarsest && P.coarsest_solver == 1) {
    coarsest_cagcr(lvl, nsys, stats, deflated);
    if (scaled) lincomb(prec, n, nsys, B.x.p, {{B.x.p, slot(lvl, kSlotScale + 1)}}, {}, {});
    return;
  }
  bool live = true;
  for (int cyc = 0; cyc < cycles && live; ++cyc) {
    if (cyc > 0) {   // restart: r = b - A x
      apply_level(lvl, B.r, B.x, nsys);
      lincomb(prec, n, nsys, B.r.p, {{B.b.p, nullptr}, {B.r.p, nullptr}}, {0, 1}, {});
    }
    int nk = 0;
    for (int k = 0; k < maxit; ++k) {
      stats.level[lvl - 1] += 1;
      if (!coarsest) kcycle(lvl, B.r, B.z[k], nsys, stats);
      else if (k == 0) copy(B.z[0], B.r, nsys);   // later directions come from the update pass
      gcr_direction(lvl, B, k, nsys, coarsest && k + 1 < maxit ? B.z[k + 1].p : nullptr);
      nk = k + 1;
      launch_conv(lmask(lvl), slot(lvl, kSlotRN), r0, tol * tol, nsys, 0, st);
      check_launch();
      if ((k + 1) % every == 0 || k + 1 == maxit) {
        if (!any_active(lvl, nsys)) { live = false; break; }
      }
    }
    gcr_flush(lvl, B, nk, nsys, cyc > 0 || deflated);
  }
  if (scaled) lincomb(prec, n, nsys, B.x.p, {{B.x.p, slot(lvl, kSlotScale + 1)}}, {}, {});
}

// x = A^{-1} b on the coarsest level (coarsest_solver 2): one column-major
// product, A^{-1} [n x n] times the nsys right-hand-side columns [n x nsys].
void Ctx::direct_apply(int lvl, int prec, void* x, const void* b, int nsys) {
  const int64_t n = L[lvl].n;
  auto fill = [&](auto& g, auto* Ainv) {
    using T = std::remove_const_t<std::remove_pointer_t<decltype(g.A)>>;
    g.A = Ainv; g.lda = n; g.sA = 0; g.a_div = 1;
    g.B = (const T*)b; g.ldb = n; g.sB = 0;
    g.C = (T*)x; g.ldc = n; g.sC = 0;
    g.m = (int)n; g.n = nsys; g.k = (int)n; g.batch = 1;
    g.alpha = 1.0; g.beta = 0.0;
    launch_bgemm(g, st);
  };
  if (prec == P64) {
    BGemmArgs<double2> g{};
    fill(g, dinv64);
  } else {
    BGemmArgs<float2> g{};
    fill(g, dinv32);
  }
  check_launch();
}

// CA-GCR(s) cycles on the coarsest level (Table 1: Chebyshev-basis CA-GCR):
// p_0 = r, p_1 = (A - c) p_0 / d, p_{j+1} = 2 (A - c) p_j / d - p_{j-1}, each
// p_j divided by g^j (g: the basis growth per step measured at set-up), with
// q_j = A p_j from the s operator applications; one Gram reduction of the
// q_j and r (FP64), an s x s Cholesky solve per system for the minimiser of
// |r - sum alpha_j q_j|, then x += sum alpha_j p_j, r -= sum alpha_j q_j.
// The cycle's result is the Krylov minimiser over K_s(A, r), whatever the
// basis; the Chebyshev one keeps the Gram matrix far better conditioned than
// powers of A.  Stops at |r| <= coarsest_tol |b| or after coarsest_restarts
// cycles.
void Ctx::coarsest_cagcr(int lvl, int nsys, SolveStats& stats, bool have_x) {
  LevelBufs& B = L[lvl];
  const int s = P.coarsest_maxiter;
  const int prec = B.prec;
  const int64_t n = B.n;
  const double c = cheb_c, d = cheb_d, gm = cheb_g;
  double2* gram = tslot(lvl, 0);
  double2* coef = tslot(lvl, 160);
  for (int cyc = 0; cyc < P.coarsest_restarts; ++cyc) {
    stats.level[lvl - 1] += s;
    copy(B.z[0], B.r, nsys);
    for (int j = 0; j < s; ++j) {
      apply_level(lvl, B.q[j], B.z[j], nsys);
      if (j + 1 == s) break;
      // p_j / gm^j: p_1 = (A - c) p_0 / (d gm), p_{j+1} = 2 (A - c) p_j / (d gm) - p_{j-1} / gm^2
      if (j == 0)
        lincomb(prec, n, nsys, B.z[1].p, {{B.q[0].p, nullptr}, {B.z[0].p, nullptr}}, {},
                {make_double2(1.0 / (d * gm), 0.0), make_double2(-c / (d * gm), 0.0)});
      else
        lincomb(prec, n, nsys, B.z[j + 1].p, {{B.q[j].p, nullptr}, {B.z[j].p, nullptr}, {B.z[j - 1].p, nullptr}}, {},
                {make_double2(2.0 / (d * gm), 0.0), make_double2(-2.0 * c / (d * gm), 0.0),
                 make_double2(-1.0 / (gm * gm), 0.0)});
    }
    auto fill = [&](auto& a) {
      using TP = decltype(a.u[0]);
      for (int j = 0; j < s; ++j) a.u[j] = (TP)B.q[j].p;
      a.u[s] = (TP)B.r.p;
      a.s = s; a.n = n; a.stride = n; a.nrhs = nsys;
    };
    if (prec == P64) {
      GramArgs<double2> a{};
      fill(a);
      launch_gram(a, part, gram, max_sys, st);
    } else {
      GramArgs<float2> a{};
      fill(a);
      launch_gram(a, part, gram, max_sys, st);
    }
    check_launch();
    launch_cagcr_solve(gram, s, nsys, max_sys, lmask(lvl), coef, st);
    check_launch();
    std::vector<std::pair<const void*, const double2*>> tx, tr;
    if (cyc > 0 || have_x) tx.push_back({B.x.p, nullptr});
    tr.push_back({B.r.p, nullptr});
    std::vector<int> nr{0};
    for (int j = 0; j < s; ++j) {
      tx.push_back({B.z[j].p, coef + (int64_t)j * max_sys});
      tr.push_back({B.q[j].p, coef + (int64_t)j * max_sys});
      nr.push_back(1);
    }
    lincomb(prec, n, nsys, B.x.p, tx, {}, {});
    lincomb(prec, n, nsys, B.r.p, tr, nr, {});
    if (cyc + 1 == P.coarsest_restarts) break;
    dots(prec, n, nsys, {{B.r.p, B.r.p}}, slot(lvl, kSlotRN));
    launch_conv(lmask(lvl), slot(lvl, kSlotRN), slot(lvl, kSlotR0), P.coarsest_tol * P.coarsest_tol, nsys, 0, st);
    check_launch();
    if (!any_active(lvl, nsys)) break;
  }
}

// Deflated start of the coarsest solve, 64 systems per pass:
// c = Q^H r, x = W' c, r -= Q c.
void Ctx::deflate_start(int lvl, int nsys) {
  LevelBufs& B = L[lvl];
  const int64_t n = B.n;
  for (int s0 = 0; s0 < nsys; s0 += kMaxDefl) {
    const int ns = std::min(kMaxDefl, nsys - s0);
    if (B.prec == P64) {
      double2* r = (double2*)B.r.p + (int64_t)s0 * n;
      double2* x = (double2*)B.x.p + (int64_t)s0 * n;
      launch_ts_gram<double2>((const double2*)defl_q, n, defl_k, r, n, ns, n, part, part_elems, defl_c, st);
      launch_ts_combine<double2>(x, n, (const double2*)defl_w, n, defl_k, ns, defl_c, n, 0, st);
      launch_ts_combine<double2>(r, n, (const double2*)defl_q, n, defl_k, ns, defl_c, n, -1, st);
    } else {
      float2* r = (float2*)B.r.p + (int64_t)s0 * n;
      float2* x = (float2*)B.x.p + (int64_t)s0 * n;
      launch_ts_gram<float2>((const float2*)defl_q, n, defl_k, r, n, ns, n, part, part_elems, defl_c, st);
      launch_ts_combine<float2>(x, n, (const float2*)defl_w, n, defl_k, ns, defl_c, n, 0, st);
      launch_ts_combine<float2>(r, n, (const float2*)defl_q, n, defl_k, ns, defl_c, n, -1, st);
    }
    check_launch();
  }
}

// Direction k of the deferred-update GCR (z_k already holds K(r)): q_k = A z_k,
// one reduction pass for every inner product the step needs (the projection
// coefficients, |q_k|^2, <q_k, r> and <q_i, r>), the scalars, and one update
// pass (projection, normalisation of q_k, r -= alpha q', |r|^2).  With znext
// the new r is also written there (the next direction of unpreconditioned GCR).
void Ctx::gcr_direction(int lvl, LevelBufs& B, int k, int nsys, void* znext) {
  const int prec = B.prec;
  const int64_t n = B.n;
  double2* T = tslot(lvl, 0);
  apply_level(lvl, B.q[k], B.z[k], nsys);
  auto run = [&](auto* tag) {
    using TP = std::remove_pointer_t<decltype(tag)>;
    GcrDotArgs<TP> d{};
    for (int i = 0; i < k; ++i) d.q[i] = (const TP*)B.q[i].p;
    d.qk = (const TP*)B.q[k].p;
    d.r = (const TP*)B.r.p;
    d.k = k; d.n = n; d.stride = n; d.nrhs = nsys;
    launch_gcr_dots(d, part, slot(lvl, 0), max_sys, st);
    launch_gcr_scalars_cgs(slot(lvl, 0), k, lmask(lvl), nsys, max_sys, T, slot(lvl, kSlotQQ + 2),
                           slot(lvl, kSlotQQ + 4), st);
    GcrUpdArgs<TP> u{};
    u.qk = (TP*)B.q[k].p;
    for (int i = 0; i < k; ++i) {
      u.q[i] = (const TP*)B.q[i].p;
      u.beta[i] = T + (int64_t)(i * kMaxNK + k) * max_sys;
    }
    u.r = (TP*)B.r.p;
    u.znext = (TP*)znext;
    u.alpha = slot(lvl, kSlotQQ + 2);
    u.inv = slot(lvl, kSlotQQ + 4);
    u.k = k; u.n = n; u.stride = n; u.nrhs = nsys;
    launch_gcr_update_cgs(u, part, slot(lvl, kSlotRN), max_sys, st);
  };
  if (prec == P64) run((double2*)nullptr);
  else run((float2*)nullptr);
  check_launch();
}

// x (+)= sum_{k < nk} gamma_k z_k with U gamma = alpha' (back substitution)
void Ctx::gcr_flush(int lvl, LevelBufs& B, int nk, int nsys, bool accumulate) {
  if (nk <= 0) return;
  double2* T = tslot(lvl, 0);
  launch_gcr_backsub(T, nk, nsys, max_sys, st);
  check_launch();
  std::vector<std::pair<const void*, const double2*>> terms;
  if (accumulate) terms.push_back({B.x.p, nullptr});
  for (int k = 0; k < nk; ++k) terms.push_back({B.z[k].p, T + (int64_t)(kTriC + k) * max_sys});
  lincomb(B.prec, B.n, nsys, B.x.p, terms, {}, {});
}

// ======================================================================== KD
// KD inverses live in max_nmass slots.  A batch needs its masses in
// consecutive slots kd_base, kd_base + 1, ...: an existing run is reused,
// otherwise a free run (or slot 0 onwards) is rebuilt.
void Ctx::ensure_kd(const std::vector<double>& masses) {
  const int nm = (int)masses.size();
  if (nm > P.max_nmass) throw Error{MG_E_ARG, "more masses than max_nmass"};
  for (int base = 0; base + nm <= P.max_nmass; ++base) {
    bool ok = true;
    for (int j = 0; j < nm && ok; ++j) ok = kd_mass[base + j] == masses[j];
    if (ok) { kd_base = base; return; }
  }
  int base = 0;
  for (int b = 0; b + nm <= P.max_nmass; ++b) {
    bool free_run = true;
    for (int j = 0; j < nm && free_run; ++j) free_run = std::isnan(kd_mass[b + j]);
    if (free_run) { base = b; break; }
  }
  for (int j = 0; j < nm; ++j) {
    const int sl = base + j;
    launch_kd_inverse(fat64, g0, masses[j], kinv64 + (int64_t)sl * kinv_slot, kinv32 + (int64_t)sl * kinv_slot, st);
    check_launch();
    kd_mass[sl] = masses[j];
  }
  kd_base = base;
}

// =================================================================== autotune
// Every tile shape of the 16-bit coarse stencil on the context's levels at
// nrhs right-hand sides, timed with HIP events; the fastest is kept for that
// rhs class.
void Ctx::autotune(int nrhs, mg_tune_info* info) {
  const int cls = rhs_class(nrhs);
  for (int l = 0; l < P.nagg; ++l) {
    mg_tune_info ti{};
    if (fmt16 < 0 || L[l + 2].prec != P32) {
      if (info) info[l] = ti;
      continue;
    }
    const int n = ncoarse[l];
    LevelBufs& B = L[l + 2];
    launch_random_normal<float2>((float2*)B.z[0].p, (int64_t)nrhs * B.n, P.seed + 99ull + l, st);
    check_launch();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_shape = [&](int rt, int mt) {
      CoarseMfmaArgs a{};
      a.out = (float2*)B.q[0].p; a.in = (const float2*)B.z[0].p; a.links = cl16[l];
      a.g = gc[l]; a.n = n; a.in_stride = a.out_stride = gc[l].V * n; a.nrhs = nrhs;
      a.inv_scale = cl16_inv_scale[l];
      a.unit_self = unit_self[l] ? 1 : 0;
      a.rt = rt; a.mt = mt;
      for (int w = 0; w < 2; ++w) launch_coarse_mfma(a, fmt16, st);
      HIPCHK(hipEventRecord(e0, st));
      for (int r = 0; r < 5; ++r) launch_coarse_mfma(a, fmt16, st);
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      return 1e3 * ms / 5.0;
    };
    try {
      ti.level = l + 2;
      ti.nrhs = nrhs;
      const int mt_def = nrhs > 16 && (n / 16) % 2 == 0 ? 2 : 1;
      const int rt_def = cls == 0 ? 1 : (cls == 1 ? 2 : 4);
      ti.us_default = time_shape(rt_def, cls == 0 ? 1 : mt_def);
      ti.us_best = ti.us_default;
      ti.rhs_per_workgroup = 16 * rt_def;
      ti.mtiles_per_wave = cls == 0 ? 1 : mt_def;
      for (const auto& sh : kCoarseTiles) {
        if ((n / 16) % sh[1]) continue;
        const double us = time_shape(sh[0], sh[1]);
        ++ti.candidates;
        if (us < ti.us_best) {
          ti.us_best = us;
          ti.rhs_per_workgroup = 16 * sh[0];
          ti.mtiles_per_wave = sh[1];
        }
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    tune[l][cls][0] = ti.rhs_per_workgroup / 16;
    tune[l][cls][1] = ti.mtiles_per_wave;
    if (info) info[l] = ti;
  }
}

}  // namespace mg
