// C ABI of the mgstag library (declared in include/mgstag.h).  Every entry
// point validates its arguments, runs the work inside a try block and maps
// failures to an mg_status with a thread-local message.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "mg.hpp"

using namespace mg;

static thread_local std::string g_err;

static mg_status fail(mg_status s, const std::string& m) {
  g_err = m;
  return s;
}

mg_status mg::set_last_error(mg_status s, const std::string& m) { return fail(s, m); }

template <typename F>
static mg_status guarded(F&& f) {
  try {
    f();
    return MG_OK;
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(MG_E_ARG, "host allocation failed");
  } catch (...) {
    return fail(MG_E_ARG, "unexpected exception");
  }
}

static bool aligned(const void* p) { return ((uintptr_t)p & 15) == 0; }

static mg_status check_vec(int32_t dtype, const void* in, const void* out, int32_t nrhs, int max) {
  if (!in || !out) return fail(MG_E_ARG, "null vector");
  if (in == out) return fail(MG_E_ARG, "input and output must be distinct");
  if (dtype != MG_C128 && dtype != MG_C64) return fail(MG_E_ARG, "dtype must be MG_C128 or MG_C64");
  if (nrhs < 1 || nrhs > max) return fail(MG_E_ARG, "nrhs out of range (1..max_nrhs)");
  if (!aligned(in) || !aligned(out)) return fail(MG_E_ALIGN, "vectors must be 16-byte aligned");
  return MG_OK;
}

mg_status mg::apply_dslash_with(Ctx& c, int32_t op, double mass, int32_t dtype, const void* in, void* out,
                                int32_t nrhs, void* stream, void* tmp) {
  mg_status s = check_vec(dtype, in, out, nrhs, c.P.max_nrhs);
  if (s != MG_OK) return s;
  if (op < 0 || op > 4) return fail(MG_E_ARG, "op must be 0..4");
  if (!std::isfinite(mass)) return fail(MG_E_ARG, "mass must be finite");
  c.st = (hipStream_t)stream;
  const int prec = dtype == MG_C128 ? P64 : P32;
  return guarded([&] {
    if (op == 0) {
      c.apply_D(prec, out, in, nrhs, true, nullptr, mass);
    } else if (op == 3) {
      // D^dag = eps D eps
      if (prec == P64) launch_eps<double2>((double2*)tmp, (const double2*)in, c.g0, nrhs, c.st);
      else launch_eps<float2>((float2*)tmp, (const float2*)in, c.g0, nrhs, c.st);
      c.apply_D(prec, out, tmp, nrhs, true, nullptr, mass, true);
    } else {
      c.ensure_kd(std::vector<double>{mass});
      c.rhs_per_slot = 0;
      const int64_t off = (int64_t)c.kd_base * c.kinv_slot;
      if (op == 4) {
        // A^dag = eps D (B + m)^{-1} eps
        c.apply_KD(prec, tmp, in, nrhs, true, false, 0);
        c.apply_D(prec, out, tmp, nrhs, c.P.kd_naik != 0, nullptr, mass, true);
      } else if (op == 2) {
        if (prec == P64) {
          KdArgs<double> a{};
          a.out = (double2*)out; a.in = (const double2*)in; a.kinv = c.kinv64 + off; a.g = c.g0;
          a.in_stride = a.out_stride = c.g0.V * 3; a.nrhs = nrhs; a.slot_stride = c.kinv_slot;
          launch_kd_apply(a, c.st);
        } else {
          KdArgs<float> a{};
          a.out = (float2*)out; a.in = (const float2*)in; a.kinv = c.kinv32 + off; a.g = c.g0;
          a.in_stride = a.out_stride = c.g0.V * 3; a.nrhs = nrhs; a.slot_stride = c.kinv_slot;
          launch_kd_apply(a, c.st);
        }
      } else {
        c.apply_kd_operator(prec, out, in, tmp, nrhs, nullptr, mass, 0);
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) throw Error{MG_E_HIP, hipGetErrorString(e)};
    }
  });
}

extern "C" {

const char* mg_last_error(void) { return g_err.c_str(); }

void mg_default_params(mg_params* p, const int32_t dims[4]) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  for (int mu = 0; mu < 4; ++mu) p->dims[mu] = dims ? dims[mu] : 4;
  p->c1 = 9.0 / 8.0;
  p->c3 = -1.0 / 24.0;
  p->kd_naik = 1;
  p->mass0 = 0.01;
  p->nagg = 2;
  for (int mu = 0; mu < 4; ++mu) { p->block[0][mu] = 4; p->block[1][mu] = 2; }
  p->nvec[0] = 64;
  p->nvec[1] = 96;
  p->setup_maxiter[0] = p->setup_maxiter[1] = 2000;
  p->setup_tol[0] = p->setup_tol[1] = 1e-6;
  p->smoother_s = 8;
  p->inner_tol = 0.25;
  p->inner_maxiter = 8;
  p->coarsest_tol = 0.25;
  p->coarsest_maxiter = 16;
  p->coarsest_restarts = 1;
  p->outer_nkrylov = 16;
  p->outer_maxiter = 500;
  p->reliable_delta = 0.1;
  p->fine_prec = MG_C64;
  p->coarse_prec = MG_C64;
  p->max_nrhs = 1;
  p->max_nmass = 1;
  p->coarsest_deflate = 0;
  p->deflate_maxiter = 300;
  p->deflate_import = 0;
  p->coarse_op = 1;   // Table 1: preconditioned coarse operators on levels 2 and 3
  p->coarsest_solver = 1;   // Table 1: Chebyshev-basis CA-GCR(16) on the coarsest level
  p->graph_coarsest = 1;
  p->compact_masses = 1;
  p->coarse_shadow = 0;   // measured no faster on the 64-rhs level-2 stencil
  p->cgne_start_import = 0;
  p->seed = 20221224ull;
}

mg_status mg_workspace_bytes(const mg_params* p, size_t* persistent, size_t* scratch) {
  if (!p || !persistent || !scratch) return fail(MG_E_ARG, "null argument");
  Arena a, b;
  std::string why;
  if (!Ctx::plan(*p, nullptr, a, b, &why)) return fail(MG_E_CONFIG, why);
  *persistent = a.off + 256;
  *scratch = b.off + 256;
  return MG_OK;
}

mg_status mg_setup(const mg_params* p, const void* fat, const void* naik, const void* const* null_vectors,
                   void* persistent_ws, size_t persistent_bytes, void* scratch_ws, size_t scratch_bytes,
                   void* stream, mg_ctx* out) {
  if (!p || !fat || !persistent_ws || !scratch_ws || !out) return fail(MG_E_ARG, "null argument");
  if (p->c3 != 0.0 && !naik) return fail(MG_E_ARG, "naik links required when c3 != 0");
  if (((uintptr_t)persistent_ws & 255) || ((uintptr_t)scratch_ws & 255))
    return fail(MG_E_ALIGN, "workspaces must be 256-byte aligned");
  if (!aligned(fat) || (naik && !aligned(naik))) return fail(MG_E_ALIGN, "links must be 16-byte aligned");
  size_t need_p = 0, need_s = 0;
  mg_status s = mg_workspace_bytes(p, &need_p, &need_s);
  if (s != MG_OK) return s;
  if (persistent_bytes < need_p || scratch_bytes < need_s) return fail(MG_E_WORKSPACE, "workspace too small");
  if (null_vectors)
    for (int l = 0; l < p->nagg + (p->coarsest_deflate > 0 && p->deflate_import ? 1 : 0); ++l)
      if (null_vectors[l] && !aligned(null_vectors[l])) return fail(MG_E_ALIGN, "null vectors must be 16-byte aligned");
  mg_ctx ctx = new (std::nothrow) mg_ctx_s;
  if (!ctx) return fail(MG_E_ARG, "host allocation failed");
  Arena pa, sa;
  pa.base = (char*)persistent_ws;
  pa.cap = persistent_bytes;
  sa.base = (char*)scratch_ws;
  sa.cap = scratch_bytes;
  std::string why;
  if (!Ctx::plan(*p, &ctx->c, pa, sa, &why)) {
    delete ctx;
    return fail(MG_E_CONFIG, why);
  }
  ctx->c.st = (hipStream_t)stream;
  s = noalloc_init_current_device();   // static work array of mg_apply_dslash_noalloc on this device
  if (s != MG_OK) {
    delete ctx;
    return s;
  }
  s = guarded([&] { ctx->c.setup(fat, naik, null_vectors); });
  if (s != MG_OK) {
    delete ctx;
    return s;
  }
  *out = ctx;
  return MG_OK;
}


mg_status mg_apply_dslash(mg_ctx ctx, int32_t op, double mass, int32_t dtype, const void* in, void* out,
                          int32_t nrhs, void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  // work batch: the first K-cycle direction of level 0 (FP64-sized, max_sys systems)
  return apply_dslash_with(ctx->c, op, mass, dtype, in, out, nrhs, stream, ctx->c.L[0].z[0].p);
}

mg_status mg_apply_coarse(mg_ctx ctx, int32_t level, int32_t dtype, const void* in, void* out, int32_t nrhs,
                          void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  mg_status s = check_vec(dtype, in, out, nrhs, c.P.max_nrhs);
  if (s != MG_OK) return s;
  if (level < 2 || level > 1 + c.P.nagg) return fail(MG_E_ARG, "level must be 2..1+nagg");
  c.st = (hipStream_t)stream;
  return guarded([&] { c.apply_coarse(level, dtype == MG_C128 ? P64 : P32, out, in, nrhs, false); });
}

mg_status mg_restrict(mg_ctx ctx, int32_t level, int32_t dtype, const void* fine, void* coarse, int32_t nrhs,
                      void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  mg_status s = check_vec(dtype, fine, coarse, nrhs, c.P.max_nrhs);
  if (s != MG_OK) return s;
  if (level < 1 || level > c.P.nagg) return fail(MG_E_ARG, "level must be 1..nagg");
  c.st = (hipStream_t)stream;
  return guarded([&] { c.restrict_(level, dtype == MG_C128 ? P64 : P32, coarse, fine, nrhs); });
}

mg_status mg_prolong(mg_ctx ctx, int32_t level, int32_t dtype, const void* coarse, void* fine,
                     int32_t accumulate, int32_t nrhs, void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  mg_status s = check_vec(dtype, coarse, fine, nrhs, c.P.max_nrhs);
  if (s != MG_OK) return s;
  if (level < 1 || level > c.P.nagg) return fail(MG_E_ARG, "level must be 1..nagg");
  c.st = (hipStream_t)stream;
  return guarded([&] { c.prolong_(level, dtype == MG_C128 ? P64 : P32, fine, coarse, nrhs, accumulate != 0); });
}

static mg_status check_solve(Ctx& c, const double* masses, int32_t nmass, const void* b, void* x, int32_t nrhs,
                             double tol, mg_solve_info* info) {
  if (!masses || !b || !x || !info) return fail(MG_E_ARG, "null argument");
  if (nmass < 1 || nrhs < 1) return fail(MG_E_ARG, "nmass and nrhs must be >= 1");
  if (nrhs > c.P.max_nrhs) return fail(MG_E_ARG, "nrhs exceeds max_nrhs");
  if (std::min(nmass, std::max(1, c.P.max_nrhs / nrhs)) > c.P.max_nmass)
    return fail(MG_E_ARG, "a batch would hold more masses than max_nmass");
  for (int j = 0; j < nmass; ++j)
    if (!(masses[j] > 0.0) || !std::isfinite(masses[j])) return fail(MG_E_ARG, "masses must be positive and finite");
  if (!(tol > 0.0)) return fail(MG_E_ARG, "tol must be positive");
  if (!aligned(b) || !aligned(x)) return fail(MG_E_ALIGN, "vectors must be 16-byte aligned");
  if (b == x) return fail(MG_E_ARG, "b and x must be distinct");
  return MG_OK;
}

mg_status mg_solve(mg_ctx ctx, const double* masses, int32_t nmass, const void* b, void* x, int32_t nrhs,
                   double tol, mg_solve_info* info, void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  mg_status s = check_solve(c, masses, nmass, b, x, nrhs, tol, info);
  if (s != MG_OK) return s;
  c.st = (hipStream_t)stream;
  s = guarded([&] { c.solve(masses, nmass, b, x, nrhs, tol, info); });
  if (s != MG_OK) return s;
  for (int i = 0; i < nmass * nrhs; ++i)
    if (info[i].status != MG_OK) return fail((mg_status)info[i].status, "a system did not converge");
  return MG_OK;
}

mg_status mg_cg_solve(mg_ctx ctx, const double* masses, int32_t nmass, const void* b, void* x, int32_t nrhs,
                      double tol, int32_t maxiter, mg_solve_info* info, void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  mg_status s = check_solve(c, masses, nmass, b, x, nrhs, tol, info);
  if (s != MG_OK) return s;

  if (maxiter < 1) return fail(MG_E_ARG, "maxiter must be >= 1");
  c.st = (hipStream_t)stream;
  s = guarded([&] { c.cg_solve(masses, nmass, b, x, nrhs, tol, maxiter, info); });
  if (s != MG_OK) return s;
  for (int i = 0; i < nmass * nrhs; ++i)
    if (info[i].status != MG_OK) return fail((mg_status)info[i].status, "a system did not converge");
  return MG_OK;
}

mg_status mg_msc_solve(mg_ctx ctx, const double* masses, int32_t nmass, const void* b, void* x, int32_t nrhs,
                       double tol, int32_t maxiter, mg_solve_info* info, void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  if (!masses || !b || !x || !info) return fail(MG_E_ARG, "null argument");
  if (nmass < 1 || nmass > 16) return fail(MG_E_ARG, "nmass must be in 1..16");
  if (nrhs < 1 || nrhs > c.P.max_nrhs) return fail(MG_E_ARG, "nrhs out of range (1..max_nrhs)");
  for (int j = 0; j < nmass; ++j)
    if (!(masses[j] > 0.0) || !std::isfinite(masses[j])) return fail(MG_E_ARG, "masses must be positive and finite");
  if (!(tol > 0.0)) return fail(MG_E_ARG, "tol must be positive");
  if (maxiter < 1) return fail(MG_E_ARG, "maxiter must be >= 1");
  if (!aligned(b) || !aligned(x)) return fail(MG_E_ALIGN, "vectors must be 16-byte aligned");
  if (b == x) return fail(MG_E_ARG, "b and x must be distinct");
  c.st = (hipStream_t)stream;
  mg_status s = guarded([&] { c.msc_solve(masses, nmass, b, x, nrhs, tol, maxiter, info); });
  if (s != MG_OK) return s;
  for (int i = 0; i < nmass * nrhs; ++i)
    if (info[i].status != MG_OK) return fail((mg_status)info[i].status, "a system did not converge");
  return MG_OK;
}

mg_status mg_solve_backward(mg_ctx ctx, double mass, const void* phi, void* X, void* Y, void* grad_fat,
                            void* grad_naik, int32_t nrhs, double tol, double* action, mg_solve_info* info,
                            void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  if (!phi || !X || !Y || !grad_fat || !info) return fail(MG_E_ARG, "null argument");
  if (c.P.c3 != 0.0 && !grad_naik) return fail(MG_E_ARG, "grad_naik required when c3 != 0");
  if (nrhs < 1 || nrhs > c.P.max_nrhs) return fail(MG_E_ARG, "nrhs out of range (1..max_nrhs)");
  if (!(mass > 0.0) || !std::isfinite(mass)) return fail(MG_E_ARG, "mass must be positive and finite");
  if (!(tol > 0.0)) return fail(MG_E_ARG, "tol must be positive");
  if (phi == X || phi == Y || X == Y) return fail(MG_E_ARG, "phi, X and Y must be distinct");
  if (!aligned(phi) || !aligned(X) || !aligned(Y) || !aligned(grad_fat) || (grad_naik && !aligned(grad_naik)))
    return fail(MG_E_ALIGN, "buffers must be 16-byte aligned");
  c.st = (hipStream_t)stream;
  mg_status s = guarded([&] { c.solve_backward(mass, phi, X, Y, grad_fat, grad_naik, nrhs, tol, action, info); });
  if (s != MG_OK) return s;
  for (int i = 0; i < 2 * nrhs; ++i)
    if (info[i].status != MG_OK) return fail((mg_status)info[i].status, "a solve did not converge");
  return MG_OK;
}

mg_status mg_update_links(mg_ctx ctx, const void* fat, const void* naik, void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  if (!fat || (c.P.c3 != 0.0 && !naik)) return fail(MG_E_ARG, "null links");
  if (!aligned(fat) || (naik && !aligned(naik))) return fail(MG_E_ALIGN, "links must be 16-byte aligned");
  c.st = (hipStream_t)stream;
  return guarded([&] { c.update_links(fat, naik); });
}

mg_status mg_export(mg_ctx ctx, int32_t what, int32_t level, void* dst, size_t bytes, size_t* bytes_needed,
                    void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  size_t need = 0;
  if (what == 0) {
    need = (size_t)c.g0.V * 22 * 4;
  } else if (what == 1) {
    if (level == c.P.nagg + 1 && c.defl_k > 0) {
      need = (size_t)c.defl_k * c.defl_n * 16;
    } else {
      if (level < 1 || level > c.P.nagg) return fail(MG_E_ARG, "level must be 1..nagg (nagg + 1: deflation vectors)");
      const Agg& a = c.A[level - 1];
      need = (size_t)a.nvec * a.nagg * 2 * a.nrows * 16;
    }
  } else if (what == 2) {
    if (level < 2 || level > 1 + c.P.nagg) return fail(MG_E_ARG, "level must be 2..1+nagg");
    const int n = c.ncoarse[level - 2];
    need = (size_t)c.gc[level - 2].V * 9 * n * n * 16;
  } else {
    return fail(MG_E_ARG, "what must be 0, 1 or 2");
  }
  if (bytes_needed) *bytes_needed = need;
  if (!dst) return MG_OK;
  if (bytes < need) return fail(MG_E_ARG, "destination too small");
  c.st = (hipStream_t)stream;
  return guarded([&] {
    if (what == 0) {
      launch_export_fine_index((int32_t*)dst, c.g0, c.A[0], c.st);
    } else if (what == 1) {
      hipError_t e = hipMemcpyAsync(dst, c.nv[level - 1], need, hipMemcpyDeviceToDevice, c.st);   // nv[nagg]: deflation
      if (e != hipSuccess) throw Error{MG_E_HIP, hipGetErrorString(e)};
    } else {
      launch_export_links(c.cl64[level - 2], (double2*)dst, c.gc[level - 2].V, c.ncoarse[level - 2], c.st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{MG_E_HIP, hipGetErrorString(e)};
  });
}

mg_status mg_apply_coarse_multi(const mg_ctx* ctxs, int32_t nprob, int32_t level, const void* const* in,
                                void* const* out, const int32_t* nrhs, void* stream) {
  if (!ctxs || !in || !out || !nrhs) return fail(MG_E_ARG, "null argument");
  if (nprob < 1 || nprob > kMaxMulti) return fail(MG_E_ARG, "nprob must be in 1..8");
  CoarseMultiArgs m{};
  int fmt = -1;
  int64_t start = 0;
  for (int p = 0; p < nprob; ++p) {
    if (!ctxs[p]) return fail(MG_E_ARG, "null context");
    Ctx& c = ctxs[p]->c;
    if (level < 2 || level > 1 + c.P.nagg) return fail(MG_E_ARG, "level must be 2..1+nagg of every context");
    if (c.fmt16 < 0) return fail(MG_E_ARG, "every context needs 16-bit coarse links");
    if (fmt >= 0 && c.fmt16 != fmt) return fail(MG_E_ARG, "contexts must share the 16-bit format");
    fmt = c.fmt16;
    const int l = level - 2;
    if (p > 0 && c.ncoarse[l] != m.p[0].n) return fail(MG_E_ARG, "contexts must share 2 Nvec on the level");
    mg_status s = check_vec(MG_C64, in[p], out[p], nrhs[p], c.P.max_nrhs);
    if (s != MG_OK) return s;
    CoarseMfmaArgs& a = m.p[p];
    a.out = (float2*)out[p]; a.in = (const float2*)in[p]; a.links = c.cl16[l];
    a.g = c.gc[l]; a.n = c.ncoarse[l]; a.in_stride = a.out_stride = c.gc[l].V * c.ncoarse[l]; a.nrhs = nrhs[p];
    a.inv_scale = c.cl16_inv_scale[l];
    a.unit_self = c.unit_self[l] ? 1 : 0;
    m.start[p] = start;
    start += c.gc[l].V * ((nrhs[p] + 15) / 16);
  }
  m.start[nprob] = start;
  m.nprob = nprob;
  return guarded([&] {
    launch_coarse_mfma_multi(m, fmt, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{MG_E_HIP, hipGetErrorString(e)};
  });
}

mg_status mg_autotune(mg_ctx ctx, int32_t nrhs, mg_tune_info* info, void* stream) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  Ctx& c = ctx->c;
  if (nrhs < 1 || nrhs > c.P.max_nrhs) return fail(MG_E_ARG, "nrhs out of range (1..max_nrhs)");
  c.st = (hipStream_t)stream;
  if (info) std::memset(info, 0, 2 * sizeof(mg_tune_info));
  return guarded([&] { c.autotune(nrhs, info); });
}

mg_status mg_profile_start(mg_ctx ctx, int32_t op, int32_t level, int32_t nrhs) {
  if (!ctx) return fail(MG_E_ARG, "null context");
  if (op < MG_PROF_COARSE || op > MG_PROF_PROLONG) return fail(MG_E_ARG, "op must be an mg_prof_op");
  if (nrhs < 0) return fail(MG_E_ARG, "nrhs must be 0 (every launch) or positive");
  Ctx& c = ctx->c;
  c.prof_op = op;
  c.prof_level = level;
  c.prof_nrhs = nrhs;
  c.prof_used = 0;
  return MG_OK;
}

mg_status mg_profile_stop(mg_ctx ctx, int32_t* launches, double* total_ms) {
  if (!ctx || !launches || !total_ms) return fail(MG_E_ARG, "null argument");
  Ctx& c = ctx->c;
  return guarded([&] {
    double sum = 0.0;
    const size_t pairs = c.prof_used / 2;
    if (pairs > 0) {
      hipError_t e = hipEventSynchronize(c.prof_events[2 * pairs - 1]);
      if (e != hipSuccess) throw Error{MG_E_HIP, std::string("hipEventSynchronize: ") + hipGetErrorString(e)};
      for (size_t i = 0; i < pairs; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, c.prof_events[2 * i], c.prof_events[2 * i + 1]);
        if (e != hipSuccess) throw Error{MG_E_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e)};
        sum += ms;
      }
    }
    *launches = (int32_t)pairs;
    *total_ms = sum;
    c.prof_op = -1;
    c.prof_used = 0;
  });
}

mg_status mg_destroy(mg_ctx ctx) {
  delete ctx;
  return MG_OK;
}

}  // extern "C"
