// Host-side multigrid context: workspace layout, hierarchy set-up and the
// GCR / CA-GCR / K-cycle / CG drivers.
#pragma once
#include <map>
#include <string>
#include <vector>

#include "../../include/mgstag.h"
#include "kernels.hpp"

namespace mg {

struct Error {
  mg_status code;
  std::string msg;
};

// Records the thread-local message that mg_last_error returns; returns s.
mg_status set_last_error(mg_status s, const std::string& msg);

// A batch of nrhs vectors of n complex numbers each, contiguous per rhs.
struct Vec {
  void* p = nullptr;
  int prec = P64;
  int64_t n = 0;
};

// Bump allocator over a caller-owned workspace; a dry run (base == nullptr)
// measures the size.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

struct LevelBufs {
  int prec = P32;
  int64_t n = 0;            // complex numbers per system
  Vec b, x, r, t, tmp;
  Vec z[kMaxNK], q[kMaxNK];
  Vec sm[kMaxS];
  int nk = 0;
};

struct SolveStats {
  int outer = 0, reliable = 0;
  int level[4] = {0, 0, 0, 0};
};

struct Ctx {
  mg_params P{};
  hipStream_t st = nullptr;
  int nlev = 0;             // levels: 0 (D), 1 (A), 2, 3
  Geom g0{};                // fine lattice
  Geom gc[2]{};             // coarse lattices of levels 2 and 3
  Agg A[2]{};               // aggregation 1 -> 2 and 2 -> 3
  int ncoarse[2]{};         // 2 nvec per level

  // persistent
  double2 *fat64 = nullptr, *lng64 = nullptr;
  float2 *fat32 = nullptr, *lng32 = nullptr;
  float4* fat32p = nullptr;   // FP32 fat links as element pairs [4][5][V]
  double2* lng64c = nullptr;  // Naik links in 13-real form [4][7][V] (used when they are unitary)
  float2* lng32c = nullptr;
  bool naik_compressed = false;
  double2* kinv64 = nullptr;
  float2* kinv32 = nullptr;
  int64_t kinv_slot = 0;    // complex per slot
  std::vector<double> kd_mass;   // mass of each slot (NaN: empty)
  double2* nv[3]{};         // null vectors, canonical per-level layout; nv[nagg]: coarsest deflation vectors
  // coarsest deflation: k vectors of n; Q = A W R^{-1}, W' = W R^{-1} (level precision),
  // coefficients c [k][max_sys], Gram / R / R^{-1} k x k (FP64)
  int defl_k = 0;
  int64_t defl_n = 0;
  void* defl_q = nullptr;
  void* defl_w = nullptr;
  double2* defl_c = nullptr;
  double2* defl_g = nullptr;
  double2* defl_rm = nullptr;
  double2* defl_rinv = nullptr;
  double2 *pp64[2]{}, *pr64[2]{};
  float2 *pp32[2]{}, *pr32[2]{};
  double2* cl64[2]{};       // coarse links of levels 2 and 3
  float2* cl32[2]{};
  uint16_t* cl16[2]{};      // 16-bit MFMA fragments (coarse_prec BF16 / FP16)
  float cl16_inv_scale[2]{1.0f, 1.0f};
  double2* xinv64[2]{};     // coarse_op 1: X^{-1} per coarse site [site][col][row]
  bool unit_self[2]{};      // the stored self block is exactly the identity (the 16-bit stencil skips it)
  uint32_t* shadow16[2][2]{};   // 16-bit copies of the smoother chain's outputs per coarse level (coarse_shadow)
  double cheb_c = 1.0, cheb_d = 1.0;   // CA-GCR coarsest solver: Chebyshev basis of (A - c) / d
  double cheb_g = 1.0;                 // its per-step growth: basis vector j is divided by cheb_g^j
  int tune[2][3][2]{};      // autotuned (rt, mt) of the 16-bit stencil per level and rhs class (0: built-in)
  std::map<int, hipGraphExec_t> coarsest_graphs;   // captured coarsest solves, by system count
  hipStream_t capture_st = nullptr;
  bool capturing = false;
  // a K-cycle on the active masses only: their group indices (nrhs systems
  // each, in batch order); kc_compact while it runs (masses, level-0 mask)
  std::vector<int> kc_groups;
  int kc_nrhs = 0;
  bool kc_compact = false;
  std::vector<int> kc_mask;
  float2* xinv32[2]{};
  int fmt16 = -1;           // -1: none, 0: bf16, 1: fp16
  bool setup_phase = false;
  int* status_dev = nullptr;

  // scratch (solver)
  int max_sys = 0;
  LevelBufs L[4];
  Vec x0s, r0s, e0s;        // level-0 K-cycle in fine precision (x0s unused)
  double2* part = nullptr;  // reduction partials
  double2* scal = nullptr;  // scalar slots [level][kMaxSlots][max_sys]
  double2* tri = nullptr;   // deferred-update GCR scalars [level][kTriSlots][max_sys]
  double* mass64 = nullptr; // per-system masses (device)
  float* mass32 = nullptr;
  int* mask = nullptr;      // per-system active flag (device)
  // scratch (set-up, aliases the solver scratch)
  char* scratch_base = nullptr;
  size_t scratch_cap = 0;
  size_t part_elems = 0;     // double2 entries of the reduction partials

  // current batch
  int nsys = 0;
  int rhs_per_slot = 0;     // systems per KD slot in the current batch
  int kd_base = 0;          // first KD slot of the current batch

  std::vector<double> host_buf;

  // kernel timing: while prof_op >= 0, every launch of that operator (at
  // prof_level where it has one) is bracketed by a pair of HIP events
  int prof_op = -1, prof_level = 0, prof_nrhs = 0;   // prof_nrhs > 0: only launches over that many systems
  std::vector<hipEvent_t> prof_events;
  size_t prof_used = 0;
  void prof_mark(int op, int level, int nsys);   // records the next event when (op, level, nsys) is profiled
  ~Ctx();

  // ---- layout
  static bool plan(const mg_params& p, Ctx* c, Arena& pers, Arena& scr, std::string* why);

  // ---- operators (all on stream st, batch of nsys systems)
  void apply_level(int lvl, const Vec& out, const Vec& in, int nsys);
  void apply_D(int prec, void* out, const void* in, int nsys, bool naik, const void* mass_rhs, double mass,
               bool eps_out = false);
  void apply_KD(int prec, void* out, const void* in, int nsys, bool eps_in, bool eps_out, int rhs_per_slot);
  void apply_kd_operator(int prec, void* out, const void* in, void* tmp, int nsys, const void* mass_rhs,
                         double mass, int rps);   // (B+m)^{-1} D, as 1 + (B+m)^{-1} D_off where it can
  void apply_coarse(int lvl, int prec, void* out, const void* in, int nsys, bool dag,
                    const uint32_t* in16 = nullptr, uint32_t* out16 = nullptr);
  void restrict_(int lvl, int prec, void* out, const void* in, int nsys);
  void prolong_(int lvl, int prec, void* out, const void* in, int nsys, bool acc);

  // ---- BLAS helpers
  double2* slot(int lvl, int s) { return scal + ((int64_t)lvl * kMaxSlots + s) * max_sys; }
  double2* tslot(int lvl, int s) { return tri + ((int64_t)lvl * kTriSlots + s) * max_sys; }
  int* lmask(int lvl) { return mask + (int64_t)(lvl == 0 && kc_compact ? 4 : lvl) * max_sys; }
  void dots(int prec, int64_t n, int nsys, const std::vector<std::pair<const void*, const void*>>& pairs,
            double2* res);
  void lincomb(int prec, int64_t n, int nsys, void* out,
               const std::vector<std::pair<const void*, const double2*>>& terms, const std::vector<int>& neg,
               const std::vector<double2>& consts);
  void copy(const Vec& dst, const Vec& src, int nsys);
  void zero(const Vec& v, int nsys);
  void norms_host(int prec, int64_t n, int nsys, const void* v, double2* res_dev, std::vector<double>& out);

  // ---- solvers
  void smoother(int lvl, const Vec& e, const Vec& t, int nsys);
  void kcycle(int lvl, const Vec& r, const Vec& e, int nsys, SolveStats& stats);
  void level_solve(int lvl, int nsys, SolveStats& stats);   // L[lvl].b -> L[lvl].x
  void gcr_step(int lvl, LevelBufs& B, const Vec& X, int k, int nsys);
  void gcr_direction(int lvl, LevelBufs& B, int k, int nsys, void* znext);
  void gcr_flush(int lvl, LevelBufs& B, int nk, int nsys, bool accumulate);
  void project(int prec, int64_t n, int nsys, LevelBufs& B, int k, const double2* beta);
  std::vector<double> read_norms(const double2* dev, int nsys);
  bool any_active(int lvl, int nsys);
  void ensure_kd(const std::vector<double>& masses);

  // ---- set-up
  void setup(const void* fat, const void* naik, const void* const* nvs);
  void solve(const double* masses, int nmass, const void* b, void* x, int nrhs, double tol, mg_solve_info* info);
  void solve_batch(const double* masses, int nmass, const void* b, void* x, int nrhs, double tol,
                   mg_solve_info* info);
  void cg_solve(const double* masses, int nmass, const void* b, void* x, int nrhs, double tol, int maxiter,
                mg_solve_info* info, bool guess = false);
  void msc_solve(const double* masses, int nmass, const void* b, void* x, int nrhs, double tol, int maxiter,
                 mg_solve_info* info);
  void solve_backward(double mass, const void* phi, void* X, void* Y, void* gw, void* gn, int nrhs, double tol,
                      double* action, mg_solve_info* info);
  void update_links(const void* fat, const void* naik);
  void build_level(int l, const void* nv_import);
  void pack_naik(const void* naik);
  void cgne_null(int l, int nvec, int64_t n, int maxiter, double tol, double2* out, const double2* start = nullptr);
  void build_deflation(const void* nv_import);
  void deflate_start(int lvl, int nsys);
  void coarsest_cagcr(int lvl, int nsys, SolveStats& stats, bool have_x);
  void estimate_lambda_max();
  double2* dinv64 = nullptr;            // coarsest_solver 2: A^{-1} of the coarsest operator (column-major)
  float2* dinv32 = nullptr;
  void build_direct();                  // set-up: dense coarsest inverse by Gauss-Jordan
  void direct_apply(int lvl, int prec, void* x, const void* b, int nsys);   // x = A^{-1} b
  void galerkin(int l);
  void finish_links(int l);          // FP32 copy and 16-bit fragments of cl64[l]
  void precondition_links(int l);    // X^{-1} and cl64[l] <- X^{-1} cl64[l] (coarse_op 1)
  void apply_xinv(int lvl, int prec, void* out, const void* in, int nsys);
  void autotune(int nrhs, mg_tune_info* info);
  static int rhs_class(int nrhs) { return nrhs <= 16 ? 0 : (nrhs <= 32 ? 1 : 2); }
};

// Body of mg_apply_dslash with the work batch given: tmp holds nrhs fine
// vectors of the dtype (ops 1, 3 and 4 stage an intermediate there).
mg_status apply_dslash_with(Ctx& c, int32_t op, double mass, int32_t dtype, const void* in, void* out,
                            int32_t nrhs, void* stream, void* tmp);
// Looks up the device address of the static work array of
// mg_apply_dslash_noalloc on the current device (once per device).
mg_status noalloc_init_current_device();

}  // namespace mg

struct mg_ctx_s {
  mg::Ctx c;
};
