// Outer solvers: MG-preconditioned flexible GCR in FP64 (Sec. 2.1, Table 1)
// and the single-parity Schur CG baseline (Sec. 3.2).  Both stop on the true
// residual ||b - D(m) x|| / ||b|| recomputed in FP64.
#include <chrono>
#include <cmath>

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

static double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Per-system masses of a [nmass][nrhs] batch on the device (FP64 and FP32)
static void set_masses(Ctx& c, const double* masses, int nmass, int nrhs) {
  const int ns = nmass * nrhs;
  std::vector<double> m64(ns);
  std::vector<float> m32(ns);
  for (int j = 0; j < nmass; ++j)
    for (int r = 0; r < nrhs; ++r) { m64[j * nrhs + r] = masses[j]; m32[j * nrhs + r] = (float)masses[j]; }
  HIPCHK(hipMemcpyAsync(c.mass64, m64.data(), ns * sizeof(double), hipMemcpyHostToDevice, c.st));
  HIPCHK(hipMemcpyAsync(c.mass32, m32.data(), ns * sizeof(float), hipMemcpyHostToDevice, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
}

// Systems are solved in lockstep batches of at most max_nrhs (mass, rhs)
// pairs: whole masses per batch, all right-hand sides of a mass together.
void Ctx::solve(const double* masses, int nmass, const void* b, void* x, int nrhs, double tol, mg_solve_info* info) {
  if (nrhs > P.max_nrhs) throw Error{MG_E_ARG, "nrhs exceeds max_nrhs"};
  const int per = std::max(1, P.max_nrhs / nrhs);
  for (int j0 = 0; j0 < nmass; j0 += per) {
    const int nm = std::min(per, nmass - j0);
    solve_batch(masses + j0, nm, b, (char*)x + (size_t)j0 * nrhs * g0.V * 3 * 16, nrhs, tol, info + j0 * nrhs);
  }
}

void Ctx::solve_batch(const double* masses, int nmass, const void* b, void* x, int nrhs, double tol,
                      mg_solve_info* info) {
  const int ns = nmass * nrhs;
  const double t0 = now();
  std::vector<double> ms(masses, masses + nmass);
  ensure_kd(ms);
  rhs_per_slot = nrhs;
  set_masses(*this, masses, nmass, nrhs);
  kc_groups.clear();
  kc_nrhs = nrhs;
  int ngroups_active = nmass;
  LevelBufs& B = L[0];
  const int64_t n = B.n;
  Vec X{x, P64, n};
  // b replicated per mass
  for (int j = 0; j < nmass; ++j)
    HIPCHK(hipMemcpyAsync((char*)B.b.p + (size_t)j * nrhs * n * 16, b, (size_t)nrhs * n * 16,
                          hipMemcpyDeviceToDevice, st));
  zero(X, ns);
  copy(B.r, B.b, ns);
  std::vector<double> bn, rn;
  norms_host(P64, n, ns, B.b.p, slot(0, kSlotNorm), bn);
  std::vector<int> act(ns), stat(ns, MG_OK);
  std::vector<double> rlast(bn);
  int nact = 0;
  for (int s = 0; s < ns; ++s) {
    if (!std::isfinite(bn[s])) { stat[s] = MG_E_NONFINITE; act[s] = 0; }
    else act[s] = bn[s] > 0.0;
    nact += act[s];
  }
  int* mk = lmask(0);
  HIPCHK(hipMemcpyAsync(mk, act.data(), ns * sizeof(int), hipMemcpyHostToDevice, st));
  SolveStats stats;
  std::vector<int> iters(ns, 0), rel_upd(ns, 0);
  int k = 0;
  auto true_residual = [&]() {   // r = b - D x for every system (FP64)
    apply_level(0, B.r, X, ns);
    lincomb(P64, n, ns, B.r.p, {{B.b.p, nullptr}, {B.r.p, nullptr}}, {0, 1}, {});
    norms_host(P64, n, ns, B.r.p, slot(0, kSlotNorm), rn);
  };
  for (int it = 0; it < P.outer_maxiter && nact > 0; ++it) {
    kcycle(0, B.r, B.z[k], ns, stats);
    gcr_step(0, B, X, k, ns);
    rn = read_norms(slot(0, kSlotRN), ns);
    bool check = false, reliable = false, nonfinite = false;
    for (int s = 0; s < ns; ++s) {
      if (!act[s]) continue;
      iters[s] += 1;
      if (!std::isfinite(rn[s])) nonfinite = true;
      else if (rn[s] <= tol * bn[s]) check = true;
      else if (rn[s] < P.reliable_delta * rlast[s]) reliable = true;
    }
    const bool restart = k + 1 == P.outer_nkrylov;
    if (check || reliable || restart || nonfinite) {
      // reliable update: replace the recursive residual by b - D x (FP64)
      true_residual();
      bool changed = false;
      for (int s = 0; s < ns; ++s) {
        if (!act[s]) continue;
        rel_upd[s] += 1;
        rlast[s] = rn[s];
        if (!std::isfinite(rn[s])) { act[s] = 0; --nact; stat[s] = MG_E_NONFINITE; changed = true; }
        else if (rn[s] <= tol * bn[s]) { act[s] = 0; --nact; changed = true; }
      }
      if (changed && nact > 0) HIPCHK(hipMemcpyAsync(mk, act.data(), ns * sizeof(int), hipMemcpyHostToDevice, st));
      if (changed && nact > 0 && P.compact_masses && nmass > 1) {
        // masses whose systems have all converged leave the K-cycle's batch
        std::vector<int> groups;
        for (int j = 0; j < nmass; ++j) {
          bool on = false;
          for (int r = 0; r < nrhs; ++r) on = on || act[j * nrhs + r];
          if (on) groups.push_back(j);
        }
        if ((int)groups.size() < ngroups_active) {
          ngroups_active = (int)groups.size();
          kc_groups = groups;
          std::vector<double> gm;
          for (int j : groups) gm.push_back(masses[j]);
          ensure_kd(gm);   // the K-cycle's masses in consecutive inverse slots
          const int nc = (int)groups.size() * nrhs;
          std::vector<double> m64(nc);
          std::vector<float> m32(nc);
          for (size_t ci = 0; ci < groups.size(); ++ci)
            for (int r = 0; r < nrhs; ++r) {
              m64[ci * nrhs + r] = masses[groups[ci]];
              m32[ci * nrhs + r] = (float)masses[groups[ci]];
            }
          HIPCHK(hipMemcpyAsync(mass64 + max_sys, m64.data(), nc * sizeof(double), hipMemcpyHostToDevice, st));
          HIPCHK(hipMemcpyAsync(mass32 + max_sys, m32.data(), nc * sizeof(float), hipMemcpyHostToDevice, st));
          HIPCHK(hipStreamSynchronize(st));   // before the host arrays go
        }
        if (!kc_groups.empty()) {   // level-0 mask of the K-cycle's systems
          kc_mask.resize((size_t)kc_groups.size() * nrhs);
          for (size_t ci = 0; ci < kc_groups.size(); ++ci)
            for (int r = 0; r < nrhs; ++r) kc_mask[ci * nrhs + r] = act[kc_groups[ci] * nrhs + r];
          HIPCHK(hipMemcpyAsync(mask + (int64_t)4 * max_sys, kc_mask.data(), kc_mask.size() * sizeof(int),
                                hipMemcpyHostToDevice, st));
          HIPCHK(hipStreamSynchronize(st));   // host buffers are reused
        }
      }
      k = restart ? 0 : k + 1;
    } else {
      k += 1;
    }
  }
  kc_groups.clear();
  true_residual();
  HIPCHK(hipStreamSynchronize(st));
  const double t1 = now();
  for (int s = 0; s < ns; ++s) {
    mg_solve_info& I = info[s];
    I.outer_iters = iters[s];
    I.reliable_updates = rel_upd[s];
    for (int l = 0; l < 4; ++l) I.level_iters[l] = stats.level[l];
    I.true_rel_residual = bn[s] > 0 ? rn[s] / bn[s] : 0.0;
    I.seconds = t1 - t0;
    if (stat[s] == MG_OK && !(I.true_rel_residual <= tol)) stat[s] = MG_E_NOCONV;
    I.status = stat[s];
  }
}

// Fermion force (HMC use of the solver, Sec. 4.2): X = (D^dag D)^{-1} phi and
// Y = D X from two MG solves, D^dag = eps D eps giving Y = eps D^{-1} (eps phi)
// and then X = D^{-1} Y, followed by the outer-product kernel.
void Ctx::solve_backward(double mass, const void* phi, void* X, void* Y, void* gw, void* gn, int nrhs, double tol,
                         double* action, mg_solve_info* info) {
  launch_eps<double2>((double2*)X, (const double2*)phi, g0, nrhs, st);
  check_launch();
  solve(&mass, 1, X, Y, nrhs, tol, info);
  launch_eps<double2>((double2*)Y, (const double2*)Y, g0, nrhs, st);
  check_launch();
  solve(&mass, 1, Y, X, nrhs, tol, info + nrhs);
  launch_force((const double2*)X, (const double2*)Y, (double2*)gw, P.c3 != 0.0 ? (double2*)gn : nullptr, g0, nrhs,
               P.c1, P.c3, 0, st);
  check_launch();
  if (action) {   // S_r = Re <phi_r, X_r>, one FP64 reduction per right-hand side
    dots(P64, g0.V * 3, nrhs, {{phi, X}}, slot(0, kSlotNorm));
    std::vector<double2> h(nrhs);
    HIPCHK(hipMemcpyAsync(h.data(), slot(0, kSlotNorm), nrhs * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) action[r] = h[r].x;
  }
  HIPCHK(hipStreamSynchronize(st));
}

// New gauge links for an existing hierarchy: the fine operator and the KD
// inverses follow the new links, the near-null vectors, transfers and coarse
// operators stay those built at set-up (the hierarchy is then a
// preconditioner for a nearby operator; the outer solve is exact).
void Ctx::update_links(const void* fat, const void* naik) {
  launch_pack_links((const double2*)fat, fat64, fat32, fat32p, g0, 0.5 * P.c1, st);
  check_launch();
  if (P.c3 != 0.0) {
    pack_naik(naik);
    check_launch();
  }
  for (auto& m : kd_mass) m = NAN;
  HIPCHK(hipStreamSynchronize(st));
}

// Single-parity Schur CG (Sec. 3.2) for every (mass, rhs) system, one mass
// at a time with the right-hand sides batched.
void Ctx::cg_solve(const double* masses, int nmass, const void* b, void* x, int nrhs, double tol, int maxiter,
                   mg_solve_info* info, bool guess) {
  if (P.outer_nkrylov < 2) throw Error{MG_E_CONFIG, "the CG baseline needs outer_nkrylov >= 2 (work vectors)"};
  const int64_t V = g0.V;
  const int64_t n = V * 3, nh = V / 2 * 3;
  LevelBufs& B = L[0];
  // half-lattice batches carved from the outer GCR work vectors
  const size_t hb = (size_t)nrhs * nh * 16;
  double2* be = (double2*)B.z[0].p;
  double2* bo = (double2*)((char*)B.z[0].p + hb);
  double2* xe = (double2*)B.q[0].p;
  double2* r = (double2*)((char*)B.q[0].p + hb);
  double2* p = (double2*)B.z[1].p;
  double2* Ap = (double2*)((char*)B.z[1].p + hb);
  double2* to = (double2*)B.q[1].p;
  double2* rhs = (double2*)((char*)B.q[1].p + hb);
  double2* xo = (double2*)B.r.p;     // odd half, then the full residual
  double2* rfull = (double2*)B.b.p;
  int* mk = lmask(0);
  double2 *rr = slot(0, kSlotQQ), *rrn = slot(0, kSlotQQ + 1), *al = slot(0, kSlotQQ + 2),
          *nal = slot(0, kSlotQQ + 3), *bt = slot(0, kSlotQQ + 4), *pap = slot(0, kSlotQQ + 5);
  for (int j = 0; j < nmass; ++j) {
    const double t0 = now();
    const double m = masses[j];
    double2* xj = (double2*)x + (size_t)j * nrhs * n;
    auto cbd = [&](double2* out, const double2* in, const double2* xs, int par, double ac, double bc) {
      DslashArgs<double> d{};
      d.out = out; d.in = in; d.xs = xs; d.fat = fat64; d.lng = lng64;
      d.lng_c = naik_compressed ? lng64c : nullptr;
      d.g = g0;
      d.in_stride = d.out_stride = d.xs_stride = nh; d.nrhs = nrhs; d.a_coef = ac; d.b_coef = bc; d.parity = par;
      launch_dslash(d, P.c3 != 0.0, true, false, st);
      check_launch();
    };
    launch_cb_split((const double2*)b, be, bo, g0, nrhs, st);
    check_launch();
    cbd(rhs, bo, be, 0, m, -1.0);   // m b_e - K_eo b_o
    std::vector<double> bn, rn;
    norms_host(P64, n, nrhs, b, slot(0, kSlotNorm), bn);
    std::vector<int> act(nrhs), stat(nrhs, MG_OK), its(nrhs, 0);
    int nact = 0;
    for (int s = 0; s < nrhs; ++s) {
      act[s] = bn[s] > 0.0 && std::isfinite(bn[s]);
      if (!std::isfinite(bn[s])) stat[s] = MG_E_NONFINITE;
      nact += act[s];
    }
    if (guess) {
      // start from the even half of the caller's x (xo is scratch here)
      launch_cb_split(xj, xe, xo, g0, nrhs, st);
      check_launch();
    } else {
      HIPCHK(hipMemsetAsync(xe, 0, hb, st));
    }
    int total = 0, restarts = 0;
    std::vector<double> rel(nrhs, 0.0);
    while (true) {
      // r = rhs - M xe,  M = m^2 - K_eo K_oe
      cbd(to, xe, nullptr, 1, 0.0, 1.0);
      cbd(r, to, xe, 0, m * m, -1.0);
      lincomb(P64, nh, nrhs, r, {{rhs, nullptr}, {r, nullptr}}, {0, 1}, {});
      HIPCHK(hipMemcpyAsync(p, r, hb, hipMemcpyDeviceToDevice, st));
      norms_host(P64, nh, nrhs, r, rr, rn);
      HIPCHK(hipMemcpyAsync(mk, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
      auto done = [&](int s) { return !(rn[s] > m * tol * bn[s]); };
      int live = 0;
      for (int s = 0; s < nrhs; ++s) if (act[s] && !done(s)) ++live;
      for (int s = 0; s < nrhs; ++s) if (act[s] && done(s)) act[s] = 0;
      HIPCHK(hipMemcpyAsync(mk, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
      // device-side convergence: a system stops updating once |r| <= m tol |b|
      // (its alpha becomes 0); the host looks at the flags every few iterations
      std::vector<double2> tgt(nrhs);
      for (int s = 0; s < nrhs; ++s) tgt[s] = make_double2(bn[s] * bn[s], 0.0);
      double2* b2 = slot(0, kSlotR0);
      HIPCHK(hipMemcpyAsync(b2, tgt.data(), nrhs * sizeof(double2), hipMemcpyHostToDevice, st));
      const double tol2 = (m * tol) * (m * tol);
      int since = 0;
      while (live > 0 && total < maxiter) {
        cbd(to, p, nullptr, 1, 0.0, 1.0);
        cbd(Ap, to, p, 0, m * m, -1.0);
        dots(P64, nh, nrhs, {{p, Ap}}, pap);
        launch_cg_alpha(rr, pap, mk, nrhs, al, nal, st);
        check_launch();
        launch_cg_update(xe, r, p, Ap, al, nh, nrhs, part, rrn, max_sys, st);
        check_launch();
        launch_conv(mk, rrn, b2, tol2, nrhs, 0, st);
        launch_cg_beta(rr, rrn, mk, nrhs, bt, st);
        check_launch();
        lincomb(P64, nh, nrhs, p, {{r, nullptr}, {p, bt}}, {}, {});
        ++total;
        for (int s = 0; s < nrhs; ++s) if (act[s]) its[s] += 1;
        if (++since == 4 || total >= maxiter) {
          since = 0;
          std::vector<int> h(nrhs);
          HIPCHK(hipMemcpyAsync(h.data(), mk, nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          live = 0;
          for (int s = 0; s < nrhs; ++s) {
            if (act[s] && !h[s]) act[s] = 0;
            live += act[s];
          }
        }
      }
      // x_o = (b_o - K_oe x_e) / m, then the true residual of the full system
      cbd(xo, xe, bo, 1, 1.0 / m, -1.0 / m);
      launch_cb_merge(xj, xe, xo, g0, nrhs, st);
      check_launch();
      apply_D(P64, rfull, xj, nrhs, true, nullptr, m);
      lincomb(P64, n, nrhs, rfull, {{b, nullptr}, {rfull, nullptr}}, {0, 1}, {});
      std::vector<double> tr;
      norms_host(P64, n, nrhs, rfull, slot(0, kSlotNorm), tr);
      bool again = false;
      for (int s = 0; s < nrhs; ++s) {
        rel[s] = bn[s] > 0 ? tr[s] / bn[s] : 0.0;
        act[s] = stat[s] == MG_OK && bn[s] > 0 && !(rel[s] <= tol) && std::isfinite(rel[s]);
        if (!std::isfinite(rel[s])) stat[s] = MG_E_NONFINITE;
        again = again || act[s];
      }
      if (!again || total >= maxiter || restarts >= 5) break;
      ++restarts;
    }
    HIPCHK(hipStreamSynchronize(st));
    const double t1 = now();
    for (int s = 0; s < nrhs; ++s) {
      mg_solve_info& I = info[j * nrhs + s];
      I.outer_iters = its[s];
      I.reliable_updates = restarts;
      for (int l = 0; l < 4; ++l) I.level_iters[l] = 0;
      I.true_rel_residual = rel[s];
      I.seconds = t1 - t0;
      if (stat[s] == MG_OK && !(rel[s] <= tol)) stat[s] = MG_E_NOCONV;
      I.status = stat[s];
    }
  }
}

// Multi-shift CG over all masses at once (Sec. 3.3 workflow).  D(m)^{-1} b =
// (m - K) y with (m^2 - K^2) y = b; m^2 - K^2 is block-diagonal in parity,
// so each parity is one CG on the smallest shift sigma_0 = m_0^2 whose
// Krylov space also gives every (sigma_j - K_pq K_qp) y_j = b_p, with
// collinear residuals zeta_j r.  A shift stops at |zeta_j r| <= tol |b| / 2
// per parity; x_j = m_j y_j - K y_j is then checked on the true residual and a
// system that misses tol is finished by the single-mass Schur CG from x_j.
void Ctx::msc_solve(const double* masses, int nmass, const void* b, void* x, int nrhs, double tol, int maxiter,
                    mg_solve_info* info) {
  if (nmass > kMaxShift) throw Error{MG_E_ARG, "multi-shift CG takes at most 16 masses"};
  if (P.outer_nkrylov < 2) throw Error{MG_E_CONFIG, "multi-shift CG needs outer_nkrylov >= 2 (work vectors)"};
  const double t0 = now();
  const int64_t V = g0.V;
  const int64_t n = V * 3, nh = V / 2 * 3;
  LevelBufs& B = L[0];
  const size_t hb = (size_t)nrhs * nh * 16;
  // sources of both parities, base residual, A p and K p
  double2* be = (double2*)B.b.p;
  double2* bo = (double2*)((char*)B.b.p + hb);
  double2* r = (double2*)B.r.p;
  double2* Ap = (double2*)((char*)B.r.p + hb);
  double2* to = (double2*)B.q[0].p;
  // search directions: blocks of nrhs half vectors in z[0..], q[1..]
  std::vector<double2*> pblk;
  const int per = (int)((2 * (int64_t)P.max_nrhs) / nrhs);
  for (int k = 0; k < P.outer_nkrylov; ++k)
    for (int h = 0; h < per; ++h) {
      pblk.push_back((double2*)((char*)B.z[k].p + h * hb));
      if (k > 0) pblk.push_back((double2*)((char*)B.q[k].p + h * hb));
    }
  if ((int)pblk.size() < nmass)
    throw Error{MG_E_CONFIG, "multi-shift CG: nmass x nrhs exceeds the work space (raise outer_nkrylov or max_nrhs)"};
  int base = 0;
  for (int j = 1; j < nmass; ++j)
    if (masses[j] < masses[base]) base = j;
  const double s0 = masses[base] * masses[base];
  double2* stt = tslot(1, 0);   // shifted-system state (the inner GCR scalars are idle here)
  const int ld = max_sys;
  int* mk = lmask(0);
  double2 *rr = slot(0, kSlotQQ), *rrn = slot(0, kSlotQQ + 1), *al = slot(0, kSlotQQ + 2),
          *nal = slot(0, kSlotQQ + 3), *pap = slot(0, kSlotQQ + 5), *tg = slot(0, kSlotR0);
  std::vector<double> bn;
  norms_host(P64, n, nrhs, b, slot(0, kSlotNorm), bn);
  std::vector<int> stat(nrhs, MG_OK);
  std::vector<double2> tgt(nrhs);
  for (int s = 0; s < nrhs; ++s) {
    if (!std::isfinite(bn[s])) stat[s] = MG_E_NONFINITE;
    const double t = 0.5 * tol * bn[s];
    tgt[s] = make_double2(std::isfinite(t) ? t * t : 0.0, 0.0);
  }
  HIPCHK(hipMemcpyAsync(tg, tgt.data(), nrhs * sizeof(double2), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(x, 0, (size_t)nmass * nrhs * n * 16, st));
  launch_cb_split((const double2*)b, be, bo, g0, nrhs, st);
  check_launch();
  // v (half, parity 1 - par) -> out (half, parity par): out = ac xs + bc K v
  auto cbd = [&](double2* out, const double2* in, const double2* xs, int par, double ac, double bc, int64_t sin,
                 int64_t sxs) {
    DslashArgs<double> d{};
    d.out = out; d.in = in; d.xs = xs; d.fat = fat64; d.lng = lng64;
    d.lng_c = naik_compressed ? lng64c : nullptr;
    d.g = g0;
    d.in_stride = sin; d.xs_stride = sxs; d.out_stride = nh; d.nrhs = nrhs; d.a_coef = ac; d.b_coef = bc;
    d.parity = par;
    launch_dslash(d, P.c3 != 0.0, true, false, st);
    check_launch();
  };
  std::vector<double> iters_sys((size_t)nmass * nrhs, 0.0);
  int total = 0;
  for (int par = 0; par < 2; ++par) {
    const double2* bp = par == 0 ? be : bo;
    HIPCHK(hipMemcpyAsync(r, bp, hb, hipMemcpyDeviceToDevice, st));
    for (int j = 0; j < nmass; ++j) HIPCHK(hipMemcpyAsync(pblk[j], bp, hb, hipMemcpyDeviceToDevice, st));
    dots(P64, nh, nrhs, {{r, r}}, rr);
    launch_msc_init(stt, rr, tg, mk, nmass, nrhs, ld, st);
    check_launch();
    MscScalArgs sa{};
    sa.st = stt; sa.rr = rr; sa.rrnew = rrn; sa.alpha = al; sa.target2 = tg; sa.mask = mk;
    for (int j = 0; j < nmass; ++j) sa.delta[j] = masses[j] * masses[j] - s0;
    sa.nshift = nmass; sa.base = base; sa.nrhs = nrhs; sa.ld = ld;
    MscUpdArgs ua{};
    for (int j = 0; j < nmass; ++j) {
      ua.x[j] = (double2*)x + (size_t)j * nrhs * n + par * nh;
      ua.p[j] = pblk[j];
    }
    ua.r = r; ua.st = stt; ua.n = nh; ua.x_stride = n; ua.p_stride = nh; ua.r_stride = nh;
    ua.nshift = nmass; ua.nrhs = nrhs; ua.ld = ld;
    double2* pb = pblk[base];
    int live = nrhs, it = 0, since = 0;
    while (live > 0 && it < maxiter) {
      // A0 p = sigma_0 p - K_pq K_qp p
      cbd(to, pb, nullptr, 1 - par, 0.0, 1.0, nh, nh);
      cbd(Ap, to, pb, par, s0, -1.0, nh, nh);
      dots(P64, nh, nrhs, {{pb, Ap}}, pap);
      launch_cg_alpha(rr, pap, mk, nrhs, al, nal, st);
      check_launch();
      // r -= alpha A p and |r|^2 (every x, the base's included, is updated below)
      launch_cg_update(nullptr, r, pb, Ap, al, nh, nrhs, part, rrn, max_sys, st);
      check_launch();
      launch_msc_scalars(sa, st);
      check_launch();
      launch_msc_update(ua, st);
      check_launch();
      ++it;
      if (++since == 4 || it >= maxiter) {
        since = 0;
        std::vector<int> h(nrhs);
        HIPCHK(hipMemcpyAsync(h.data(), mk, nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        live = 0;
        for (int s = 0; s < nrhs; ++s) live += h[s] != 0;
      }
    }
    total += it;
    std::vector<double2> cnt((size_t)nmass * ld);
    for (int j = 0; j < nmass; ++j)
      HIPCHK(hipMemcpyAsync(cnt.data() + (size_t)j * ld, stt + (int64_t)(kMscPer * j + 7) * ld, ld * sizeof(double2),
                            hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int j = 0; j < nmass; ++j)
      for (int s = 0; s < nrhs; ++s) iters_sys[(size_t)j * nrhs + s] += cnt[(size_t)j * ld + s].x;
  }
  // x_j = (m_j - K) y_j, parity by parity into the r / A p halves, then merged
  double2* te = r;
  double2* tod = Ap;
  double2* rfull = (double2*)B.b.p;
  std::vector<int> redo(nmass, 0);
  std::vector<double> rel((size_t)nmass * nrhs, 0.0);
  for (int j = 0; j < nmass; ++j) {
    const double m = masses[j];
    double2* yj = (double2*)x + (size_t)j * nrhs * n;
    cbd(te, yj + nh, yj, 0, m, -1.0, n, n);
    cbd(tod, yj, yj + nh, 1, m, -1.0, n, n);
    launch_cb_merge(yj, te, tod, g0, nrhs, st);
    check_launch();
    apply_D(P64, rfull, yj, nrhs, true, nullptr, m);
    lincomb(P64, n, nrhs, rfull, {{b, nullptr}, {rfull, nullptr}}, {0, 1}, {});
    std::vector<double> tr;
    norms_host(P64, n, nrhs, rfull, slot(0, kSlotNorm), tr);
    for (int s = 0; s < nrhs; ++s) {
      const double q = bn[s] > 0 ? tr[s] / bn[s] : 0.0;
      rel[(size_t)j * nrhs + s] = q;
      if (stat[s] == MG_OK && bn[s] > 0 && !(q <= tol)) redo[j] = 1;
    }
  }
  const double t1 = now();
  for (int j = 0; j < nmass; ++j)
    for (int s = 0; s < nrhs; ++s) {
      mg_solve_info& I = info[j * nrhs + s];
      I.outer_iters = (int)iters_sys[(size_t)j * nrhs + s];
      I.reliable_updates = 0;
      for (int l = 0; l < 4; ++l) I.level_iters[l] = 0;
      I.level_iters[0] = total;
      I.true_rel_residual = rel[(size_t)j * nrhs + s];
      I.seconds = t1 - t0;
      I.status = stat[s] != MG_OK ? stat[s] : MG_OK;
    }
  // finish the systems the iterated residual let through (rounding drift)
  for (int j = 0; j < nmass; ++j) {
    if (!redo[j]) continue;
    std::vector<mg_solve_info> fix(nrhs);
    cg_solve(masses + j, 1, b, (double2*)x + (size_t)j * nrhs * n, nrhs, tol, maxiter, fix.data(), true);
    for (int s = 0; s < nrhs; ++s) {
      mg_solve_info& I = info[j * nrhs + s];
      I.outer_iters += fix[s].outer_iters;
      I.reliable_updates = 1 + fix[s].reliable_updates;
      I.true_rel_residual = fix[s].true_rel_residual;
      I.status = fix[s].status;
    }
  }
}

}  // namespace mg
