"""Oracle solvers and the multigrid hierarchy: flexible GCR, the minimal
residual smoother, the K-cycle, CGNE near-null vectors and the Schur CG
baseline.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy, complex128.

Readings of the paper used here (it leaves these open):
  * inner solves stop at ||r|| <= 0.25 ||r_in|| or 8 iterations, whichever
    comes first (Table 1);
  * the smoother CA-GCR(s) is defined by what it computes, the minimiser of
    ||r - A v|| over the Krylov space K_s(A, r) from a zero guess; the oracle
    computes that minimiser with s steps of Arnoldi (MGS) and a small
    least-squares solve;
  * the coarsest level is unpreconditioned GCR to a tolerance / iteration
    cap, or a dense LU solve; its deflation (Table 1 deflates it with
    singular vectors) is read as a minimal-residual start on the span of
    given low modes of the coarsest operator (mr_deflation);
  * near-null vectors: CG on A A^dag y = -A phi0, phi = phi0 + A^dag y
    (CGNE on the homogeneous system, Sec. 2.1 and Table 1), stopping at
    ||A phi|| <= tol ||A phi0|| or maxiter.  PARITY UNPINNED: a long random
    iteration; tests only check quality metrics.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import operators as ops


def _norm(v):
    return float(np.sqrt(np.vdot(v, v).real))


# --------------------------------------------------------------------------
# Krylov building blocks
# --------------------------------------------------------------------------

@dataclass
class SolveInfo:
    iters: int = 0
    converged: bool = False
    history: list = field(default_factory=list)   # recursive ||r|| / ||b|| per iteration
    true_rel_residual: float = float("nan")
    restarts: int = 0


def gcr(op, b, precond=None, tol=1e-10, maxiter=1000, nkrylov=16, true_residual=False):
    """Flexible GCR (Sec. 2.1) with modified Gram-Schmidt, zero initial guess.

    Each iteration: z = K(r), q = A z, orthogonalise q against the stored
    q_i (applying the same combination to z), normalise, then
    x += alpha z, r -= alpha q with alpha = <q, r>.  After nkrylov
    directions the space is discarded and r = b - A x recomputed.
    With true_residual=True the stop test is the recomputed ||b - A x||.
    """
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = _norm(b)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged = True
        info.true_rel_residual = 0.0
        return x, info
    Z, Q = [], []
    for it in range(maxiter):
        z = precond(r) if precond is not None else r.copy()
        q = op(z)
        for zi, qi in zip(Z, Q):
            beta = np.vdot(qi, q)
            q = q - beta * qi
            z = z - beta * zi
        g = _norm(q)
        q = q / g
        z = z / g
        alpha = np.vdot(q, r)
        x = x + alpha * z
        r = r - alpha * q
        Z.append(z)
        Q.append(q)
        info.iters = it + 1
        rel = _norm(r) / bnorm
        info.history.append(rel)
        if rel <= tol:
            if not true_residual:
                info.converged = True
                break
            r = b - op(x)
            Z, Q = [], []
            info.restarts += 1
            if _norm(r) / bnorm <= tol:
                info.converged = True
                break
            continue
        if len(Z) == nkrylov:
            r = b - op(x)
            Z, Q = [], []
            info.restarts += 1
    if true_residual:
        info.true_rel_residual = _norm(b - op(x)) / bnorm
    return x, info


def mr_deflation(op, Wv):
    """Coarsest-level deflation space (Sec. 2.3 / Table 1: the coarsest solve is
    deflated with low modes of its operator).  Reading used here: the space is
    spanned by given vectors W (rows of Wv, near-null vectors of the coarsest
    operator A), and the deflated start is the minimal-residual one,
        x0 = W y,  y = argmin ||b - A W y||,
    formed through a Cholesky QR of Z = A W:  Z^H Z = R^H R (R upper),
    Q = Z R^{-1}, W' = W R^{-1}, so x0 = W' Q^H b and r0 = b - Q Q^H b.
    Returns (Q, W') as rows.  Pinned by a least-squares solve
    (tests/test_oracle_solvers.py)."""
    Wm = np.stack([w.reshape(-1) for w in Wv], axis=1)             # n x k
    Zm = np.stack([op(w).reshape(-1) for w in Wv], axis=1)         # n x k
    G = Zm.conj().T @ Zm
    R = np.linalg.cholesky(G).conj().T                               # G = R^H R
    Rinv = np.linalg.inv(R)
    return (Zm @ Rinv).T, (Wm @ Rinv).T


def mr_deflate(Q, Wp, b):
    """x0 = W' Q^H b and r0 = b - Q Q^H b for the space of mr_deflation."""
    c = Q.conj() @ b.reshape(-1)
    return (Wp.T @ c).reshape(b.shape), (b.reshape(-1) - Q.T @ c).reshape(b.shape)


def mr_smoother(op, r, s):
    """v = argmin_{v in K_s(A, r)} ||r - A v||  (the smoother's result).

    Computed with s steps of Arnoldi (MGS) from v_0 = r/||r|| and the
    (s+1) x s least-squares problem min ||beta e_1 - H y||.
    """
    beta = _norm(r)
    if beta == 0.0:
        return np.zeros_like(r)
    V = [r / beta]
    H = np.zeros((s + 1, s), dtype=np.complex128)
    k = s
    for j in range(s):
        w = op(V[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = _norm(w)
        if H[j + 1, j].real <= 1e-300:
            k = j + 1
            break
        V.append(w / H[j + 1, j])
    rhs = np.zeros(k + 1, dtype=np.complex128)
    rhs[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)[0]
    return sum(y[i] * V[i] for i in range(k))


def cagcr(op, b, s, tol, cycles):
    """Restarted CA-GCR(s) (Table 1, the coarsest solver), by what a cycle
    computes: from x, the correction minimising ||r - A v|| over K_s(A, r),
    r = b - A x (the basis the GPU builds it in, Chebyshev or another, does
    not change the minimiser); cycles until ||r|| <= tol ||b||."""
    x = np.zeros_like(b)
    bn = _norm(b)
    if bn == 0.0:
        return x
    r = b.copy()
    for _ in range(cycles):
        x = x + mr_smoother(op, r, s)
        r = b - op(x)
        if _norm(r) <= tol * bn:
            break
    return x


def cgne_null_vector(op, op_dag, phi0, tol, maxiter):
    """Near-null vector by CGNE on A phi = 0 from phi0 (Sec. 2.1, Table 1).

    CG on A A^dag y = -A phi0 from y = 0; phi = phi0 + A^dag y.  The CG
    residual equals -A phi, so the stop test ||r|| <= tol ||A phi0|| is the
    test on ||A phi||.  Returns (phi, iterations, ||A phi|| / ||A phi0||).
    """
    r = -op(phi0)
    r0 = _norm(r)
    y = np.zeros_like(phi0)
    p = r.copy()
    rr = np.vdot(r, r).real
    it = 0
    for it in range(1, maxiter + 1):
        Ap = op(op_dag(p))
        alpha = rr / np.vdot(p, Ap).real
        y = y + alpha * p
        r = r - alpha * Ap
        rr_new = np.vdot(r, r).real
        if np.sqrt(rr_new) <= tol * r0:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    phi = phi0 + op_dag(y)
    return phi, it, _norm(op(phi)) / r0


# --------------------------------------------------------------------------
# Schur CG baseline (Sec. 3.2)
# --------------------------------------------------------------------------

def cg_schur(W, N, mass, c1, c3, b, tol=1e-10, maxiter=100000):
    """Single-parity (even) Schur CG for D x = b, D = m + K.

    (m^2 - K_eo K_oe) x_e = m b_e - K_eo b_o, then x_o = (b_o - K_oe x_e)/m.
    The full residual is the even Schur residual divided by m, so CG runs to
    ||r_e|| <= m * tol * ||b|| (the m x 1e-10 of Sec. 3.2) and the stop test
    is confirmed on the true ||b - D x||; a miss restarts CG from the current
    x_e.  Returns (x, iterations, true relative residual).
    """
    T, Z, Y, X = b.shape[:4]
    epsf = ops.epsilon((X, Y, Z, T))[..., None]
    Pe = (epsf > 0).astype(np.float64)
    Po = 1.0 - Pe

    def K(v):
        return ops.dslash(v, W, N, 0.0, c1, c3)

    def M(v):  # m^2 v_e - K_eo K_oe v_e on even sites
        return mass * mass * v - Pe * K(Po * K(Pe * v))

    bnorm = _norm(b)
    rhs = Pe * (mass * b - K(Po * b))
    xe = np.zeros_like(b)
    iters = 0
    while True:
        r = rhs - M(xe)
        p = r.copy()
        rr = np.vdot(r, r).real
        while np.sqrt(rr) > mass * tol * bnorm and iters < maxiter:
            Ap = M(p)
            alpha = rr / np.vdot(p, Ap).real
            xe = xe + alpha * p
            r = r - alpha * Ap
            rr_new = np.vdot(r, r).real
            p = r + (rr_new / rr) * p
            rr = rr_new
            iters += 1
        x = xe + Po * (b - K(xe)) / mass
        rel = _norm(b - ops.dslash(x, W, N, mass, c1, c3)) / bnorm
        if rel <= tol or iters >= maxiter:
            return x, iters, rel


# --------------------------------------------------------------------------
# Multi-shift CG of the propagator workflow (Sec. 3.3)
# --------------------------------------------------------------------------

def multishift_cg(W, N, masses, c1, c3, b, tol=1e-10, maxiter=100000):
    """D(m_j) x_j = b for every mass at once, by multi-shift CG (Sec. 3.3).

    K = D(0) is anti-Hermitian and couples even sites to odd ones only, so
    D(m)^dag D(m) = m^2 - K^2 is block-diagonal in parity and
    D(m)^{-1} b = (m - K) y with (m^2 - K^2) y = b.  On each parity p the
    systems (sigma_j + A_p) y_p = b_p, A_p = -K_pq K_qp, sigma_j = m_j^2,
    differ by a shift only, and CG on the smallest shift sigma_0 builds the
    Krylov space of all of them (the propagators of the paper's workflow:
    one even and one odd solve per source).

    Shifted systems have residuals collinear with the base one,
    r_j = zeta_j r.  With the base CG steps
        r' = r - alpha A0 p,  p' = r' + beta p,  A0 = A_p + sigma_0,
    matching the three-term residual recurrence of CG on A0 + d_j
    (d_j = sigma_j - sigma_0) gives
        zeta'_j = zeta_j zeta''_j a_prev
                  / (alpha b_prev (zeta''_j - zeta_j) + zeta''_j a_prev (1 + alpha d_j))
    (zeta'' the previous value, a_prev, b_prev the previous base alpha and
    beta; a_prev = 1, b_prev = 0 and zeta'' = zeta = 1 at the start) and
        alpha_j = alpha zeta'_j / zeta_j,  beta_j = beta (zeta'_j / zeta_j)^2,
        x_j += alpha_j p_j,  p_j = zeta'_j r' + beta_j p_j.
    A shift stops updating when |zeta_j| |r| <= tol |b| / 2 on its parity,
    so both parities together leave |b - D x_j| <= tol |b| / sqrt(2) in exact
    arithmetic; the true residual is reported.

    Returns (list of x_j, iterations per parity, list of true relative
    residuals).  Pinned by dense solves (tests/test_oracle_solvers.py).
    """
    masses = [float(m) for m in masses]
    T, Z, Y, X = b.shape[:4]
    epsf = ops.epsilon((X, Y, Z, T))[..., None]
    par = [(epsf > 0).astype(np.float64), (epsf < 0).astype(np.float64)]

    def K(v):
        return ops.dslash(v, W, N, 0.0, c1, c3)

    bnorm = _norm(b)
    sig = [m * m for m in masses]
    base = int(np.argmin(sig))
    ns = len(masses)
    y = [np.zeros_like(b) for _ in range(ns)]
    iters = []
    for Pp in par:
        # A0 v = sigma_0 v - K_pq K_qp v on parity p
        def A0(v):
            return sig[base] * v - Pp * K((1.0 - Pp) * K(Pp * v))

        r = Pp * b
        ps = [r.copy() for _ in range(ns)]
        zeta = [1.0] * ns
        zeta_old = [1.0] * ns
        a_prev, b_prev = 1.0, 0.0
        rr = np.vdot(r, r).real
        target = 0.5 * tol * bnorm
        on = [np.sqrt(rr) > target for _ in range(ns)]
        it = 0
        while any(on) and it < maxiter:
            Ap = A0(ps[base])
            alpha = rr / np.vdot(ps[base], Ap).real
            zeta_new = [1.0] * ns
            for j in range(ns):
                if j == base or not on[j]:
                    continue
                d = sig[j] - sig[base]
                zeta_new[j] = zeta[j] * zeta_old[j] * a_prev / (
                    alpha * b_prev * (zeta_old[j] - zeta[j]) + zeta_old[j] * a_prev * (1.0 + alpha * d))
            for j in range(ns):
                if on[j]:
                    y[j] = y[j] + alpha * zeta_new[j] / zeta[j] * ps[j]
            r = r - alpha * Ap
            rr_new = np.vdot(r, r).real
            beta = rr_new / rr
            for j in range(ns):
                if on[j]:
                    ps[j] = zeta_new[j] * r + beta * (zeta_new[j] / zeta[j]) ** 2 * ps[j]
            for j in range(ns):
                if on[j]:
                    zeta_old[j], zeta[j] = zeta[j], zeta_new[j]
                    on[j] = abs(zeta[j]) * np.sqrt(rr_new) > target
            a_prev, b_prev, rr = alpha, beta, rr_new
            it += 1
        iters.append(it)
    xs, rels = [], []
    for j, m in enumerate(masses):
        x = m * y[j] - K(y[j])
        xs.append(x)
        rels.append(_norm(b - ops.dslash(x, W, N, m, c1, c3)) / bnorm)
    return xs, iters, rels


# --------------------------------------------------------------------------
# Hierarchy and K-cycle (Sec. 2.1, Sec. 2.3, Table 1)
# --------------------------------------------------------------------------

@dataclass
class MGParams:
    dims: tuple
    c1: float
    c3: float
    kd_naik: bool = True
    blocks: tuple = ((4, 4, 4, 4), (2, 2, 2, 2))   # one entry per aggregation level
    smoother_s: int = 8
    inner_tol: float = 0.25
    inner_maxiter: int = 8
    coarsest_tol: float = 0.25
    coarsest_maxiter: int = 16
    coarsest_direct: bool = False
    coarsest_solver: str = "gcr"     # "gcr", or "cagcr": cycles of CA-GCR(s), s = coarsest_maxiter (Table 1)
    coarsest_cycles: int = 1
    outer_nkrylov: int = 16
    dense_coarse_limit: int = 6144   # coarse levels up to this many dof are tabulated densely
    coarse_op: str = "galerkin"      # "galerkin": A_l = R A_{l-1} P; "block": X_l^{-1} R A_{l-1} P


class Hierarchy:
    """Levels of the KD multigrid (Sec. 2.3, Table 1):

      level 0   D(m)            (full, non-Schur HISQ operator)
      level 1   A = (B+m)^{-1} D (KD "pseudo-fine": same space, no coarsening;
                                 Naik dropped inside it when kd_naik is False)
      level 2   P1^dag A P1     (Galerkin, chirally split block-orthonormal P1)
      level 3   P2^dag A2 P2    (optional second aggregation)

    With coarse_op "block" every coarse level l >= 2 is the block-preconditioned
    operator  A_l = X_l^{-1} (P_l^dag A_{l-1} P_l),  X_l the coarse-site
    (self) block of the Galerkin product, and the next level coarsens that
    preconditioned operator (Sec. 2.3: the near-null vectors come from the
    coarse operator, the block-preconditioned version is what is coarsened;
    Table 1 marks levels 2 and 3 "Schur-preconditioned").  A level solve then
    solves A_l x = X_l^{-1} b, which has the same solution as the Galerkin
    system.

    Transfers: level 0 -> 1 is r1 = (B+m)^{-1} r0 with identity prolongation
    (so A e1 = r1 is D e1 = r0); deeper transfers are R = P^dag and P.
    The coarse operators are applied matrix-free as R A P (their definition).
    """

    def __init__(self, p: MGParams, W, N, mass, null_vectors):
        self.p = p
        self.W, self.N, self.mass = W, N, mass
        self.c3_kd = p.c3 if p.kd_naik else 0.0
        self.Kinv = ops.kd_inverse(W, mass, p.c1)
        self.transfers = []
        dims = p.dims
        agg, chi = ops.fine_dof_labels(dims, p.blocks[0])
        self.transfers.append(ops.Transfer(null_vectors[0], agg, chi))
        cdims = tuple(d // b for d, b in zip(dims, p.blocks[0]))
        self.cdims = [cdims]
        for lvl in range(1, len(p.blocks)):
            nv = self.transfers[-1].nvec
            agg, chi = ops.coarse_dof_labels(cdims, nv, p.blocks[lvl])
            self.transfers.append(ops.Transfer(null_vectors[lvl], agg, chi))
            cdims = tuple(d // b for d, b in zip(cdims, p.blocks[lvl]))
            self.cdims.append(cdims)
        self.nlevels = 2 + len(self.transfers)
        self._dense_lu = None
        self._dense = {}
        self._xinv = {}
        self.deflation = None

    def set_coarsest_deflation(self, Wv):
        """Deflate the coarsest solve with the span of the vectors Wv."""
        lvl = self.nlevels - 1
        self.deflation = mr_deflation(lambda v: self.op(lvl, v), Wv)

    # --- level operators --------------------------------------------------
    def op(self, lvl, v):
        p = self.p
        if lvl == 0:
            return ops.dslash(v, self.W, self.N, self.mass, p.c1, p.c3)
        if lvl == 1:
            return ops.kd_operator(v, self.W, self.N, self.Kinv, self.mass, p.c1, self.c3_kd)
        if v.size <= p.dense_coarse_limit:
            # the same R A P, tabulated column by column once for a small level
            if lvl not in self._dense:
                self._dense[lvl] = ops.dense_matrix(lambda u: self._galerkin(lvl, u), v.shape)
            return (self._dense[lvl] @ v.reshape(-1)).reshape(v.shape)
        return self._galerkin(lvl, v)

    def _galerkin(self, lvl, v):
        """R A P v for the operator A of level lvl - 1 (Galerkin, Sec. 2.1),
        block-preconditioned by X_lvl^{-1} with coarse_op "block"."""
        t = self.transfers[lvl - 2]
        fine = t.prolong(v)
        shape = self.fine_shape(lvl - 1)
        y = t.restrict(self.op(lvl - 1, fine.reshape(shape))).reshape(v.shape)
        return self.xinv_apply(lvl, y) if self.p.coarse_op == "block" else y

    def xinv_apply(self, lvl, v, dagger=False):
        """X_lvl^{-1} v (or X_lvl^{-dag} v) coarse site by coarse site, X_lvl(a)
        the coarse-site diagonal block of P^dag A_{lvl-1} P (from the level's
        explicit links)."""
        if lvl not in self._xinv:
            self.level_links(lvl)
        Xi = self._xinv[lvl]
        if dagger:
            Xi = np.swapaxes(Xi.conj(), -1, -2)
        return np.einsum("aij,aj->ai", Xi, v.reshape(Xi.shape[0], -1)).reshape(v.shape)

    def level_links(self, lvl):
        """Explicit links [Vc][9][n][n] of coarse level lvl (as applied: block-
        preconditioned with coarse_op "block"), built once."""
        if not hasattr(self, "_links"):
            self._links = {}
        if lvl not in self._links:
            p = self.p
            t = self.transfers[lvl - 2]
            nc = int(np.prod(self.cdims[lvl - 2]))
            if lvl == 2:
                def pieces(v):
                    ps = ops.dslash_pieces(v, self.W, self.N, self.mass, p.c1, self.c3_kd, p.blocks[0])
                    return [ops.kd_apply(self.Kinv, q) for q in ps]
            else:
                Lp = self.level_links(lvl - 1)
                pieces = lambda v: ops.coarse_pieces(Lp, self.cdims[lvl - 3], v, p.blocks[lvl - 2])
            L = ops.galerkin_links(t, pieces, self.fine_shape(lvl - 1), nc)
            if p.coarse_op == "block":
                # X(a): the coarse-site diagonal block, the self piece plus the
                # +-mu pieces that return to the site (coarse extent 1)
                cd = self.cdims[lvl - 2]
                X = L[:, 0].copy()
                for mu in range(4):
                    if cd[mu] == 1:
                        X += L[:, 1 + 2 * mu] + L[:, 2 + 2 * mu]
                self._xinv[lvl] = np.linalg.inv(X)
                L = np.einsum("aij,adjk->adik", self._xinv[lvl], L)
            self._links[lvl] = L
        return self._links[lvl]

    def op_dag(self, lvl, v):
        p = self.p
        if lvl == 0:
            return ops.dslash_dagger(v, self.W, self.N, self.mass, p.c1, p.c3)
        if lvl == 1:
            return ops.kd_operator_dagger(v, self.W, self.N, self.Kinv, self.mass, p.c1, self.c3_kd)
        if self.p.coarse_op == "block":   # (X^{-1} R A P)^dag = R A^dag P X^{-dag}
            v = self.xinv_apply(lvl, v, dagger=True)
        t = self.transfers[lvl - 2]
        fine = t.prolong(v)
        shape = self.fine_shape(lvl - 1)
        return t.restrict(self.op_dag(lvl - 1, fine.reshape(shape))).reshape(v.shape)

    def fine_shape(self, lvl):
        X, Y, Z, T = self.p.dims
        if lvl <= 1:
            return (T, Z, Y, X, 3)
        Xc, Yc, Zc, Tc = self.cdims[lvl - 2]
        return (Tc, Zc, Yc, Xc, 2, self.transfers[lvl - 2].nvec)

    def restrict(self, lvl, r):
        """level lvl -> lvl + 1"""
        if lvl == 0:
            return ops.kd_apply(self.Kinv, r)
        t = self.transfers[lvl - 1]
        return t.restrict(r).reshape(self.fine_shape(lvl + 1))

    def prolong(self, lvl, e):
        """level lvl + 1 -> lvl"""
        if lvl == 0:
            return e
        t = self.transfers[lvl - 1]
        return t.prolong(e).reshape(self.fine_shape(lvl))

    # --- cycle -------------------------------------------------------------
    def kcycle(self, lvl, r):
        """K_l(r): no pre-smoothing; restrict; solve on level l+1; prolong;
        post-smooth with the minimal-residual smoother (Sec. 2.1, Table 1)."""
        rc = self.restrict(lvl, r)
        ec = self.solve_level(lvl + 1, rc)
        e = self.prolong(lvl, ec)
        return e + mr_smoother(lambda v: self.op(lvl, v), r - self.op(lvl, e), self.p.smoother_s)

    def solve_level(self, lvl, b):
        p = self.p
        if p.coarse_op == "block" and lvl >= 2:
            b = self.xinv_apply(lvl, b)   # A_l x = X^{-1} b: the Galerkin system's solution
        if lvl == self.nlevels - 1:
            if p.coarsest_direct:
                if self._dense_lu is None:
                    self._dense_lu = ops.dense_matrix(lambda v: self.op(lvl, v), b.shape)
                return np.linalg.solve(self._dense_lu, b.reshape(-1)).reshape(b.shape)
            if self.deflation is not None:
                # deflated start, then GCR on the remaining residual with the
                # stop test still relative to ||b||
                Q, Wp = self.deflation
                x0, r0 = mr_deflate(Q, Wp, b)
                bn, rn = _norm(b), _norm(r0)
                if bn == 0.0 or rn == 0.0:
                    return x0
                e, _ = gcr(lambda v: self.op(lvl, v), r0, None, p.coarsest_tol * bn / rn,
                           p.coarsest_maxiter, p.coarsest_maxiter)
                return x0 + e
            if p.coarsest_solver == "cagcr":
                return cagcr(lambda v: self.op(lvl, v), b, p.coarsest_maxiter, p.coarsest_tol, p.coarsest_cycles)
            x, _ = gcr(lambda v: self.op(lvl, v), b, None, p.coarsest_tol,
                       p.coarsest_maxiter, p.coarsest_maxiter)
            return x
        x, _ = gcr(lambda v: self.op(lvl, v), b, lambda r: self.kcycle(lvl, r),
                   p.inner_tol, p.inner_maxiter, p.inner_maxiter)
        return x

    def solve(self, b, tol=1e-10, maxiter=200):
        """Outer flexible GCR on D, preconditioned by K_0, stop on the true
        residual ||b - D x|| / ||b|| <= tol (Sec. 3.2)."""
        return gcr(lambda v: self.op(0, v), b, lambda r: self.kcycle(0, r), tol, maxiter,
                   self.p.outer_nkrylov, true_residual=True)


def hierarchy_links(H):
    """Explicit direction-split coarse links of every coarse level of the
    hierarchy H ([Vc][9][n][n] row-major), built from the pieces of the level
    operators (the Galerkin definition written out block by block; with
    coarse_op "block" each level's links are multiplied by X^{-1} and the next
    level is built from those)."""
    return [H.level_links(lvl) for lvl in range(2, H.nlevels)]


# --------------------------------------------------------------------------
# Fermion force: gradient of S = phi^dag (D^dag D)^{-1} phi (HMC use, Sec. 4.2)
# --------------------------------------------------------------------------

def force(W, N, mass, c1, c3, phi, tol=1e-12):
    """S = phi^dag (D^dag D)^{-1} phi and its gradients with respect to the
    fat and Naik links in PyTorch's convention (dS/dRe U + i dS/dIm U):

      X = (D^dag D)^{-1} phi,  Y = D X  (so D^dag Y = phi),
      G^W_mu(x) = -c1 eta_mu(x) [ Y(x) X(x+mu)^dag  - X(x) Y(x+mu)^dag  ]
      G^N_mu(x) = -c3 eta_mu(x) [ Y(x) X(x+3mu)^dag - X(x) Y(x+3mu)^dag ]

    from dS = -2 Re(Y^dag dD X).  The two solves are D^dag Y = phi and D X = Y
    (Schur CG, FP64).  Pinned by central finite differences."""
    T, Z, Yd, X = phi.shape[:4]
    dims = (X, Yd, Z, T)
    eta = ops.staggered_eta(dims)
    # D^dag = eps D eps: Y = eps D^{-1} (eps phi)
    e = ops.epsilon(dims)[..., None]
    y1, _, _ = cg_schur(W, N, mass, c1, c3, e * phi, tol=tol)
    Yv = e * y1
    Xv, _, _ = cg_schur(W, N, mass, c1, c3, Yv, tol=tol)
    S = float(np.vdot(phi, Xv).real)

    def outer(a, b):
        return np.einsum("...i,...j->...ij", a, b.conj())

    gW = np.empty_like(W)
    gN = np.empty_like(N)
    for mu in range(4):
        ax = ops.axis_of(mu)
        et = eta[mu][..., None, None]
        X1, Y1 = np.roll(Xv, -1, axis=ax), np.roll(Yv, -1, axis=ax)
        gW[mu] = -c1 * et * (outer(Yv, X1) - outer(Xv, Y1))
        X3, Y3 = np.roll(Xv, -3, axis=ax), np.roll(Yv, -3, axis=ax)
        gN[mu] = -c3 * et * (outer(Yv, X3) - outer(Xv, Y3))
    return S, gW, gN, Xv, Yv


def action(W, N, mass, c1, c3, phi, tol=1e-13):
    """S = phi^dag (D^dag D)^{-1} phi = |D^{-dag} phi|^2 (one Schur CG solve)."""
    T, Z, Yd, X = phi.shape[:4]
    e = ops.epsilon((X, Yd, Z, T))[..., None]
    y1, _, _ = cg_schur(W, N, mass, c1, c3, e * phi, tol=tol)
    return float(np.vdot(y1, y1).real)
