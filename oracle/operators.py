"""Oracle operators: lattice geometry, the staggered/HISQ Dirac operator, the
Kahler-Dirac (KD) block preconditioner, chirally split block-orthonormal
transfer operators and the Galerkin coarse operator.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy, complex128.

Conventions (readings of the paper where it is silent, Sec. 2.2):
  * lattice extents (X, Y, Z, T), even; periodic in every direction (an
    antiperiodic time boundary is a sign on the links, the caller's choice);
  * fine vector shape [T][Z][Y][X][3]; link field [4][T][Z][Y][X][3][3];
  * staggered phases eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y),
    eta_3 = (-1)^(x+y+z) and the normalisation 1/2 (the paper fixes neither);
  * epsilon(x) = (-1)^(x+y+z+t) generates the staggered chiral symmetry and
    the chiral projectors (1 +- epsilon)/2 (Sec. 2.2);
  * hypercubes of the KD decomposition have their origin at even coordinates,
    local index s = sum_mu (x_mu mod 2) 2^mu, KD row 3 s + colour.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------

def coords(dims):
    """Integer coordinate arrays (x, y, z, t), each of shape [T][Z][Y][X]."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    return x, y, z, t


def axis_of(mu: int) -> int:
    """Array axis of direction mu in a [T][Z][Y][X] field."""
    return 3 - mu


@lru_cache(maxsize=8)
def staggered_eta(dims) -> np.ndarray:
    """eta_mu(x) for mu = 0..3 as a [4][T][Z][Y][X] array of +-1 (read-only)."""
    x, y, z, t = coords(dims)
    eta = np.empty((4,) + x.shape)
    eta[0] = 1.0
    eta[1] = (-1.0) ** x
    eta[2] = (-1.0) ** (x + y)
    eta[3] = (-1.0) ** (x + y + z)
    eta.flags.writeable = False
    return eta


def epsilon(dims) -> np.ndarray:
    """epsilon(x) = (-1)^(x+y+z+t) (Sec. 2.2), shape [T][Z][Y][X]."""
    x, y, z, t = coords(dims)
    return (-1.0) ** (x + y + z + t)


def _mv(U, v):
    return np.einsum("...ij,...j->...i", U, v)


def _dag(U):
    return np.swapaxes(U.conj(), -1, -2)


# --------------------------------------------------------------------------
# Fine operator (Sec. 2.2, Sec. 3.1)
# --------------------------------------------------------------------------

def dslash(x, W, N, mass: float, c1: float, c3: float):
    """y = D x, the staggered (c3 = 0, W = U) or HISQ-style operator:

      (D x)(x) = m x(x) + 1/2 sum_mu eta_mu(x) [ c1 (W_mu(x) x(x+mu) - W_mu(x-mu)^dag x(x-mu))
                                                + c3 (N_mu(x) x(x+3mu) - N_mu(x-3mu)^dag x(x-3mu)) ]

    one-hop fat links W and three-hop Naik links N (Sec. 2.2, Sec. 3.1).
    Pinned by the free-field closed-form spectrum, anti-Hermiticity of D - m,
    epsilon-Hermiticity and gauge covariance (tests/test_oracle_operators.py).
    """
    dims = (int(x.shape[3]), int(x.shape[2]), int(x.shape[1]), int(x.shape[0]))
    eta = staggered_eta(dims)
    y = mass * x
    for mu in range(4):
        ax = axis_of(mu)
        hop = c1 * (_mv(W[mu], np.roll(x, -1, axis=ax))
                    - _mv(_dag(np.roll(W[mu], 1, axis=ax)), np.roll(x, 1, axis=ax)))
        if c3 != 0.0:
            hop = hop + c3 * (_mv(N[mu], np.roll(x, -3, axis=ax))
                              - _mv(_dag(np.roll(N[mu], 3, axis=ax)), np.roll(x, 3, axis=ax)))
        y = y + 0.5 * eta[mu][..., None] * hop
    return y


def dslash_dagger(x, W, N, mass: float, c1: float, c3: float):
    """y = D^dag x.  D - m is anti-Hermitian (Sec. 2.2: the spectrum is
    anti-Hermitian up to the real mass), so D^dag = 2m - D.  Pinned against the
    dense conjugate transpose."""
    return 2.0 * mass * x - dslash(x, W, N, mass, c1, c3)


def dense_matrix(apply, shape):
    """Dense matrix of a linear map on arrays of `shape` (small lattices)."""
    n = int(np.prod(shape))
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        M[:, j] = apply(e.reshape(shape)).reshape(-1)
    return M


# --------------------------------------------------------------------------
# Kahler-Dirac block preconditioner (Sec. 2.2 Eq. 1-2, Sec. 3.1)
# --------------------------------------------------------------------------

def hypercube_index(dims):
    """(hc, s): hypercube id (lexicographic over dims/2) and local index
    s = sum_mu (x_mu mod 2) 2^mu for every site, each [T][Z][Y][X]."""
    X, Y, Z, T = dims
    x, y, z, t = coords(dims)
    hx, hy, hz, ht = X // 2, Y // 2, Z // 2, T // 2
    hc = (x // 2) + hx * ((y // 2) + hy * ((z // 2) + hz * (t // 2)))
    s = (x % 2) + 2 * (y % 2) + 4 * (z % 2) + 8 * (t % 2)
    return hc, s


def kd_block_matrices(W, mass: float, c1: float) -> np.ndarray:
    """Dense (B + m) for every 2^4 hypercube, shape [nhc][48][48].

    B holds the one-hop (fat-link) terms of D whose two sites lie in the same
    hypercube (Sec. 2.2, dual decomposition D = (B + m) + C): a forward hop
    x -> x+mu with x_mu even, a backward hop x -> x-mu with x_mu odd.  Naik
    hops move three sites and always leave the hypercube, so they sit in C.
    Row / column index 3 s + colour.
    """
    T, Z, Y, X = W.shape[1:5]
    dims = (X, Y, Z, T)
    eta = staggered_eta(dims)
    hc, s = hypercube_index(dims)
    nhc = (X * Y * Z * T) // 16
    Bm = np.zeros((nhc, 16, 3, 16, 3), dtype=np.complex128)
    for sl in range(16):
        Bm[:, sl, :, sl, :] = mass * np.eye(3)
    c = coords(dims)
    for mu in range(4):
        ax = axis_of(mu)
        even = (c[mu] % 2) == 0
        # forward hops inside the cube: x (x_mu even) -> x + mu
        blk = 0.5 * c1 * eta[mu][even][:, None, None] * W[mu][even]
        Bm[hc[even], s[even], :, s[even] + (1 << mu), :] += blk
        # backward hops inside the cube: x (x_mu odd) -> x - mu
        odd = ~even
        Wb = np.roll(W[mu], 1, axis=ax)  # W_mu(x - mu) at x
        blk = -0.5 * c1 * eta[mu][odd][:, None, None] * _dag(Wb[odd])
        Bm[hc[odd], s[odd], :, s[odd] - (1 << mu), :] += blk
    return Bm.reshape(nhc, 48, 48)


def kd_inverse(W, mass: float, c1: float) -> np.ndarray:
    """(B + m)^{-1} per hypercube by dense LU (numpy.linalg.inv), [nhc][48][48]
    (the explicit inverse the paper stores per 2^d sites, Sec. 3.1)."""
    return np.linalg.inv(kd_block_matrices(W, mass, c1))


@lru_cache(maxsize=8)
def _hc_gather_index(dims):
    """flat site index of (hc, s), shape [nhc][16] (read-only)."""
    hc, s = hypercube_index(dims)
    X, Y, Z, T = dims
    idx = np.empty((X * Y * Z * T // 16, 16), dtype=np.int64)
    idx[hc.reshape(-1), s.reshape(-1)] = np.arange(X * Y * Z * T)
    idx.flags.writeable = False
    return idx


def kd_apply(Kb, x, dagger: bool = False):
    """y = (B + m)^{-1} x (or its adjoint) with per-hypercube blocks Kb."""
    T, Z, Y, X = (int(n) for n in x.shape[:4])
    idx = _hc_gather_index((X, Y, Z, T))
    xf = x.reshape(-1, 3)[idx].reshape(idx.shape[0], 48)
    M = np.swapaxes(Kb.conj(), -1, -2) if dagger else Kb
    yh = np.einsum("hij,hj->hi", M, xf)
    y = np.empty_like(x.reshape(-1, 3))
    y[idx.reshape(-1)] = yh.reshape(-1, 3)
    return y.reshape(x.shape)


def kd_operator(x, W, N, Kinv, mass, c1, c3):
    """A x = (B + m)^{-1} D x: the KD-preconditioned ("pseudo-fine") operator
    of Sec. 2.3, applied literally as in Sec. 3.1.  With c3 = 0 this is the
    truncated operator (Naik term dropped inside the KD level)."""
    return kd_apply(Kinv, dslash(x, W, N, mass, c1, c3))


def kd_operator_dagger(x, W, N, Kinv, mass, c1, c3):
    """A^dag x = D^dag (B + m)^{-dag} x (plain definition)."""
    return dslash_dagger(kd_apply(Kinv, x, dagger=True), W, N, mass, c1, c3)


# --------------------------------------------------------------------------
# Transfer: chiral doubling + block orthonormalisation (Sec. 2.1, Sec. 2.3)
# --------------------------------------------------------------------------

def fine_dof_labels(dims, block):
    """(aggregate, chirality) of every fine degree of freedom (site*3 + c).

    aggregate = lexicographic index of floor(x_mu / block_mu); chirality 0 for
    epsilon(x) = +1 and 1 for epsilon(x) = -1 (the two chiral projections)."""
    X, Y, Z, T = dims
    bx, by, bz, bt = block
    x, y, z, t = coords(dims)
    cX, cY, cZ = X // bx, Y // by, Z // bz
    agg = (x // bx) + cX * ((y // by) + cY * ((z // bz) + cZ * (t // bt)))
    chi = ((x + y + z + t) % 2).astype(np.int64)
    agg = np.repeat(agg.reshape(-1), 3)
    chi = np.repeat(chi.reshape(-1), 3)
    return agg, chi


def coarse_dof_labels(cdims, nvec, block):
    """(aggregate, chirality) of every coarse dof (site*2N + spin*N + k) when a
    coarse lattice is aggregated again: the chirality of a coarse dof is its
    spin index (the coarse epsilon is diag(+1, -1) x 1_Nvec)."""
    X, Y, Z, T = cdims
    bx, by, bz, bt = block
    x, y, z, t = coords(cdims)
    cX, cY, cZ = X // bx, Y // by, Z // bz
    agg = (x // bx) + cX * ((y // by) + cY * ((z // bz) + cZ * (t // bt)))
    agg = np.repeat(agg.reshape(-1), 2 * nvec)
    chi = np.tile(np.repeat(np.arange(2), nvec), X * Y * Z * T)
    return agg, chi


def qr_positive(V):
    """Thin QR with real positive diag(R); this Q is unique for full-rank V.
    V: [..., rows, cols]."""
    Q, R = np.linalg.qr(V)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    return Q * ph[..., None, :], np.abs(d)


class Transfer:
    """P (and R = P^dag) for one aggregation step.

    Each near-null vector is split by the chiral projectors (1 +- eps)/2 and the
    pieces are orthonormalised block by block (Sec. 2.1): for every aggregate a
    and chirality sigma, Q_{a,sigma} is the thin-QR Q factor (positive diag R)
    of the null vectors restricted to the rows of (a, sigma).  Coarse dof index
    (a, sigma, k), sigma = +1 first.  P = R^dag (Galerkin, Sec. 2.1).
    """

    def __init__(self, null_vectors, agg, chi):
        V = np.asarray(null_vectors).reshape(len(null_vectors), -1).T  # [nflat][nvec]
        self.nflat, self.nvec = V.shape
        self.nagg = int(agg.max()) + 1
        order = np.lexsort((np.arange(self.nflat), chi, agg))  # group by (agg, chi), rows ascending
        self.rows = order.reshape(self.nagg, 2, -1)
        Vb = V[self.rows]  # [nagg][2][nrows][nvec]
        if Vb.shape[2] < self.nvec:
            raise ValueError("aggregate has fewer rows than near-null vectors")
        self.Q, self.rdiag = qr_positive(Vb)

    def restrict(self, r):
        """r_c[a, sigma, k] = sum_{rows of (a, sigma)} conj(Q[row, k]) r[row]."""
        rf = np.asarray(r).reshape(-1)[self.rows]
        return np.einsum("asrk,asr->ask", self.Q.conj(), rf)

    def prolong(self, ec):
        """e[row] = sum_k Q[row, k] e_c[a, sigma, k]."""
        e = np.zeros(self.nflat, dtype=np.complex128)
        e[self.rows] = np.einsum("asrk,ask->asr", self.Q, np.asarray(ec).reshape(self.nagg, 2, self.nvec))
        return e


# --------------------------------------------------------------------------
# Explicit direction-split coarse links (Sec. 2.1 Galerkin; 9-point stencil)
# --------------------------------------------------------------------------

def dslash_pieces(x, W, N, mass, c1, c3, block):
    """D x split by where each hop goes relative to the aggregate of the
    output site: piece 0 keeps hops that stay inside the aggregate (and the
    mass), piece 1 + 2 mu the hops that leave through its +mu face, piece
    2 + 2 mu through its -mu face.  The nine pieces sum to D x."""
    dims = (int(x.shape[3]), int(x.shape[2]), int(x.shape[1]), int(x.shape[0]))
    eta = staggered_eta(dims)
    co = coords(dims)
    out = [np.zeros_like(x) for _ in range(9)]
    out[0] = out[0] + mass * x
    for mu in range(4):
        ax = axis_of(mu)
        u = (co[mu] % block[mu])[..., None]
        for h, coef, F in ((1, c1, W), (3, c3, N)):
            if coef == 0.0:
                continue
            fwd = 0.5 * coef * eta[mu][..., None] * _mv(F[mu], np.roll(x, -h, axis=ax))
            bwd = -0.5 * coef * eta[mu][..., None] * _mv(_dag(np.roll(F[mu], h, axis=ax)), np.roll(x, h, axis=ax))
            leave_f = (u + h) >= block[mu]
            leave_b = (u - h) < 0
            out[1 + 2 * mu] = out[1 + 2 * mu] + np.where(leave_f, fwd, 0)
            out[0] = out[0] + np.where(leave_f, 0, fwd)
            out[2 + 2 * mu] = out[2 + 2 * mu] + np.where(leave_b, bwd, 0)
            out[0] = out[0] + np.where(leave_b, 0, bwd)
    return out


def coarse_neighbours(cdims):
    """[Vc][9] site index of the self / +mu / -mu neighbours (periodic)."""
    X, Y, Z, T = cdims
    V = X * Y * Z * T
    s = np.arange(V)
    c = [s % X, (s // X) % Y, (s // (X * Y)) % Z, s // (X * Y * Z)]
    nb = np.empty((V, 9), dtype=np.int64)
    nb[:, 0] = s
    for mu in range(4):
        for d, h in ((1 + 2 * mu, 1), (2 + 2 * mu, -1)):
            cc = list(c)
            cc[mu] = (c[mu] + h) % cdims[mu]
            nb[:, d] = cc[0] + X * (cc[1] + Y * (cc[2] + Z * cc[3]))
    return nb, c


def coarse_apply_links(L, cdims, x):
    """y(a) = sum_d L[a, d] x(nb_d(a)) for links L [Vc][9][n][n] (row-major)."""
    nb, _ = coarse_neighbours(cdims)
    xv = x.reshape(L.shape[0], -1)
    y = np.einsum("adij,adj->ai", L, xv[nb])
    return y.reshape(x.shape)


def coarse_pieces(L, cdims, x, block):
    """The coarse stencil split like dslash_pieces, relative to the aggregates
    (blocks `block`) of the next coarsening."""
    nb, c = coarse_neighbours(cdims)
    xv = x.reshape(L.shape[0], -1)
    out = [np.zeros_like(xv) for _ in range(9)]
    out[0] = out[0] + np.einsum("aij,aj->ai", L[:, 0], xv)
    for mu in range(4):
        u = c[mu] % block[mu]
        for d, leave in ((1 + 2 * mu, u == block[mu] - 1), (2 + 2 * mu, u == 0)):
            y = np.einsum("aij,aj->ai", L[:, d], xv[nb[:, d]])
            out[d] = out[d] + np.where(leave[:, None], y, 0)
            out[0] = out[0] + np.where(leave[:, None], 0, y)
    return [o.reshape(x.shape) for o in out]


def galerkin_links(transfer, pieces_of, fine_shape, ncoarse_sites):
    """Coarse links [Vc][9][n][n] (row-major blocks) of R A P: column j of
    every block is R applied to piece d of A acting on P e_j (e_j on every
    aggregate at once)."""
    n = 2 * transfer.nvec
    L = np.zeros((ncoarse_sites, 9, n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros((ncoarse_sites, n), dtype=np.complex128)
        e[:, j] = 1.0
        v = transfer.prolong(e).reshape(fine_shape)
        for d, p in enumerate(pieces_of(v)):
            L[:, d, :, j] = transfer.restrict(p).reshape(ncoarse_sites, n)
    return L


def round_bf16(a):
    """Round to bfloat16 (round to nearest, ties to even), returned as float64;
    the input is first taken to float32."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_fp16(a):
    """Round to IEEE binary16 (numpy's float16 conversion is round to nearest
    even), returned as float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float16).astype(np.float64)
