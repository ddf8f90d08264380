"""Seeded synthetic inputs for staggered/HISQ multigrid: gauge links, fat and
Naik links, right-hand sides, near-null starting vectors and gauge transforms.

This module draws random numbers and builds the *inputs* of the operator; it
contains none of the method's arithmetic (no Dirac operator, no Kahler-Dirac
blocks, no transfer, no solver).  Both the CPU oracle's tests and the GPU path
take their inputs from here, so that the two see bit-identical data.

Canonical layouts (complex128, C order):
  link field  [4][T][Z][Y][X][3][3]   mu = 0,1,2,3 is x,y,z,t; row-major 3x3
  fine vector [T][Z][Y][X][3]         (a batch prepends [nrhs])
  coarse vec  [Tc][Zc][Yc][Xc][2][Nvec]  spin index 0 is chirality +1

Recipe (the synthetic stand-in for a thermalised HISQ ensemble; the paper's
MILC 144^3x288 configuration (Sec. 3.2) is not available):
  * U_mu(x) = exp(i eps H), H = (A + A^dag)/2 minus its trace/3, A with i.i.d.
    standard complex normal entries (E|A_ij|^2 = 1), exponentiated through
    eigh(H).
  * fat links  W = U + 0.1 G, G i.i.d. standard complex normal (generic 3x3,
    not unitary: the one-hop HISQ links of Sec. 2.2 are smeared sums).
  * Naik links N_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu) (products of three
    gauge links, so in U(3) as Sec. 3.1 notes for the long links).
  * right-hand sides: standard complex normal.
Draw order for one seed: H-generator A, then G, then whatever the caller asks.
"""
from __future__ import annotations

import numpy as np

# Seeds recorded per workload.
SEEDS = {
    "c0_4x4_naive": 20221224,
    "c1_16x4_hisq": 20221225,
    "c2_32x4_hisq": 20221226,
    "small_8x4_hisq": 20221227,
}


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """Standard complex normal (E|z|^2 = 1), drawn as interleaved (re, im)."""
    z = rng.standard_normal(tuple(shape) + (2,))
    return (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)


def _su3_exp(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for a stack of Hermitian 3x3 matrices, via eigh."""
    w, V = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ik,...k,...jk->...ij", V, ph, V.conj(), optimize=False)


def random_hermitian_traceless(rng, shape) -> np.ndarray:
    A = complex_normal(rng, tuple(shape) + (3, 3))
    H = 0.5 * (A + np.swapaxes(A.conj(), -1, -2))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[..., None, None] * np.eye(3)
    return H


def gauge_field(dims, eps: float, rng: np.random.Generator, chunk: int = 1 << 18) -> np.ndarray:
    """U_mu(x) = exp(i eps H_mu(x)); returns [4][T][Z][Y][X][3][3] complex128."""
    X, Y, Z, T = dims
    nsite = 4 * T * Z * Y * X
    H = random_hermitian_traceless(rng, (nsite,))
    U = np.empty_like(H)
    for s in range(0, nsite, chunk):
        U[s:s + chunk] = _su3_exp(H[s:s + chunk], eps)
    return U.reshape(4, T, Z, Y, X, 3, 3)


def _axis(mu: int) -> int:
    """Array axis of direction mu in a [T][Z][Y][X] field."""
    return 3 - mu


def naik_links(U: np.ndarray) -> np.ndarray:
    """N_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu) (periodic)."""
    N = np.empty_like(U)
    for mu in range(4):
        ax = _axis(mu)
        U1 = np.roll(U[mu], -1, axis=ax)
        U2 = np.roll(U[mu], -2, axis=ax)
        N[mu] = U[mu] @ U1 @ U2
    return N


def hisq_style_links(dims, eps: float, seed: int, fat_noise: float = 0.1):
    """Fat (W) and Naik (N) links of the HISQ-style synthetic ensemble."""
    rng = np.random.default_rng(seed)
    U = gauge_field(dims, eps, rng)
    G = complex_normal(rng, U.shape)
    W = U + fat_noise * G
    N = naik_links(U)
    return W, N, rng


def naive_links(dims, eps: float, seed: int):
    """Unimproved staggered: W = U, no Naik term (returns zero N)."""
    rng = np.random.default_rng(seed)
    U = gauge_field(dims, eps, rng)
    return U, np.zeros_like(U), rng


def unit_links(dims):
    X, Y, Z, T = dims
    U = np.zeros((4, T, Z, Y, X, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def fine_vectors(dims, n: int, rng: np.random.Generator) -> np.ndarray:
    X, Y, Z, T = dims
    return complex_normal(rng, (n, T, Z, Y, X, 3))


def coarse_vectors(cdims, nspin_vec: int, n: int, rng) -> np.ndarray:
    X, Y, Z, T = cdims
    return complex_normal(rng, (n, T, Z, Y, X, 2, nspin_vec))


def gauge_transform(dims, rng) -> np.ndarray:
    """Random SU(3) matrix per site, [T][Z][Y][X][3][3]."""
    X, Y, Z, T = dims
    H = random_hermitian_traceless(rng, (T * Z * Y * X,))
    return _su3_exp(H, 1.0).reshape(T, Z, Y, X, 3, 3)


def log_masses(m0: float = 0.005, m1: float = 0.2, n: int = 8):
    """m_j = m0 (m1/m0)^(j/(n-1)): the log-spaced mass ladder of the
    multi-mass workload (light to heavy)."""
    return [m0 * (m1 / m0) ** (j / (n - 1)) for j in range(n)]
