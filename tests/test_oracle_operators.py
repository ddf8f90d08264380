"""Pins of the oracle's operators against what physics and mathematics fix
(free-field closed forms, symmetries, gauge covariance, brute-force loops).
CPU only."""
import itertools

import numpy as np
import pytest

from oracle import operators as ops
from paper_2212_12559_amd import latgen

C1H, C3H = 9.0 / 8.0, -1.0 / 24.0


def rand_links(dims, seed, naik=True):
    W, N, rng = latgen.hisq_style_links(dims, 0.5, seed)
    if not naik:
        N = np.zeros_like(N)
    return W, N, rng


def free_spectrum(dims, mass, c1, c3):
    """Closed form: eigenvalues m +- i sqrt(sum_mu f(p_mu)^2),
    f(p) = c1 sin p + c3 sin 3p, p = 2 pi n / L; colour multiplicity 3,
    symmetric in +-.  Returned as the sorted multiset of |Im lambda|."""
    vals = []
    for n in itertools.product(*[range(L) for L in dims]):
        p = [2 * np.pi * n[i] / dims[i] for i in range(4)]
        f2 = sum((c1 * np.sin(q) + c3 * np.sin(3 * q)) ** 2 for q in p)
        vals += [np.sqrt(f2)] * 3
    return np.sort(np.array(vals))


@pytest.mark.parametrize("dims,c1,c3", [((4, 4, 4, 4), 1.0, 0.0), ((4, 4, 6, 6), C1H, C3H)])
def test_free_field_spectrum(dims, c1, c3):
    """Sec. 2.2: the staggered spectrum is anti-Hermitian up to the real mass;
    the free-field values follow from the momentum-space form."""
    mass = 0.1
    U = latgen.unit_links(dims)
    X, Y, Z, T = dims
    D = ops.dense_matrix(lambda v: ops.dslash(v, U, U, mass, c1, c3), (T, Z, Y, X, 3))
    lam = np.linalg.eigvals(D)
    assert np.max(np.abs(lam.real - mass)) < 1e-12
    got = np.sort(np.abs(lam.imag))
    want = free_spectrum(dims, mass, c1, c3)
    assert np.max(np.abs(got - want)) < 1e-11
    # +- symmetry of the nonzero eigenvalues
    nz = np.abs(lam.imag) > 1e-8
    assert np.sum(lam.imag[nz] > 0) == np.sum(lam.imag[nz] < 0)


def test_free_plane_wave_8x4():
    """(D - m)^2 e^{ipx} v = -sum_mu f(p_mu)^2 e^{ipx} v on unit links at a larger
    lattice: the square of the hopping term is diagonal in momentum."""
    dims = (8, 8, 8, 8)
    U = latgen.unit_links(dims)
    x, y, z, t = ops.coords(dims)
    n = (1, 3, 2, 5)
    p = [2 * np.pi * n[i] / 8 for i in range(4)]
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    v = np.array([0.3 + 0.1j, -0.7j, 1.1])
    psi = phase[..., None] * v
    K2 = ops.dslash(ops.dslash(psi, U, U, 0.0, C1H, C3H), U, U, 0.0, C1H, C3H)
    f2 = sum((C1H * np.sin(q) + C3H * np.sin(3 * q)) ** 2 for q in p)
    assert np.max(np.abs(K2 + f2 * psi)) < 1e-12


def brute_dense_dslash(dims, W, N, mass, c1, c3):
    """Dense D from explicit loops over sites, directions and hops with modular
    neighbour arithmetic (independent of the np.roll formulation)."""
    X, Y, Z, T = dims
    L = [X, Y, Z, T]
    V = X * Y * Z * T

    def idx(c):
        return c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))

    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    for c in itertools.product(range(T), range(Z), range(Y), range(X)):
        co = [c[3], c[2], c[1], c[0]]
        i = idx(co)
        D[3 * i:3 * i + 3, 3 * i:3 * i + 3] += mass * np.eye(3)
        for mu in range(4):
            eta = (-1) ** sum(co[:mu])
            for hop, coef, F in ((1, c1, W), (3, c3, N)):
                if coef == 0.0:
                    continue
                fw = list(co)
                fw[mu] = (co[mu] + hop) % L[mu]
                bw = list(co)
                bw[mu] = (co[mu] - hop) % L[mu]
                j, k = idx(fw), idx(bw)
                Uf = F[mu, co[3], co[2], co[1], co[0]]
                Ub = F[mu, bw[3], bw[2], bw[1], bw[0]]
                D[3 * i:3 * i + 3, 3 * j:3 * j + 3] += 0.5 * eta * coef * Uf
                D[3 * i:3 * i + 3, 3 * k:3 * k + 3] -= 0.5 * eta * coef * Ub.conj().T
    return D


def test_dslash_matches_brute_force_loops():
    dims = (4, 4, 4, 6)
    W, N, _ = rand_links(dims, 11)
    X, Y, Z, T = dims
    D = ops.dense_matrix(lambda v: ops.dslash(v, W, N, 0.07, C1H, C3H), (T, Z, Y, X, 3))
    Db = brute_dense_dslash(dims, W, N, 0.07, C1H, C3H)
    assert np.max(np.abs(D - Db)) < 1e-14


def test_antihermitian_and_eps_hermitian():
    """D - m anti-Hermitian for generic (non-unitary) fat links; eps D eps = D^dag
    (Sec. 2.2); the oracle's D^dag equals the dense conjugate transpose."""
    dims = (4, 4, 4, 4)
    W, N, _ = rand_links(dims, 12)
    m = 0.05
    D = ops.dense_matrix(lambda v: ops.dslash(v, W, N, m, C1H, C3H), (4, 4, 4, 4, 3))
    K = D - m * np.eye(D.shape[0])
    assert np.max(np.abs(K + K.conj().T)) < 1e-14
    e = np.repeat(ops.epsilon(dims).reshape(-1), 3)
    assert np.max(np.abs(e[:, None] * D * e[None, :] - D.conj().T)) < 1e-14
    Dd = ops.dense_matrix(lambda v: ops.dslash_dagger(v, W, N, m, C1H, C3H), (4, 4, 4, 4, 3))
    assert np.max(np.abs(Dd - D.conj().T)) < 1e-14


def test_gauge_covariance():
    """D[W^g, N^g] (g x) = g (D[W, N] x) with W^g_mu(x) = g(x) W_mu(x) g(x+mu)^dag and
    N^g_mu(x) = g(x) N_mu(x) g(x+3mu)^dag."""
    dims = (6, 4, 4, 8)
    W, N, rng = rand_links(dims, 13)
    g = latgen.gauge_transform(dims, rng)
    Wg = np.empty_like(W)
    Ng = np.empty_like(N)
    for mu in range(4):
        ax = ops.axis_of(mu)
        g1 = np.roll(g, -1, axis=ax)
        g3 = np.roll(g, -3, axis=ax)
        Wg[mu] = g @ W[mu] @ np.swapaxes(g1.conj(), -1, -2)
        Ng[mu] = g @ N[mu] @ np.swapaxes(g3.conj(), -1, -2)
    x = latgen.fine_vectors(dims, 1, rng)[0]
    lhs = ops.dslash(np.einsum("...ij,...j->...i", g, x), Wg, Ng, 0.02, C1H, C3H)
    rhs = np.einsum("...ij,...j->...i", g, ops.dslash(x, W, N, 0.02, C1H, C3H))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


# ----------------------------------------------------------------------------
# Kahler-Dirac block
# ----------------------------------------------------------------------------

def dense_B(dims, W, c1):
    Bm = ops.kd_block_matrices(W, 0.0, c1)
    idx = ops._hc_gather_index(dims)
    V = int(np.prod(dims))
    B = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    rows = (3 * idx[:, :, None] + np.arange(3)).reshape(idx.shape[0], 48)
    for h in range(idx.shape[0]):
        B[np.ix_(rows[h], rows[h])] = Bm[h]
    return B


def test_kd_B_is_in_cube_part_of_D():
    """B = the one-hop terms of D between sites of the same 2^4 hypercube
    (Sec. 2.2); D = (B + m) + C with C coupling different hypercubes only."""
    dims = (4, 4, 4, 4)
    W, _, _ = rand_links(dims, 14)
    m = 0.1
    D = ops.dense_matrix(lambda v: ops.dslash(v, W, W, m, C1H, 0.0), (4, 4, 4, 4, 3))
    B = dense_B(dims, W, C1H)
    hc, _ = ops.hypercube_index(dims)
    h3 = np.repeat(hc.reshape(-1), 3)
    same = h3[:, None] == h3[None, :]
    C = D - m * np.eye(D.shape[0]) - B
    assert np.max(np.abs(C[same])) < 1e-15
    assert np.max(np.abs(B[~same])) == 0.0
    assert np.max(np.abs(B + B.conj().T)) < 1e-15  # anti-Hermitian for any links


def test_kd_free_field():
    """Free field (Sec. 2.2): B^dag B = C^dag C = c1^2 I, so
    (B+m)^{-1} = (m - B)/(m^2 + c1^2), and the naive KD operator
    A = (B+m)^{-1} D has its spectrum on the circle |lambda - 1| = c1/sqrt(m^2+c1^2)
    (the overlap-like shifted circle of Eq. 2)."""
    dims = (4, 4, 4, 4)
    U = latgen.unit_links(dims)
    m, c1 = 0.1, 1.0
    B = dense_B(dims, U, c1)
    D = ops.dense_matrix(lambda v: ops.dslash(v, U, U, m, c1, 0.0), (4, 4, 4, 4, 3))
    I = np.eye(D.shape[0])
    C = D - m * I - B
    assert np.max(np.abs(B.conj().T @ B - c1 ** 2 * I)) < 1e-14
    assert np.max(np.abs(C.conj().T @ C - c1 ** 2 * I)) < 1e-14
    Kinv = ops.kd_inverse(U, m, c1)
    Bb = ops.kd_block_matrices(U, 0.0, c1)
    closed = (m * np.eye(48) - Bb) / (m * m + c1 * c1)
    assert np.max(np.abs(Kinv - closed)) < 1e-14
    A = ops.dense_matrix(lambda v: ops.kd_operator(v, U, U, Kinv, m, c1, 0.0), (4, 4, 4, 4, 3))
    lam = np.linalg.eigvals(A)
    assert np.max(np.abs(np.abs(lam - 1.0) - c1 / np.sqrt(m * m + c1 * c1))) < 1e-12


def test_kd_inverse_and_operator_adjoint():
    dims = (4, 4, 4, 4)
    W, N, rng = rand_links(dims, 15)
    m = 0.01
    Kinv = ops.kd_inverse(W, m, C1H)
    Bm = ops.kd_block_matrices(W, m, C1H)
    assert np.max(np.abs(Kinv @ Bm - np.eye(48))) < 1e-10
    shape = (4, 4, 4, 4, 3)
    A = ops.dense_matrix(lambda v: ops.kd_operator(v, W, N, Kinv, m, C1H, C3H), shape)
    Ad = ops.dense_matrix(lambda v: ops.kd_operator_dagger(v, W, N, Kinv, m, C1H, C3H), shape)
    assert np.max(np.abs(Ad - A.conj().T)) < 1e-10 * np.max(np.abs(A))
    # with the Naik term kept, A is an exact left preconditioning of D (Sec. 3.1)
    D = ops.dense_matrix(lambda v: ops.dslash(v, W, N, m, C1H, C3H), shape)
    B = dense_B(dims, W, C1H) + m * np.eye(D.shape[0])
    assert np.max(np.abs(B @ A - D)) < 1e-12


# ----------------------------------------------------------------------------
# Transfer and Galerkin
# ----------------------------------------------------------------------------

def test_transfer_orthonormal_chiral_local():
    dims = (8, 4, 4, 4)
    block = (4, 2, 2, 2)
    rng = np.random.default_rng(3)
    nvec = 12
    nv = latgen.fine_vectors(dims, nvec, rng)
    agg, chi = ops.fine_dof_labels(dims, block)
    t = ops.Transfer(nv, agg, chi)
    ncoarse = t.nagg * 2 * nvec
    Pm = np.stack([t.prolong(np.eye(ncoarse)[j]) for j in range(ncoarse)], axis=1)
    assert np.max(np.abs(Pm.conj().T @ Pm - np.eye(ncoarse))) < 1e-14
    # restrict is the adjoint of prolong
    r = latgen.fine_vectors(dims, 1, rng)[0].reshape(-1)
    assert np.max(np.abs(t.restrict(r).reshape(-1) - Pm.conj().T @ r)) < 1e-13
    # each column lives on one aggregate and one chirality
    e = np.repeat(ops.epsilon(dims).reshape(-1), 3)
    for j in range(ncoarse):
        a, s = j // (2 * nvec), (j // nvec) % 2
        col = Pm[:, j]
        nz = np.abs(col) > 0
        assert np.all(agg[nz] == a)
        assert np.all(e[nz] == (1 - 2 * s))
    # span: each null vector's chiral projections lie in range(P)
    for k in range(nvec):
        v = nv[k].reshape(-1)
        for sgn in (1, -1):
            pv = 0.5 * (1 + sgn * e) * v
            assert np.linalg.norm(Pm @ (Pm.conj().T @ pv) - pv) < 1e-12 * np.linalg.norm(pv)


def test_qr_positive_unique():
    rng = np.random.default_rng(4)
    V = latgen.complex_normal(rng, (30, 7))
    Q, rd = ops.qr_positive(V)
    R = Q.conj().T @ V
    assert np.max(np.abs(np.tril(R, -1))) < 1e-13
    assert np.all(np.abs(np.diag(R).imag) < 1e-13) and np.all(np.diag(R).real > 0)
    # Gram-Schmidt by hand gives the same Q (uniqueness of positive-diag QR)
    G = np.zeros_like(V)
    for k in range(7):
        w = V[:, k].copy()
        for j in range(k):
            w -= np.vdot(G[:, j], w) * G[:, j]
        for j in range(k):
            w -= np.vdot(G[:, j], w) * G[:, j]
        G[:, k] = w / np.linalg.norm(w)
    assert np.max(np.abs(G - Q)) < 1e-13


def test_coarse_dof_labels_pinned_by_restriction_and_chirality():
    """The labels of a second aggregation (coarse_dof_labels) follow from what
    the first one produces, not from their own formula: a fine vector on one
    chirality restricts onto the coarse dofs labelled with it, a fine vector on
    one first-level aggregate restricts onto the dofs of that coarse site, and
    the coarse aggregates are those of a brute-force loop over coarse
    coordinates.  The coarse chirality they define is the one the physics
    fixes: eps_hat P1^dag D P1 eps_hat = (P1^dag D P1)^dag (eps D eps = D^dag,
    Sec. 2.2), and it carries over to the third level."""
    dims, b1, b2, nvec = (8, 4, 4, 4), (2, 2, 2, 2), (2, 1, 1, 2), 6
    cd = tuple(d // b for d, b in zip(dims, b1))          # (4, 2, 2, 2)
    cd3 = tuple(d // b for d, b in zip(cd, b2))           # (2, 2, 2, 1)
    rng = np.random.default_rng(11)
    W, N, rng = rand_links(dims, 16)
    nv = latgen.fine_vectors(dims, nvec, rng)
    t1 = ops.Transfer(nv, *ops.fine_dof_labels(dims, b1))
    agg1, chi1 = ops.coarse_dof_labels(cd, nvec, (1, 1, 1, 1))
    nc = int(np.prod(cd)) * 2 * nvec
    assert agg1.shape == chi1.shape == (nc,)
    eps = ops.epsilon(dims)[..., None]
    r = latgen.fine_vectors(dims, 1, rng)[0]
    # chirality: restriction of each chiral half lands on the dofs with that label
    for sgn, lab in ((1, 0), (-1, 1)):
        rc = t1.restrict(0.5 * (1 + sgn * eps) * r).reshape(-1)
        assert np.all(np.abs(rc[chi1 != lab]) == 0.0)
        assert np.all(np.abs(rc[chi1 == lab]) > 0.0)
    # aggregates: fine sites of first-level aggregate c (brute-force coordinates)
    X, Y, Z, T = dims
    owner = np.zeros((T, Z, Y, X), dtype=np.int64)
    for t in range(T):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    owner[t, z, y, x] = (x // b1[0]) + cd[0] * ((y // b1[1]) + cd[1] * ((z // b1[2]) + cd[2] * (t // b1[3])))
    for c in (0, 5, int(np.prod(cd)) - 1):
        rc = t1.restrict(np.where((owner == c)[..., None], r, 0)).reshape(-1)
        assert np.all(rc[agg1 != c] == 0.0) and np.all(np.abs(rc[agg1 == c]) > 0.0)
    # second aggregation: coarse site c at coordinates from a loop, aggregate by floor(x / b2)
    agg2, chi2 = ops.coarse_dof_labels(cd, nvec, b2)
    assert np.array_equal(chi2, chi1)
    site = 0
    for t in range(cd[3]):
        for z in range(cd[2]):
            for y in range(cd[1]):
                for x in range(cd[0]):
                    want = (x // b2[0]) + cd3[0] * ((y // b2[1]) + cd3[1] * ((z // b2[2]) + cd3[2] * (t // b2[3])))
                    assert np.all(agg2[site * 2 * nvec:(site + 1) * 2 * nvec] == want)
                    site += 1
    # physics: the labelled chirality makes the Galerkin operator eps-hermitian
    m = 0.05
    P1 = np.stack([t1.prolong(np.eye(nc)[j]) for j in range(nc)], axis=1)
    D1 = P1.conj().T @ np.stack([ops.dslash(P1[:, j].reshape(T, Z, Y, X, 3), W, N, m, C1H, C3H).reshape(-1)
                                 for j in range(nc)], axis=1)
    e2 = 1.0 - 2.0 * chi1
    assert np.max(np.abs(e2[:, None] * D1 * e2[None, :] - D1.conj().T)) < 1e-12 * np.max(np.abs(D1))
    # a swapped labelling (spin index taken as the fast one) breaks it
    bad = np.tile(np.arange(2 * nvec) % 2, nc // (2 * nvec))
    eb = 1.0 - 2.0 * bad
    assert np.max(np.abs(eb[:, None] * D1 * eb[None, :] - D1.conj().T)) > 1e-3 * np.max(np.abs(D1))
    # third level: columns on one aggregate and one chirality, null vectors' chiral halves in range(P2),
    # and the level-3 operator is eps-hermitian with the labels of its own layout
    nvec2 = 5
    nv2 = latgen.coarse_vectors(cd, nvec, nvec2, rng)
    t2 = ops.Transfer(nv2, agg2, chi2)
    nc3 = int(np.prod(cd3)) * 2 * nvec2
    P2 = np.stack([t2.prolong(np.eye(nc3)[j]) for j in range(nc3)], axis=1)
    assert np.max(np.abs(P2.conj().T @ P2 - np.eye(nc3))) < 1e-13
    for j in range(nc3):
        nz = np.abs(P2[:, j]) > 0
        assert np.all(agg2[nz] == j // (2 * nvec2)) and np.all(chi2[nz] == (j // nvec2) % 2)
    for k in range(nvec2):
        v = nv2[k].reshape(-1)
        for sgn in (1, -1):
            pv = 0.5 * (1 + sgn * e2) * v
            assert np.linalg.norm(P2 @ (P2.conj().T @ pv) - pv) < 1e-12 * np.linalg.norm(pv)
    D2 = P2.conj().T @ D1 @ P2
    _, chi3 = ops.coarse_dof_labels(cd3, nvec2, (1, 1, 1, 1))
    e3 = 1.0 - 2.0 * chi3
    assert np.max(np.abs(e3[:, None] * D2 * e3[None, :] - D2.conj().T)) < 1e-12 * np.max(np.abs(D2))
