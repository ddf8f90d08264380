"""Shared helpers of the GPU parity tests: seeded configurations, oracle
counterparts and error metrics."""
import sys

import numpy as np

from oracle import operators as ops
from oracle import solvers as sol
from paper_2212_12559_amd import latgen

C1H, C3H = 9.0 / 8.0, -1.0 / 24.0

# name: dims, coefficients, kd_naik, blocks, nvec, mass0
CONFIGS = {
    # 4^4 naive, KD then 2^4 aggregation, Nvec 24 (square P)
    "c0": dict(dims=(4, 4, 4, 4), c1=1.0, c3=0.0, kd_naik=1, blocks=[(2, 2, 2, 2)], nvec=(24,), mass0=0.1,
               eps=0.3, seed=latgen.SEEDS["c0_4x4_naive"]),
    # 8^4 HISQ-style, two aggregations (coarse 2^4, then 1^4)
    "cubic": dict(dims=(8, 8, 8, 8), c1=C1H, c3=C3H, kd_naik=1, blocks=[(4, 4, 4, 4), (2, 2, 2, 2)], nvec=(8, 8),
                  mass0=0.05, eps=0.5, seed=latgen.SEEDS["small_8x4_hisq"]),
    # ragged: V = 2304 (9 blocks of 256), odd coarse extent 3, extents 1
    "ragged": dict(dims=(8, 4, 6, 12), c1=C1H, c3=C3H, kd_naik=0, blocks=[(4, 4, 6, 4), (2, 1, 1, 3)],
                   nvec=(10, 12), mass0=0.07, eps=0.5, seed=424242),
    # widest 16-bit coarse stencil: Nvec 128 (n = 256, sixteen MFMA row tiles),
    # coarse lattice 2x1x1x1
    "wide": dict(dims=(8, 4, 4, 4), c1=C1H, c3=C3H, kd_naik=1, blocks=[(4, 4, 4, 4)], nvec=(128,), mass0=0.05,
                 eps=0.5, seed=515151),
    # the production level shapes (Nvec 64 / 96: level 2 n = 128, level 3 n = 192) on a 4x4x4x1
    # level-2 lattice (odd x, y and z = 2, 3 mod 4 all present) at the light mass 0.005, Naik truncated
    # in the KD level as in the 32^4 multi-mass workload
    "prod": dict(dims=(16, 16, 16, 4), c1=C1H, c3=C3H, kd_naik=0, blocks=[(4, 4, 4, 4), (2, 2, 2, 1)],
                 nvec=(64, 96), mass0=0.005, eps=0.5, seed=626262),
    # the same level shapes with every coarse extent >= 2 (2x4x4x2, then 2^4): with block-preconditioned
    # coarse levels the self block is then exactly the identity and the 16-bit stencil adds the input
    # instead of reading it
    "prodblk": dict(dims=(8, 16, 16, 8), c1=C1H, c3=C3H, kd_naik=0, blocks=[(4, 4, 4, 4), (1, 2, 2, 1)],
                    nvec=(64, 96), mass0=0.005, eps=0.5, seed=636363),
    # the 16^4 HISQ-style hierarchy shape: KD, 4^4 / Nvec 64, 2^4 / Nvec 96
    "c1": dict(dims=(16, 16, 16, 16), c1=C1H, c3=C3H, kd_naik=1, blocks=[(4, 4, 4, 4), (2, 2, 2, 2)],
               nvec=(64, 96), mass0=0.01, eps=0.5, seed=latgen.SEEDS["c1_16x4_hisq"]),
}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def links(cfg):
    if cfg["c3"] == 0.0:
        W, N, rng = latgen.naive_links(cfg["dims"], cfg["eps"], cfg["seed"])
    else:
        W, N, rng = latgen.hisq_style_links(cfg["dims"], cfg["eps"], cfg["seed"])
    return W, N, rng


def coarse_dims(dims, block):
    return tuple(d // b for d, b in zip(dims, block))


def random_null_vectors(cfg, rng):
    """Full-rank random near-null vectors (inputs only; any full-rank set
    defines a valid transfer for operator parity)."""
    nv = [latgen.fine_vectors(cfg["dims"], cfg["nvec"][0], rng)]
    if len(cfg["blocks"]) > 1:
        cd = coarse_dims(cfg["dims"], cfg["blocks"][0])
        nv.append(latgen.coarse_vectors(cd, cfg["nvec"][0], cfg["nvec"][1], rng))
    return nv


def oracle_hierarchy(cfg, W, N, mass, nvs, **kw):
    p = sol.MGParams(dims=cfg["dims"], c1=cfg["c1"], c3=cfg["c3"], kd_naik=bool(cfg["kd_naik"]),
                     blocks=tuple(cfg["blocks"]), **kw)
    return sol.Hierarchy(p, W, N, mass, nvs)


def gpu_params(mg, cfg, **kw):
    # coarse_op 0 (Galerkin) and the GCR coarsest solver unless asked for: the oracle hierarchies default to them
    p = mg.default_params(cfg["dims"], c1=cfg["c1"], c3=cfg["c3"], kd_naik=cfg["kd_naik"],
                          nagg=len(cfg["blocks"]), block=cfg["blocks"], nvec=tuple(cfg["nvec"]) + (1,) * (2 - len(cfg["nvec"])),
                          mass0=cfg["mass0"], coarse_op=0, coarsest_solver=0)
    for k, v in kw.items():
        if k in ("setup_maxiter", "setup_tol", "nvec"):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(p, k, v)
    return p


_LINKS = {}


def cached_hierarchy_links(name, H):
    """The oracle's explicit coarse links of the hierarchy of CONFIGS[name]
    with its seeded random null vectors (computed once per process: about a
    minute for "prod")."""
    if name not in _LINKS:
        _LINKS[name] = sol.hierarchy_links(H)
    return _LINKS[name]


def abs1(a):
    """|Re a| + |Im a|: bounds |a| and makes the error bounds of complex sums
    of products a sum over real products."""
    return np.abs(np.real(a)) + np.abs(np.imag(a))


def gamma(k, u):
    """Higham's gamma_k = k u / (1 - k u): the relative error bound of a sum of
    k real products accumulated in any order with unit roundoff u."""
    return k * u / (1.0 - k * u)


def abs_dslash(xa, W, N, mass, c1, c3):
    """sum_j |D_ij|_1 xa_j for the staggered operator: every hop with its link
    entries' |Re| + |Im| and a positive coefficient (phases and signs dropped),
    for the a-priori bound of a floating-point application of D."""
    out = abs(mass) * xa
    for mu in range(4):
        ax = ops.axis_of(mu)
        for h, coef, F in ((1, c1, W), (3, c3, N)):
            if coef == 0.0:
                continue
            Fa = abs1(F[mu])
            fwd = np.einsum("...ab,...b->...a", Fa, np.roll(xa, -h, axis=ax))
            Fb = np.roll(Fa, h, axis=ax)
            bwd = np.einsum("...ba,...b->...a", Fb, np.roll(xa, h, axis=ax))
            out = out + 0.5 * abs(coef) * (fwd + bwd)
    return out


def rel_err(got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))
