"""GPU solves through the C ABI: MG-GCR (FP64 and mixed precision), the
Schur CG baseline, multi-mass batches, GPU-generated near-null vectors and the
error paths.  The true residual of every solution is recomputed by the
oracle's FP64 operator."""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import solvers as sol
from paper_2212_12559_amd import latgen

from gpu_common import CONFIGS, gpu_params, links, log, oracle_hierarchy, rel_err  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mg(torch):
    from paper_2212_12559_amd import mgstag
    return mgstag


def true_rel(cfg, W, N, m, x, b):
    r = b - ops.dslash(x, W, N, m, cfg["c1"], cfg["c3"])
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def cgne_vectors(cfg, W, N, rng, iters=(30, 20)):
    """Oracle near-null vectors: short CGNE on each level's operator."""
    m = cfg["mass0"]
    c3kd = cfg["c3"] if cfg["kd_naik"] else 0.0
    Kinv = ops.kd_inverse(W, m, cfg["c1"])
    A = lambda v: ops.kd_operator(v, W, N, Kinv, m, cfg["c1"], c3kd)
    Ad = lambda v: ops.kd_operator_dagger(v, W, N, Kinv, m, cfg["c1"], c3kd)
    phi0 = latgen.fine_vectors(cfg["dims"], cfg["nvec"][0], rng)
    nv1 = np.stack([sol.cgne_null_vector(A, Ad, phi0[k], 1e-6, iters[0])[0] for k in range(len(phi0))])
    out = [nv1]
    if len(cfg["blocks"]) > 1:
        H1 = oracle_hierarchy(dict(cfg, blocks=cfg["blocks"][:1]), W, N, m, [nv1])
        shape = H1.fine_shape(2)
        phi2 = latgen.complex_normal(rng, (cfg["nvec"][1],) + shape)
        nv2 = np.stack([sol.cgne_null_vector(lambda v: H1.op(2, v), lambda v: H1.op_dag(2, v), phi2[k], 1e-6,
                                             iters[1])[0] for k in range(len(phi2))])
        out.append(nv2)
    return out


@pytest.fixture(scope="module")
def cubic(torch):
    cfg = CONFIGS["cubic"]
    W, N, rng = links(cfg)
    nvs = cgne_vectors(cfg, W, N, rng)
    b = latgen.fine_vectors(cfg["dims"], 2, rng)
    return cfg, W, N, nvs, b


def make_ctx(torch, mg, cfg, W, N, nvs, **kw):
    dev = "cuda:0"
    p = gpu_params(mg, cfg, **kw)
    nvt = [torch.from_numpy(v).to(dev) for v in nvs] if nvs is not None else None
    return mg.setup(p, torch.from_numpy(W).to(dev), torch.from_numpy(N).to(dev) if cfg["c3"] else None, nvt)


def test_fp64_kcycle_matches_oracle(torch, mg, cubic):
    """All-FP64 GPU MG-GCR vs the oracle's K-cycle with the same null
    vectors: same outer iteration count (+-1), both at true residual 1e-10,
    residual histories agreeing over the first iterations, and
    ||x - x_oracle|| within the bound 2e-10 ||b|| / m."""
    cfg, W, N, nvs, b = cubic
    m = cfg["mass0"]
    log("[solve] cubic fp64 vs oracle")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128, max_nrhs=1)
    x, info, st = ctx.solve([m], torch.from_numpy(b[:1]).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()[0, 0]
    H = oracle_hierarchy(cfg, W, N, m, nvs)
    xo, io = H.solve(b[0], tol=1e-10)
    assert io.converged
    assert abs(info[0]["outer_iters"] - io.iters) <= 1, (info[0], io.iters)
    assert true_rel(cfg, W, N, m, x, b[0]) <= 1e-10
    assert np.linalg.norm(x - xo) <= 2e-10 * np.linalg.norm(b[0]) / m


def test_fp64_block_kcycle_matches_oracle(torch, mg, cubic):
    """Block-preconditioned coarse levels (coarse_op 1, Sec. 2.3 / Table 1),
    all FP64: the GPU's K-cycle and the oracle's with coarse_op "block" and the
    same null vectors take the same outer iterations (+-1) and agree within
    2e-10 ||b|| / m at true residual 1e-10; the coarse solves of the block
    hierarchy are compared with the Galerkin ones in iteration counts (log)."""
    cfg, W, N, nvs, b = cubic
    m = cfg["mass0"]
    log("[solve] cubic fp64 block-preconditioned vs oracle")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128, max_nrhs=1,
                   coarse_op=1)
    x, info, st = ctx.solve([m], torch.from_numpy(b[:1]).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()[0, 0]
    H = oracle_hierarchy(cfg, W, N, m, nvs, coarse_op="block")
    xo, io = H.solve(b[0], tol=1e-10)
    assert io.converged
    assert abs(info[0]["outer_iters"] - io.iters) <= 1, (info[0], io.iters)
    assert true_rel(cfg, W, N, m, x, b[0]) <= 1e-10
    assert np.linalg.norm(x - xo) <= 2e-10 * np.linalg.norm(b[0]) / m
    ctx_g = make_ctx(torch, mg, cfg, W, N, nvs, fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128, max_nrhs=1)
    xg, info_g, st = ctx_g.solve([m], torch.from_numpy(b[:1]).to("cuda:0"), tol=1e-10)
    log(f"    block: outer {info[0]['outer_iters']} levels {info[0]['level_iters']}; "
        f"galerkin: outer {info_g[0]['outer_iters']} levels {info_g[0]['level_iters']}")


def test_fp64_cagcr_coarsest_matches_oracle(torch, mg, cubic):
    """Coarsest level solved by CA-GCR(16) in a Chebyshev basis
    (coarsest_solver 1, Table 1), with block-preconditioned coarse levels, all
    FP64: a cycle computes the Krylov minimiser over K_16, as the oracle's
    CA-GCR does by Arnoldi and least squares, so the K-cycles take the same
    outer iterations (+-1) and the solutions agree within 2e-10 ||b|| / m."""
    cfg, W, N, nvs, b = cubic
    m = cfg["mass0"]
    log("[solve] cubic fp64 CA-GCR(16) coarsest vs oracle")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128, max_nrhs=1,
                   coarse_op=1, coarsest_solver=1, coarsest_maxiter=16, coarsest_restarts=1)
    x, info, st = ctx.solve([m], torch.from_numpy(b[:1]).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()[0, 0]
    H = oracle_hierarchy(cfg, W, N, m, nvs, coarse_op="block", coarsest_solver="cagcr", coarsest_maxiter=16,
                         coarsest_cycles=1)
    xo, io = H.solve(b[0], tol=1e-10)
    assert io.converged
    log(f"    outer {info[0]['outer_iters']} (oracle {io.iters}), levels {info[0]['level_iters']}")
    assert abs(info[0]["outer_iters"] - io.iters) <= 1, (info[0], io.iters)
    assert true_rel(cfg, W, N, m, x, b[0]) <= 1e-10
    assert np.linalg.norm(x - xo) <= 2e-10 * np.linalg.norm(b[0]) / m


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_cagcr_coarsest_lockstep_16bit(torch, mg, cubic, fmt):
    """CA-GCR(16) coarsest solver with FP32 vectors and 16-bit links in a
    16 rhs x 2 masses lockstep solve (two restart cycles): every system
    reaches 1e-10 on the oracle's true residual."""
    cfg, W, N, nvs, _ = cubic
    masses = [0.05, 0.11]
    rng = np.random.default_rng(4323)
    b = latgen.fine_vectors(cfg["dims"], 16, rng)
    log(f"[solve] cubic 16 rhs x 2 masses {fmt}, CA-GCR(16) coarsest")
    cp = mg.MG_CBF16 if fmt == "bf16" else mg.MG_CF16
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=32, max_nmass=2, coarse_prec=cp, coarse_op=1,
                   coarsest_solver=1, coarsest_maxiter=16, coarsest_restarts=2)
    x, info, st = ctx.solve(masses, torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()
    for j, m in enumerate(masses):
        for r in range(16):
            assert info[j * 16 + r]["status"] == "MG_OK"
            assert true_rel(cfg, W, N, m, x[j, r], b[r]) <= 1e-10, (m, r)
    log(f"    outer iterations {[i['outer_iters'] for i in info]}, levels {info[0]['level_iters']}")


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_default_hierarchy_16bit_production_shapes(torch, mg, fmt):
    """The library defaults (block-preconditioned coarse levels, CA-GCR(16)
    coarsest solver in a Chebyshev basis) with 16-bit coarse links on the
    production level shapes (Nvec 64 / 96: level 2 n = 128, level 3 n = 192,
    a 2x2x2x1 coarsest lattice) at the light mass 0.005, GPU null vectors:
    8 systems reach 1e-10 on the oracle's true residual.  For this
    non-Hermitian coarsest operator the Chebyshev basis grows off the real
    axis; its set-up growth estimate keeps the fp16 stencil inputs in range."""
    cfg = CONFIGS["prod"]
    W, N, rng = links(cfg)
    m = cfg["mass0"]
    b = latgen.fine_vectors(cfg["dims"], 8, rng)
    log(f"[solve] prod shapes {fmt}, library defaults")
    cp = mg.MG_CBF16 if fmt == "bf16" else mg.MG_CF16
    ctx = make_ctx(torch, mg, cfg, W, N, None, max_nrhs=8, coarse_prec=cp, coarse_op=1, coarsest_solver=1,
                   setup_maxiter=(300, 100))
    x, info, st = ctx.solve([m], torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()
    log(f"    outer iterations {[i['outer_iters'] for i in info]}, levels {info[0]['level_iters']}")
    for r in range(8):
        assert info[r]["status"] == "MG_OK"
        assert true_rel(cfg, W, N, m, x[0, r], b[r]) <= 1e-10, r
    ctx.destroy()


def test_lockstep_truncated_kd_two_masses(torch, mg):
    """Two masses x 16 rhs in one lockstep solve with the Naik term truncated
    in the KD level on the production level shapes: the KD-level operator runs
    as 1 + (B+m)^{-1} D_off with a KD inverse slot per mass (16-rhs tiles), and
    every system reaches 1e-10 on the oracle's true residual."""
    cfg = CONFIGS["prod"]
    W, N, rng = links(cfg)
    masses = [0.005, 0.02]
    b = latgen.fine_vectors(cfg["dims"], 16, rng)
    log("[solve] prod shapes 16 rhs x 2 masses, truncated KD, fp16")
    ctx = make_ctx(torch, mg, cfg, W, N, None, max_nrhs=32, max_nmass=2, coarse_prec=mg.MG_CF16, coarse_op=1,
                   coarsest_solver=1, setup_maxiter=(300, 100))
    x, info, st = ctx.solve(masses, torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()
    log(f"    outer iterations {[i['outer_iters'] for i in info]}, levels {info[0]['level_iters']}")
    for j, m in enumerate(masses):
        for r in range(16):
            assert info[j * 16 + r]["status"] == "MG_OK"
            assert true_rel(cfg, W, N, m, x[j, r], b[r]) <= 1e-10, (m, r)
    ctx.destroy()


def test_fp64_direct_coarsest_matches_oracle(torch, mg):
    """coarsest_solver 2: the coarsest operator's dense inverse (Gauss-Jordan
    with partial pivoting at set-up) applied as one product per coarsest
    solve, all FP64, on the 4^4 two-level hierarchy (coarsest 2^4 x 48 = 768
    dof, block-preconditioned), against the oracle's K-cycle with a dense LU
    coarsest solve: same outer iterations (+-1), both at true residual 1e-10,
    solutions within 2e-10 ||b|| / m."""
    from gpu_common import random_null_vectors
    cfg = CONFIGS["c0"]
    W, N, rng = links(cfg)
    nvs = random_null_vectors(cfg, rng)
    b = latgen.fine_vectors(cfg["dims"], 1, rng)
    m = cfg["mass0"]
    log("[solve] c0 fp64 direct coarsest vs oracle")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128, max_nrhs=1,
                   coarse_op=1, coarsest_solver=2)
    x, info, st = ctx.solve([m], torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()[0, 0]
    H = oracle_hierarchy(cfg, W, N, m, nvs, coarse_op="block", coarsest_direct=True)
    xo, io = H.solve(b[0], tol=1e-10)
    assert io.converged
    log(f"    outer {info[0]['outer_iters']} (oracle {io.iters}), levels {info[0]['level_iters']}")
    assert abs(info[0]["outer_iters"] - io.iters) <= 1, (info[0], io.iters)
    assert true_rel(cfg, W, N, m, x, b[0]) <= 1e-10
    assert np.linalg.norm(x - xo) <= 2e-10 * np.linalg.norm(b[0]) / m
    ctx.destroy()


def test_direct_coarsest_small_lattice_bf16(torch, mg):
    """8^4 two-level hierarchy of the uneven batch (KD + 4^4 / Nvec 48: a
    coarsest level of 2^4 x 96 = 1536 dof), mass 0.01, GPU null vectors, bf16
    links, 12 rhs: with the exact coarsest solve the outer iteration count
    drops from hundreds (16-step GCR on the coarsest level) to a few dozen,
    and every system reaches 1e-10 on the oracle's true residual."""
    dims, m = (8, 8, 8, 8), 0.01
    cfg = dict(c1=9.0 / 8.0, c3=-1.0 / 24.0)
    W, N, rng = latgen.hisq_style_links(dims, 0.5, 20221229)
    b = latgen.fine_vectors(dims, 12, rng)
    dev = "cuda:0"
    outer = {}
    for cs in (0, 2):
        log(f"[solve] 8^4 uneven hierarchy, coarsest_solver {cs}")
        p = mg.default_params(dims, mass0=m, nagg=1, nvec=(48, 1), block=[(4, 4, 4, 4)], setup_maxiter=(300, 1),
                              max_nrhs=12, kd_naik=0, coarse_prec=mg.MG_CBF16, outer_nkrylov=8, outer_maxiter=2000,
                              coarse_op=0, coarsest_solver=cs)
        ctx = mg.setup(p, torch.from_numpy(W).to(dev), torch.from_numpy(N).to(dev))
        x, info, st = ctx.solve([m], torch.from_numpy(b).to(dev), tol=1e-10)
        x = x.cpu().numpy()
        outer[cs] = max(i["outer_iters"] for i in info)
        for r in range(12):
            assert info[r]["status"] == "MG_OK"
            assert true_rel(cfg, W, N, m, x[0, r], b[r]) <= 1e-10, (cs, r)
        ctx.destroy()
    log(f"    outer iterations: GCR(16) coarsest {outer[0]}, direct {outer[2]}")
    assert outer[2] <= 60 and outer[2] * 3 < outer[0], outer


def test_mass_compaction_is_exact(torch, mg, cubic):
    """compact_masses 1: once all right-hand sides of a mass have converged,
    that mass leaves the K-cycle's batch (its residuals are no longer
    gathered); every system is independent in the batch, so the solutions
    equal bit for bit, and the outer iteration counts, those of a context
    that keeps every mass in the K-cycle; all at true residual 1e-10."""
    cfg, W, N, nvs, _ = cubic
    masses = [0.05, 0.11, 0.3]
    rng = np.random.default_rng(4325)
    b = latgen.fine_vectors(cfg["dims"], 8, rng)
    bt = torch.from_numpy(b).to("cuda:0")
    res = {}
    for cm in (0, 1):
        log(f"[compact] compact_masses {cm}")
        ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=24, max_nmass=6, coarse_prec=mg.MG_CBF16, coarse_op=1,
                       coarsest_solver=1, compact_masses=cm)
        x, info, st = ctx.solve(masses, bt, tol=1e-10)
        res[cm] = (x.cpu().numpy(), [i["outer_iters"] for i in info], info[0]["level_iters"])
        ctx.destroy()
    log(f"    outer {res[1][1]}; level iterations without / with compaction {res[0][2]} / {res[1][2]}")
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])
    assert len(set(res[1][1][j * 8] for j in range(3))) > 1   # the masses converge at different iterations
    for j, m in enumerate(masses):
        for r in range(8):
            assert true_rel(cfg, W, N, m, res[1][0][j, r], b[r]) <= 1e-10, (m, r)


def test_coarse_shadow_is_exact(torch, mg, cubic):
    """coarse_shadow 1: in the level-2 smoother's chain the 16-bit stencil also
    stores its output rounded to the link format and the next application
    stages those values instead of rounding the FP32 vector again; the
    rounding is the same, so the solutions equal bit for bit those without
    the copies (bf16 and fp16 links)."""
    cfg, W, N, nvs, _ = cubic
    rng = np.random.default_rng(4326)
    b = latgen.fine_vectors(cfg["dims"], 4, rng)
    bt = torch.from_numpy(b).to("cuda:0")
    for fmt, cp in (("bf16", mg.MG_CBF16), ("fp16", mg.MG_CF16)):
        res = []
        for sh in (0, 1):
            log(f"[shadow] {fmt} coarse_shadow {sh}")
            ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=4, coarse_prec=cp, coarse_op=1, coarsest_solver=1,
                           coarse_shadow=sh)
            x, info, st = ctx.solve([0.05], bt, tol=1e-10)
            res.append((x.cpu().numpy(), [i["outer_iters"] for i in info]))
            ctx.destroy()
        assert res[0][1] == res[1][1], fmt
        assert np.array_equal(res[0][0], res[1][0]), fmt
        for r in range(4):
            assert true_rel(cfg, W, N, 0.05, res[1][0][0, r], b[r]) <= 1e-10


def test_graph_coarsest_replays_match_eager(torch, mg, cubic):
    """The coarsest solve captured into a HIP graph (graph_coarsest 1, one
    CA-GCR cycle) and replayed: three solves of the same batch on one
    context, with eager work and synchronisations between them, each equal
    bit for bit to the solve of a context that launches eagerly; every
    system at true residual 1e-10."""
    cfg, W, N, nvs, _ = cubic
    masses = [0.05, 0.11]
    rng = np.random.default_rng(4324)
    b = latgen.fine_vectors(cfg["dims"], 16, rng)
    bt = torch.from_numpy(b).to("cuda:0")
    kw = dict(max_nrhs=32, max_nmass=2, coarse_prec=mg.MG_CBF16, coarse_op=1, coarsest_solver=1,
              coarsest_maxiter=16, coarsest_restarts=1)
    log("[graph] eager reference")
    ctx_e = make_ctx(torch, mg, cfg, W, N, nvs, graph_coarsest=0, **kw)
    xe, ie, _ = ctx_e.solve(masses, bt, tol=1e-10)
    xe = xe.cpu().numpy()
    ctx_g = make_ctx(torch, mg, cfg, W, N, nvs, graph_coarsest=1, **kw)
    for rep in range(3):
        log(f"[graph] replay {rep}")
        xg, ig, _ = ctx_g.solve(masses, bt, tol=1e-10)
        assert np.array_equal(xg.cpu().numpy(), xe), rep
        assert [i["outer_iters"] for i in ig] == [i["outer_iters"] for i in ie]
        ctx_g.apply_dslash(0, 0.1, bt)   # eager work between the replays
        torch.cuda.synchronize()
    for j, m in enumerate(masses):
        for r in range(16):
            assert true_rel(cfg, W, N, m, xe[j, r], b[r]) <= 1e-10, (m, r)


def test_block_lockstep_bf16(torch, mg, cubic):
    """Block-preconditioned coarse levels with 16-bit links (the links
    multiplied by X^{-1} before rounding) in a 16 rhs x 2 masses lockstep
    solve: every system reaches 1e-10 on the oracle's true residual."""
    cfg, W, N, nvs, _ = cubic
    masses = [0.05, 0.11]
    rng = np.random.default_rng(4322)
    b = latgen.fine_vectors(cfg["dims"], 16, rng)
    log("[solve] cubic 16 rhs x 2 masses bf16, block-preconditioned coarse levels")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=32, max_nmass=2, coarse_prec=mg.MG_CBF16, coarse_op=1)
    x, info, st = ctx.solve(masses, torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()
    for j, m in enumerate(masses):
        for r in range(16):
            assert info[j * 16 + r]["status"] == "MG_OK"
            assert true_rel(cfg, W, N, m, x[j, r], b[r]) <= 1e-10, (m, r)
    log(f"    outer iterations {[i['outer_iters'] for i in info]}")


def test_mixed_precision_solve_and_cg(torch, mg, cubic):
    """FP32 K-cycle inside the FP64 outer GCR reaches 1e-10 on the true
    residual; the Schur CG baseline reaches it too and agrees with MG within
    the bound from ||D^{-1}|| <= 1/m."""
    cfg, W, N, nvs, b = cubic
    m = 0.02
    log("[solve] cubic fp32 mixed + CG")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=2)
    bt = torch.from_numpy(b).to("cuda:0")
    x, info, st = ctx.solve([m], bt, tol=1e-10)
    xc, ic, stc = ctx.cg_solve([m], bt, tol=1e-10)
    x, xc = x.cpu().numpy()[0], xc.cpu().numpy()[0]
    for r in range(2):
        assert true_rel(cfg, W, N, m, x[r], b[r]) <= 1e-10
        assert true_rel(cfg, W, N, m, xc[r], b[r]) <= 1e-10
        assert np.linalg.norm(x[r] - xc[r]) <= 2e-10 * np.linalg.norm(b[r]) / m
        assert info[r]["status"] == "MG_OK" and ic[r]["status"] == "MG_OK"
    assert info[0]["outer_iters"] < ic[0]["outer_iters"]


def test_multi_mass_batch(torch, mg, cubic):
    """One hierarchy (built at mass0) serves several masses with exact per-mass
    KD inverses; every (mass, rhs) system converges."""
    cfg, W, N, nvs, b = cubic
    masses = [0.05, 0.11, 0.3]
    log("[solve] cubic multi-mass")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=6, max_nmass=3)
    x, info, st = ctx.solve(masses, torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()
    for j, m in enumerate(masses):
        for r in range(2):
            assert true_rel(cfg, W, N, m, x[j, r], b[r]) <= 1e-10, (m, r)


_iters16 = {}


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_lockstep_16rhs_two_masses_16bit(torch, mg, cubic, fmt):
    """The production batch shape: 16 right-hand sides for each of two masses
    in one lockstep solve (KD on the matrix cores with one inverse slot per
    mass, 16-bit coarse links); every system reaches 1e-10 on the oracle's
    true residual.  Near the end of the solve the K-cycle's input is about
    1e-10 of b, far below FP16's normal range: the coarse levels solve for a
    power-of-two multiple of their right-hand side, so FP16 links keep
    preconditioning as well as bf16 ones (outer iterations compared)."""
    cfg, W, N, nvs, _ = cubic
    masses = [0.05, 0.11]
    rng = np.random.default_rng(4321)
    b = latgen.fine_vectors(cfg["dims"], 16, rng)
    log(f"[solve] cubic 16 rhs x 2 masses {fmt}")
    cp = mg.MG_CBF16 if fmt == "bf16" else mg.MG_CF16
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=32, max_nmass=2, coarse_prec=cp)
    x, info, st = ctx.solve(masses, torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()
    for j, m in enumerate(masses):
        for r in range(16):
            assert info[j * 16 + r]["status"] == "MG_OK"
            assert true_rel(cfg, W, N, m, x[j, r], b[r]) <= 1e-10, (m, r)
    _iters16[fmt] = [i["outer_iters"] for i in info]
    log(f"    outer iterations {fmt}: {_iters16[fmt]}")
    if len(_iters16) == 2:
        for ib, ih in zip(_iters16["bf16"], _iters16["fp16"]):
            assert ih <= ib + 2, (_iters16["bf16"], _iters16["fp16"])


def test_lockstep_truncated_kd_matches_solo(torch, mg, cubic):
    """Truncated KD level in FP32 (plane-staged stencil with per-rhs masses,
    KD inverse with per-mass slots): a lockstep batch of 2 masses x 16 rhs
    gives every system the iterations and solution of that mass solved alone
    (systems are independent in a batch), all at true residual 1e-10."""
    cfg, W, N, nvs, b0 = cubic
    cfg = dict(cfg, kd_naik=0)
    rng = np.random.default_rng(41)
    b = latgen.fine_vectors(cfg["dims"], 16, rng)
    bt = torch.from_numpy(b).to("cuda:0")
    masses = [0.05, 0.11]
    log("[solve] truncated KD, 2 masses x 16 rhs lockstep vs solo")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=32, max_nmass=2)
    x, info, st = ctx.solve(masses, bt, tol=1e-10)
    x = x.cpu().numpy()
    for j, m in enumerate(masses):
        xs, infos, sts = ctx.solve([m], bt, tol=1e-10)
        xs = xs.cpu().numpy()[0]
        for r in (0, 7, 15):
            assert info[j * 16 + r]["outer_iters"] == infos[r]["outer_iters"], (m, r)
            assert true_rel(cfg, W, N, m, x[j, r], b[r]) <= 1e-10
            assert np.linalg.norm(x[j, r] - xs[r]) <= 1e-6 * np.linalg.norm(xs[r]), (m, r)


def test_c0_exact_two_level(torch, mg):
    """4^4 naive, KD + 2^4 aggregation with Nvec = 24 (square, unitary P): with
    the coarsest level solved to 1e-14 the K-cycle is the exact inverse and the
    outer GCR converges in one iteration."""
    cfg = CONFIGS["c0"]
    W, N, rng = links(cfg)
    nvs = cgne_vectors(cfg, W, N, rng, iters=(50,))
    b = latgen.fine_vectors(cfg["dims"], 1, rng)
    log("[solve] c0 exact two-level")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128,
                   coarsest_tol=1e-14, coarsest_maxiter=16, coarsest_restarts=200, max_nrhs=1)
    x, info, st = ctx.solve([cfg["mass0"]], torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    assert info[0]["outer_iters"] == 1
    assert true_rel(cfg, W, N, cfg["mass0"], x.cpu().numpy()[0, 0], b[0]) <= 1e-10


def test_gpu_cgne_matches_oracle(torch, mg):
    """The set-up's CGNE from imported starting vectors (cgne_start_import 1,
    FP64 levels) against the oracle's cgne_null_vector from the same starts:
    the level-1 vectors after 12 iterations on the KD operator (Naik kept),
    then the level-2 vectors after 8 iterations on the Galerkin operator the
    oracle builds from its own level-1 vectors, element by element.  CG in
    FP64 over a dozen steps keeps the two within 1e-9 of each other."""
    from gpu_common import random_null_vectors
    cfg = CONFIGS["cubic"]
    W, N, rng = links(cfg)
    m = cfg["mass0"]
    starts = random_null_vectors(cfg, rng)
    log("[setup] cubic GPU CGNE from imported starts vs oracle")
    ctx = make_ctx(torch, mg, cfg, W, N, starts, fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128, max_nrhs=1,
                   cgne_start_import=1, setup_maxiter=(12, 8), setup_tol=(0.0, 0.0))
    nv1 = ctx.export(1, 1).cpu().numpy().reshape(starts[0].shape)
    nv2 = ctx.export(1, 2).cpu().numpy().reshape(starts[1].shape)
    ctx.destroy()
    c3kd = cfg["c3"] if cfg["kd_naik"] else 0.0
    Kinv = ops.kd_inverse(W, m, cfg["c1"])
    A = lambda v: ops.kd_operator(v, W, N, Kinv, m, cfg["c1"], c3kd)
    Ad = lambda v: ops.kd_operator_dagger(v, W, N, Kinv, m, cfg["c1"], c3kd)
    want1 = np.stack([sol.cgne_null_vector(A, Ad, starts[0][k], 0.0, 12)[0] for k in range(len(starts[0]))])
    e1 = rel_err(nv1, want1)
    H1 = oracle_hierarchy(dict(cfg, blocks=cfg["blocks"][:1]), W, N, m, [want1])
    want2 = np.stack([sol.cgne_null_vector(lambda v: H1.op(2, v), lambda v: H1.op_dag(2, v), starts[1][k], 0.0, 8)[0]
                      for k in range(len(starts[1]))])
    e2 = rel_err(nv2, want2)
    log(f"    level 1 rel err {e1:.2e}, level 2 rel err {e2:.2e}")
    assert e1 < 1e-9 and e2 < 1e-9, (e1, e2)


def test_gpu_null_vectors(torch, mg):
    """Null vectors generated on the GPU (CGNE on each level's operator from
    the GPU's own seeded random starts, so checked by their properties rather
    than element by element): the transfer built from them is orthonormal
    (R P = 1) and the vectors are much closer to the near-null space than
    random vectors; the MG solve converges with them."""
    cfg = CONFIGS["cubic"]
    W, N, rng = links(cfg)
    log("[setup] cubic GPU CGNE")
    ctx = make_ctx(torch, mg, cfg, W, N, None, setup_maxiter=(40, 30), max_nrhs=1)
    nv1 = ctx.export(1, 1).cpu().numpy().reshape((cfg["nvec"][0],) + (8, 8, 8, 8, 3))
    m = cfg["mass0"]
    Kinv = ops.kd_inverse(W, m, cfg["c1"])
    A = lambda v: ops.kd_operator(v, W, N, Kinv, m, cfg["c1"], cfg["c3"])
    q = [np.linalg.norm(A(v)) / np.linalg.norm(v) for v in nv1]
    rv = latgen.fine_vectors(cfg["dims"], 4, rng)
    q0 = [np.linalg.norm(A(v)) / np.linalg.norm(v) for v in rv]
    assert max(q) < 0.5 * min(q0)
    ec = torch.from_numpy(latgen.complex_normal(rng, (1, 2, 2, 2, 2, 2, cfg["nvec"][0]))).to("cuda:0")
    back = ctx.restrict(1, ctx.prolong(1, ec))
    assert rel_err(back.cpu().numpy(), ec.cpu().numpy()) < 1e-5
    b = latgen.fine_vectors(cfg["dims"], 1, rng)
    x, info, st = ctx.solve([m], torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    assert true_rel(cfg, W, N, m, x.cpu().numpy()[0, 0], b[0]) <= 1e-10


def test_error_paths(torch, mg, cubic):
    cfg, W, N, nvs, b = cubic
    log("[errors] cubic")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=1, outer_maxiter=1)
    bt = torch.from_numpy(b[:1]).to("cuda:0")
    # one outer iteration cannot reach 1e-10: MG_E_NOCONV, last iterate kept
    x, info, st = ctx.solve([cfg["mass0"]], bt, tol=1e-10, check=False)
    assert st == mg.MG_E_NOCONV and info[0]["status"] == "MG_E_NOCONV"
    assert info[0]["true_rel_residual"] < 1.0
    # NaN in b
    bn = bt.clone()
    bn[0, 0, 0, 0, 0, 0] = float("nan")
    x, info, st = ctx.solve([cfg["mass0"]], bn, tol=1e-10, check=False)
    assert st == mg.MG_E_NONFINITE
    # too many right-hand sides, bad level, bad dtype
    with pytest.raises(mg.MGError) as e:
        ctx.solve([cfg["mass0"]], torch.from_numpy(b).to("cuda:0"))
    assert e.value.status == mg.MG_E_ARG
    z = torch.zeros(4096, dtype=torch.complex128, device="cuda:0")
    z2 = torch.zeros_like(z)
    st = mg.LIB.mg_apply_coarse(ctx.ctx, 4, mg.MG_C128, z.data_ptr(), z2.data_ptr(), 1, None)
    assert st == mg.MG_E_ARG
    st = mg.LIB.mg_apply_coarse(ctx.ctx, 2, mg.MG_CBF16, z.data_ptr(), z2.data_ptr(), 1, None)
    assert st == mg.MG_E_ARG
    st = mg.LIB.mg_apply_dslash(ctx.ctx, 0, 0.1, mg.MG_C128, z.data_ptr(), z.data_ptr(), 1, None)
    assert st == mg.MG_E_ARG
    # rank-deficient null vectors: two identical vectors
    bad = [v.copy() for v in nvs]
    bad[0][1] = bad[0][0]
    with pytest.raises(mg.MGError) as e:
        make_ctx(torch, mg, cfg, W, N, bad, max_nrhs=1)
    assert e.value.status == mg.MG_E_RANK


@pytest.fixture(scope="module")
def cubic1(torch):
    """8^4 HISQ-style with one aggregation (coarsest level 2^4 x 16 = 256 dof)."""
    cfg = dict(CONFIGS["cubic"], blocks=[(4, 4, 4, 4)], nvec=(8,))
    W, N, rng = links(cfg)
    nvs = cgne_vectors(cfg, W, N, rng)
    b = latgen.fine_vectors(cfg["dims"], 2, rng)
    return cfg, W, N, nvs, b


def test_fp64_deflated_kcycle_matches_oracle(torch, mg, cubic1):
    """Coarsest solve deflated with 32 near-null vectors of its operator, made
    by the oracle (CGNE on its coarsest operator from seeded starts) and
    imported into the library: the all-FP64 MG-GCR solves of both sides with
    the same deflation space agree (outer iterations +-1,
    ||x - x_oracle|| <= 2e-10 ||b|| / m)."""
    cfg, W, N, nvs, b = cubic1
    m = cfg["mass0"]
    log("[deflate] cubic1 fp64 vs oracle")
    H = oracle_hierarchy(cfg, W, N, m, nvs)
    lc = H.nlevels - 1
    rng = np.random.default_rng(2718)
    starts = latgen.complex_normal(rng, (32,) + H.fine_shape(lc))
    wd = np.stack([sol.cgne_null_vector(lambda v: H.op(lc, v), lambda v: H.op_dag(lc, v), s0, 1e-6, 100)[0]
                   for s0 in starts])
    ctx = make_ctx(torch, mg, cfg, W, N, list(nvs) + [wd], fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128,
                   max_nrhs=1, coarsest_deflate=32, deflate_maxiter=100, deflate_import=1)
    assert np.array_equal(ctx.export(1, 2).cpu().numpy().reshape(wd.shape), wd)
    x, info, st = ctx.solve([m], torch.from_numpy(b[:1]).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()[0, 0]
    H.set_coarsest_deflation(list(wd))
    xo, io = H.solve(b[0], tol=1e-10)
    assert io.converged
    assert abs(info[0]["outer_iters"] - io.iters) <= 1, (info[0], io.iters)
    assert true_rel(cfg, W, N, m, x, b[0]) <= 1e-10
    assert np.linalg.norm(x - xo) <= 2e-10 * np.linalg.norm(b[0]) / m


def test_deflated_bf16_solve(torch, mg, cubic1):
    """16-bit coarse links (the matrix-core stencil builds Z = A W) with a
    deflated coarsest level (16 vectors): both right-hand sides reach 1e-10,
    as they do without deflation."""
    cfg, W, N, nvs, b = cubic1
    m = 0.02
    bt = torch.from_numpy(b).to("cuda:0")
    its = {}
    for k in (0, 16):
        log(f"[deflate] cubic1 bf16 k={k}")
        ctx = make_ctx(torch, mg, cfg, W, N, nvs, coarse_prec=mg.MG_CBF16, max_nrhs=2, coarsest_deflate=k,
                       deflate_maxiter=200)
        x, info, st = ctx.solve([m], bt, tol=1e-10)
        x = x.cpu().numpy()[0]
        for r in range(2):
            assert info[r]["status"] == "MG_OK"
            assert true_rel(cfg, W, N, m, x[r], b[r]) <= 1e-10
        its[k] = info[0]["level_iters"][1] / max(1, info[0]["level_iters"][0])
        ctx.destroy()
    # the iteration counts are logged, not compared: on this small lattice the
    # near-null vectors barely change the coarsest level's convergence
    log(f"[deflate] coarsest iterations per KD-level iteration {its}")


def test_concurrent_contexts_match_sequential(torch, mg, cubic, cubic1):
    """Two contexts (different hierarchies) solved at the same time from two
    host threads on two streams give exactly the results of solving them one
    after the other: the library keeps no state outside a context.  Every
    concurrent solution's true residual, recomputed by the oracle's FP64 D,
    meets the 1e-10 target."""
    import threading
    log("[solve] two contexts on two streams")
    probs = []
    for cfg, W, N, nvs, b in (cubic, cubic1):
        ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=2)
        probs.append((ctx, torch.from_numpy(b).to("cuda:0")))
    seq = [ctx.solve([0.05], bt, tol=1e-10)[0].cpu().numpy() for ctx, bt in probs]
    out = [None, None]

    def run(k):
        ctx, bt = probs[k]
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            x, info, st = ctx.solve([0.05], bt, tol=1e-10)
            s.synchronize()
            out[k] = x.cpu().numpy()
    ts = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for k in range(2):
        assert out[k] is not None
        assert np.array_equal(out[k], seq[k]), k
        cfg, W, N, nvs, b = (cubic, cubic1)[k]
        for r in range(b.shape[0]):
            res = b[r] - ops.dslash(out[k][0, r], W, N, 0.05, cfg["c1"], cfg["c3"])
            rel = np.linalg.norm(res) / np.linalg.norm(b[r])
            assert rel <= 1.001e-10, (k, r, rel)


def test_multishift_cg_matches_oracle(torch, mg, cubic):
    """Multi-shift CG over unsorted masses with a repeat (Sec. 3.3 workflow):
    every (mass, rhs) system at true residual 1e-10 and within 2e-10 ||b|| / m
    of the oracle's multi-shift solution; the lightest shift takes the
    oracle's iteration count (both parities, within 5%), a repeated mass the
    same count, and heavier shifts freeze earlier."""
    cfg, W, N, nvs, b = cubic
    masses = [0.3, 0.02, 0.07, 0.02]
    log("[msc] cubic 4 masses x 2 rhs")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=2)
    x, info, st = ctx.multishift_cg_solve(masses, torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    x = x.cpu().numpy()
    for r in range(2):
        xo, io, relo = sol.multishift_cg(W, N, masses, cfg["c1"], cfg["c3"], b[r], tol=1e-10)
        for j, m in enumerate(masses):
            I = info[j * 2 + r]
            assert I["status"] == "MG_OK" and I["reliable_updates"] == 0, I
            assert true_rel(cfg, W, N, m, x[j, r], b[r]) <= 1e-10, (m, r)
            assert np.linalg.norm(x[j, r] - xo[j]) <= 2e-10 * np.linalg.norm(b[r]) / m, (m, r)
        # ~900 CG steps per parity: rounding in a different summation order
        # moves the step at which 1e-10 is reached by a few percent
        assert abs(info[1 * 2 + r]["outer_iters"] - sum(io)) <= 0.05 * sum(io), (info[2 + r], io)
        assert info[3 * 2 + r]["outer_iters"] == info[1 * 2 + r]["outer_iters"]
        assert info[0 * 2 + r]["outer_iters"] < info[2 * 2 + r]["outer_iters"] < info[1 * 2 + r]["outer_iters"]


def test_multishift_cg_limits(torch, mg, cubic):
    """Work-space and argument limits of the multi-shift CG: 16 shifts at most,
    and the shifts' directions must fit in the outer GCR work vectors."""
    cfg, W, N, nvs, b = cubic
    log("[msc] limits")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=1, outer_nkrylov=2)
    bt = torch.from_numpy(b[:1]).to("cuda:0")
    x, info, st = ctx.multishift_cg_solve([0.1] * 6, bt, tol=1e-8, check=False)
    assert st == mg.MG_OK
    x, info, st = ctx.multishift_cg_solve([0.1] * 7, bt, tol=1e-8, check=False)
    assert st == mg.MG_E_CONFIG
    x, info, st = ctx.multishift_cg_solve([0.1] * 17, bt, tol=1e-8, check=False)
    assert st == mg.MG_E_ARG
    x, info, st = ctx.multishift_cg_solve([0.1, -0.2], bt, tol=1e-8, check=False)
    assert st == mg.MG_E_ARG


def test_force_matches_oracle(torch, mg, cubic):
    """Fermion-force gradients from the MG solves and the outer-product kernel
    against the oracle's (FD-pinned) force on the same links and source;
    through torch.autograd as well."""
    cfg, W, N, nvs, b = cubic
    m = 0.1
    log("[force] cubic")
    ctx = make_ctx(torch, mg, cfg, W, N, nvs, max_nrhs=2, fine_prec=mg.MG_C128, coarse_prec=mg.MG_C128)
    phi = b
    X, Y, gw, gn, info = ctx.solve_backward(m, torch.from_numpy(phi).to("cuda:0"), tol=1e-13)
    gw, gn = gw.cpu().numpy(), gn.cpu().numpy()
    Sw = np.zeros_like(W)
    Sn = np.zeros_like(N)
    S = 0.0
    for r in range(phi.shape[0]):
        s_, gW, gN, Xo, Yo = sol.force(W, N, m, cfg["c1"], cfg["c3"], phi[r], tol=1e-13)
        S += s_
        Sw += gW
        Sn += gN
    assert rel_err(gw, Sw) < 1e-9
    assert rel_err(gn, Sn) < 1e-9
    # the library returns the action per right-hand side (S_r = Re <phi_r, X_r>)
    assert len(ctx.last_action) == phi.shape[0]
    assert abs(sum(ctx.last_action) - S) < 1e-9 * abs(S)
    Wt = torch.from_numpy(W).to("cuda:0").requires_grad_(True)
    Nt = torch.from_numpy(N).to("cuda:0").requires_grad_(True)
    St = mg.fermion_action(Wt, Nt, torch.from_numpy(phi).to("cuda:0"), ctx, m, 1e-13)
    St.backward()
    assert abs(St.item() - S) < 1e-9 * abs(S)
    assert rel_err(Wt.grad.cpu().numpy(), Sw) < 1e-9
    assert rel_err(Nt.grad.cpu().numpy(), Sn) < 1e-9


def test_force24_against_oracle_fixture(torch, mg):
    """The fermion force at 24^4 (the force benchmark's lattice: HISQ-style
    links with eps 0.5, m = 0.01, one Gaussian phi, same seeds) against the
    FP64 oracle's gradient at 256 fat and 256 Naik link positions and its
    action, stored by tests/golden/make_force24_fixture.py (oracle solves to
    1e-11).  The GPU solves run to 1e-11 through the default hierarchy
    (short set-up); with ||D^{-1}|| <= 1/m the solution errors are below
    1e-11 ||phi|| / m^2 relative, far inside the 1e-6 bar on the gradient
    entries (relative to the largest entry) and 1e-8 on S."""
    import os
    f = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "force24_oracle_sample.npz")
    if not os.path.exists(f):
        pytest.skip("oracle fixture not generated (tests/golden/make_force24_fixture.py)")
    d = np.load(f)
    dims = (24, 24, 24, 24)
    m = 0.01
    W, N, rng = latgen.hisq_style_links(dims, 0.5, 20221228)
    phi = latgen.fine_vectors(dims, 1, rng)
    log("[force24] setup")
    p = mg.default_params(dims, mass0=m, kd_naik=0, coarse_prec=mg.MG_CBF16, setup_maxiter=(200, 100), max_nrhs=1)
    dev = "cuda:0"
    ctx = mg.setup(p, torch.from_numpy(W).to(dev), torch.from_numpy(N).to(dev))
    log("[force24] solves")
    X, Y, gw, gn, info = ctx.solve_backward(m, torch.from_numpy(phi).to(dev), tol=1e-11)
    gw, gn = gw.cpu().numpy(), gn.cpu().numpy()
    S = sum(ctx.last_action)
    ew = max(np.max(np.abs(gw[tuple(q)] - g)) for q, g in zip(d["pos_fat"], d["grad_fat"])) / float(d["max_abs_fat"])
    en = max(np.max(np.abs(gn[tuple(q)] - g)) for q, g in zip(d["pos_naik"], d["grad_naik"])) / float(d["max_abs_naik"])
    log(f"    S {S!r} (oracle {float(d['S'])!r}); sampled gradient errors fat {ew:.2e}, naik {en:.2e}")
    assert abs(S - float(d["S"])) <= 1e-8 * abs(float(d["S"]))
    assert ew <= 1e-6 and en <= 1e-6
    ctx.destroy()
