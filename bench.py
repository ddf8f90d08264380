"""Benchmark: MG-GCR time-to-1e-10 against plain FP64 CG on a 32^4 HISQ-style
lattice on one MI355X, plus the roofline of the dominant kernel and the CPU
oracle baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2batch|...]

A step is one MG-GCR solve of the workload's whole batch (default: 16
Gaussian right-hand sides x 8 masses, 128 systems) to ||b - D x|| / ||b|| <=
1e-10, with every input resident in HBM; the hierarchy set-up is excluded (as
in the paper, Sec. 3.2) and reported separately.  A step takes about a
minute, so the run keeps to a wall-time budget (--budget-s, counted from the
start of the process): it times as many of the requested steps as fit beside
the comparators and reports the requested and the timed counts.  One JSON line
is printed, also when a later leg fails.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # 32^4 HISQ-style, eps 0.5 (as the 16^4 workload), mass 0.005, KD + 4^4/Nvec 64 + 2^4/Nvec 96
    "c2": dict(dims=(32, 32, 32, 32), mass=0.005, nrhs=1, eps=0.5, seed=20221226, kd_naik=0,
               nvec=(64, 96), blocks=[(4, 4, 4, 4), (2, 2, 2, 2)], setup_iters=(2000, 300)),
    # the multi-mass batch: 32^4, 16 rhs x 8 masses (log-spaced 0.005..0.2), 16-bit coarse links (fp16:
    # its 10-bit significand is the closer IEEE match to the paper's 16-bit fixed point, and with it the
    # K-cycle takes fewer level-2 iterations than with bf16); 4 masses (64 systems) per lockstep solve
    "c2batch": dict(dims=(32, 32, 32, 32), mass=0.005, nrhs=16, eps=0.5, seed=20221226, kd_naik=0,
                    nvec=(64, 96), blocks=[(4, 4, 4, 4), (2, 2, 2, 2)], setup_iters=(2000, 300),
                    masses=(0.005, 0.0084691, 0.014345, 0.024298, 0.041156, 0.069711, 0.11808, 0.2),
                    coarse_prec="fp16", mass_batch=4),
    # MG against CG toward lighter masses (the Sec. 3.2 mass dependence): the 32^4 fields of c2batch, 16 rhs
    # per mass, a hierarchy per mass, fp16 coarse links
    "massscan": dict(dims=(32, 32, 32, 32), mass=0.0005, nrhs=16, eps=0.5, seed=20221226, kd_naik=0,
                     nvec=(64, 96), blocks=[(4, 4, 4, 4), (2, 2, 2, 2)], setup_iters=(2000, 300),
                     masses=(0.005, 0.002, 0.001, 0.0005), coarse_prec="fp16", kind="massscan"),
    # fermion force (the HMC gradient of phi^dag (D^dag D)^-1 phi) at 24^4 HISQ-style, mass 0.01, one phi
    "force24": dict(dims=(24, 24, 24, 24), mass=0.01, nrhs=1, eps=0.5, seed=20221228, kd_naik=0,
                    nvec=(64, 96), blocks=[(4, 4, 4, 4), (2, 2, 2, 2)], setup_iters=(2000, 300), kind="force",
                    coarse_prec="bf16"),
    # uneven batch: 12 systems on each of 8^4, 12^4, 16^4 and 24^4, every lattice with its own fields and
    # hierarchy (KD + one aggregation, Nvec 48: coarse 2^4, 3^4, 4^4, 6^4 with 96 dof per site; the Table 1
    # set-up of 2000 CGNE iterations per null vector), solved one lattice after another and then all four
    # at once on separate streams
    "uneven": dict(dims_list=((8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (24, 24, 24, 24)), mass=0.01,
                   nrhs=12, eps=0.5, seed=20221229, kd_naik=0, nvec=(48,), blocks=[(4, 4, 4, 4)],
                   setup_iters=(2000,), kind="uneven", coarse_prec="bf16"),
    # 16^4 HISQ-style, mass 0.01
    "c1": dict(dims=(16, 16, 16, 16), mass=0.01, nrhs=1, eps=0.5, seed=20221225, kd_naik=0,
               nvec=(64, 96), blocks=[(4, 4, 4, 4), (2, 2, 2, 2)], setup_iters=(2000, 2000)),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- HBM traffic
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "coarse_mfma_level2_traffic.json")
DOM_SOURCE = os.path.join(ROOT, "paper_2212_12559_amd", "csrc", "coarse_mfma.hip")


def hbm_traffic(nrhs, mode=None):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, each scaled by what
    the counter reads for a copy of known size), or None when those runs were
    taken on another version of the kernel's source, another rhs count or
    another link format / coarse operator (mode)."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter run committed"
    rec = json.load(open(TRAFFIC_FILE))
    sha = hashlib.sha256(open(DOM_SOURCE, "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None, "counters taken on an older version of the kernel"
    if rec.get("nrhs") != nrhs:
        return None, f"counters taken at {rec.get('nrhs')} rhs per launch"
    if mode is not None and rec.get("mode") != mode:
        return None, f"counters taken with {rec.get('mode')}"
    return rec["bytes_per_launch"], os.path.relpath(TRAFFIC_FILE, ROOT)


def coarse_mode(cprec, coarse_op):
    return f"{cprec} links, coarse_op {coarse_op}"


def summarize_counters(fetch_dir, write_dir, wl, mode):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the level-2 coarse
    stencil and of the 512 MiB calibration copy -> bytes per launch."""
    import csv
    import glob
    import hashlib

    def per_dispatch(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        out = {}
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            out[int(r["Dispatch_Id"])] = (r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"]))
        return out

    nr = wl["nrhs"] * wl.get("mass_batch", 1)
    Vc = int(np.prod(wl["dims"])) // 256
    # the level-2 launch shape at nr rhs (work-items): one workgroup per coarse
    # site and rhs group, 64 threads per m-tile pair (one per m-tile at 16 rhs)
    mt_n = 2 * wl["nvec"][0] // 16
    rt = 1 if nr <= 16 else (2 if nr <= 32 else 4)
    mt = 2 if nr > 16 and mt_n % 2 == 0 else 1
    g_dom = Vc * 64 * (mt_n // mt) * ((nr + 16 * rt - 1) // (16 * rt))
    res = {}
    for name, d, counter, copy_kib in (("fetch", fetch_dir, "FETCH_SIZE", 512 * 1024),
                                       ("write", write_dir, "WRITE_SIZE", 512 * 1024)):
        rows = per_dispatch(d, counter)
        # the calibration copy is the last large copy of the run
        cal = [rows[max(i for i, (k, g, v) in rows.items() if "copyBuffer" in k and g >= (1 << 17))][2]]
        dom = [v for (k, g, v) in rows.values() if "coarse_mfma_kernel" in k and g == g_dom]
        factor = copy_kib / (sum(cal) / len(cal))
        res[name] = {"counter": counter, "kib_per_launch_raw": sum(dom) / len(dom), "launches": len(dom),
                     "copy_kib_raw": sum(cal) / len(cal), "copy_kib_true": copy_kib, "scale": factor,
                     "bytes_per_launch": sum(dom) / len(dom) * factor * 1024}
    sha = hashlib.sha256(open(DOM_SOURCE, "rb").read()).hexdigest()
    rec = {"kernel": "coarse_mfma_kernel (level-2 coarse stencil)", "nrhs": nr, "mode": mode, "source_sha256": sha,
           "fetch": res["fetch"], "write": res["write"],
           "bytes_per_launch": res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(rec, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(rec, indent=1))


# ---------------------------------------------------------------- op counts
def op_counts(info, s, nlev):
    """Operator applications one MG solve performed, from its iteration
    counts (the K-cycle's structure is fixed: see the solver's K-cycle)."""
    outer = info["outer_iters"]
    rel = info["reliable_updates"]
    l1, l2, l3 = info["level_iters"][0], info["level_iters"][1], info["level_iters"][2]
    c = {
        "dslash_fp64": outer + rel + 1,
        "dslash_fp32_level0": outer * (s + 1),
        "kd_fp32": outer + l1 * (s + 2),
        "dslash_fp32_level1": l1 * (s + 2),
        "restrict1": l1, "prolong1": l1,
        "coarse2": l2 * (s + 2) if nlev > 3 else l2,
        "restrict2": l2 if nlev > 3 else 0, "prolong2": l2 if nlev > 3 else 0,
        "coarse3": l3,
    }
    return c


# ---------------------------------------------------------------- bytes
def coarse_link_blocks(ctx, level, link_csz):
    """Link blocks per coarse site that the stencil reads: 8 when the level is
    block-preconditioned with an identity self block that the 16-bit stencil
    adds instead of reading (every coarse extent >= 2, n a multiple of 32),
    else all 9."""
    p = ctx.params
    shape = ctx.coarse_shapes[level - 2]
    n = 2 * shape[-1]
    implicit = p.coarse_op == 1 and link_csz == 4 and min(shape[:4]) >= 2 and n % 32 == 0
    return 8 if implicit else 9


def algorithmic_bytes(dims, nvec, nrhs=1, csz=8, naik=True, link_csz=8, blocks2=9):
    """Per-apply algorithmic HBM bytes (each operand read or written once);
    link_csz is the size of one stored complex coarse-link entry, blocks2 the
    link blocks per level-2 site the stencil reads."""
    V = int(np.prod(dims))
    links = 8 * 9 * csz          # fat + Naik, 4 directions each, 3x3 complex (op 0 always has Naik)
    vec = 3 * csz
    b = {
        "dslash": V * (links + 2 * vec * nrhs),
        "kd": V * (144 * csz + 2 * vec * nrhs),
        # A = (B+m)^-1 D of the KD level: the one-hop (truncated) or full stencil, then (B+m)^-1
        "kd_operator": V * ((4 if not naik else 8) * 9 * csz + 2 * vec * nrhs) + V * (144 * csz + 2 * vec * nrhs),
        "restrict": V * (3 * nvec[0] * csz + vec * nrhs) + (V // 256) * 2 * nvec[0] * csz * nrhs,
        "prolong": V * (3 * nvec[0] * csz + vec * nrhs) + (V // 256) * 2 * nvec[0] * csz * nrhs,
    }
    Vc = V // 256
    n = 2 * nvec[0]
    b["coarse2"] = Vc * (blocks2 * n * n * link_csz + 2 * n * csz * nrhs)
    return b


def kernel_rates(torch, ctx, wl, reps, mg, link_csz=8):
    """Average duration of each hot-path kernel at the workload's shape,
    timed with HIP events on torch's current stream (the library's stream)."""
    dims, m = wl["dims"], wl["mass"]
    dev = "cuda:0"
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    X, Y, Z, T = dims
    nr = wl["nrhs"] * wl.get("mass_batch", 1)
    x = torch.randn((nr, T, Z, Y, X, 3), dtype=torch.complex64, device=dev, generator=gen)
    xc = torch.randn((nr,) + ctx.coarse_shapes[0], dtype=torch.complex64, device=dev, generator=gen)
    xc3 = torch.randn((nr,) + ctx.coarse_shapes[1], dtype=torch.complex64, device=dev, generator=gen)
    y = torch.empty_like(x)
    yc = torch.empty_like(xc)
    yc3 = torch.empty_like(xc3)
    k2, k3 = coarse_link_blocks(ctx, 2, link_csz), coarse_link_blocks(ctx, 3, link_csz)
    b = algorithmic_bytes(dims, wl["nvec"], nrhs=nr, naik=wl["kd_naik"] != 0, link_csz=link_csz, blocks2=k2)
    n3 = 2 * wl["nvec"][1]
    Vc3 = int(np.prod(ctx.coarse_shapes[1][:4]))
    b["coarse3"] = Vc3 * (k3 * n3 * n3 * link_csz + 2 * n3 * 8 * nr)
    n2 = 2 * wl["nvec"][0]
    Vc2 = int(np.prod(ctx.coarse_shapes[0][:4]))
    flops = {"coarse2": 8.0 * Vc2 * n2 * k2 * n2 * nr, "coarse3": 8.0 * Vc3 * n3 * k3 * n3 * nr}
    ops = {
        "dslash": lambda: ctx.apply_dslash(0, m, x, y),
        "kd": lambda: ctx.apply_dslash(2, m, x, y),
        "kd_operator": lambda: ctx.apply_dslash(1, m, x, y),
        "restrict": lambda: ctx.restrict(1, x, yc),
        "prolong": lambda: ctx.prolong(1, xc, y),
        "coarse2": lambda: ctx.apply_coarse(2, xc, yc),
        "coarse3": lambda: ctx.apply_coarse(3, xc3, yc3),
    }
    out = {}
    for name, f in ops.items():
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out[name] = {"us": us, "bytes": b[name], "GBps": b[name] / (us * 1e-6) / 1e9}
        if name in flops:
            out[name]["TFLOPs"] = flops[name] / (us * 1e-6) / 1e12
        log(f"[bench] kernel {name}: {us:.1f} us, {out[name]['GBps']:.0f} GB/s"
            + (f", {out[name]['TFLOPs']:.1f} TFLOP/s" if name in flops else ""))
    return out


def _oracle_sample_worker(job):
    """One oracle sample, run in a process of its own (one thread): one
    application of each hot-path operator on a 16^4 lattice of the workload's
    kind.  Returns the seconds of each application."""
    dims, eps, seed, nvec, kd_naik, block, m = job
    from threadpoolctl import threadpool_limits

    from oracle import operators as ops
    from oracle import solvers as sol
    from paper_2212_12559_amd import latgen

    c1, c3 = 9.0 / 8.0, -1.0 / 24.0
    t = {}
    with threadpool_limits(1):
        W, N, rng = latgen.hisq_style_links(dims, eps, seed)
        x = latgen.fine_vectors(dims, 1, rng)[0]
        t0 = time.perf_counter()
        ops.dslash(x, W, N, m, c1, c3)
        t["dslash"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        ops.dslash(x, W, N, m, c1, c3 if kd_naik else 0.0)
        t["dslash_kd"] = time.perf_counter() - t0
        Kinv = ops.kd_inverse(W, m, c1)
        t0 = time.perf_counter()
        ops.kd_apply(Kinv, x)
        t["kd"] = time.perf_counter() - t0
        del Kinv
        nv1 = latgen.fine_vectors(dims, nvec, rng)
        p = sol.MGParams(dims=dims, c1=c1, c3=c3, kd_naik=bool(kd_naik), blocks=(tuple(block),))
        H = sol.Hierarchy(p, W, N, m, [nv1])
        t0 = time.perf_counter()
        rc = H.restrict(1, x)
        t["restrict"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        H.prolong(1, rc)
        t["prolong"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        H.op(2, rc)
        t["coarse"] = time.perf_counter() - t0
    return t


def host_cpu():
    """CPU model and the cores this process may use (capped at the 16-core
    share of one GPU)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, max(1, min(16, n))


def cpu_baseline(wl, batch_infos, s, oracle_check=None):
    """The FP64 oracle (numpy) timed on the host's cores: every core runs one
    sample (one application of each hot-path operator on a 16^4 lattice, in a
    process of its own), so their combined rate is the oracle's throughput on
    this host; scaled to the workload's volume (every operator is local, so
    its cost is proportional to the volume) and multiplied by the operator
    counts of the measured MG solves, it gives the oracle's time for the same
    work (Krylov BLAS omitted: a lower bound).

    oracle_check: optional (dims, links (W, N), [(mass, rhs, b, x)]) of GPU
    solutions; their true residuals ||b - D(m) x|| / ||b|| are recomputed with
    the oracle's FP64 operator, with the error bound ||x - x*|| <= ||r|| / m
    that holds because D = m + K with K anti-Hermitian (so ||D^-1|| <= 1 / m)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    model, cores = host_cpu()
    dims = wl["dims"]
    sd = (16, 16, 16, 16)
    scale = float(np.prod(dims)) / float(np.prod(sd))
    job = (sd, wl["eps"], wl["seed"], wl["nvec"][0], wl["kd_naik"], wl["blocks"][0], wl["mass"])
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        samples = list(ex.map(_oracle_sample_worker, [job] * cores))
    sample_s = time.perf_counter() - t0
    # combined rate of the cores -> seconds per application on the whole host, at the workload's volume
    per_op = {k: scale / sum(1.0 / smp[k] for smp in samples) for k in samples[0]}
    est = 0.0
    for info in batch_infos:
        cnt = op_counts(info, s, 4)
        est += wl["nrhs"] * (cnt["dslash_fp64"] * per_op["dslash"] + cnt["dslash_fp32_level0"] * per_op["dslash"]
                             + cnt["dslash_fp32_level1"] * per_op["dslash_kd"] + cnt["kd_fp32"] * per_op["kd"]
                             + cnt["restrict1"] * per_op["restrict"] + cnt["prolong1"] * per_op["prolong"]
                             + (cnt["coarse2"] + cnt["coarse3"]) * per_op["coarse"])
    log(f"[bench] cpu oracle on {cores} cores ({model}): per application at {'x'.join(map(str, dims))} "
        + ", ".join(f"{k} {v:.3f}s" for k, v in per_op.items()) + f" -> {est:.0f} s")
    out = {"value": est, "unit": "s", "cores": cores, "cpu_model": model, "kind": "oracle",
           "sample": (f"{cores} processes (one thread each) each applied the numpy FP64 oracle's D, D of the KD "
                      f"level, (B+m)^-1, R, P and the level-2 operator R A P once on a 16^4 lattice (took "
                      f"{sample_s:.1f} s); their combined rate, scaled by the volume ratio {scale:.0f} to "
                      f"{'x'.join(map(str, dims))}, times the operator counts of the measured MG solves (level-3 "
                      f"applies priced as level 2, Krylov BLAS omitted): a lower bound for the oracle's time"),
           "per_op_s": per_op}
    if oracle_check is not None:
        from oracle import operators as ops
        cdims, (W, N), systems = oracle_check
        rows = []
        for mass, rhs, b, x in systems:
            r = b - ops.dslash(x, W, N, mass, 9.0 / 8.0, -1.0 / 24.0)
            rn, bn, xn = np.linalg.norm(r), np.linalg.norm(b), np.linalg.norm(x)
            rows.append({"mass": mass, "rhs": rhs, "true_rel_residual": rn / bn, "err_bound_rel_x": rn / (mass * xn)})
            log(f"[bench] oracle check mass {mass} rhs {rhs}: residual {rn / bn:.3e}, "
                f"|x - x*| / |x| <= {rn / (mass * xn):.2e}")
        out["oracle_check"] = {"what": "true residual of GPU solutions recomputed by the oracle's FP64 D at full "
                                       "size (rhs 0 and 1 of every mass), with the bound |x - x*| <= |r| / m",
                               "systems": rows,
                               "worst_true_rel_residual": max(r["true_rel_residual"] for r in rows),
                               "worst_err_bound_rel_x": max(r["err_bound_rel_x"] for r in rows)}
    return out


def force_bench(args, wl, torch, latgen, mg):
    """Fermion force at the workload's lattice: mg_solve_backward (two MG
    solves and the outer-product kernel) timed over the steps, then the
    gradient checked at full size by a central finite difference of the
    action along a random direction of the fat links (the property
    dS = Re sum conj(G) dW holds at any size)."""
    dims, m = wl["dims"], wl["mass"]
    dev = "cuda:0"
    log(f"[bench] force workload {dims} mass {m}: generating links")
    W, N, rng = latgen.hisq_style_links(dims, wl["eps"], wl["seed"])
    phi = torch.from_numpy(latgen.fine_vectors(dims, wl["nrhs"], rng)).to(dev)
    dW = torch.from_numpy(latgen.complex_normal(rng, W.shape)).to(dev)
    Wt, Nt = torch.from_numpy(W).to(dev), torch.from_numpy(N).to(dev)
    del W, N
    cp = {"fp32": mg.MG_C64, "bf16": mg.MG_CBF16, "fp16": mg.MG_CF16}[args.coarse_prec or wl.get("coarse_prec", "fp32")]
    setup_iters = tuple(int(v) for v in args.setup_iters.split(",")) if args.setup_iters else wl["setup_iters"]
    p = mg.default_params(dims, mass0=m, nvec=wl["nvec"], block=wl["blocks"], setup_maxiter=setup_iters,
                          max_nrhs=wl["nrhs"], kd_naik=wl["kd_naik"], coarse_prec=cp)
    log("[bench] setup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = mg.setup(p, Wt, Nt)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup {setup_s:.2f} s")
    for i in range(args.warmup):
        ctx.solve_backward(m, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        X, Y, gw, gn, info = ctx.solve_backward(m, phi)
        res = ", ".join(f"{d['true_rel_residual']:.2e}" for d in info)
        log(f"[bench] step {i}: outer {[d['outer_iters'] for d in info]}, residuals {res}")
    torch.cuda.synchronize()
    t_force = (time.perf_counter() - t0) / args.steps
    S0 = float(torch.sum(torch.conj(phi) * X).real)
    # directional derivative along dW (fat links only) by central differences
    h = 1e-3 * float(torch.linalg.vector_norm(Wt)) / float(torch.linalg.vector_norm(dW))
    Sp = []
    for sgn in (1.0, -1.0):
        ctx.update_links((Wt + sgn * h * dW).contiguous(), Nt)
        Xs, _, _, _, _ = ctx.solve_backward(m, phi)
        Sp.append(float(torch.sum(torch.conj(phi) * Xs).real))
    ctx.update_links(Wt, Nt)
    fd = (Sp[0] - Sp[1]) / (2 * h)
    an = float(torch.sum(torch.conj(gw) * dW).real)
    rel = abs(fd - an) / abs(an)
    log(f"[bench] force {t_force:.3f} s; S = {S0:.6e}; dS/dh finite difference {fd:.8e} vs gradient {an:.8e} "
        f"(rel {rel:.1e})")
    out = {"metric": "fermion force (MG adjoint solves + outer product) time at 24^4 HISQ", "value": t_force,
           "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_force * 1e3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128 outer / c64 K-cycle",
           "data": "synthetic",
           "config": {"workload": f"{'x'.join(map(str, dims))} HISQ-style eps {wl['eps']}, mass {m}, {wl['nrhs']} phi, "
                                  f"truncated-KD={not wl['kd_naik']}, coarse links "
                                  f"{args.coarse_prec or wl.get('coarse_prec', 'fp32')}"},
           "setup_s": setup_s, "solve_infos": info, "action": S0,
           "gradient_check": {"direction": "Gaussian on every fat-link entry", "step": h, "finite_difference": fd,
                              "gradient": an, "rel_diff": rel}}
    # against the oracle's force stored for this lattice, mass, eps and seeds (tests/golden: written by a
    # script that runs only the oracle): 256 fat and 256 Naik link positions and the action
    fx = os.path.join(ROOT, "tests", "golden", "force24_oracle_sample.npz")
    if tuple(dims) == (24, 24, 24, 24) and m == 0.01 and wl["eps"] == 0.5 and wl["seed"] == 20221228 \
            and os.path.exists(fx):
        ref = np.load(fx)
        gwn, gnn = gw.cpu().numpy(), gn.cpu().numpy()
        ew = max(float(np.max(np.abs(gwn[tuple(q)] - g))) for q, g in zip(ref["pos_fat"], ref["grad_fat"]))
        en = max(float(np.max(np.abs(gnn[tuple(q)] - g))) for q, g in zip(ref["pos_naik"], ref["grad_naik"]))
        out["oracle_fixture_check"] = {
            "what": "gradient entries at the 256 + 256 stored positions and the action, against the FP64 oracle's",
            "fat_max_err_rel_to_largest": ew / float(ref["max_abs_fat"]),
            "naik_max_err_rel_to_largest": en / float(ref["max_abs_naik"]),
            "action_rel_err": abs(S0 - float(ref["S"])) / abs(float(ref["S"]))}
        log(f"[bench] against the oracle's stored force: {out['oracle_fixture_check']}")
    print(json.dumps(out), flush=True)


def massscan_bench(args, wl, torch, latgen, mg):
    """MG-GCR and FP64 Schur CG on the same 16 right-hand sides at masses
    down to 0.0005, each mass with its own hierarchy (set-up timed apart, as
    in Sec. 3.2): MG's outer iteration count stays nearly flat while CG's
    grows, the behaviour Sec. 3.2 reports; the line gives the per-mass times
    and where MG overtakes CG."""
    dims = wl["dims"]
    dev = "cuda:0"
    W, N, rng = latgen.hisq_style_links(dims, wl["eps"], wl["seed"])
    Wt, Nt = torch.from_numpy(W).to(dev), torch.from_numpy(N).to(dev)
    del W, N
    bt = torch.from_numpy(latgen.fine_vectors(dims, wl["nrhs"], rng)).to(dev)
    cp = {"fp32": mg.MG_C64, "bf16": mg.MG_CBF16, "fp16": mg.MG_CF16}[args.coarse_prec or wl["coarse_prec"]]
    setup_iters = tuple(int(v) for v in args.setup_iters.split(",")) if args.setup_iters else wl["setup_iters"]
    masses = list(wl["masses"])[:args.nmass]
    rows = []
    for m in masses:
        p = mg.default_params(dims, mass0=m, nvec=wl["nvec"], block=wl["blocks"], setup_maxiter=setup_iters,
                              max_nrhs=wl["nrhs"], max_nmass=1, kd_naik=wl["kd_naik"], coarse_prec=cp,
                              outer_nkrylov=8, outer_maxiter=300)
        log(f"[bench] massscan m {m}: set-up")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = mg.setup(p, Wt, Nt)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        ctx.autotune(wl["nrhs"])
        log(f"[bench] massscan m {m}: set-up {setup_s:.1f} s; MG solve")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info, st = ctx.solve([m], bt, tol=1e-10, check=False)
        torch.cuda.synchronize()
        mg_s = time.perf_counter() - t0
        del x
        log(f"[bench] massscan m {m}: MG {mg_s:.2f} s ({max(i['outer_iters'] for i in info)} outer); CG solve")
        t0 = time.perf_counter()
        xc, info_cg, _ = ctx.cg_solve([m], bt, tol=1e-10)
        torch.cuda.synchronize()
        cg_s = time.perf_counter() - t0
        del xc
        row = {"mass": m, "setup_s": setup_s, "mg_s": mg_s, "mg_status": st,
               "mg_outer_iters": max(i["outer_iters"] for i in info), "mg_level_iters": info[0]["level_iters"],
               "mg_worst_residual": max(i["true_rel_residual"] for i in info), "cg_s": cg_s,
               "cg_iters": max(i["outer_iters"] for i in info_cg),
               "cg_worst_residual": max(i["true_rel_residual"] for i in info_cg), "cg_over_mg": cg_s / mg_s}
        rows.append(row)
        log(f"[bench] massscan m {m}: MG {mg_s:.2f} s ({row['mg_outer_iters']} outer), CG {cg_s:.2f} s "
            f"({row['cg_iters']} iterations): CG / MG {cg_s / mg_s:.2f}")
        ctx.destroy()
        del ctx
        torch.cuda.empty_cache()
    faster = [r["mass"] for r in rows if r["cg_s"] > r["mg_s"]]
    out = {"metric": "MG-GCR vs FP64 Schur CG time-to-1e-10 against the mass, 32^4 HISQ-style, 16 rhs per mass",
           "value": rows[-1]["cg_s"] / rows[-1]["mg_s"], "unit": "CG time / MG time at the lightest mass",
           "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": sum(r["mg_s"] for r in rows) * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 outer GCR, f32 K-cycle, 16-bit coarse links (f32 accumulate); f64 CG", "data": "synthetic",
           "config": {"workload": f"{'x'.join(map(str, dims))} HISQ-style eps {wl['eps']}, masses {masses}, "
                                  f"{wl['nrhs']} rhs per mass, a hierarchy per mass"},
           "per_mass": rows, "mg_faster_at": faster}
    print(json.dumps(out), flush=True)


def uneven_bench(args, wl, torch, latgen, mg):
    """Uneven batch: one context (fields, hierarchy, workspaces) per lattice
    size, 12 systems each.  The lattices are solved one after another, then
    all at once from one host thread and one HIP stream per lattice (the
    library holds no global state; each solve synchronises its own stream).
    Reports per-lattice latency in both modes and the aggregate systems/s."""
    import threading
    m, nr = wl["mass"], wl["nrhs"]
    dev = "cuda:0"
    cp = {"fp32": mg.MG_C64, "bf16": mg.MG_CBF16, "fp16": mg.MG_CF16}[args.coarse_prec or wl.get("coarse_prec", "fp32")]
    setup_iters = tuple(int(v) for v in args.setup_iters.split(",")) if args.setup_iters else wl["setup_iters"]
    probs = []
    for i, dims in enumerate(wl["dims_list"]):
        W, N, rng = latgen.hisq_style_links(dims, wl["eps"], wl["seed"] + i)
        b = torch.from_numpy(latgen.fine_vectors(dims, nr, rng)).to(dev)
        # block-preconditioned coarse levels only where every coarse extent is >= 4: on the 2^4 and 3^4
        # coarse lattices of 8^4 and 12^4 they raise the outer iteration count with an iterative coarsest
        # solve (373 -> 615 at 8^4); coarsest levels of at most 8192 dof (8^4: 1536, 12^4: 7776) are solved
        # exactly (dense inverse formed at set-up), the larger ones by CA-GCR(16)
        cdims = [d // b for d, b in zip(dims, wl["blocks"][0])]
        ncl = int(np.prod(cdims)) * 2 * wl["nvec"][0]
        p = mg.default_params(dims, mass0=m, nagg=1, nvec=wl["nvec"], block=wl["blocks"],
                              setup_maxiter=setup_iters + (1,), max_nrhs=nr, kd_naik=wl["kd_naik"], coarse_prec=cp,
                              outer_nkrylov=8, outer_maxiter=2000, coarse_op=1 if min(cdims) >= 4 else 0,
                              coarsest_solver=2 if ncl <= 8192 and not args.no_direct else 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = mg.setup(p, torch.from_numpy(W).to(dev), torch.from_numpy(N).to(dev))
        xk = torch.zeros((1,) + ctx.fine_shape, dtype=torch.complex64, device=dev)
        ctx.apply_dslash(2, m, xk)   # the KD inverse of the mass, outside the timed solves
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        tune = ctx.autotune(nr) if cp != mg.MG_C64 else []
        log(f"[bench] uneven {dims}: setup {setup_s:.2f} s ({probs_cs(p)} coarsest solve), coarse tiles {tune}")
        probs.append({"dims": dims, "ctx": ctx, "b": b, "setup_s": setup_s, "tune": tune,
                      "coarsest_solver": ["GCR", "CA-GCR(16)", "direct"][p.coarsest_solver]})
    coarse_multi = None
    if cp != mg.MG_C64:
        # the four lattices' level-2 operators: one launch each against one persistent launch over
        # their common (lattice, site, rhs tile) work list
        xs = [torch.randn((nr,) + pr["ctx"].coarse_shapes[0], dtype=torch.complex64, device=dev) for pr in probs]
        ys = [torch.empty_like(x) for x in xs]
        ctxs = [pr["ctx"] for pr in probs]

        def timed(f, reps=20):
            f()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                f()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) * 1e3 / reps

        sep_us = timed(lambda: [c.apply_coarse(2, x, y) for c, x, y in zip(ctxs, xs, ys)])
        multi_us = timed(lambda: mg.apply_coarse_multi(ctxs, 2, xs, ys))
        coarse_multi = {"separate_launches_us": sep_us, "one_persistent_launch_us": multi_us}
        log(f"[bench] level-2 operators of the four lattices: {sep_us:.1f} us in four launches, "
            f"{multi_us:.1f} us in one persistent launch")
        del xs, ys
    for pr in probs:   # warm-up solve of each lattice
        pr["ctx"].solve([m], pr["b"], tol=1e-10)
    torch.cuda.synchronize()
    seq = []
    t0 = time.perf_counter()
    for pr in probs:
        t1 = time.perf_counter()
        x, info, st = pr["ctx"].solve([m], pr["b"], tol=1e-10)
        torch.cuda.synchronize()
        seq.append({"s": time.perf_counter() - t1, "outer": max(i["outer_iters"] for i in info),
                    "residual": max(i["true_rel_residual"] for i in info)})
        del x
    seq_s = time.perf_counter() - t0
    conc = [None] * len(probs)

    keep = [None] * len(probs)   # rhs 0 of every concurrent solution (for the oracle's residual check)

    def run(k):
        pr = probs[k]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            t1 = time.perf_counter()
            x, info, st = pr["ctx"].solve([m], pr["b"], tol=1e-10)
            stream.synchronize()
            conc[k] = {"s": time.perf_counter() - t1, "outer": max(i["outer_iters"] for i in info),
                       "residual": max(i["true_rel_residual"] for i in info)}
            keep[k] = x[0, 0].cpu().numpy()
    threads = [threading.Thread(target=run, args=(k,)) for k in range(len(probs))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    conc_s = time.perf_counter() - t0
    nsys = nr * len(probs)
    for pr, a, c in zip(probs, seq, conc):
        log(f"[bench] uneven {pr['dims']}: alone {a['s']:.2f} s ({a['outer']} outer), concurrent {c['s']:.2f} s, "
            f"residual {max(a['residual'], c['residual']):.2e}")
    log(f"[bench] uneven: one after another {seq_s:.2f} s, concurrent {conc_s:.2f} s")
    out = {"metric": "uneven batch: 4 lattices (8^4..24^4) x 12 systems to 1e-10, wall time with one stream per "
                     "lattice", "value": conc_s, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": conc_s * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "c128 outer / c64 K-cycle", "data": "synthetic",
           "config": {"workload": f"HISQ-style eps 0.5 lattices {[list(p['dims']) for p in probs]}, mass {m}, "
                                  f"{nr} rhs each, truncated-KD={not wl['kd_naik']}, KD + 4^4/Nvec {wl['nvec'][0]}, "
                                  f"coarse links {args.coarse_prec or wl.get('coarse_prec', 'fp32')}"},
           "sequential_s": seq_s, "systems_per_s_concurrent": nsys / conc_s, "systems_per_s_sequential": nsys / seq_s,
           "per_lattice": [{"dims": list(p["dims"]), "setup_s": p["setup_s"], "coarse_tiles": p["tune"],
                            "coarsest_solver": p["coarsest_solver"],
                            "alone": a, "concurrent": c} for p, a, c in zip(probs, seq, conc)],
           "coarse_level2_multi": coarse_multi}
    if not args.no_cpu:
        out["cpu_baseline"] = uneven_oracle_leg(wl, probs, keep)
    print(json.dumps(out), flush=True)


def probs_cs(p):
    return ["GCR", "CA-GCR(16)", "direct"][p.coarsest_solver]


def uneven_oracle_leg(wl, probs, keep):
    """The oracle on the host for the uneven batch: its FP64 D recomputes the
    true residual of rhs 0 of every lattice's concurrent solution (fields
    regenerated from the same seeds); the time of those applications is the
    reported oracle figure."""
    from oracle import operators as ops
    from paper_2212_12559_amd import latgen

    c1, c3 = 9.0 / 8.0, -1.0 / 24.0
    model, _ = host_cpu()
    checks, t_ops = [], 0.0
    for i, (pr, x) in enumerate(zip(probs, keep)):
        W, N, rng = latgen.hisq_style_links(pr["dims"], wl["eps"], wl["seed"] + i)
        b = latgen.fine_vectors(pr["dims"], wl["nrhs"], rng)[0]
        t0 = time.perf_counter()
        r = b - ops.dslash(x, W, N, wl["mass"], c1, c3)
        t_ops += time.perf_counter() - t0
        rel = float(np.linalg.norm(r) / np.linalg.norm(b))
        checks.append({"dims": list(pr["dims"]), "true_rel_residual": rel})
        log(f"[bench] uneven {pr['dims']}: oracle true residual of rhs 0 {rel:.3e}")
    return {"value": t_ops, "unit": "s", "cores": 1, "cpu_model": model, "kind": "oracle",
            "sample": "one application of the numpy FP64 oracle's D per lattice (8^4, 12^4, 16^4, 24^4), "
                      "the residual check below",
            "oracle_check": {"what": "true residual of rhs 0 of every lattice's concurrent solution, "
                                     "recomputed by the oracle's FP64 D",
                             "systems": checks,
                             "worst_true_rel_residual": max(c["true_rel_residual"] for c in checks)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2batch", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-cg", action="store_true", help="skip the CG comparator")
    ap.add_argument("--no-msc", action="store_true", help="skip the multi-shift CG workflow comparison")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-time budget of the whole run from process start; the timed steps stop early to fit")
    ap.add_argument("--reserve-s", type=float, default=150.0,
                    help="time kept for the comparators, the oracle and the ceilings after the timed steps")
    ap.add_argument("--no-oracle-check", dest="oracle_check", action="store_false",
                    help="skip the oracle's residual check of the GPU solutions")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set up, time the hot kernels and copy a known-size buffer (for counter runs)")
    ap.add_argument("--coarse-prec", default=None, choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--eps", type=float, default=None,
                    help="roughness of the synthetic links (U = exp(i eps H)); default: the workload's")
    ap.add_argument("--no-direct", action="store_true",
                    help="uneven workload: CA-GCR(16) on every coarsest level (no exact small-level solve)")
    ap.add_argument("--mass-batch", type=int, default=None,
                    help="masses per lockstep solve (default: the workload's)")
    ap.add_argument("--nmass", type=int, default=None, help="solve only the first NMASS masses (profiling runs)")
    ap.add_argument("--setup-iters", default=None, help="CGNE iterations per level, e.g. 10,10 (kernel timing runs)")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=VALUE",
                    help="override one solver parameter (mg_params field), e.g. coarsest_restarts=4")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="turn two rocprofv3 --pmc runs of --kernels-only (FETCH_SIZE, WRITE_SIZE) into the "
                         "committed traffic record of the dominant kernel, then exit")
    args = ap.parse_args()
    if args.summarize_counters:
        from paper_2212_12559_amd import mgstag as mg
        wl = WORKLOADS[args.workload]
        cop = mg.default_params(wl["dims"]).coarse_op
        for kv in args.set:
            if kv.split("=", 1)[0] == "coarse_op":
                cop = int(kv.split("=", 1)[1])
        summarize_counters(*args.summarize_counters, wl, coarse_mode(args.coarse_prec or wl["coarse_prec"], cop))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2212_12559_amd import latgen, mgstag as mg

    wl = dict(WORKLOADS[args.workload])
    if args.eps is not None:
        wl["eps"] = args.eps
    if args.mass_batch is not None:
        wl["mass_batch"] = args.mass_batch
    if wl.get("kind") == "force":
        force_bench(args, wl, torch, latgen, mg)
        return
    if wl.get("kind") == "uneven":
        uneven_bench(args, wl, torch, latgen, mg)
        return
    if wl.get("kind") == "massscan":
        massscan_bench(args, wl, torch, latgen, mg)
        return
    out = {"metric": "MG-GCR time-to-1e-10 vs plain CG at 32^4 HISQ; Dslash/coarse GB/s, MFMA %",
           "value": None, "unit": "s", "n_gpus": 1, "steps": 0, "warmup": 0, "ms_per_step": None,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 outer GCR, f32 K-cycle, 16-bit coarse links (f32 accumulate)", "data": "synthetic",
           "steps_requested": args.steps, "warmup_requested": args.warmup, "budget_s": args.budget_s}
    try:
        c2batch_bench(args, wl, torch, latgen, mg, out)
    except Exception as e:   # report what was measured, then fail
        import traceback
        traceback.print_exc()
        out["error"] = f"{type(e).__name__}: {e}"
        print(json.dumps(out), flush=True)
        sys.exit(1)
    print(json.dumps(out), flush=True)


def elapsed():
    return time.perf_counter() - T_START


def c2batch_bench(args, wl, torch, latgen, mg, out):
    """The headline: MG-GCR solves of the multi-mass batch timed over as many
    of the requested steps as the budget allows, then the FP64 Schur CG
    comparator, the dominant kernel's roofline, the oracle baseline (with the
    oracle's residual check of a sample of the solutions), measured ceilings
    and, when time is left, the multi-shift CG workflow comparison."""
    dims, m = wl["dims"], wl["mass"]
    dev = "cuda:0"
    log(f"[bench] workload {args.workload} dims {dims} mass {m}: generating links")
    W, N, rng = latgen.hisq_style_links(dims, wl["eps"], wl["seed"])
    b = latgen.fine_vectors(dims, wl["nrhs"], rng)
    Wt, Nt = torch.from_numpy(W).to(dev), torch.from_numpy(N).to(dev)
    bt = torch.from_numpy(b).to(dev)
    masses = list(wl.get("masses", (m,)))[:args.nmass]
    cprec = args.coarse_prec or wl.get("coarse_prec", "fp32")
    cp = {"fp32": mg.MG_C64, "bf16": mg.MG_CBF16, "fp16": mg.MG_CF16}[cprec]
    setup_iters = tuple(int(v) for v in args.setup_iters.split(",")) if args.setup_iters else wl["setup_iters"]
    mb = wl.get("mass_batch", 1)
    nr = wl["nrhs"]
    p = mg.default_params(dims, mass0=m, nvec=wl["nvec"], block=wl["blocks"], setup_maxiter=setup_iters,
                          max_nrhs=nr * mb, max_nmass=len(masses), kd_naik=wl["kd_naik"], coarse_prec=cp,
                          outer_nkrylov=8 if nr > 1 else 16)
    for kv in args.set:
        k, v = kv.split("=", 1)
        setattr(p, k, type(getattr(p, k))(float(v)) if isinstance(getattr(p, k), float) else int(v))
        log(f"[bench] parameter {k} = {getattr(p, k)}")
    out["config"] = {"workload": f"{'x'.join(map(str, dims))} HISQ-style eps {wl['eps']}, masses {masses}, "
                                 f"{nr} rhs per mass, {mb} masses per lockstep solve, "
                                 f"truncated-KD={not wl['kd_naik']}, KD + {wl['blocks'][0]}/Nvec {wl['nvec'][0]} + "
                                 f"{wl['blocks'][1]}/Nvec {wl['nvec'][1]}, coarse links {cprec}",
                     "systems": nr * len(masses), "lattice": list(dims)}
    out["dtype"] = f"f64 outer GCR, f32 K-cycle, {cprec} coarse links (f32 accumulate)"
    log(f"[bench] setup ({elapsed():.0f} s into the run)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = mg.setup(p, Wt, Nt)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    out["setup_s"] = setup_s
    log(f"[bench] setup {setup_s:.2f} s")
    if cprec != "fp32":   # tile shapes of the 16-bit coarse stencil at the batch's rhs count
        out["autotune"] = ctx.autotune(nr * mb)
        log(f"[bench] coarse tiles {out['autotune']}")

    if args.kernels_only:
        kern = kernel_rates(torch, ctx, wl, args.kernel_reps, mg, 8 if cprec == "fp32" else 4)
        src = torch.empty(1 << 29, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)   # known-size copy (512 MiB read + 512 MiB write) to calibrate byte counters
        torch.cuda.synchronize()
        out["kernels"] = {k: {"us": v["us"], "bytes": v["bytes"]} for k, v in kern.items()}
        return

    # per-mass set-up (the exact KD inverse of every mass, Sec. 3.1) outside the timed region
    xk = torch.zeros((1,) + ctx.fine_shape, dtype=torch.complex64, device=dev)
    for mj in masses:
        ctx.apply_dslash(2, mj, xk)
    torch.cuda.synchronize()
    del xk

    batch_s = []
    keep = {}   # rhs 0 and 1 of every mass from the last step (for the oracle's residual check)

    def mg_step(tag, tol=1e-10, chunks=None):
        # lockstep batches of mb masses x nrhs systems; a line per batch and mass
        info_all = []
        batch_s.clear()
        for j0 in range(0, len(masses), mb):
            if chunks is not None and j0 // mb >= chunks:
                break
            chunk = masses[j0:j0 + mb]
            x, info, st = ctx.solve(chunk, bt, tol=tol)
            info_all += info
            batch_s.append(info[0]["seconds"])
            for j, mj in enumerate(chunk):
                ij = info[j * nr:(j + 1) * nr]
                log(f"[bench] {tag} mass {mj}: {max(i['outer_iters'] for i in ij)} outer, batch level iters "
                    f"{ij[0]['level_iters']}, batch {ij[0]['seconds']:.2f} s, "
                    f"max residual {max(i['true_rel_residual'] for i in ij):.2e}")
                keep[mj] = x[j, :2].clone()   # rhs 0 and 1
            del x
        return info_all

    # warm-up: one lockstep batch to a loose tolerance runs every kernel of the
    # solve once (the library is compiled ahead of time: nothing else to warm)
    if args.warmup > 0:
        mg_step("warmup", tol=1e-2, chunks=1)
        out["warmup"] = 1
        out["warmup_kind"] = f"one lockstep batch ({nr * mb} systems) solved to 1e-2"
    torch.cuda.synchronize()
    # the dominant kernel (level-2 coarse stencil) is timed inside the timed
    # solves: the library brackets each of its launches over the full batch
    # (the rhs count its algorithmic bytes are taken at; a batch shrinks as
    # its systems converge) with HIP events on the stream it runs on
    ctx.profile_start(mg.MG_PROF_COARSE, 2, nrhs=nr * mb)
    infos = []
    t_steps = time.perf_counter()
    while len(infos) < max(1, args.steps):
        t1 = time.perf_counter()
        infos.append(mg_step(f"step {len(infos)}"))
        torch.cuda.synchronize()
        step_s = time.perf_counter() - t1
        # the rest of the run (comparators, oracle, ceilings) needs about args.reserve_s
        if elapsed() + step_s + args.reserve_s > args.budget_s:
            break
    torch.cuda.synchronize()
    mg_s = (time.perf_counter() - t_steps) / len(infos)
    last_batch_s = list(batch_s)
    dom_launches, dom_ms = ctx.profile_stop()
    res = max(s_["true_rel_residual"] for i in infos for s_ in i)
    out.update({"value": mg_s, "steps": len(infos), "ms_per_step": mg_s * 1e3, "mg_info": infos[-1][0],
                "mg_outer_iters_per_mass": [max(i["outer_iters"] for i in infos[-1][j * nr:(j + 1) * nr])
                                            for j in range(len(masses))],
                "mg_batch_s": last_batch_s, "true_rel_residual": res})
    log(f"[bench] MG {mg_s:.2f} s per step over {len(infos)} steps ({elapsed():.0f} s into the run)")

    if not args.no_cg:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cg_iters = []
        for mj in masses:
            xc, cinfo, st = ctx.cg_solve([mj], bt, tol=1e-10, maxiter=200000)
            cg_iters.append(max(i["outer_iters"] for i in cinfo))
            log(f"[bench] CG mass {mj}: {cg_iters[-1]} iterations, {cinfo[0]['seconds']:.2f} s")
            del xc
        torch.cuda.synchronize()
        cg_s = time.perf_counter() - t0
        out.update({"cg_s": cg_s, "cg_iters_per_mass": cg_iters, "speedup_vs_cg": cg_s / mg_s})
        log(f"[bench] CG {cg_s:.3f} s")

    # ---- roofline of the dominant kernel (its launches inside the timed solves)
    kern = kernel_rates(torch, ctx, wl, args.kernel_reps, mg, 8 if cprec == "fp32" else 4)
    dom_bytes = kern["coarse2"]["bytes"]          # algorithmic bytes at the batch's rhs count
    dom_us = dom_ms / max(dom_launches, 1) * 1e3
    dom_gbs = dom_bytes / (dom_us * 1e-6) / 1e9
    kname = ("coarse_kernel<float,float2>" if cprec == "fp32" else f"coarse_mfma_kernel<{cprec}>")
    traffic, traffic_src = hbm_traffic(nr * mb, coarse_mode(cprec, p.coarse_op))
    out["roofline"] = {"bound": "hbm", "kernel": f"{kname} (level-2 coarse stencil, {nr * mb} rhs per launch)",
                       "achieved": dom_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": dom_gbs / HBM_PEAK_GBS, "traffic": traffic,
                       "bytes_per_launch": dom_bytes, "avg_launch_us": dom_us, "launches_timed": dom_launches,
                       "timing": f"HIP events around every launch over the full batch ({nr * mb} systems) "
                                 "inside the timed solves",
                       "traffic_source": traffic_src}
    out["kernels"] = {k: {kk: round(vv, 2) for kk, vv in v.items() if kk != "bytes"} for k, v in kern.items()}
    out["mfma_frac_coarse2"] = (kern["coarse2"].get("TFLOPs", 0.0) / 2500.0) if cprec != "fp32" else None

    # ---- measured ceilings: a 4 GiB copy and a loop of 16-bit matrix-core products
    src = torch.empty(1 << 32, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    copy_gbs = mg.peak_copy(src, dst, reps=5)
    del src, dst
    mfma_tf = mg.peak_mfma(cp if cp in (mg.MG_CBF16, mg.MG_CF16) else mg.MG_CBF16)
    out["ceilings"] = {"copy_4GiB_GBps": copy_gbs, "mfma16_TFLOPs": mfma_tf,
                       "roofline_frac_of_copy": dom_gbs / copy_gbs}
    log(f"[bench] ceilings: copy {copy_gbs:.0f} GB/s, 16-bit MFMA {mfma_tf:.0f} TFLOP/s")

    if not args.no_cpu:
        # one info per lockstep batch (one mass, nrhs systems): counts x nrhs single applications
        batch_infos = [infos[-1][j * nr] for j in range(len(masses))]
        sample = ([(mj, r, b[r], keep[mj][r].cpu().numpy()) for mj in masses for r in range(min(2, nr))]
                  if args.oracle_check else [])
        out["cpu_baseline"] = cpu_baseline(wl, batch_infos, p.smoother_s,
                                           oracle_check=(dims, (W, N), sample) if sample else None)
    log(f"[bench] {elapsed():.0f} s into the run")

    # ---- propagator workflow (Sec. 3.3, the Table 2 comparison): multi-shift CG
    # over every mass, against MG for the lightest lockstep batch plus
    # multi-shift CG for the rest; only when the budget has room for it
    if not args.no_msc and len(masses) > mb and elapsed() + 40 < args.budget_s:
        def msc(ms, tag):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xm, minfo, st = ctx.multishift_cg_solve(list(ms), bt, tol=1e-10, maxiter=200000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            per = [max(i["outer_iters"] for i in minfo[j * nr:(j + 1) * nr]) for j in range(len(ms))]
            worst = max(i["true_rel_residual"] for i in minfo)
            fixed = sum(1 for i in minfo if i["reliable_updates"] > 0)
            log(f"[bench] multi-shift CG {tag}: {dt:.2f} s, base iterations {minfo[0]['level_iters'][0]}, "
                f"per-mass {per}, worst residual {worst:.2e}, finished by CG {fixed}")
            del xm
            return dt, per, worst, fixed
        msc_all, per_all, worst_all, fix_all = msc(masses, "all masses")
        msc_heavy, per_heavy, worst_heavy, fix_heavy = msc(masses[mb:], "heavier masses")
        mg_light = last_batch_s[0]
        out["workflow"] = {
            "masses_mg": masses[:mb], "masses_msc": masses[mb:],
            "msc_all_s": msc_all, "msc_all_iters_per_mass": per_all,
            "mg_light_s": mg_light, "msc_heavy_s": msc_heavy,
            "mg_plus_msc_s": mg_light + msc_heavy, "speedup_vs_msc": msc_all / (mg_light + msc_heavy),
            "worst_true_rel_residual": max(worst_all, worst_heavy),
            "systems_finished_by_cg": fix_all + fix_heavy,
            # Table 2: propagators after which the set-up is paid back (None: MG + multi-shift is
            # not faster per propagator, so it never is)
            "break_even_propagators": (setup_s / (msc_all - mg_light - msc_heavy)
                                       if msc_all > mg_light + msc_heavy else None)}
        log(f"[bench] workflow {out['workflow']}")
    out["wall_s"] = elapsed()
    log(f"[bench] done, {elapsed():.0f} s")


if __name__ == "__main__":
    main()
