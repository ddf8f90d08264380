"""Python binding of the mgstag C ABI (include/mgstag.h).

Argument marshalling only: every operation runs in the HIP library
libmgstag.so next to this file.  PyTorch provides device memory (the
workspaces are torch uint8 tensors owned by the Context object) and streams
(torch's current stream is passed to every call).  Importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgstag.so")

MG_OK, MG_E_ARG, MG_E_CONFIG, MG_E_ALIGN, MG_E_RANK, MG_E_NOCONV, MG_E_NONFINITE, MG_E_HIP, MG_E_STATE, \
    MG_E_WORKSPACE = range(10)
MG_C128, MG_C64, MG_CBF16, MG_CF16 = range(4)
MG_PROF_COARSE, MG_PROF_DSLASH, MG_PROF_KD, MG_PROF_RESTRICT, MG_PROF_PROLONG = range(5)
STATUS_NAMES = ["MG_OK", "MG_E_ARG", "MG_E_CONFIG", "MG_E_ALIGN", "MG_E_RANK", "MG_E_NOCONV",
                "MG_E_NONFINITE", "MG_E_HIP", "MG_E_STATE", "MG_E_WORKSPACE"]


class MGParams(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32 * 4),
        ("c1", ctypes.c_double), ("c3", ctypes.c_double),
        ("kd_naik", ctypes.c_int32),
        ("mass0", ctypes.c_double),
        ("nagg", ctypes.c_int32),
        ("block", (ctypes.c_int32 * 4) * 2),
        ("nvec", ctypes.c_int32 * 2),
        ("setup_maxiter", ctypes.c_int32 * 2),
        ("setup_tol", ctypes.c_double * 2),
        ("smoother_s", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("inner_maxiter", ctypes.c_int32),
        ("coarsest_tol", ctypes.c_double),
        ("coarsest_maxiter", ctypes.c_int32),
        ("coarsest_restarts", ctypes.c_int32),
        ("outer_nkrylov", ctypes.c_int32),
        ("outer_maxiter", ctypes.c_int32),
        ("reliable_delta", ctypes.c_double),
        ("fine_prec", ctypes.c_int32),
        ("coarse_prec", ctypes.c_int32),
        ("max_nrhs", ctypes.c_int32),
        ("max_nmass", ctypes.c_int32),
        ("coarsest_deflate", ctypes.c_int32),
        ("deflate_maxiter", ctypes.c_int32),
        ("deflate_import", ctypes.c_int32),
        ("coarse_op", ctypes.c_int32),
        ("coarsest_solver", ctypes.c_int32),
        ("graph_coarsest", ctypes.c_int32),
        ("compact_masses", ctypes.c_int32),
        ("coarse_shadow", ctypes.c_int32),
        ("cgne_start_import", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


class MGTuneInfo(ctypes.Structure):
    _fields_ = [
        ("level", ctypes.c_int32),
        ("nrhs", ctypes.c_int32),
        ("rhs_per_workgroup", ctypes.c_int32),
        ("mtiles_per_wave", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("us_best", ctypes.c_double),
        ("us_default", ctypes.c_double),
    ]


class MGSolveInfo(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int32),
        ("reliable_updates", ctypes.c_int32),
        ("level_iters", ctypes.c_int32 * 4),
        ("true_rel_residual", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("status", ctypes.c_int32),
    ]

    def as_dict(self):
        return {"outer_iters": self.outer_iters, "reliable_updates": self.reliable_updates,
                "level_iters": list(self.level_iters), "true_rel_residual": self.true_rel_residual,
                "seconds": self.seconds, "status": STATUS_NAMES[self.status]}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"mgstag HIP library not built: {LIB_PATH} is missing "
                          "(run python -m paper_2212_12559_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, vp, sz, i32, f64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    sig = {
        "mg_default_params": (None, [P(MGParams), P(ctypes.c_int32 * 4)]),
        "mg_workspace_bytes": (i32, [P(MGParams), P(sz), P(sz)]),
        "mg_setup": (i32, [P(MGParams), vp, vp, P(vp), vp, sz, vp, sz, vp, P(vp)]),
        "mg_apply_dslash": (i32, [vp, i32, f64, i32, vp, vp, i32, vp]),
        "mg_apply_dslash_noalloc": (i32, [vp, i32, f64, i32, vp, vp, i32, vp]),
        "mg_noalloc_scratch_bytes": (sz, []),
        "mg_apply_coarse": (i32, [vp, i32, i32, vp, vp, i32, vp]),
        "mg_restrict": (i32, [vp, i32, i32, vp, vp, i32, vp]),
        "mg_prolong": (i32, [vp, i32, i32, vp, vp, i32, i32, vp]),
        "mg_solve": (i32, [vp, P(f64), i32, vp, vp, i32, f64, P(MGSolveInfo), vp]),
        "mg_cg_solve": (i32, [vp, P(f64), i32, vp, vp, i32, f64, i32, P(MGSolveInfo), vp]),
        "mg_msc_solve": (i32, [vp, P(f64), i32, vp, vp, i32, f64, i32, P(MGSolveInfo), vp]),
        "mg_export": (i32, [vp, i32, i32, vp, sz, P(sz), vp]),
        "mg_solve_backward": (i32, [vp, f64, vp, vp, vp, vp, vp, i32, f64, P(f64), P(MGSolveInfo), vp]),
        "mg_update_links": (i32, [vp, vp, vp, vp]),
        "mg_autotune": (i32, [vp, i32, P(MGTuneInfo), vp]),
        "mg_apply_coarse_multi": (i32, [P(vp), i32, i32, P(vp), P(vp), P(i32), vp]),
        "mg_profile_start": (i32, [vp, i32, i32, i32]),
        "mg_profile_stop": (i32, [vp, P(i32), P(f64)]),
        "mg_peak_copy": (i32, [vp, vp, sz, i32, vp, P(f64)]),
        "mg_peak_mfma": (i32, [i32, i32, vp, vp, P(f64)]),
        "mg_destroy": (i32, [vp]),
        "mg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


class MGError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = LIB.mg_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES[status] if 0 <= status < 10 else status}: {msg}")


def _check(status, where):
    if status != MG_OK:
        raise MGError(status, where)


def default_params(dims, **overrides) -> MGParams:
    p = MGParams()
    d = (ctypes.c_int32 * 4)(*dims)
    LIB.mg_default_params(ctypes.byref(p), ctypes.byref(d))
    for k, v in overrides.items():
        if k == "block":
            for l in range(2):
                for mu in range(4):
                    p.block[l][mu] = v[l][mu] if l < len(v) else 1
        elif k in ("nvec", "setup_maxiter", "setup_tol", "dims"):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(p, k, v)
    return p


def workspace_bytes(p: MGParams):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(LIB.mg_workspace_bytes(ctypes.byref(p), ctypes.byref(a), ctypes.byref(b)), "mg_workspace_bytes")
    return a.value, b.value


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.complex128:
        return MG_C128
    if t.dtype == torch.complex64:
        return MG_C64
    raise TypeError(f"unsupported dtype {t.dtype} (complex128 or complex64)")


def _dev(t, name):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _check_batch(t, name, per_rhs, dtype=None, nrhs=None):
    """The library takes raw pointers: check what it will read or write.
    t must hold a whole number of vectors of per_rhs complex elements (of the
    given dtype, complex128/complex64 otherwise) and, when nrhs is given,
    exactly nrhs of them; returns the number of vectors."""
    torch = _torch()
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dtype not in (torch.complex128, torch.complex64):
        raise TypeError(f"{name} must be complex128 or complex64, got {t.dtype}")
    n = t.numel()
    if n == 0 or n % per_rhs:
        raise ValueError(f"{name} has {n} elements, not a positive multiple of {per_rhs} (one vector)")
    if nrhs is not None and n != nrhs * per_rhs:
        raise ValueError(f"{name} has {n // per_rhs} vectors, expected {nrhs}")
    return n // per_rhs


class Context:
    """An mg_ctx with its two caller-owned device workspaces."""

    def __init__(self, params: MGParams, fat, naik=None, null_vectors=None):
        torch = _torch()
        self.ctx = None
        self._init_shapes(params)
        pb, sb = workspace_bytes(params)   # validates the parameters first
        nlink = 4 * self.V * 9
        _check_batch(fat, "fat", nlink, torch.complex128, 1)
        if params.c3 != 0.0:
            if naik is None:
                raise ValueError("naik links are required when c3 != 0")
            _check_batch(naik, "naik", nlink, torch.complex128, 1)
        dev = fat.device
        # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
        self.persistent = torch.empty(pb, dtype=torch.uint8, device=dev)
        self.scratch = torch.empty(sb, dtype=torch.uint8, device=dev)
        nvp = None
        self._keep = []
        if null_vectors is not None:
            # levels 1 .. nagg, then (deflate_import) the coarsest level's deflation vectors
            nent = params.nagg + (1 if params.coarsest_deflate > 0 and params.deflate_import else 0)
            if len(null_vectors) > nent:
                raise ValueError(f"null_vectors: at most {nent} entries with these parameters")
            arr = (ctypes.c_void_p * 3)()
            for l in range(nent):
                v = null_vectors[l] if l < len(null_vectors) else None
                if v is not None:
                    defl = l == params.nagg
                    _check_batch(v, f"null_vectors[{l}]", self._level_size(l + 1), torch.complex128,
                                 params.coarsest_deflate if defl else params.nvec[l])
                    _dev(v, f"null_vectors[{l}]")
                    self._keep.append(v)
                    arr[l] = v.data_ptr()
            nvp = arr
        ctx = ctypes.c_void_p()
        st = LIB.mg_setup(ctypes.byref(params), _dev(fat, "fat"),
                          _dev(naik, "naik") if naik is not None else None,
                          nvp, ctypes.c_void_p(self.persistent.data_ptr()), pb,
                          ctypes.c_void_p(self.scratch.data_ptr()), sb, _stream(), ctypes.byref(ctx))
        _check(st, "mg_setup")
        self.ctx = ctx

    def _init_shapes(self, params):
        """Lattice and level shapes (host only)."""
        self.params = params
        self.dims = tuple(params.dims)
        X, Y, Z, T = self.dims
        self.V = X * Y * Z * T
        self.fine_shape = (T, Z, Y, X, 3)
        self.coarse_shapes = []
        cd = list(self.dims)
        for l in range(params.nagg):
            cd = [cd[mu] // params.block[l][mu] for mu in range(4)]
            self.coarse_shapes.append((cd[3], cd[2], cd[1], cd[0], 2, params.nvec[l]))

    def _level_size(self, level):
        """Complex elements of one vector of `level` (1: fine, 2, 3: coarse)."""
        if level == 1:
            return 3 * self.V
        n = 1
        for v in self.coarse_shapes[level - 2]:
            n *= v
        return n

    def _out(self, out, like, shape, name="out"):
        torch = _torch()
        if out is None:
            return torch.empty(shape, dtype=like.dtype, device=like.device)
        n = 1
        for v in shape:
            n *= v
        _check_batch(out, name, n, like.dtype, 1)
        if out.data_ptr() == like.data_ptr():
            raise ValueError(f"{name} must not alias the input")
        return out

    # ---------------------------------------------------------------- applies
    def apply_dslash(self, op, mass, x, out=None):
        nrhs = _check_batch(x, "x", self._level_size(1))
        out = self._out(out, x, tuple(x.shape))
        _check(LIB.mg_apply_dslash(self.ctx, op, mass, _dtype_code(x), _dev(x, "x"), _dev(out, "out"), nrhs,
                                   _stream()), "mg_apply_dslash")
        return out

    def apply_dslash_noalloc(self, op, mass, x, out):
        """apply_dslash through the entry point that allocates nothing (its
        work batch is the library's static device array); out is required."""
        nrhs = _check_batch(x, "x", self._level_size(1))
        out = self._out(out, x, tuple(x.shape))
        _check(LIB.mg_apply_dslash_noalloc(self.ctx, op, mass, _dtype_code(x), _dev(x, "x"), _dev(out, "out"),
                                           nrhs, _stream()), "mg_apply_dslash_noalloc")
        return out

    def apply_coarse(self, level, x, out=None):
        if not 2 <= level <= 1 + self.params.nagg:
            raise ValueError(f"level must be in 2..{1 + self.params.nagg}")
        nrhs = _check_batch(x, "x", self._level_size(level))
        out = self._out(out, x, tuple(x.shape))
        _check(LIB.mg_apply_coarse(self.ctx, level, _dtype_code(x), _dev(x, "x"), _dev(out, "out"), nrhs,
                                   _stream()), "mg_apply_coarse")
        return out

    def restrict(self, level, x, out=None):
        if not 1 <= level <= self.params.nagg:
            raise ValueError(f"level must be in 1..{self.params.nagg}")
        nrhs = _check_batch(x, "x", self._level_size(level))
        out = self._out(out, x, (nrhs,) + self.coarse_shapes[level - 1])
        _check(LIB.mg_restrict(self.ctx, level, _dtype_code(x), _dev(x, "x"), _dev(out, "out"), nrhs, _stream()),
               "mg_restrict")
        return out

    def prolong(self, level, xc, out=None, accumulate=False):
        torch = _torch()
        if not 1 <= level <= self.params.nagg:
            raise ValueError(f"level must be in 1..{self.params.nagg}")
        nrhs = _check_batch(xc, "xc", self._level_size(level + 1))
        shape = (nrhs,) + tuple(self.fine_shape if level == 1 else self.coarse_shapes[level - 2])
        if out is None:
            out = torch.zeros(shape, dtype=xc.dtype, device=xc.device)
        else:
            out = self._out(out, xc, shape)
        _check(LIB.mg_prolong(self.ctx, level, _dtype_code(xc), _dev(xc, "xc"), _dev(out, "out"),
                              1 if accumulate else 0, nrhs, _stream()), "mg_prolong")
        return out

    # ---------------------------------------------------------------- solves
    def _solve(self, fn, masses, b, tol, extra=()):
        torch = _torch()
        nrhs = _check_batch(b, "b", self._level_size(1), torch.complex128)
        nm = len(masses)
        if nm < 1:
            raise ValueError("at least one mass")
        x = torch.empty((nm, nrhs) + self.fine_shape, dtype=torch.complex128, device=b.device)
        infos = (MGSolveInfo * (nm * nrhs))()
        m = (ctypes.c_double * nm)(*masses)
        st = fn(self.ctx, m, nm, _dev(b, "b"), _dev(x, "x"), nrhs, tol, *extra, infos, _stream())
        return st, x, [i.as_dict() for i in infos]

    def solve(self, masses, b, tol=1e-10, check=True):
        """MG-GCR solve of D(m) x = b for every mass; b [nrhs][T][Z][Y][X][3] complex128."""
        st, x, info = self._solve(LIB.mg_solve, masses, b, tol)
        if check:
            _check(st, "mg_solve")
        return x, info, st

    def cg_solve(self, masses, b, tol=1e-10, maxiter=100000, check=True):
        st, x, info = self._solve(LIB.mg_cg_solve, masses, b, tol, (maxiter,))
        if check:
            _check(st, "mg_cg_solve")
        return x, info, st

    def multishift_cg_solve(self, masses, b, tol=1e-10, maxiter=100000, check=True):
        """Multi-shift CG over all masses at once (at most 16); same layouts as solve."""
        st, x, info = self._solve(LIB.mg_msc_solve, masses, b, tol, (maxiter,))
        if check:
            _check(st, "mg_msc_solve")
        return x, info, st

    def solve_backward(self, mass, phi, tol=1e-10):
        """X = (D^dag D)^{-1} phi, Y = D X, the action S_r = Re <phi_r, X_r> per
        right-hand side and the fermion-force gradients of S = sum_r S_r with
        respect to the fat and Naik links (PyTorch convention), all computed
        by the library.  phi [nrhs][T][Z][Y][X][3] complex128."""
        torch = _torch()
        nrhs = _check_batch(phi, "phi", self._level_size(1), torch.complex128)
        X = torch.empty_like(phi)
        Y = torch.empty_like(phi)
        T_, Z_, Y_, X_ = self.fine_shape[:4]
        gw = torch.empty((4, T_, Z_, Y_, X_, 3, 3), dtype=torch.complex128, device=phi.device)
        gn = torch.empty_like(gw) if self.params.c3 != 0.0 else None
        infos = (MGSolveInfo * (2 * nrhs))()
        action = (ctypes.c_double * nrhs)()
        st = LIB.mg_solve_backward(self.ctx, mass, _dev(phi, "phi"), _dev(X, "X"), _dev(Y, "Y"), _dev(gw, "grad_fat"),
                                   _dev(gn, "grad_naik") if gn is not None else None, nrhs, tol, action, infos,
                                   _stream())
        _check(st, "mg_solve_backward")
        self.last_action = list(action)
        return X, Y, gw, gn, [i.as_dict() for i in infos]

    def update_links(self, fat, naik=None):
        torch = _torch()
        nlink = 4 * self.V * 9
        _check_batch(fat, "fat", nlink, torch.complex128, 1)
        if naik is not None:
            _check_batch(naik, "naik", nlink, torch.complex128, 1)
        _check(LIB.mg_update_links(self.ctx, _dev(fat, "fat"), _dev(naik, "naik") if naik is not None else None,
                                   _stream()), "mg_update_links")

    def export(self, what, level=1):
        torch = _torch()
        need = ctypes.c_size_t()
        _check(LIB.mg_export(self.ctx, what, level, None, 0, ctypes.byref(need), _stream()), "mg_export")
        dt = torch.int32 if what == 0 else torch.complex128
        esz = 4 if what == 0 else 16
        out = torch.empty(need.value // esz, dtype=dt, device=self.persistent.device)
        _check(LIB.mg_export(self.ctx, what, level, _dev(out, "dst"), need.value, None, _stream()), "mg_export")
        return out

    def autotune(self, nrhs):
        """Tile shapes of the 16-bit coarse stencil timed at nrhs rhs; the
        fastest is kept.  Returns one dict per coarse level (the shape
        chosen, its time and the built-in shape's time in microseconds)."""
        info = (MGTuneInfo * 2)()
        _check(LIB.mg_autotune(self.ctx, nrhs, info, _stream()), "mg_autotune")
        return [{"level": t.level, "nrhs": t.nrhs, "rhs_per_workgroup": t.rhs_per_workgroup,
                 "mtiles_per_wave": t.mtiles_per_wave, "candidates": t.candidates, "us_best": t.us_best,
                 "us_default": t.us_default} for t in info if t.level > 0]

    def profile_start(self, op, level=0, nrhs=0):
        """Time every launch of one operator (MG_PROF_*) with HIP events; with
        nrhs > 0 only its launches over exactly nrhs systems."""
        _check(LIB.mg_profile_start(self.ctx, op, level, nrhs), "mg_profile_start")

    def profile_stop(self):
        """(launches, total milliseconds) since profile_start."""
        n = ctypes.c_int32()
        ms = ctypes.c_double()
        _check(LIB.mg_profile_stop(self.ctx, ctypes.byref(n), ctypes.byref(ms)), "mg_profile_stop")
        return n.value, ms.value

    def destroy(self):
        if getattr(self, "ctx", None):
            LIB.mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def peak_copy(src, dst, reps=5):
    """Measured HBM ceiling: GB/s (read + write) of the library's copy kernel."""
    if src.numel() * src.element_size() != dst.numel() * dst.element_size():
        raise ValueError("src and dst must have the same size")
    g = ctypes.c_double()
    _check(LIB.mg_peak_copy(_dev(src, "src"), _dev(dst, "dst"), src.numel() * src.element_size(), reps, _stream(),
                            ctypes.byref(g)), "mg_peak_copy")
    return g.value


def peak_mfma(fmt=MG_CBF16, iters=20000, device="cuda:0"):
    """Measured dense 16-bit matrix-core rate in TFLOP/s."""
    torch = _torch()
    sink = torch.empty(8192, dtype=torch.uint8, device=device)
    t = ctypes.c_double()
    _check(LIB.mg_peak_mfma(fmt, iters, _dev(sink, "sink"), _stream(), ctypes.byref(t)), "mg_peak_mfma")
    return t.value


def apply_coarse_multi(ctxs, level, xs, outs=None):
    """Level-`level` coarse operators of several contexts (16-bit links, same
    2 Nvec) applied in one persistent launch; xs[p] are complex64 batches of
    ctxs[p]'s level vectors.  Returns the outputs."""
    torch = _torch()
    n = len(ctxs)
    if not 1 <= n <= 8 or len(xs) != n:
        raise ValueError("1..8 contexts, one input batch each")
    outs = list(outs) if outs is not None else [None] * n
    cv, iv, ov, nv = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)(), (ctypes.c_int32 * n)()
    for p, (c, x) in enumerate(zip(ctxs, xs)):
        if not 2 <= level <= 1 + c.params.nagg:
            raise ValueError(f"level must be in 2..{1 + c.params.nagg}")
        nv[p] = _check_batch(x, f"xs[{p}]", c._level_size(level), torch.complex64)
        outs[p] = c._out(outs[p], x, tuple(x.shape), f"outs[{p}]")
        cv[p] = c.ctx.value
        iv[p] = _dev(x, f"xs[{p}]").value
        ov[p] = _dev(outs[p], f"outs[{p}]").value
    _check(LIB.mg_apply_coarse_multi(cv, n, level, iv, ov, nv, _stream()), "mg_apply_coarse_multi")
    return outs


def setup(params, fat, naik=None, null_vectors=None) -> Context:
    return Context(params, fat, naik, null_vectors)


def _fermion_action_class():
    torch = _torch()

    class FermionAction(torch.autograd.Function):
        """S = sum_r phi_r^dag (D^dag D)^{-1} phi_r as a differentiable function
        of the fat and Naik links; the forward pass runs the two MG solves and
        the force kernel of the library, the backward pass scales the stored
        gradients.  `ctx_mg` is a Context whose links are replaced by (W, N)."""

        @staticmethod
        def forward(ctx, W, N, phi, ctx_mg, mass, tol):
            ctx_mg.update_links(W.detach().contiguous(), N.detach().contiguous() if N is not None else None)
            X, Y, gw, gn, info = ctx_mg.solve_backward(mass, phi.detach().contiguous(), tol)
            ctx.save_for_backward(gw, gn if gn is not None else gw)
            ctx.has_naik = gn is not None
            return torch.tensor(sum(ctx_mg.last_action), dtype=torch.float64, device=W.device)

        @staticmethod
        def backward(ctx, g):
            gw, gn = ctx.saved_tensors
            return g * gw, (g * gn if ctx.has_naik else None), None, None, None, None

    return FermionAction


def fermion_action(W, N, phi, ctx_mg, mass, tol=1e-10):
    """Differentiable S(W, N) = sum_r phi_r^dag (D^dag D)^{-1} phi_r (see FermionAction)."""
    return _fermion_action_class().apply(W, N, phi, ctx_mg, mass, tol)
