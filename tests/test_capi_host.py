"""The C-ABI library loads, exports every symbol include/mgstag.h declares,
and its host-only entry points (defaults, workspace sizing, validation)
behave as documented.  No GPU work is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mgstag.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def m():
    from paper_2212_12559_amd import mgstag
    return mgstag


def test_header_symbols_exported(m):
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(m.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in mgstag.h but not exported"


def declared_prototypes():
    """name -> (return type, [parameter types]) of every function the header
    declares (comments removed, parameter names dropped)."""
    src = open(os.path.join(ROOT, "include", "mgstag.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for ret, name, params in re.findall(r"([A-Za-z_][\w\s\*]*?)\b(mg_[a-z_]+)\s*\(([^)]*)\)\s*;", src):
        ps = [q.strip() for q in params.split(",")]
        ps = [] if ps == ["void"] or ps == [""] else ps
        types = []
        for q in ps:
            arr = re.search(r"\[[^]]*\]$", q) is not None
            q = re.sub(r"\s*\[[^]]*\]$", "", q)
            q = re.sub(r"\b\w+$", "", q).strip()   # drop the parameter name
            types.append(q + "*" if arr else q)      # an array parameter is a pointer
        out[name] = (ret.split()[-1].strip() if "*" not in ret else ret.strip(), types)
    return out


def _kind(ctype):
    """'ptr', 'i32', 'f64', 'size' or 'void' for a C type or a ctypes type."""
    if isinstance(ctype, str):
        if "*" in ctype or ctype in ("mg_ctx",):
            return "ptr"
        base = ctype.replace("const", "").strip()
        return {"int32_t": "i32", "mg_status": "i32", "double": "f64", "size_t": "size", "void": "void"}[base]
    if ctype is None:
        return "void"
    if ctype in (ctypes.c_void_p, ctypes.c_char_p) or hasattr(ctype, "_type_") and issubclass(
            ctype, ctypes._Pointer):
        return "ptr"
    return {ctypes.c_int32: "i32", ctypes.c_double: "f64", ctypes.c_size_t: "size"}[ctype]


def test_binding_signatures_match_header(m):
    """Every function of include/mgstag.h has a ctypes prototype in the
    binding with the same return kind and the same number and kind of
    arguments (pointer, int32, double, size_t): a stale prototype would
    pass wrong arguments through the C ABI without any error on the host."""
    protos = declared_prototypes()
    assert len(protos) == len(declared_functions())
    for name, (ret, params) in protos.items():
        f = getattr(m.LIB, name)
        assert f.argtypes is not None, f"{name}: no ctypes prototype in the binding"
        assert [_kind(t) for t in f.argtypes] == [_kind(t) for t in params], name
        assert _kind(f.restype) == _kind(ret), name


def test_params_struct_matches_header(m, tmp_path):
    """sizeof and field offsets of mg_params / mg_solve_info as the C compiler
    lays them out from the header equal the ctypes mirrors."""
    import subprocess
    fields = [f for f, _ in m.MGParams._fields_]
    src = tmp_path / "layout.c"
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#define __HIP_PLATFORM_AMD__',
             '#include "mgstag.h"', 'int main(void) {',
             '  printf("%zu %zu\\n", sizeof(mg_params), sizeof(mg_solve_info));']
    lines += [f'  printf("%zu\\n", offsetof(mg_params, {f}));' for f in fields]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run(["gcc", "-I", inc, "-I", "/opt/rocm/include", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(m.MGParams)
    assert int(out[1]) == ctypes.sizeof(m.MGSolveInfo)
    for f, off in zip(fields, out[2:]):
        assert getattr(m.MGParams, f).offset == int(off), f


def test_default_params_table1(m):
    """Defaults against the values of the paper's Table 1 (tests/golden)."""
    import json
    t = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_mg_parameters.json")))
    p = m.default_params((16, 16, 16, 16))
    assert p.smoother_s == t["smoother_s"] and p.inner_tol == t["inner_tol"]
    assert p.inner_maxiter == t["inner_maxiter"]
    assert p.setup_maxiter[0] == t["setup_maxiter"] and p.setup_tol[0] == t["setup_tol"]
    assert p.setup_maxiter[1] == t["setup_maxiter"] and p.setup_tol[1] == t["setup_tol"]
    assert p.coarsest_maxiter == t["coarsest_basis"]
    assert list(p.nvec) == [t["nvec_level1"], t["nvec_level2"]]
    assert abs(p.c1 - 9 / 8) < 1e-15 and abs(p.c3 + 1 / 24) < 1e-15
    assert p.coarse_op == (1 if t["coarse_preconditioned"] else 0)
    assert p.coarsest_solver == (1 if "CA-GCR" in t["coarsest_solver"] else 0)
    assert p.coarsest_maxiter == 16 and p.coarsest_restarts == 1


@pytest.mark.parametrize("bad,why", [
    (dict(dims=(5, 4, 4, 4)), "even"),
    (dict(dims=(2, 4, 4, 4)), "even"),
    (dict(nagg=3), "nagg"),
    (dict(block=[(3, 4, 4, 4), (2, 2, 2, 2)]), "block"),
    (dict(block=[(2, 2, 2, 2), (2, 2, 2, 2)]), "Naik"),
    (dict(nvec=(200, 96)), "nvec"),
    (dict(c3=0.0, nvec=(64, 96), block=[(2, 2, 2, 4), (2, 2, 2, 2)]), "rows"),
    (dict(smoother_s=9), "smoother_s"),
    (dict(inner_maxiter=0), "inner_maxiter"),
    (dict(fine_prec=7), "fine_prec"),
    (dict(mass0=0.0), "mass0"),
    (dict(coarsest_deflate=20), "coarsest_deflate"),
    (dict(coarsest_deflate=80), "coarsest_deflate"),
    (dict(coarsest_deflate=16, deflate_maxiter=0), "deflate_maxiter"),
    (dict(deflate_import=2), "deflate_import"),
    (dict(coarse_op=2), "coarse_op"),
    (dict(coarsest_solver=3), "coarsest_solver"),
    (dict(dims=(32, 32, 32, 32), coarsest_solver=2), "8192"),
    (dict(coarsest_solver=2, coarsest_deflate=16), "iterative"),
    (dict(graph_coarsest=2), "graph_coarsest"),
    (dict(compact_masses=5), "compact_masses"),
    (dict(coarse_shadow=3), "coarse_shadow"),
    (dict(cgne_start_import=2), "cgne_start_import"),
    (dict(dims=(8, 8, 8, 8), nvec=(8, 8), coarsest_deflate=32), "dimension"),
])
def test_workspace_validation(m, bad, why):
    bad = dict(bad)
    dims = bad.pop("dims", (16, 16, 16, 16))
    p = m.default_params(dims, **bad)
    with pytest.raises(m.MGError) as e:
        m.workspace_bytes(p)
    assert e.value.status == m.MG_E_CONFIG
    assert why.lower() in str(e.value).lower()


def test_deflation_workspace(m):
    """Deflation vectors add persistent storage (FP64 vectors, Q and W' in the
    coarse precision) and set-up scratch for their CGNE."""
    base = m.workspace_bytes(m.default_params((32, 32, 32, 32)))
    p = m.default_params((32, 32, 32, 32), coarsest_deflate=64)
    pd, sd = m.workspace_bytes(p)
    n = 4 ** 4 * 2 * 96                      # coarsest level of the default 32^4 hierarchy
    assert pd - base[0] >= 64 * n * (16 + 8 + 8)
    assert sd >= base[1]


def test_workspace_sizes_scale(m):
    small = m.workspace_bytes(m.default_params((16, 16, 16, 16)))
    big = m.workspace_bytes(m.default_params((32, 32, 32, 32)))
    assert 15 < big[0] / small[0] < 17   # persistent state is proportional to the volume
    naive = m.default_params((4, 4, 4, 4), c1=1.0, c3=0.0, nagg=1, block=[(2, 2, 2, 2)], nvec=(24,))
    pb, sb = m.workspace_bytes(naive)
    assert pb > 0 and sb > 0


def test_profile_entry_points_validate(m):
    """The kernel-timing entry points reject a null context and null outputs
    before touching any device state."""
    n = ctypes.c_int32()
    ms = ctypes.c_double()
    assert m.LIB.mg_profile_start(None, m.MG_PROF_COARSE, 2, 0) == m.MG_E_ARG
    assert m.LIB.mg_profile_stop(None, ctypes.byref(n), ctypes.byref(ms)) == m.MG_E_ARG


def _shell(m, dims=(8, 8, 8, 8), **kw):
    """A Context with its shapes but no device state: the binding's checks run
    before any library call, so they can be exercised on the host."""
    c = object.__new__(m.Context)
    c.ctx = None
    c._init_shapes(m.default_params(dims, **kw))
    return c


def test_binding_rejects_wrong_sizes_and_dtypes(m):
    """The library reads and writes through raw pointers: the binding checks
    dtype and element count of every buffer it hands over (a tensor that
    would make the library run past its end is refused on the host)."""
    import torch
    c = _shell(m, nvec=(8, 8), max_nrhs=4)
    V = 8 ** 4
    fine = torch.zeros((2, 8, 8, 8, 8, 3), dtype=torch.complex128)
    # a solve needs complex128 right-hand sides
    with pytest.raises(TypeError):
        c.solve([0.1], fine.to(torch.complex64))
    # a partial vector
    with pytest.raises(ValueError):
        c.solve([0.1], torch.zeros(3 * V - 3, dtype=torch.complex128))
    with pytest.raises(ValueError):
        c.apply_dslash(0, 0.1, torch.zeros(3 * V + 1, dtype=torch.complex64))
    # real tensors are not vectors
    with pytest.raises(TypeError):
        c.apply_dslash(0, 0.1, torch.zeros(6 * V, dtype=torch.float64))
    # an output of the wrong size or dtype
    with pytest.raises(ValueError):
        c.apply_dslash(0, 0.1, fine, out=torch.zeros((1, 8, 8, 8, 8, 3), dtype=torch.complex128))
    with pytest.raises(TypeError):
        c.apply_dslash(0, 0.1, fine, out=torch.zeros_like(fine, dtype=torch.complex64))
    # coarse vectors: level 2 is 2^4 x 2 x 8 per rhs; level 3 1^4 x 2 x 8
    with pytest.raises(ValueError):
        c.apply_coarse(2, torch.zeros(2 ** 4 * 2 * 8 + 2, dtype=torch.complex64))
    with pytest.raises(ValueError):
        c.apply_coarse(4, torch.zeros(16, dtype=torch.complex64))
    with pytest.raises(ValueError):
        c.restrict(1, torch.zeros(3 * V, dtype=torch.complex64), out=torch.zeros(7, dtype=torch.complex64))
    with pytest.raises(ValueError):
        c.prolong(1, torch.zeros(2 ** 4 * 2 * 8, dtype=torch.complex64), out=torch.zeros(5, dtype=torch.complex64))
    # links: complex128, one full field
    with pytest.raises(TypeError):
        c.update_links(torch.zeros(4 * V * 9, dtype=torch.complex64))
    with pytest.raises(ValueError):
        c.update_links(torch.zeros(4 * V * 9 - 9, dtype=torch.complex128))
    with pytest.raises(TypeError):
        c.solve_backward(0.1, fine.to(torch.complex64))
