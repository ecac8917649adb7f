"""C ABI checks that need no GPU: the library loads, exports every entry point declared in
include/vsie.h, and rejects invalid problems before any device work (host-side validation)."""
import os
import re

import numpy as np
import pytest

import vsie_synth as synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vsie.h")).read()
    return sorted(set(re.findall(r"\b(vsie_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def vs():
    from paper_2206_12409_amd import build, vsie
    if not os.path.exists(vsie.LIB_PATH):
        build.build()
    vsie.load()
    return vsie


def test_every_declared_symbol_is_exported(vs):
    lib = vs.load()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(vs.EXPORTED) == names


def test_default_options(vs):
    o = vs.default_options()
    assert o.tt_tol == 1e-3 and o.aca_tol == 1e-3 and o.tt_rank_max == 96 and o.precorrect_dist == 2
    assert o.precision == vs.VSIE_PREC_MIXED and o.basis == vs.VSIE_BASIS_PWC and o.stencil == 5
    assert (o.quad_near_vol, o.quad_near_surf, o.quad_far_vol, o.quad_far_surf) == (8, 5, 1, 1)


@pytest.mark.parametrize("field,value,code", [
    ("basis", 1, 9),            # piecewise-linear basis (Sec. II-B): not built
    ("basis", 7, 1),
    ("stencil", 4, 9),          # pFFT block other than 5x5x5 (Sec. IV-B)
    ("quad_near_vol", 27, 9),   # coupling rules other than 8 x 5 / 1 x 1 (Sec. IV-C)
    ("quad_far_surf", 3, 9),
    ("precision", 2, 1),
    ("tt_tol", 0.0, 1),
])
def test_rejects_unsupported_options(vs, field, value, code):
    """Options outside the built discretisation are refused before any device work."""
    with pytest.raises(vs.VsieError) as e:
        vs.Operator(synth.small_case(), stream=0, **{field: value})
    assert e.value.code == code, str(e.value)


def _expect(vs, problem, code):
    with pytest.raises(vs.VsieError) as e:
        vs.Operator(problem, stream=0)
    assert e.value.code == code, str(e.value)


def test_rejects_non_finite_material(vs):
    p = synth.small_case()
    p.grid.eps_r[0, 0, 0] = np.nan
    _expect(vs, p, 1)


def test_rejects_inconsistent_mesh(vs):
    p = synth.small_case()
    t = p.meshes[1].tris.copy()
    t[0] = t[0][::-1]
    p.meshes[1].tris = t
    _expect(vs, p, 2)


def test_rejects_bad_port_edge(vs):
    p = synth.small_case()
    p.meshes[1].port_edges = np.array([[0, 999 % len(p.meshes[1].verts)]], np.int32)
    p.meshes[1].port_id = np.array([0], np.int32)
    _expect(vs, p, 2)


def test_rejects_rwg_pair_larger_than_stencil(vs):
    """Sec. IV-B: every near RWG pair must fit the 5x5x5 expansion block."""
    p = synth.small_case()
    g = p.grid
    p.grid = synth.Grid(g.n, 1e-3, g.origin * 0.2, g.eps_r, g.sigma, g.labels)
    _expect(vs, p, 3)


def test_rejects_bad_sizes(vs):
    p = synth.small_case()
    p.grid = synth.Grid(p.grid.n, -1.0, p.grid.origin, p.grid.eps_r, p.grid.sigma, p.grid.labels)
    _expect(vs, p, 1)


def test_new_entry_points_reject_bad_arguments(vs):
    """Argument checks of the elimination and dense-solve entry points happen before any device
    work: null handles and invalid sizes give E_ARG; default solve options ask for the
    preconditioner."""
    import ctypes as C
    lib = vs.load()
    vp = C.c_void_p
    dummy = vp(16)   # never dereferenced: every call below fails its argument check first
    assert lib.vsie_schur_setup(None, 1) == 1
    assert lib.vsie_schur_info(None, None, None, None) == 1
    assert lib.vsie_schur_matvec(None, dummy, dummy, None) == 1
    assert lib.vsie_schur_precond(None, dummy, dummy, None) == 1
    assert lib.vsie_dense_lu_solve(-1, dummy, 1, dummy, 1, 1, None) == 1
    assert lib.vsie_dense_lu_solve(4, dummy, 3, dummy, 1, 1, None) == 1     # lda < n
    assert lib.vsie_dense_lu_solve(4, dummy, 4, dummy, 1, 2, None) == 1     # ldb < nrhs
    assert lib.vsie_dense_lu_solve(4, None, 4, dummy, 1, 1, None) == 1
    assert lib.vsie_dense_lu_solve(0, None, 0, None, 0, 0, None) == 0       # empty system: nothing to do
    nmax, rmax = vs.LU_NOALLOC_MAX_N, vs.LU_NOALLOC_MAX_NRHS
    assert lib.vsie_dense_lu_solve_noalloc(nmax + 1, dummy, nmax + 1, dummy, 1, 1, None) == 1
    assert lib.vsie_dense_lu_solve_noalloc(8, dummy, 8, dummy, rmax + 1, rmax + 1, None) == 1
    assert lib.vsie_dense_lu_solve_noalloc(4, dummy, 3, dummy, 1, 1, None) == 1
    assert lib.vsie_dense_lu_solve_noalloc(0, None, 0, None, 0, 0, None) == 0
    o = vs.SolveOpts()
    lib.vsie_default_solve_opts(C.byref(o))
    assert o.precond == 1 and o.method == vs.VSIE_GMRES64 and o.restart == 50 and o.tol == 1e-6
    assert o.reorth == 0.1
    assert lib.vsie_solve(None, C.byref(o), 1, dummy, dummy, None, None) == 1
    ports = (C.c_int32 * 1)(0)
    assert lib.vsie_solve_ports(None, C.byref(o), 1, ports, dummy, None, None) == 1
    assert lib.vsie_rhs(None, 0, 0, dummy, None) == 1
    # checkpoint of the compressed far coupling: null handle or path
    assert lib.vsie_checkpoint_save(None, b"/nonexistent/ckpt") == 1
    assert lib.vsie_checkpoint_load(None, b"/nonexistent/ckpt") == 1
    assert lib.vsie_checkpoint_save(dummy, None) == 1
    assert lib.vsie_checkpoint_load(dummy, None) == 1


def test_binding_structs_match_the_header(vs, tmp_path):
    """Every ctypes mirror in the binding has the size and field offsets that a C compiler gives
    the structs of include/vsie.h (compiled here with gcc against the header itself)."""
    import ctypes as C
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    mirrors = {"vsie_mesh": vs.Mesh, "vsie_problem": vs.ProblemC, "vsie_options": vs.Options,
               "vsie_sizes_t": vs.Sizes, "vsie_solve_opts": vs.SolveOpts, "vsie_solve_stats": vs.SolveStats}
    lines = ['#include <stdio.h>', '#include "vsie.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_noalloc_limits_match_the_header(vs):
    import re as _re
    src = open(os.path.join(ROOT, "include", "vsie.h")).read()
    assert int(_re.search(r"#define VSIE_LU_NOALLOC_MAX_N (\d+)", src).group(1)) == vs.LU_NOALLOC_MAX_N
    assert int(_re.search(r"#define VSIE_LU_NOALLOC_MAX_NRHS (\d+)", src).group(1)) == vs.LU_NOALLOC_MAX_NRHS


def test_binding_rejects_bad_vectors_before_any_call(vs):
    """Operator.matvec and Operator.solve check shape, contiguity, dtype and device of every vector
    (and of a caller-supplied output) before they reach the library, so that a short or strided
    buffer is never handed to a kernel."""
    import torch
    op = vs.Operator.__new__(vs.Operator)
    op._h = None
    op.N = 10
    good = torch.zeros(10, dtype=torch.complex128)
    bad = [torch.zeros(9, dtype=torch.complex128),                  # short
           torch.zeros(20, dtype=torch.complex128)[::2],            # strided
           torch.zeros((2, 3, 10), dtype=torch.complex128),         # wrong rank
           torch.zeros(10, dtype=torch.float64)]                    # real
    for x in bad:
        with pytest.raises((ValueError, TypeError)):
            op.matvec(x)
        with pytest.raises((ValueError, TypeError)):
            op.solve(x)
    with pytest.raises(ValueError):
        op.solve(good.to(torch.complex64))
    # a well-formed host tensor is refused for not being on the device
    with pytest.raises(ValueError):
        op.matvec(good)
    with pytest.raises(ValueError):
        op.solve(good)
    # outputs: shape, dtype and contiguity must match x
    for out in (torch.zeros(9, dtype=torch.complex128), torch.zeros(10, dtype=torch.complex64),
                torch.zeros(20, dtype=torch.complex128)[::2]):
        with pytest.raises(ValueError):
            op.matvec(good, out=out)
