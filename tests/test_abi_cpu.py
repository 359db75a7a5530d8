"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/tomg.h declares, and its host-only calls (configuration,
level count, workspace sizing) behave as documented."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tomg.h")
LIB = os.path.join(ROOT, "paper_2602_01888_amd", "libtomg.so")


def header_text():
    """The header without preprocessor lines (macros are not declarations)."""
    return re.sub(r"^[ \t]*#.*$", "", open(HEADER).read(), flags=re.M)


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", header_text(), flags=re.S)
    names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\([^;{]*\)\s*;", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtomg.so is not built (run __graft_entry__.build())")
    from paper_2602_01888_amd import _lib
    return _lib.load(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("setup_coeffs", "vcycle", "solve", "residual_norm", "tomg_workspace_bytes",
              "tomg_create", "tomg_destroy", "tomg_solve_batch"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2602_01888_amd import _lib
    names = declared_functions()
    assert sorted(_lib.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n), n


def test_missing_library_fails_loudly(tmp_path):
    from paper_2602_01888_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            _lib.load(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved


def cfg(nx, ny, dx=None, dy=None, **kw):
    import paper_2602_01888_amd as t
    return t.make_config(nx, ny, dx or 1.0 / (nx - 1), dy or 1.0 / (ny - 1), **kw)


def test_levels_and_workspace(lib):
    import paper_2602_01888_amd as t
    assert t.num_levels(cfg(129, 129)) == 5
    assert t.num_levels(cfg(4097, 4097)) == 10
    assert t.num_levels(cfg(129, 65)) == 5
    # the 201 x 201 grid of Section 4.1 stops halving at 26 x 26 (a large
    # coarsest level, inverted through a band LU); 1001 would stop at 126 x 126
    assert t.num_levels(cfg(201, 201)) == 4
    assert t.workspace_bytes(cfg(201, 201)) > 0
    assert t.num_levels(cfg(1001, 1001)) == 0
    assert t.workspace_bytes(cfg(1001, 1001)) == 0
    w64 = t.workspace_bytes(cfg(4097, 4097))
    w32 = t.workspace_bytes(cfg(4097, 4097, precision="fp32_ir"))
    n = 4097 * 4097
    # level 0: 6 double fields + flags; coarse levels about 11/3 doubles per fine node
    assert 6 * 8 * n < w64 < (6 * 8 + 1 + 40) * n
    assert w32 > w64 + 5 * 4 * n
    assert t.workspace_bytes(cfg(129, 129)) % 256 == 0


@pytest.mark.parametrize("kw", [dict(nu1=0, nu2=0), dict(nu1=5), dict(smoother="jacobi",
                                                                          jacobi_omega=1.5),
                                dict(precision="fp32_ir", ir_inner_cycles=0)])
def test_invalid_configs_size_to_zero(lib, kw):
    import paper_2602_01888_amd as t
    assert t.workspace_bytes(cfg(65, 65, **kw)) == 0


def test_stored_stencil_mixed_precision_configs(lib):
    """Neumann edges and the flux form keep the level-0 stencil stored; with
    FP32 inner cycles an FP32 copy of it is added.  Every smoother but the
    alternating zebra (whose transposed levels are FP64 only) takes that
    combination."""
    import paper_2602_01888_amd as t
    n = 4097 * 4097
    w64 = t.workspace_bytes(cfg(4097, 4097, neumann=t.TOMG_NEU_S))
    w32 = t.workspace_bytes(cfg(4097, 4097, neumann=t.TOMG_NEU_S, precision="fp32_ir"))
    w32d = t.workspace_bytes(cfg(4097, 4097, precision="fp32_ir"))
    w64d = t.workspace_bytes(cfg(4097, 4097))
    assert w64 - w64d >= 9 * 8 * n
    assert w32 - w32d >= 9 * 8 * n + 9 * 4 * n
    assert t.workspace_bytes(cfg(129, 129, flux=True, precision="fp32_ir")) > 0
    for sm in ("jacobi", "zebra_x"):
        assert t.workspace_bytes(cfg(129, 129, flux=True, precision="fp32_ir", smoother=sm)) > 0
        assert t.workspace_bytes(cfg(129, 129, neumann=1, precision="fp32_ir", smoother=sm)) > 0
    assert t.workspace_bytes(cfg(129, 129, flux=True, precision="fp32_ir",
                                 smoother="zebra_xy")) == 0
    assert t.workspace_bytes(cfg(129, 129, neumann=1, precision="fp32_ir",
                                 smoother="zebra_xy")) == 0


def test_create_rejects_bad_arguments_before_touching_the_device(lib):
    """NULL workspace, misaligned workspace and undersized workspace are
    rejected by host checks alone."""
    import paper_2602_01888_amd as t
    c = cfg(65, 65)
    need = t.workspace_bytes(c)
    h = C.c_void_p()
    assert lib.tomg_create(C.byref(c), None, need, None, C.byref(h)) == t.TOMG_EINVAL
    assert lib.tomg_create(C.byref(c), C.c_void_p(0x1000 + 8), need, None,
                           C.byref(h)) == t.TOMG_EINVAL
    assert lib.tomg_create(C.byref(c), C.c_void_p(0x100000), need - 256, None,
                           C.byref(h)) == t.TOMG_ENOMEM
    bad = cfg(66, 65)
    assert lib.tomg_create(C.byref(bad), C.c_void_p(0x100000), 1 << 30, None,
                           C.byref(h)) == t.TOMG_EINVAL
    assert h.value is None


def test_null_problem_calls(lib):
    import paper_2602_01888_amd as t
    assert lib.setup_coeffs(None, None, None, None, None, None, None) == t.TOMG_EINVAL
    assert lib.vcycle(None, None) == t.TOMG_EINVAL
    assert lib.solve(None, None, 1e-10, 10, None, None) == t.TOMG_EINVAL
    assert lib.residual_norm(None, None, None, None) == t.TOMG_EINVAL
    assert lib.tomg_last_error(None) == b"null problem"


# Declarations that carry out a step of the paper's method; each must cite
# the passage (section or equation) that defines it.
PAPER_CALLS = ["setup_coeffs", "tomg_setup_coeffs_async", "tomg_update_rhs", "vcycle", "solve",
               "residual_norm", "tomg_solve_batch", "tomg_batch_step", "tomg_batch_launch",
               "tomg_laplace_grid", "tomg_field", "tomg_setup_coeffs_desc",
               "tomg_update_rhs_desc", "tomg_residual_history"]


def declaration_comments():
    """name -> the comment block written directly above its declaration."""
    text = header_text()
    out = {}
    for m in re.finditer(r"/\*((?:(?!\*/).)*)\*/\s*\n([^/;{}]*?)\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;",
                         text, flags=re.S):
        out[m.group(3)] = m.group(1)
    return out


def test_every_declaration_is_documented():
    docs = declaration_comments()
    for name in declared_functions():
        assert name in docs and len(docs[name].split()) >= 5, name


@pytest.mark.parametrize("name", PAPER_CALLS)
def test_paper_calls_cite_their_passage(name):
    doc = declaration_comments()[name]
    assert re.search(r"\b(Section \d|eq\. \d)", doc), f"{name} cites no passage"


def test_coarse_operator_options(lib):
    """coarse_op: the Galerkin product (default) or rediscretisation, which
    applies eq. 18 on every level and so needs Dirichlet edges and the eq. 18
    form; the workspace is the same either way."""
    import paper_2602_01888_amd as t
    g = t.workspace_bytes(cfg(129, 129))
    assert t.workspace_bytes(cfg(129, 129, coarse_op="rediscretize")) == g
    assert t.workspace_bytes(cfg(129, 129, coarse_op="rediscretize", precision="fp32_ir")) > g
    assert t.workspace_bytes(cfg(129, 129, coarse_op="rediscretize", neumann=1)) == 0
    assert t.workspace_bytes(cfg(129, 129, coarse_op="rediscretize", flux=True)) == 0
    assert t.workspace_bytes(cfg(129, 129, coarse_op="rediscretize", smoother="zebra_xy")) == 0
    c = cfg(129, 129)
    c.coarse_op = 2
    assert t.workspace_bytes(c) == 0


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of tomg_config, tomg_map_desc and tomg_source_desc
    have the C compiler's size and field offsets for include/tomg.h."""
    import shutil
    import subprocess
    from paper_2602_01888_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"tomg_config": _lib.Config, "tomg_map_desc": _lib.MapDesc,
               "tomg_source_desc": _lib.SourceDesc}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "tomg.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True,
                                                      capture_output=True,
                                                      text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[f"{cname} size"]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname} {f}"]) == getattr(py, f).offset, (cname, f)


def test_descriptor_calls_reject_bad_descriptors_on_the_host(lib):
    """NULL problem handles are rejected before any descriptor is read."""
    import paper_2602_01888_amd as t
    m = t.map_desc("circle", r_in=0.15, r_c=0.2, r_out=0.35)
    s = t.source_desc([1.0], [(0.5, 0.5)], 0.02)
    assert lib.tomg_setup_coeffs_desc(None, C.byref(m), C.byref(s), None, 0) == t.TOMG_EINVAL
    assert lib.tomg_update_rhs_desc(None, C.byref(s)) == t.TOMG_EINVAL
    with pytest.raises(t.TomgError):
        t.source_desc([1.0] * 17, [(0.5, 0.5)] * 17, 0.02)


def test_semi_coarsening_options(lib):
    """semi_levels / semi_axis: the level shapes are the oracle's (the first
    coarsenings halve one axis only); semi-coarsening needs the four-colour
    smoother and Galerkin operators, and a requested semi-coarsening that
    cannot be made refuses the grid."""
    import oracle
    import paper_2602_01888_amd as t
    for n, neu, semi, axis in ((4097, 12, 2, "x"), (257, 0, 1, "y"), (129, 0, 3, "x"),
                               (65, 3, 2, "y")):
        c = cfg(n, n, neumann=neu, semi_levels=semi, semi_axis=axis)
        want = oracle.levels(n, n, neumann=neu, semi=semi, semi_axis=0 if axis == "x" else 1)
        assert t.num_levels(c) == len(want) > 0
        assert t.workspace_bytes(c) > t.workspace_bytes(cfg(n, n, neumann=neu)) or n == 129
    assert t.workspace_bytes(cfg(129, 129, semi_levels=1, smoother="zebra_x")) == 0
    assert t.workspace_bytes(cfg(129, 129, semi_levels=1, smoother="jacobi")) == 0
    assert t.workspace_bytes(cfg(129, 129, semi_levels=1, coarse_op="rediscretize")) == 0
    assert t.workspace_bytes(cfg(9, 9, semi_levels=3)) == 0
    c = cfg(129, 129, semi_levels=1)
    c.semi_axis = 2
    assert t.workspace_bytes(c) == 0
    c = cfg(129, 129)
    c.semi_levels = -1
    assert t.workspace_bytes(c) == 0
