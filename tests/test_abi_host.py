"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point ``include/fe.h`` declares, rejects bad arguments before
touching the device, and its line-search rule matches the scripted cases."""
import os
import subprocess
import sys
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def fe():
    from paper_1508_04596_amd import fe as fe_mod
    fe_mod.lib()
    return fe_mod


def test_library_exports_every_declared_entry_point(fe):
    names = declared_functions()
    assert "fe_jvp" in names and "newton_solve" in names and "serve_submit" in names
    L = fe.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"
    assert set(fe.EXPORTS) <= set(names)


def test_version_and_error_string(fe):
    assert "gfx950" in fe.fe_version()


def test_bad_grid_is_rejected_before_any_device_call(fe):
    import ctypes
    L = fe.lib()
    h = ctypes.c_void_p()
    ph = fe.make_phys()
    for g in (fe.FeGrid(0, 4, 4, 0.1), fe.FeGrid(4, -1, 4, 0.1), fe.FeGrid(4, 4, 4, 0.0)):
        rc = L.fe_problem_create(ctypes.byref(g), ctypes.byref(ph), None, ctypes.byref(h))
        assert rc == fe.FE_EINVAL
        assert "grid" in L.fe_last_error().decode()
    bad = fe.make_phys(Ck=0.0)
    rc = L.fe_problem_create(ctypes.byref(fe.FeGrid(2, 2, 2, 0.5)), ctypes.byref(bad), None,
                             ctypes.byref(h))
    assert rc == fe.FE_EINVAL


def test_solve_option_defaults_through_the_binding(fe):
    """fe_solve_opts_default fills the C struct; reading every field back
    through the ctypes mirror checks that the two layouts agree (a field out of
    place would read another field's bytes)."""
    o = fe.solve_opts()
    want = dict(rtol_newton=1e-8, rtol_lin=1e-5, max_newton=50, restart=60, max_lin=3000,
                n_refine=3, krylov_op_prec=fe.FE_FP64, ls_lambda_min=0.05, verbose=0,
                precond=fe.FE_PC_AUTO, mg_nu=2, mg_omega=0.6, atol_newton=0.0, ramp_steps=0,
                mg_assembled_nodes=-1, mg_nu_post=1, pc_prec=fe.FE_FP64,
                mg_coarse_reuse=2)
    assert [f[0] for f in fe.FeSolveOpts._fields_] == list(want)
    for k, v in want.items():
        assert getattr(o, k) == v, k
    assert fe.solve_opts(pc_prec="fp32").pc_prec == fe.FE_FP32
    assert fe.solve_opts(krylov_op_prec="mixed").krylov_op_prec == fe.FE_FP32


def test_fp32_preconditioner_footprint(fe):
    """An FP32 preconditioner adds the FP32 copies (Krylov vectors z_j, state,
    blocks and the multigrid levels' FP32 vectors) to the footprint, as mixed
    mode does."""
    f64 = fe.fe_solve_footprint_bytes(32, 32, 32, 0.1, fe.solve_opts())
    f32 = fe.fe_solve_footprint_bytes(32, 32, 32, 0.1, fe.solve_opts(pc_prec="fp32"))
    fmx = fe.fe_solve_footprint_bytes(32, 32, 32, 0.1, fe.solve_opts(krylov_op_prec="mixed"))
    assert f64 < f32 == fmx


def test_null_handle_is_rejected(fe):
    L = fe.lib()
    assert L.fe_residual(None, None, None, None, None, None) == fe.FE_EINVAL
    assert L.fe_jvp(None, 0, None, None, None, None, None, None) == fe.FE_EINVAL
    assert L.newton_solve(None, None, None, None, None, None, None) == fe.FE_EINVAL


def test_line_search_rule_on_scripted_norms(fe):
    ls = fe.fe_line_search_lambda
    assert ls(4.0, 1.0, 0.0) == 1.0
    q = lambda l: 2.0 + 5.0 * (l - 0.3) ** 2
    assert ls(q(0), q(0.5), q(1)) == pytest.approx(0.3, rel=1e-14)
    q = lambda l: (l - 3.0) ** 2
    assert ls(q(0), q(0.5), q(1)) == 1.0
    q = lambda l: (l + 1.0) ** 2
    assert ls(q(0), q(0.5), q(1)) == 0.05
    assert ls(1.0, 1.2, 1.3) == 0.5
    assert ls(1.0, 0.98, 0.9) == 1.0


def test_footprint_grows_with_grid_and_restart(fe):
    a = fe.fe_solve_footprint_bytes(16, 16, 16)
    b = fe.fe_solve_footprint_bytes(32, 32, 32)
    assert 0 < a < b
    o = fe.solve_opts(restart=10)
    assert fe.fe_solve_footprint_bytes(32, 32, 32, opts=o) < b


def test_footprint_counts_assembled_levels(fe):
    """32^3: levels 16^3 and 8^3 (4913 and 729 nodes) are assembled by default,
    each holding 675 FP64 stencil entries per node and a second iterate of 5
    values per node for its one-kernel sweeps (plus FP32 copies when mixed)."""
    for prec in ("fp64", "mixed"):
        base = fe.fe_solve_footprint_bytes(32, 32, 32, opts=fe.solve_opts(krylov_op_prec=prec,
                                                                          mg_assembled_nodes=0))
        full = fe.fe_solve_footprint_bytes(32, 32, 32, opts=fe.solve_opts(krylov_op_prec=prec))
        per = 12 if prec == "mixed" else 8
        stencil = per * (675 + 5) * (4913 + 729)
        je = 8 * 1600 * (16 ** 3 - 4 ** 3)  # element Jacobians sized for the 16^3 level
        assert full - base == pytest.approx(stencil + je, abs=4 * 256)


def test_footprint_counts_ramping_buffers(fe):
    """Heat-source ramping keeps the initial vector (FP64 per DOF) and a scaled
    source (FP64 per element)."""
    r = lambda b: (b + 255) // 256 * 256
    a = fe.fe_solve_footprint_bytes(16, 16, 16, opts=fe.solve_opts())
    b = fe.fe_solve_footprint_bytes(16, 16, 16, opts=fe.solve_opts(ramp_steps=3))
    assert b - a == r(8 * 5 * 17 ** 3) + r(8 * 16 ** 3)


def test_product_path_fails_loudly_without_the_hip_library():
    """With the HIP library missing, every product entry point raises instead
    of computing anything on the CPU (there is no fallback path)."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1508_04596_amd import fe, inputs\n"
        "fe.LIB_PATH = '/nonexistent/libfe_hip.so'\n"
        "p = inputs.config(1)\n"
        "calls = [lambda: fe.lib(), lambda: fe.Problem.from_inputs(p, mask='solve'),\n"
        "         lambda: fe.solve_opts(), lambda: fe.fe_solve_footprint_bytes(8, 8, 8)]\n"
        "n = 0\n"
        "for c in calls:\n"
        "    try:\n"
        "        c()\n"
        "    except ImportError:\n"
        "        n += 1\n"
        "print(n)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "4"


def test_product_modules_do_not_import_the_oracle():
    """The oracle is test infrastructure: no module of the package imports it."""
    import re
    pkg = os.path.join(ROOT, "paper_1508_04596_amd")
    for name in sorted(os.listdir(pkg)):
        if name.endswith(".py"):
            src = open(os.path.join(pkg, name)).read()
            assert not re.search(r"^\s*(import|from)\s+oracle\b", src, re.M), name
            assert "libfe_oracle" not in src, name
