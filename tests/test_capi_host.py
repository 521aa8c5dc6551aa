"""Host-side checks of the C ABI: the library loads, exports every function
the header declares, and validates configurations without touching a GPU."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "imexhdg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(imexhdg_[a-z_]+)\s*\(", src)))


def test_header_compiles_as_c99(tmp_path):
    out = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c",
                          HEADER], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr


def test_library_exports_every_declared_symbol():
    from paper_1711_02751_amd import imexhdg as m
    lib = m.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(m.EXPORTS) == names


def test_validation_errors_are_host_only():
    from paper_1711_02751_amd import imexhdg as m
    good = m.default_config(nx=4, ny=3, degree=3, dt=0.01)
    assert m.validate(good) == m.OK
    bad = [dict(degree=0), dict(degree=9), dict(nx=0), dict(dt=0.0), dict(dt=-1.0),
           dict(g=0.0), dict(H=-1.0), dict(Lx=0.0), dict(scheme=7), dict(physics=3),
           dict(krylov_rtol=0.0), dict(refine_rtol=2.0), dict(krylov_max_iter=0),
           dict(check_every=0), dict(precision=9), dict(launch=5),
           dict(trace_guess=2), dict(local_sweeps=4), dict(local_sweeps=-1),
           dict(precision=2, local_sweeps=3), dict(boundary=3), dict(boundary=-1),
           dict(boundary=1, vortex=(1.0, 0.0, float("nan"), 0.0, 0.0)),
           dict(variable_depth=2), dict(variable_depth=1, boundary=1)]
    for kw in bad:
        base = dict(nx=4, ny=3, degree=3, dt=0.01)
        base.update(kw)
        cfg = m.default_config(**base)
        assert m.validate(cfg) == m.E_INVAL, kw
        assert m.load().imexhdg_last_error().decode() != ""


def test_bounded_mesh_sizes_and_ensembles():
    """A bounded mesh's device arrays hold two ghost columns and rows;
    ensembles take periodic members only."""
    import ctypes
    from paper_1711_02751_amd import imexhdg as m
    per = m.default_config(nx=30, ny=30, degree=3)
    bnd = m.default_config(nx=28, ny=28, degree=3, boundary=m.BOUNDARY_VORTEX)
    assert m.validate(bnd) == m.OK
    a, b = m.workspace_bytes(per), m.workspace_bytes(bnd)
    assert abs(a - b) < 0.01 * a
    cfgs = (m.Config * 2)(bnd, bnd)
    n = ctypes.c_size_t(0)
    assert m.load().imexhdg_ens_workspace_bytes(cfgs, 2, ctypes.byref(n)) == m.E_INVAL
    cfgs = (m.Config * 2)(per, per)
    assert m.load().imexhdg_ens_workspace_bytes(cfgs, 2, ctypes.byref(n)) == m.OK


def test_workspace_bytes_scales_with_mesh():
    from paper_1711_02751_amd import imexhdg as m
    a = m.workspace_bytes(m.default_config(nx=64, ny=64, degree=4))
    b = m.workspace_bytes(m.default_config(nx=128, ny=128, degree=4))
    assert 3.5 < b / a < 4.5
    with pytest.raises(m.ImexError):
        m.workspace_bytes(m.default_config(nx=8, ny=8, degree=0))


def test_null_arguments_rejected():
    import ctypes
    from paper_1711_02751_amd import imexhdg as m
    lib = m.load()
    assert lib.imexhdg_validate(None) == m.E_INVAL
    assert lib.imexhdg_create(None, None, None, 0, None) == m.E_INVAL
    assert lib.imexhdg_step(None, 1) == m.E_INVAL
    assert lib.imexhdg_sizes(None, None, None) == m.E_INVAL
    assert lib.imexhdg_get_schedule(None, None, None) == m.E_INVAL
    assert lib.imexhdg_set_schedule(None, 1, None) == m.E_INVAL
    assert lib.imexhdg_set_launch_geometry(None, 1024, 1024) == m.E_INVAL
    assert lib.imexhdg_autotune(None, None, None, None) == m.E_INVAL
    assert lib.imexhdg_ens_create(None, 0, None, None, 0, None) == m.E_INVAL
    assert lib.imexhdg_ens_step(None, 1) == m.E_INVAL
    assert lib.imexhdg_ens_autotune(None, None, None, None) == m.E_INVAL
    assert lib.imexhdg_set_state_device(None, m.VARS_DEPTH, m.DTYPE_F64, None) == m.E_INVAL
    assert lib.imexhdg_ens_set_state_device(None, 0, m.VARS_DEPTH, m.DTYPE_F64, None) == m.E_INVAL
    d = m.Diag()
    assert lib.imexhdg_get_diag(None, ctypes.byref(d)) == m.E_INVAL
    lib.imexhdg_ens_destroy(None)
    lib.imexhdg_destroy(None)
