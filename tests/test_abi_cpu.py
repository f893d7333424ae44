"""Host-side checks of the C ABI (no GPU needed).

* libaderdg.so loads and exports every function declared in include/aderdg.h,
  include/aderdg2d.h and include/aderdg3d.h;
* the library's host operator tables (an independent C++ construction)
  agree with the oracle's;
* argument validation returns ADERDG_E_INVAL before any device work.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import basis, limiter
from paper_2409_12483_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aderdg.h")
HEADER_2D = os.path.join(ROOT, "include", "aderdg2d.h")
HEADER_3D = os.path.join(ROOT, "include", "aderdg3d.h")
HEADER_LIM = os.path.join(ROOT, "include", "aderdg_lim.h")
HEADER_LIM2D = os.path.join(ROOT, "include", "aderdg_lim2d.h")

pytestmark = pytest.mark.skipif(not os.path.exists(abi.LIBPATH),
                                reason="libaderdg.so not built (run __graft_entry__.build())")


def _declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aderdg_\w+|aderweno_\w+|aderdg[23]d_\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ["aderdg_init", "aderdg_predict", "aderdg_correct", "aderdg_step",
                     "aderweno_step", "aderdg_free"]:
        assert required in names
    assert set(names) == set(abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(abi.LIBPATH)
    for name in (_declared_functions() + _declared_functions(HEADER_2D) + _declared_functions(HEADER_3D)
                 + _declared_functions(HEADER_LIM) + _declared_functions(HEADER_LIM2D)):
        assert hasattr(lib, name), name


def test_2d_header_declares_the_entry_points():
    assert set(_declared_functions(HEADER_2D)) == set(abi.EXPORTS_2D)


@pytest.mark.parametrize("N", range(0, 10))
def test_host_operator_tables_match_oracle(N):
    t = abi.aderdg_operators(N)
    ops = basis.build_operators(N)
    scale = max(1.0, np.abs(ops.ktil).max())
    assert np.allclose(t["xi"], ops.xi, atol=1e-15, rtol=0)
    assert np.allclose(t["w"], ops.w, atol=1e-15, rtol=0)
    assert np.allclose(t["ktil"], ops.ktil, atol=2e-14 * scale, rtol=0)
    assert np.allclose(t["kappa"], ops.kappa, atol=1e-13, rtol=0)
    assert np.allclose(t["Dtil"], ops.Dtil, atol=2e-14 * scale, rtol=0)
    assert np.allclose(t["psi0"], ops.psi0, atol=1e-13, rtol=0)
    assert np.allclose(t["psi1"], ops.psi1, atol=1e-13, rtol=0)
    assert np.allclose(t["P"], ops.P, atol=1e-13, rtol=0)
    if N >= 1:
        assert np.allclose(t["R"], limiter.subcell_R(ops), atol=1e-11, rtol=0)


def _init(pde, cfg):
    lib = abi.load()
    h = ctypes.c_void_p()
    P = (abi.PdeDesc * 1)(pde)
    C = (abi.Config * 1)(cfg)
    return lib.aderdg_init(P, C, 1, None, ctypes.byref(h)), h


@pytest.mark.parametrize("mutate,needle", [
    (lambda p, c: setattr(p, "nvars", 4), "nvars"),
    (lambda p, c: setattr(c, "N", 0), "degree"),
    (lambda p, c: setattr(c, "N", 10), "degree"),
    (lambda p, c: setattr(c, "ncells", 0), "ncells"),
    (lambda p, c: setattr(c, "x1", -1.0), "x1 > x0"),
    (lambda p, c: setattr(c, "cfl", 1.5), "cfl"),
    (lambda p, c: setattr(c, "bc", 1), "periodic"),
    (lambda p, c: setattr(c, "precision", 7), "precision"),
    (lambda p, c: setattr(p, "gamma", 1.0), "gamma"),
    (lambda p, c: setattr(p, "pde", 9), "pde"),
    (lambda p, c: (setattr(c, "scheme", abi.SCHEME_FV), setattr(c, "N", 3)), "WENO"),
    (lambda p, c: (setattr(c, "scheme", abi.SCHEME_FV), setattr(c, "N", 4), setattr(c, "ncells", 5)), "2N+1"),
])
def test_invalid_descriptors_are_rejected(mutate, needle):
    p = abi.pde_desc(abi.PDE_EULER)
    c = abi.config(3, 100)
    mutate(p, c)
    rc, h = _init(p, c)
    assert rc == abi.ADERDG_E_INVAL
    assert h.value is None
    assert needle in abi.aderdg_last_error()


def test_null_arguments_are_rejected():
    lib = abi.load()
    assert lib.aderdg_step(None, None, None, None, None, None, 1) == abi.ADERDG_E_INVAL
    assert lib.aderweno_step(None, None, None, None, None, None, 1) == abi.ADERDG_E_INVAL
    assert lib.aderdg_predict(None, 0, None, 0.0, 0.1, None, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg_correct(None, 0, None, None, 0.0, 0.1, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg_sweep_count(None, 0, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg_free(None) == abi.ADERDG_OK
    with pytest.raises(abi.AderdgError):
        abi.aderdg_operators(10)


def test_config_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors of the C structs have the header's size and field
    offsets: a C program compiled against include/aderdg.h prints them."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = {"aderdg_pde_desc": (abi.PdeDesc, [f for f, _ in abi.PdeDesc._fields_]),
              "aderdg_config": (abi.Config, [f for f, _ in abi.Config._fields_]),
              "aderdg_lim_config": (abi.LimConfig, [f for f, _ in abi.LimConfig._fields_])}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "aderdg.h"', '#include "aderdg_lim.h"',
             "int main(void) {"]
    for st, (_, names) in fields.items():
        lines.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for f in names:
            lines.append(f'  printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st, (cls, names) in fields.items():
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for f in names:
            assert got[(st, f)] == getattr(cls, f).offset, (st, f)


def _init2d(cfg):
    lib = abi.load()
    h = ctypes.c_void_p()
    return lib.aderdg2d_init(ctypes.byref(cfg), None, ctypes.byref(h)), h


@pytest.mark.parametrize("mutate,needle", [
    (lambda c: setattr(c, "N", 0), "N must"),
    (lambda c: setattr(c, "N", 10), "N must"),
    (lambda c: setattr(c, "precision", 3), "precision"),
    (lambda c: setattr(c, "cells_x", 0), "cells_x"),
    (lambda c: setattr(c, "cells_y", -2), "cells_x"),
    (lambda c: (setattr(c, "cells_x", 1 << 16), setattr(c, "cells_y", 1 << 16)), "2^31"),
    (lambda c: setattr(c, "y1", -1.0), "domain"),
    (lambda c: setattr(c, "x1", float("inf")), "domain"),
    (lambda c: setattr(c, "gamma", 0.9), "gamma"),
    (lambda c: setattr(c, "cfl", 0.0), "cfl"),
    (lambda c: setattr(c, "fixed_dt", -1.0), "fixed_dt"),
    (lambda c: setattr(c, "picard_tol", float("nan")), "picard_tol"),
])
def test_invalid_2d_configs_are_rejected(mutate, needle):
    c = abi.config2d(3, 8, 8)
    mutate(c)
    rc, h = _init2d(c)
    assert rc == abi.ADERDG_E_INVAL
    assert h.value is None
    assert needle in abi.aderdg_last_error()


def test_null_2d_arguments_are_rejected():
    lib = abi.load()
    assert lib.aderdg2d_init(None, None, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg2d_step(None, None, None, None, None, None, 1) == abi.ADERDG_E_INVAL
    assert lib.aderdg2d_predict(None, None, 0.0, 0.1, None, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg2d_sweep_count(None, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg2d_free(None) == abi.ADERDG_OK


def test_2d_config_struct_layout_matches_header():
    assert abi.Config2D.cells_x.offset == 8 and abi.Config2D.x0.offset == 24
    assert abi.Config2D.gamma.offset == 56 and abi.Config2D.picard_tol.offset == 80
    assert abi.Config2D.picard_max_iter.offset == 88 and ctypes.sizeof(abi.Config2D) == 96


def test_3d_header_declares_the_entry_points():
    assert set(_declared_functions(HEADER_3D)) == set(abi.EXPORTS_3D)


@pytest.mark.parametrize("mutate,needle", [
    (lambda c: setattr(c, "N", 0), "N must"),
    (lambda c: setattr(c, "N", 10), "N must"),
    (lambda c: (setattr(c, "N", 10), setattr(c, "precision", abi.FP32_PREDICTOR)), "N must"),
    (lambda c: setattr(c, "precision", 2), "precision"),
    (lambda c: setattr(c, "cells_z", 0), "cells_x"),
    (lambda c: (setattr(c, "cells_x", 2048), setattr(c, "cells_y", 2048), setattr(c, "cells_z", 1024)), "2^31"),
    (lambda c: setattr(c, "z1", -1.0), "domain"),
    (lambda c: setattr(c, "gamma", 1.0), "gamma"),
    (lambda c: setattr(c, "cfl", 2.0), "cfl"),
    (lambda c: setattr(c, "fixed_dt", float("nan")), "fixed_dt"),
])
def test_invalid_3d_configs_are_rejected(mutate, needle):
    c = abi.config3d(3, (4, 4, 4))
    mutate(c)
    h = ctypes.c_void_p()
    rc = abi.load().aderdg3d_init(ctypes.byref(c), None, ctypes.byref(h))
    assert rc == abi.ADERDG_E_INVAL and h.value is None
    assert needle in abi.aderdg_last_error()


def test_null_3d_arguments_are_rejected():
    lib = abi.load()
    assert lib.aderdg3d_init(None, None, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg3d_step(None, None, None, None, None, None, 1) == abi.ADERDG_E_INVAL
    assert lib.aderdg3d_predict(None, None, 0.0, 0.1, None, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg3d_sweep_count(None, None) == abi.ADERDG_E_INVAL
    assert lib.aderdg3d_free(None) == abi.ADERDG_OK


def test_3d_config_struct_layout_matches_header():
    assert abi.Config3D.cells_z.offset == 24 and abi.Config3D.x0.offset == 32
    assert abi.Config3D.gamma.offset == 80 and abi.Config3D.picard_max_iter.offset == 112
    assert ctypes.sizeof(abi.Config3D) == 120


def test_noalloc_step_rejects_a_state_beyond_its_static_scratch():
    """The allocation-free entry point checks its size limit on the host, before
    any device call: (64 MiB - 64 KiB) / 8 doubles of state."""
    lib = abi.load()
    limit = ((64 << 20) - (64 << 10)) // 8
    dummy = ctypes.c_void_p(8)          # never dereferenced: the call fails before device work
    for N, C in [(5, limit // 18 + 1), (1, limit // 6 + 1)]:
        rc = lib.aderdg_step_noalloc(ctypes.byref(abi.pde_desc(abi.PDE_EULER)), ctypes.byref(abi.config(N, C)),
                                     dummy, dummy, dummy, dummy, dummy, 1, None)
        assert rc == abi.ADERDG_E_INVAL
        assert "static scratch" in abi.aderdg_last_error()
    rc = lib.aderdg_step_noalloc(ctypes.byref(abi.pde_desc(abi.PDE_EULER)), ctypes.byref(abi.config(2, 10)),
                                 dummy, dummy, dummy, dummy, dummy, -1, None)
    assert rc == abi.ADERDG_E_INVAL


@pytest.mark.parametrize("pde,scheme", [(abi.PDE_EULER, abi.SCHEME_DG), (abi.PDE_SWE, abi.SCHEME_DG),
                                        (abi.PDE_EULER_REACT, abi.SCHEME_FV)])
def test_newton_inner_solver_only_for_dg_with_a_linear_source(pde, scheme):
    rc, _ = _init(abi.pde_desc(pde), abi.config(4, 20, scheme=scheme, inner=abi.INNER_NEWTON))
    assert rc == abi.ADERDG_E_INVAL
    assert "Newton" in abi.aderdg_last_error()


def test_limiter_header_declares_the_entry_points():
    assert set(_declared_functions(HEADER_LIM)) == set(abi.EXPORTS_LIM)
    assert set(_declared_functions(HEADER_LIM2D)) == set(abi.EXPORTS_LIM2D)


def _init_lim(cfg):
    lib = abi.load()
    h = ctypes.c_void_p()
    return lib.aderdg_lim_init(ctypes.byref(cfg), None, ctypes.byref(h)), h


@pytest.mark.parametrize("mutate,needle", [
    (lambda c: setattr(c, "N", 0), "N must"),
    (lambda c: setattr(c, "N", 10), "N must"),
    (lambda c: setattr(c, "bc", 2), "bc must"),
    (lambda c: setattr(c, "ncells", 2), "ncells"),
    (lambda c: setattr(c, "ncells", 2 ** 31 // 19 + 1), "ncells"),
    (lambda c: setattr(c, "x1", -1.0), "domain"),
    (lambda c: setattr(c, "gamma", 0.9), "gamma"),
    (lambda c: setattr(c, "cfl", 0.0), "cfl"),
    (lambda c: setattr(c, "dims", 4), "dims"),
    (lambda c: setattr(c, "picard_tol", float("inf")), "picard_tol"),
    (lambda c: setattr(c, "weno_degree", 3), "weno_degree"),
    (lambda c: setattr(c, "reserved", 1), "reserved"),
])
def test_invalid_limiter_configs_are_rejected(mutate, needle):
    cfg = abi.lim_config(9, 50)
    mutate(cfg)
    rc, h = _init_lim(cfg)
    assert rc == abi.ADERDG_E_INVAL and h.value is None
    assert needle in abi.aderdg_last_error()
    assert abi.load().aderdg_lim_free(None) == abi.ADERDG_OK


@pytest.mark.parametrize("mutate,needle", [
    (lambda c: setattr(c, "N", 0), "N must"),
    (lambda c: setattr(c, "N", 10), "N must"),
    (lambda c: setattr(c, "bc", 2), "bc must"),
    (lambda c: setattr(c, "cells_x", 2), "cells_x"),
    (lambda c: setattr(c, "cells_y", 70000), "cells_x"),
    (lambda c: setattr(c, "y1", -3.0), "domain"),
    (lambda c: setattr(c, "gamma", 1.0), "gamma"),
    (lambda c: setattr(c, "cfl", 1.5), "cfl"),
    (lambda c: setattr(c, "picard_tol", float("nan")), "picard_tol"),
    (lambda c: setattr(c, "reserved", 2), "reserved"),
])
def test_invalid_2d_limiter_configs_are_rejected(mutate, needle):
    cfg = abi.lim2d_config(3, 12, 10)
    mutate(cfg)
    h = ctypes.c_void_p()
    rc = abi.load().aderdg2d_lim_init(ctypes.byref(cfg), None, ctypes.byref(h))
    assert rc == abi.ADERDG_E_INVAL and h.value is None
    assert needle in abi.aderdg_last_error()
    assert abi.load().aderdg2d_lim_free(None) == abi.ADERDG_OK
