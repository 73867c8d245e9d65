"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/fld.h declares, and its pure-host calls (defaults,
workspace sizing, argument validation) behave as documented."""
import ctypes
import os
import re

import pytest

from conftest import ROOT, read_golden

HEADERS = [os.path.join(ROOT, "include", h)
           for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for hdr in HEADERS:
        src = open(hdr).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(fld_[a-z_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def fld():
    import paper_1306_0645_amd as m
    return m


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fld_assemble", "fld_solve", "fld_step", "fld_create",
                 "fld_destroy", "fld_batch_step", "fld_server_submit"):
        assert must in names


def test_library_exports_every_declared_symbol(fld):
    lib = ctypes.CDLL(fld.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(fld.EXPORTS)


def test_default_params_follow_the_paper(fld):
    t1 = read_golden("solver_table1.txt")
    lc = read_golden("limiter_constants.txt")
    c, L = 2.99792458e10, 2.037e22
    p = fld.fld_default_params(c, L)
    assert p.d_max == pytest.approx(float(lc["dmax_factor"]) * c * L, rel=1e-15)
    assert p.r_min == pytest.approx(float(lc["rmin_factor"]) / L, rel=1e-15)
    assert p.tau_tol == float(lc["tau_tol"])
    assert p.rtol == float(t1["cg_tolerance"])
    assert p.max_iter == int(t1["cg_max_iterations"])
    assert p.nu_pre == int(t1["mg_pre_sweeps"])
    assert p.nu_post == int(t1["mg_post_sweeps"])
    assert p.theta == 1.0 and p.precision == fld.FLD_PREC_FP64


def test_workspace_sizing_and_validation(fld):
    p = fld.fld_default_params(1.0, 1.0)
    g = fld.make_grid((32, 32, 32), (1.0, 1.0, 1.0))
    b64 = fld.fld_workspace_bytes(g, p)
    # 7 Krylov vectors + 4 coefficient arrays + E copy on the finest level
    assert b64 >= 12 * 8 * 32 ** 3
    pm = fld.fld_default_params(1.0, 1.0, precision=fld.FLD_PREC_MIXED)
    assert fld.fld_workspace_bytes(g, pm) > b64
    for bad in [(31, 32, 32), (32, 2, 32), (0, 32, 32)]:
        assert fld.fld_workspace_bytes(fld.make_grid(bad, (1, 1, 1)), p) == 0
    assert fld.fld_workspace_bytes(fld.make_grid((8, 8, 8), (1, -1, 1)), p) == 0
    for field, val in [("theta", 0.3), ("c", 0.0), ("nu_pre", 0),
                       ("precision", 7), ("max_iter", 0), ("smoother", 2),
                       ("fused_levels", -1), ("fused_levels", 13)]:
        q = fld.fld_default_params(1.0, 1.0, **{field: val})
        assert fld.fld_workspace_bytes(g, q) == 0, field
    # and carves one more iterate buffer per level; the mixed-precision fused
    # V(1,1) red/black iteration carves a second FP64 residual on the finest
    # level instead
    for prec in (fld.FLD_PREC_FP64, fld.FLD_PREC_MIXED):
        r = fld.fld_default_params(1.0, 1.0, precision=prec, nu_pre=2, nu_post=2)
        j = fld.fld_default_params(1.0, 1.0, precision=prec,
                                   smoother=fld.FLD_SMOOTH_JACOBI)
        assert p.smoother == fld.FLD_SMOOTH_RBGS
        extra = fld.fld_workspace_bytes(g, j) - fld.fld_workspace_bytes(g, r)
        w = 4 if prec == fld.FLD_PREC_MIXED else 8
        assert w * 32 ** 3 <= extra <= w * 32 ** 3 * 8 / 7 + (1 << 16), prec
        f = fld.fld_default_params(1.0, 1.0, precision=prec)
        extra = fld.fld_workspace_bytes(g, f) - fld.fld_workspace_bytes(g, r)
        if prec == fld.FLD_PREC_MIXED:
            # the second residual (FP64)
            assert 8 * 32 ** 3 <= extra <= 8 * 32 ** 3 + (1 << 12), prec
        else:
            assert extra == 0


def test_create_rejects_bad_arguments_before_any_launch(fld):
    lib = fld._lib
    p = fld.fld_default_params(1.0, 1.0)
    h = ctypes.c_void_p()
    bad = fld.make_grid((8, 8, 7), (1, 1, 1))
    assert lib.fld_create(ctypes.byref(bad), ctypes.byref(p), None,
                          ctypes.c_void_p(256), 1 << 30,
                          ctypes.byref(h)) == fld.FLD_EINVAL
    good = fld.make_grid((8, 8, 8), (1, 1, 1))
    # misaligned workspace
    assert lib.fld_create(ctypes.byref(good), ctypes.byref(p), None,
                          ctypes.c_void_p(4096 + 8), 1 << 30,
                          ctypes.byref(h)) == fld.FLD_EINVAL
    # too small
    assert lib.fld_create(ctypes.byref(good), ctypes.byref(p), None,
                          ctypes.c_void_p(4096), 16,
                          ctypes.byref(h)) == fld.FLD_ENOMEM
    assert fld.fld_strerror(fld.FLD_ENOCONV).startswith("linear solve")


def test_chem_defaults_and_validation(fld):
    g = read_golden("test1_parameters.txt")
    p = fld.fld_chem_default_params()
    assert p.alpha_b == float(g["alpha_b_cm3_s"])
    assert p.hnu == pytest.approx(float(g["photon_energy_ev"]) * 1.602176634e-12,
                                  rel=1e-15)
    assert p.sigma == 6.3e-18 and p.substeps == 1 and p.reserved == 0
    grid = fld.make_grid((8, 8, 8), (1.0, 1.0, 1.0))
    n = 8 * 8 * 8 * 8
    # fake, never dereferenced addresses: every call below fails validation
    # before any launch
    E, nh, x, k = (ctypes.c_void_p(0x10000000 + i * 0x100000) for i in range(4))
    upd = fld._lib.fld_chem_h_update

    def call(pp, dt=1.0, ptrs=(E, nh, x, k), gr=grid, a=1.0):
        return upd(ctypes.byref(gr), ctypes.byref(pp), None, *ptrs, dt, a)

    EINVAL = fld.FLD_EINVAL
    assert call(p, ptrs=(None, nh, x, k)) == EINVAL
    assert call(p, ptrs=(E, nh, x, None)) == EINVAL
    assert call(p, dt=-1.0) == EINVAL
    assert call(p, dt=float("nan")) == EINVAL
    assert call(p, a=0.0) == EINVAL
    assert call(p, a=float("inf")) == EINVAL
    for field, bad in (("substeps", 0), ("substeps", 2000000), ("c", 0.0),
                       ("hnu", 0.0), ("sigma", -1.0), ("alpha_b", float("inf")),
                       ("reserved", 1)):
        q = fld.fld_chem_default_params(**{field: bad})
        assert call(q) == EINVAL, field
    # x and kappa overlapping, or x overlapping an input
    assert call(p, ptrs=(E, nh, x, ctypes.c_void_p(x.value + n // 2))) == EINVAL
    assert call(p, ptrs=(E, x, x, k)) == EINVAL
    bad_grid = fld.make_grid((8, 8, 0), (1.0, 1.0, 1.0))
    assert call(p, gr=bad_grid) == EINVAL
    s = fld._lib.fld_chem_ionized_sum
    assert s(ctypes.byref(grid), None, None, x) == EINVAL
    assert s(ctypes.byref(grid), None, x, ctypes.c_void_p(x.value + 8)) == EINVAL


def test_struct_layouts_match_the_header(fld, tmp_path):
    """The ctypes mirrors of fld_grid, fld_params, fld_stats, fld_request and
    fld_result have the size and field offsets the C compiler gives the
    header's structs (a field added on one side only would shift every
    field after it)."""
    import subprocess
    structs = {"fld_grid": fld.Grid, "fld_params": fld.Params, "fld_stats": fld.Stats,
               "fld_request": fld.Request, "fld_result": fld.Result}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fld.h"',
             'int main(void) {']
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
