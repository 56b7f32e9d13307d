"""C ABI without a GPU: the library loads, exports every entry point the header
declares, and its host-side validation and hierarchy logic behave as documented."""
import ctypes
import os
import re

import pytest

import paper_1410_6609_amd as pkg

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "ccmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccmg_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = pkg.lib()
    decl = declared_functions()
    assert len(decl) >= 14
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(pkg.exported_symbols()) == decl


def faces(kinds, values=(0.0,) * 6):
    F = pkg._Face * 6
    return F(*[pkg._Face(k, v) for k, v in zip(kinds, values)])


def create(shape, kinds, h=1.0, **opt):
    L = pkg.lib()
    o = pkg.Options(**opt)._c()
    hd = ctypes.c_void_p()
    rc = L.ccmg_create(ctypes.byref(hd), *shape, h, faces(kinds), ctypes.byref(o), None)
    return rc, hd


ZD = (1, 1, 1, 1, 0, 0)


def test_auto_levels_and_dims():
    L = pkg.lib()
    for shape, want in [((256, 256, 256), 6), ((512, 512, 512), 7), ((32, 32, 32), 3), ((1024, 256, 256), 7)]:
        rc, hd = create(shape, ZD)
        assert rc == 0
        assert L.ccmg_num_levels(hd) == want
        d = (ctypes.c_int * 3)()
        assert L.ccmg_level_dims(hd, want - 1, d) == 0
        assert d[0] * d[1] * d[2] <= 512 * 4
        L.ccmg_destroy(hd)


def test_workspace_size_covers_hierarchy():
    L = pkg.lib()
    rc, hd = create((64, 64, 64), ZD, levels=4)
    assert rc == 0
    n = 64 ** 3
    need = L.ccmg_workspace_bytes(hd)
    # finest b-tilde and ping-pong + three arrays per coarse level, FP64
    assert need >= 8 * (2 * n + 3 * (n // 8 + n // 64 + n // 512))
    rc, hd2 = create((64, 64, 64), ZD, levels=4, precision=pkg.FP32_IR)
    assert rc == 0
    need32 = L.ccmg_workspace_bytes(hd2)
    assert need32 >= 8 * 2 * n + 4 * 3 * (n + n // 8 + n // 64 + n // 512)
    L.ccmg_destroy(hd)
    L.ccmg_destroy(hd2)


@pytest.mark.parametrize("shape,kinds,opt,code", [
    ((30, 32, 32), ZD, dict(levels=3), pkg.E_DIMS),          # 30 not divisible by 4
    ((32, 32, 32), (1,) * 6, {}, pkg.E_SINGULAR),            # all Neumann
    ((32, 32, 32), ZD, dict(nu1=0), pkg.E_ARG),
    ((32, 32, 32), ZD, dict(fuse_sweeps=3), pkg.E_ARG),
    ((256, 256, 256), ZD, dict(levels=2), pkg.E_DIMS),       # coarsest grid too large for one workgroup
    ((32, 32, 32), ZD, dict(precision=7), pkg.E_ARG),
    ((32, 32, 32), ZD, dict(bottom_cells=5000), pkg.E_ARG),
    ((32, 32, 32), (0, 0, 0, 0, 0, 5), {}, pkg.E_ARG),
])
def test_create_rejects(shape, kinds, opt, code):
    rc, _ = create(shape, kinds, **opt)
    assert rc == code
    assert pkg.lib().ccmg_last_error(None)


def test_create_rejects_bad_spacing():
    rc, _ = create((32, 32, 32), ZD, h=0.0)
    assert rc == pkg.E_ARG


def test_calls_without_workspace_fail_cleanly():
    L = pkg.lib()
    rc, hd = create((32, 32, 32), ZD)
    assert rc == 0
    assert L.ccmg_solve(hd, None, None, 1e-10, 10, None) == pkg.E_STATE
    assert L.ccmg_solve_zero(hd, None, None, 1e-10, 10, None) == pkg.E_STATE
    assert L.ccmg_vcycle(hd, None, None, None) == pkg.E_STATE
    assert b"workspace" in L.ccmg_last_error(hd)
    assert L.ccmg_set_face_values(hd, 0, None) == pkg.E_STATE
    assert L.ccmg_vcycles(hd, None, None, 1, None) == pkg.E_STATE
    assert L.ccmg_force_charge_gradient(hd, None, 0, None, None, None, 1.0, 1, 0, 1, 0, None, None, None, None,
                                        1e-10, 10, None) == pkg.E_STATE
    L.ccmg_destroy(hd)


@pytest.mark.parametrize("kinds,opt,code", [
    ((2, 0, 1, 1, 0, 0), {}, pkg.E_ARG),                        # periodic faces must pair
    ((2, 2, 2, 2, 1, 1), {}, pkg.E_SINGULAR),                   # no Dirichlet face
    ((2, 2, 1, 1, 0, 0), dict(precision=pkg.FP32_IR), pkg.E_ARG),
    ((2, 2, 1, 1, 0, 0), {}, pkg.OK),
    ((3, 3, 1, 1, 0, 0), {}, pkg.E_ARG),
])
def test_periodic_face_validation(kinds, opt, code):
    rc, hd = create((32, 32, 32), kinds, **opt)
    assert rc == code
    if rc == 0:
        # the stored-stencil workspace is reserved without asking for variable_eps
        rc0, h0 = create((32, 32, 32), ZD)
        assert pkg.lib().ccmg_workspace_bytes(hd) > pkg.lib().ccmg_workspace_bytes(h0)
        pkg.lib().ccmg_destroy(h0)
        pkg.lib().ccmg_destroy(hd)


def test_variable_permittivity_options():
    rc, _ = create((32, 32, 32), ZD, variable_eps=2)
    assert rc == pkg.E_ARG
    rc, _ = create((32, 32, 32), ZD, variable_eps=1, precision=pkg.FP32_IR)
    assert rc == pkg.E_ARG
    L = pkg.lib()
    rc, h0 = create((64, 64, 64), ZD, levels=4)
    rc1, h1 = create((64, 64, 64), ZD, levels=4, variable_eps=1)
    assert rc == 0 and rc1 == 0
    n = 64 ** 3
    # three face arrays per level
    assert L.ccmg_workspace_bytes(h1) - L.ccmg_workspace_bytes(h0) >= 8 * 3 * (n + n // 8 + n // 64 + n // 512)
    assert L.ccmg_set_permittivity(h1, None) == pkg.E_STATE   # no workspace yet
    L.ccmg_destroy(h0)
    L.ccmg_destroy(h1)


@pytest.mark.parametrize("subsample,mode", [(0, 0), (9, 0), (2, 2), (3, -1)])
def test_subsampled_deposition_rejects_arguments(subsample, mode):
    """Checked before any device access (n = 0 spheres)."""
    L = pkg.lib()
    rc, hd = create((32, 32, 32), ZD)
    assert rc == 0
    assert L.ccmg_deposit_charges_sub(hd, 0, None, None, None, 1.0, subsample, mode, None, None) == pkg.E_ARG
    assert L.ccmg_charge_gradient(hd, 0, None, None, 1.0, subsample, mode, None, None) == pkg.E_ARG
    assert L.ccmg_last_error(hd)
    assert L.ccmg_charge_gradient(hd, -1, None, None, 1.0, 2, 0, None, None) == pkg.E_ARG
    assert L.ccmg_set_face_values(hd, 7, None) == pkg.E_ARG
    L.ccmg_destroy(hd)


def test_defaults():
    o = pkg._Options()
    pkg.lib().ccmg_default_options(ctypes.byref(o))
    assert (o.nu1, o.nu2, o.omega, o.precision, o.levels) == (2, 2, 2.0, 0, 0)
    assert o.cg_rtol == 1e-13
    assert (o.fuse_sweeps, o.bottom_cells, o.variable_eps) == (2, 4096, 0)
    assert o.ir_inner_cycles == 4
    assert o.ir_cg_rtol == 1e-6


def test_static_scratch_solve_rejects_before_device_work():
    """The allocation-free solve checks the workspace size against its static
    scratch, and the solver kinds whose data live in an attached workspace,
    on the host: no device is touched for a rejected call."""
    L = pkg.lib()
    rc, hd = create((512, 512, 512), ZD)
    assert rc == 0 and L.ccmg_workspace_bytes(hd) > (64 << 20)
    rc = L.ccmg_solve_zero_static(hd, None, None, 1e-10, 10, None)
    assert rc == pkg.E_ARG
    assert b"static scratch" in L.ccmg_last_error(hd)
    L.ccmg_destroy(hd)
    rc, hd = create((32, 32, 32), (2, 2, 1, 1, 0, 0))   # periodic x
    assert rc == 0 and L.ccmg_workspace_bytes(hd) <= (64 << 20)
    assert L.ccmg_solve_zero_static(hd, None, None, 1e-10, 10, None) == pkg.E_STATE
    assert b"periodic" in L.ccmg_last_error(hd)
    L.ccmg_destroy(hd)
