"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU.  No
kernel is launched here."""
import ctypes as C
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dimp.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:dimp_status|const char\*)\s+(dimp_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["dimp_create_grid", "dimp_set_materials", "dimp_bind", "dimp_advance", "dimp_max_wavespeed",
              "dimp_destroy"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2009_14555_amd import dimp as D

    for s in declared_symbols():
        assert hasattr(D.lib, s), s
    assert sorted(D.EXPORTED) == declared_symbols()


def make_grid(D, ndim=2, n=(8, 8, 1), dx=(0.1, 0.1, 0.1), bc=(0, 0, 0)):
    h = C.c_void_p()
    rc = D.lib.dimp_create_grid(ndim, (C.c_int64 * 3)(*n), (C.c_double * 3)(*dx), (C.c_int32 * 3)(*bc),
                                C.byref(h))
    return rc, h


def test_argument_errors():
    from paper_2009_14555_amd import dimp as D
    from paper_2009_14555_amd import problems as P

    assert make_grid(D, ndim=4)[0] == D.EINVAL
    assert make_grid(D, n=(0, 8, 1))[0] == D.EINVAL
    assert make_grid(D, dx=(0.0, 0.1, 0.1))[0] == D.EINVAL
    assert make_grid(D, bc=(7, 0, 0))[0] == D.EINVAL
    assert b"bc" in D.lib.dimp_last_error()
    rc, h = make_grid(D)
    assert rc == D.OK
    try:
        # out of order: advance before materials / bind
        assert D.lib.dimp_advance(h, 1e-6) == D.ESTATE
        mats4 = (D.dimp_material * 4)(*[D.material(P.water_sg())] * 4)
        assert D.lib.dimp_set_materials(h, 4, mats4, None) == D.EUNSUPPORTED  # built for 2 or 3
        assert D.lib.dimp_set_materials(h, 1, mats4, None) == D.EUNSUPPORTED
        assert D.lib.dimp_set_materials(h, 5, mats4, None) == D.EINVAL
        rc3, h3 = make_grid(D, ndim=3)
        assert rc3 == D.OK
        assert D.lib.dimp_set_materials(h3, 3, mats4, None) == D.EUNSUPPORTED  # three on 1-D and 2-D grids
        D.lib.dimp_destroy(h3)
        assert D.lib.dimp_set_materials(h, 3, mats4, None) == D.OK
        nf3 = C.c_int()
        nc3 = C.c_int64()
        assert D.lib.dimp_nfields(h, C.byref(nf3), C.byref(nc3)) == D.OK and nf3.value == 13
        bad = D.material(P.water_sg())
        bad.gamma = 0.5
        mats = (D.dimp_material * 2)(bad, D.material(P.solid_c2()))
        assert D.lib.dimp_set_materials(h, 2, mats, None) == D.EINVAL
        mats = (D.dimp_material * 2)(D.material(P.water_sg()), D.material(P.solid_c2()))
        assert D.lib.dimp_set_materials(h, 2, mats, None) == D.OK
        nf, nc = C.c_int(), C.c_int64()
        assert D.lib.dimp_nfields(h, C.byref(nf), C.byref(nc)) == D.OK
        assert (nf.value, nc.value) == (11, 64)
        assert D.lib.dimp_advance(h, 1e-6) == D.ESTATE  # nothing bound
        assert D.lib.dimp_bind(h, None, None, None, 0, 0, None) == D.EINVAL
        assert D.lib.dimp_bind(h, C.c_void_p(16), C.c_void_p(16), None, 0, 0, None) == D.EINVAL
        # a Romenskii reactive component is valid input but not built
        rx = D.reactive(P.generic_explosive(0))
        rx.reactant = D.material(P.solid_c2())
        assert D.lib.dimp_set_materials(h, 2, mats, C.byref(rx)) == D.EUNSUPPORTED
        o = D.options(P.Problem(ndim=2, n=(8, 8, 1), dx=(1, 1, 1)))
        o.limiter = 9
        assert D.lib.dimp_set_options(h, C.byref(o)) == D.EINVAL
        # refinement entry points: null handles and unbound grids are refused
        # before any device work
        out = C.c_void_p()
        box = (C.c_int64 * 4)(3, 3, 5, 5)
        assert D.lib.dimp_amr_create(None, h, box, C.c_void_p(256), 1 << 20, C.byref(out)) == D.EINVAL
        assert D.lib.dimp_amr_create(h, h, box, C.c_void_p(256), 1 << 20, C.byref(out)) == D.ESTATE  # not bound
        assert D.lib.dimp_amr_nest(None, None) == D.EINVAL
        assert D.lib.dimp_amr_group(None, None) == D.EINVAL
        assert D.lib.dimp_amr_advance(None, 1e-6) == D.EINVAL
        dt = C.c_double()
        assert D.lib.dimp_amr_dt(None, 0.5, C.byref(dt)) == D.EINVAL
        assert D.lib.dimp_amr_destroy(None) == D.OK
    finally:
        assert D.lib.dimp_destroy(h) == D.OK
    assert D.lib.dimp_destroy(None) == D.OK


def test_workspace_query_and_bind_checks():
    """dimp_workspace_bytes: the regions of the caller-owned workspace
    (reduction words, tag extent, wave-speed slots; RK3 stage buffers;
    adjoint buffers), and dimp_bind's refusal of a workspace that is too
    small, misaligned or given for unknown purposes -- all before any device
    work"""
    from paper_2009_14555_amd import dimp as D
    from paper_2009_14555_amd import problems as P

    rc, h = make_grid(D, n=(100, 70, 1))
    assert rc == D.OK
    try:
        nb = C.c_size_t()
        assert D.lib.dimp_workspace_bytes(h, 0, C.byref(nb)) == D.ESTATE  # materials not set
        mats = (D.dimp_material * 2)(D.material(P.water_sg()), D.material(P.solid_c2()))
        assert D.lib.dimp_set_materials(h, 2, mats, None) == D.OK
        assert D.lib.dimp_workspace_bytes(h, 4, C.byref(nb)) == D.EINVAL  # unknown purpose bit
        sizes = {}
        for purposes in (0, D.WS_RK3, D.WS_ADJOINT, D.WS_RK3 | D.WS_ADJOINT):
            assert D.lib.dimp_workspace_bytes(h, purposes, C.byref(nb)) == D.OK
            sizes[purposes] = nb.value
            assert nb.value % 256 == 0
        F, ncell = 11, 100 * 70
        # wave-speed slots: 2 segments of 58 cells x 70 rows (x), 25 tiles of 4
        # columns x 2 segments x 4 waves (y); three doubles each, plus the
        # reduction's first stage (one block) -- after two 256-byte words
        slots = max(2 * 70, 25 * 2 * 4)
        assert sizes[0] == 256 + 256 + -(-(slots + 1) * 3 * 8 // 256) * 256
        rk = sizes[D.WS_RK3] - sizes[0]
        assert rk == -(-2 * F * ncell * 8 // 256) * 256  # two more states in 2-D
        adj = sizes[D.WS_ADJOINT] - sizes[0]
        assert (3 * F + 2) * ncell * 8 <= adj < (3 * F + 2) * ncell * 8 + (1 << 20)
        assert sizes[D.WS_RK3 | D.WS_ADJOINT] == sizes[0] + rk + adj
        # bind refuses before touching the device
        buf0, buf1 = C.c_void_p(1 << 20), C.c_void_p(1 << 21)
        ws = C.c_void_p(1 << 22)
        assert D.lib.dimp_bind(h, buf0, buf1, ws, sizes[0] - 8, 0, None) == D.EINVAL
        assert b"too small" in D.lib.dimp_last_error()
        assert D.lib.dimp_bind(h, buf0, buf1, C.c_void_p((1 << 22) + 8), sizes[0], 0, None) == D.EINVAL
        assert D.lib.dimp_bind(h, buf0, buf1, ws, sizes[D.WS_RK3], 8, None) == D.EINVAL
        assert D.lib.dimp_bind(h, buf0, buf1, None, 0, D.WS_RK3, None) == D.EINVAL
        assert D.lib.dimp_bind(h, buf0, buf1, ws, sizes[0], D.WS_RK3, None) == D.EINVAL
        assert D.lib.dimp_set_integrator(h, D.INTEGRATOR_RK3) == D.OK  # not bound yet
        assert D.lib.dimp_bind(h, buf0, buf1, ws, sizes[0], 0, None) == D.EINVAL  # RK3 needs its region
        assert b"DIMP_WS_RK3" in D.lib.dimp_last_error()
    finally:
        assert D.lib.dimp_destroy(h) == D.OK


def test_no_device_allocation_after_bind():
    """the C-ABI source allocates device memory only where a patch set is
    created (its patch table and work lists, before any bind); every other
    device buffer is the caller's (state buffers, workspace, snapshot,
    hierarchy workspace)"""
    src = open(os.path.join(ROOT, "paper_2009_14555_amd", "csrc", "dimp_capi.cpp")).read()
    funcs = []
    for m in re.finditer(r"\bhipMalloc\w*\s*\(", src):
        # the enclosing function: the last definition opened before the call
        head = src[:m.start()]
        defs = list(re.finditer(r"^(?:static\s+)?[\w:<>*]+\s+(\w+)\([^;{]*\)\s*\{", head, re.M))
        funcs.append(defs[-1].group(1))
    assert funcs and set(funcs) <= {"upload_list", "dimp_create_patch_set"}, funcs
    for lib_src in ("dimp_kernels.hip", "dimp_sweeps.hpp", "dimp_sweeps3.hip", "dimp_sweeps_n3.hip", "dimp_patches.hpp",
                    "dimp_patches.hip", "dimp_patches_rx.hip", "dimp_patches_n3.hip", "dimp_adjoint.hip", "dimp_amr.hip",
                    "dimp_velocity.hip"):
        text = open(os.path.join(ROOT, "paper_2009_14555_amd", "csrc", lib_src)).read()
        assert "hipMalloc" not in text, lib_src


def test_field_counts_match_layout():
    from paper_2009_14555_amd import dimp as D
    from paper_2009_14555_amd import problems as P

    for ndim, rx, F in [(1, False, 8), (2, False, 11), (3, False, 16), (3, True, 17), (2, True, 12)]:
        rc, h = make_grid(D, ndim=ndim)
        mats = (D.dimp_material * 2)(D.material(P.placeholder_for_reactive()), D.material(P.solid_c2()))
        r = D.reactive(P.generic_explosive(0)) if rx else D.reactive(P.Reactive())
        assert D.lib.dimp_set_materials(h, 2, mats, C.byref(r)) == D.OK
        nf, nc = C.c_int(), C.c_int64()
        D.lib.dimp_nfields(h, C.byref(nf), C.byref(nc))
        pb = P.Problem(ndim=ndim, n=(8, 8, 1), dx=(1, 1, 1), materials=[P.water_sg(), P.solid_c2()],
                       reactive=P.generic_explosive(0) if rx else P.Reactive())
        assert nf.value == F == P.layout(pb).nfields
        D.lib.dimp_destroy(h)


def test_patch_set_host_side():
    from paper_2009_14555_amd import dimp as D

    h = C.c_void_p()
    sizes = np.array([[16, 20], [3, 1], [128, 64]], dtype=np.int32)
    dx = (C.c_double * 2)(0.1, 0.1)
    bad = np.array([[16, 0]], dtype=np.int32)
    assert D.lib.dimp_create_patch_set(1, bad.ctypes.data_as(C.POINTER(C.c_int32)), dx, C.byref(h)) == D.EINVAL
    rc = D.lib.dimp_create_patch_set(3, sizes.ctypes.data_as(C.POINTER(C.c_int32)), dx, C.byref(h))
    if rc == D.EHIP:
        pytest.skip("no HIP device for the task-list upload")
    assert rc == D.OK
    offs = (C.c_int64 * 4)()
    assert D.lib.dimp_patch_offsets(h, offs) == D.OK
    assert list(offs) == [0, 20 * 24, 20 * 24 + 7 * 5, 20 * 24 + 7 * 5 + 132 * 68]
    assert D.lib.dimp_set_patch_launch(h, 0, 4, 5) == D.EINVAL
    assert D.lib.dimp_set_patch_launch(h, 0, 3, 4) == D.EINVAL
    assert D.lib.dimp_set_patch_launch(h, 2, 4, 4) == D.EINVAL
    assert D.lib.dimp_set_patch_launch(h, 1, 2, 8) == D.OK
    D.lib.dimp_destroy(h)


def test_patch_packing_layout():
    from paper_2009_14555_amd import problems as P
    from paper_2009_14555_amd.solver import GHOST, pack_patches, patch_offsets

    tmpl, sizes, prims = P.patch_set(5, seed=4, dx=1.0 / 256)
    F = P.layout(tmpl).nfields
    G = pack_patches(F, sizes, prims)
    offs = patch_offsets(sizes)
    assert G.shape == (F, offs[-1])
    for p, ((nx, ny), W) in enumerate(zip(sizes, prims)):
        blk = G[:, offs[p]:offs[p + 1]].reshape(F, ny + 2 * GHOST, nx + 2 * GHOST)
        assert np.array_equal(blk[:, GHOST:-GHOST, GHOST:-GHOST], W)
        assert np.array_equal(blk[:, 0], blk[:, GHOST]) and np.array_equal(blk[:, -1], blk[:, -1 - GHOST])
        assert np.array_equal(blk[:, :, 0], blk[:, :, GHOST]) and np.array_equal(blk[:, :, -1], blk[:, :, -1 - GHOST])
    with pytest.raises(ValueError):
        pack_patches(F, sizes, [W[:, :-1] for W in prims])
    s = P.patch_sizes(4096, seed=0)
    assert s.min() >= 16 and s.max() <= 128
