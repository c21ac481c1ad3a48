"""The no-allocation step (dimp_advance_static): a handle bound without a
workspace, stepped through the C-ABI with the library's static scratch,
matches dimp_advance on a twin handle bit for bit (state and wave speed),
on two calls in a row on a larger and then a smaller grid, and the
entry point refuses what it cannot serve."""
import ctypes as C

import numpy as np
import pytest

from paper_2009_14555_amd import problems as P

pytestmark = pytest.mark.gpu


def _pair(n, seed):
    import torch

    from paper_2009_14555_amd import dimp as D
    from paper_2009_14555_amd import solver as S

    pb, W = P.shock_disc(n, seed=seed)
    ref = S.Grid(pb)
    ref.set_primitive(W)
    new = S.Grid(pb)
    new.set_primitive(W)
    torch.cuda.synchronize()
    # rebind without a workspace: this handle can only take the static step
    D.call("dimp_bind", new.h, C.c_void_p(new.bufs[0].data_ptr()), C.c_void_p(new.bufs[1].data_ptr()), None, 0, 0,
           C.c_void_p(new.stream.cuda_stream))
    new.ws = None
    return pb, ref, new


def test_static_step_matches_advance():
    import torch

    from paper_2009_14555_amd import dimp as D

    smax = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
    for n, seed in [(96, 1), (40, 2)]:  # a larger grid, then a smaller one
        pb, ref, new = _pair(n, seed)
        assert D.lib.dimp_advance(new.h, 1e-8) == D.ESTATE  # no workspace bound
        for k in range(2):
            dt = ref.dt_cfl()
            ref.advance(dt)
            D.call("dimp_advance_static", new.h, float(dt), C.c_void_p(smax.data_ptr()))
            torch.cuda.synchronize()
            assert torch.equal(new.state, ref.state), (n, k)
            want = ref.max_wavespeed()
            got = smax.cpu().numpy()
            assert np.array_equal(got[:2], want) and got[2] == 0.0, (n, k, got, want)
        ref.close()
        new.close()


def test_static_step_refusals():
    import torch

    from paper_2009_14555_amd import dimp as D
    from paper_2009_14555_amd import solver as S

    pb, W = P.shock_disc(16, seed=0)
    g = S.Grid(pb)
    g.set_primitive(W)
    smax = torch.zeros(3, dtype=torch.float64, device="cuda")
    assert D.lib.dimp_advance_static(g.h, 0.0, C.c_void_p(smax.data_ptr())) == D.EINVAL
    assert D.lib.dimp_advance_static(g.h, 1e-8, None) == D.EINVAL
    g.set_integrator("rk3")
    assert D.lib.dimp_advance_static(g.h, 1e-8, C.c_void_p(smax.data_ptr())) == D.EUNSUPPORTED
    g.close()
    # a grid whose wave-speed slots exceed the static array (not allocated:
    # the size check comes first)
    h = C.c_void_p()
    n = (C.c_int64 * 3)(59, 200000, 1)
    assert D.lib.dimp_create_grid(2, n, (C.c_double * 3)(1e-3, 1e-3, 1.0), (C.c_int32 * 3)(0, 0, 0),
                                  C.byref(h)) == D.OK
    mats = (D.dimp_material * 2)(D.material(P.water_sg()), D.material(P.solid_c2()))
    assert D.lib.dimp_set_materials(h, 2, mats, None) == D.OK
    buf = torch.empty(2, dtype=torch.float64, device="cuda")  # never touched: the call fails first
    assert D.lib.dimp_bind(h, C.c_void_p(buf.data_ptr()), C.c_void_p(buf.data_ptr() + 8), None, 0, 0, None) == D.OK
    assert D.lib.dimp_advance_static(h, 1e-8, C.c_void_p(smax.data_ptr())) == D.EINVAL
    assert b"static scratch" in D.lib.dimp_last_error()
    D.lib.dimp_destroy(h)
