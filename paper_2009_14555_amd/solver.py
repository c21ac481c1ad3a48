"""Grid solver object: device state in torch tensors, every step in HIP.

    g = Grid(problem)                 # C-ABI handle, two state buffers on cuda
    g.set_primitive(W)                # numpy/torch primitive fields -> conserved
    g.advance(dt)                     # one full step (sweeps + sources + wave speed)
    g.max_wavespeed()                 # per-direction max |u_d| + c_L (syncs)
    g.state                           # the current conserved state (F, *shape)

    ps = PatchSet(template, sizes)    # independent 2-D patches with 2 ghost layers
    ps.set_primitive(list_of_W)       # interior primitive fields per patch
    ps.advance_graph(nsteps)          # pairs of steps replayed from a HIP graph
    ps.patch(p)                       # conserved state of patch p (F, ny+4, nx+4)
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import dimp as _d
from . import problems as _p


class Grid:
    def __init__(self, pb: _p.Problem, device: str = "cuda", stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the diffuse-interface solver needs a ROCm GPU (no CPU path)")
        self.pb = pb
        self.device = torch.device(device)
        h = C.c_void_p()
        n = (C.c_int64 * 3)(*[int(pb.n[d]) if d < pb.ndim else 1 for d in range(3)])
        dx = (C.c_double * 3)(*[float(pb.dx[d]) for d in range(3)])
        bc = (C.c_int32 * 3)(*[int(pb.bc[d]) for d in range(3)])
        _d.call("dimp_create_grid", pb.ndim, n, dx, bc, C.byref(h))
        self.h = h
        mats = (_d.dimp_material * pb.nmat)(*[_d.material(m) for m in pb.materials])
        rx = _d.reactive(pb.reactive)
        _d.call("dimp_set_materials", h, pb.nmat, mats, C.byref(rx))
        opt = _d.options(pb)
        _d.call("dimp_set_options", h, C.byref(opt))
        if getattr(pb, "geom", 0):
            _d.call("dimp_set_geometry", h, int(pb.geom), float(pb.lo[0]))
        nf, nc = C.c_int(), C.c_int64()
        _d.call("dimp_nfields", h, C.byref(nf), C.byref(nc))
        self.F, self.ncell = nf.value, nc.value
        shape = (self.F,) + pb.shape
        with torch.cuda.device(self.device):
            self.bufs = [torch.zeros(shape, dtype=torch.float64, device=self.device) for _ in range(2)]
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws_purposes = 0
        self._bind(0)

    def _bind(self, purposes: int) -> None:
        """bind the state buffers with a workspace for `purposes` (torch
        allocates it; the library allocates no device memory after this)"""
        nb = C.c_size_t()
        _d.call("dimp_workspace_bytes", self.h, int(purposes), C.byref(nb))
        with torch.cuda.device(self.device):
            ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        if ws.data_ptr() % 256:
            raise RuntimeError("the workspace must be 256-byte aligned")
        _d.call("dimp_bind", self.h, C.c_void_p(self.bufs[0].data_ptr()), C.c_void_p(self.bufs[1].data_ptr()),
                C.c_void_p(ws.data_ptr()), nb, int(purposes), C.c_void_p(self.stream.cuda_stream))
        self.ws = ws
        self.ws_purposes = int(purposes)

    def ensure_workspace(self, purposes: int) -> None:
        """rebind with a workspace that also serves `purposes` (WS_RK3,
        WS_ADJOINT); the state stays (its buffer becomes buffer 0)"""
        if (self.ws_purposes & purposes) == purposes:
            return
        cur = self.current()
        self.stream.synchronize()  # the old workspace is released below
        if cur == 1:
            self.bufs = [self.bufs[1], self.bufs[0]]
        self._bind(self.ws_purposes | purposes)

    def set_materials(self, materials, reactive=None) -> None:
        """replace the materials (same count and reactive setting)"""
        mats = (_d.dimp_material * len(materials))(*[_d.material(m) for m in materials])
        rx = _d.reactive(self.pb.reactive if reactive is None else reactive)
        _d.call("dimp_set_materials", self.h, len(materials), mats, C.byref(rx))
        self.pb = self.pb.replace(materials=list(materials))

    def close(self):
        if getattr(self, "h", None):
            _d.lib.dimp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ state
    @property
    def state(self) -> torch.Tensor:
        return self.bufs[self.current()]

    @property
    def other(self) -> torch.Tensor:
        """the bound buffer that does not hold the state (after a 2-D split
        step on a Cartesian single grid: the step's first sweep)"""
        return self.bufs[1 - self.current()]

    def current(self) -> int:
        """index of the bound buffer that holds the state"""
        w = C.c_int()
        _d.call("dimp_current", self.h, C.byref(w))
        return w.value

    def _dev(self, a) -> torch.Tensor:
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        a = a.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(a.shape) != (self.F,) + self.pb.shape:
            raise ValueError(f"expected shape {(self.F,) + self.pb.shape}, got {tuple(a.shape)}")
        return a

    def set_primitive(self, W) -> None:
        Wd = self._dev(W)
        _d.call("dimp_prim_to_cons", self.h, C.c_void_p(Wd.data_ptr()))
        self._keep = Wd  # alive until the conversion has run on the stream

    def set_conserved(self, U) -> None:
        Ud = self._dev(U)
        _d.call("dimp_set_conserved", self.h, C.c_void_p(Ud.data_ptr()))
        self._keep = Ud  # alive until the copy has run on the stream

    def primitive(self) -> torch.Tensor:
        out = torch.empty_like(self.state)
        _d.call("dimp_cons_to_prim", self.h, C.c_void_p(out.data_ptr()))
        return out

    # -------------------------------------------------------------- step
    def advance(self, dt: float) -> None:
        _d.call("dimp_advance", self.h, float(dt))

    def advance_cfl(self, nsteps: int = 1, cfl: float | None = None, dt_log: torch.Tensor | None = None) -> None:
        """nsteps steps with the CFL time step computed on the device"""
        cfl = self.pb.cfl if cfl is None else cfl
        ptr = C.c_void_p(dt_log.data_ptr()) if dt_log is not None else None
        _d.call("dimp_advance_cfl", self.h, float(cfl), int(nsteps), ptr)

    def sweep(self, dt: float, d: int) -> None:
        _d.call("dimp_sweep", self.h, float(dt), int(d))

    def sources(self, dt: float) -> None:
        _d.call("dimp_sources", self.h, float(dt))

    def set_step_index(self, k: int) -> None:
        _d.call("dimp_set_step_index", self.h, int(k))

    def set_integrator(self, name: str) -> None:
        """'split' (dimensionally split MUSCL-Hancock, the default) or 'rk3'
        (the unsplit operator with the SSP-RK3 of Sec. 3.1)"""
        kinds = {"split": _d.INTEGRATOR_SPLIT, "rk3": _d.INTEGRATOR_RK3}
        if name not in kinds:
            raise ValueError(f"integrator must be one of {sorted(kinds)}")
        if name == "rk3":
            self.ensure_workspace(_d.WS_RK3)
        _d.call("dimp_set_integrator", self.h, kinds[name])

    def max_wavespeed(self) -> np.ndarray:
        s = (C.c_double * 3)()
        _d.call("dimp_max_wavespeed", self.h, s)
        return np.array(s[: self.pb.ndim])

    def max_wavespeed_device(self, out: torch.Tensor) -> None:
        _d.call("dimp_max_wavespeed_device", self.h, C.c_void_p(out.data_ptr()))

    def dt_cfl(self, cfl: float | None = None) -> float:
        cfl = self.pb.cfl if cfl is None else cfl
        s = self.max_wavespeed()
        return cfl * min(self.pb.dx[d] / s[d] for d in range(self.pb.ndim))

    def set_kernel_timing(self, on: bool) -> None:
        _d.call("dimp_set_kernel_timing", self.h, 1 if on else 0)

    def kernel_times(self):
        """{(dir, fused): (total_ms, count)} since the last query"""
        ms = (C.c_double * 6)()
        cnt = (C.c_int64 * 6)()
        _d.call("dimp_kernel_times", self.h, ms, cnt)
        return {(k // 2, bool(k % 2)): (ms[k], cnt[k]) for k in range(6) if cnt[k]}

    def advance_graph(self, nsteps: int, cfl: float | None = None) -> None:
        """nsteps steps, pairs of them replayed from a captured HIP graph"""
        cfl = self.pb.cfl if cfl is None else cfl
        _d.call("dimp_advance_graph", self.h, float(cfl), int(nsteps))

    # ------------------------------------------------------------ adjoint
    def _adj_io(self, *arrays):
        self.ensure_workspace(_d.WS_ADJOINT)
        out = []
        for a in arrays:
            t = self._dev(a)
            out.append(t)
        return out

    def adjoint_sweep(self, state_in, adj_out, dt: float, d: int, dparams: torch.Tensor) -> torch.Tensor:
        """dJ/dU before one sweep from dJ/dU after it (dparams accumulates)"""
        U, lo = self._adj_io(state_in, adj_out)
        li = torch.empty_like(lo)
        _d.call("dimp_adjoint_sweep", self.h, float(dt), int(d), C.c_void_p(U.data_ptr()), C.c_void_p(lo.data_ptr()),
                C.c_void_p(li.data_ptr()), C.c_void_p(dparams.data_ptr()))
        self._keep = (U, lo)
        return li

    def adjoint_plastic(self, state_in, adj_out, dparams: torch.Tensor) -> torch.Tensor:
        U, lo = self._adj_io(state_in, adj_out)
        li = torch.empty_like(lo)
        _d.call("dimp_adjoint_plastic", self.h, C.c_void_p(U.data_ptr()), C.c_void_p(lo.data_ptr()),
                C.c_void_p(li.data_ptr()), C.c_void_p(dparams.data_ptr()))
        self._keep = (U, lo)
        return li

    def adjoint_step(self, state_in, adj_out, dt: float, step: int, dparams: torch.Tensor,
                     first_sweep=None) -> torch.Tensor:
        """first_sweep: the step's kept first sweep (dimp_adjoint_step_kept)"""
        U, lo = self._adj_io(state_in, adj_out)
        li = torch.empty_like(lo)
        if first_sweep is None:
            _d.call("dimp_adjoint_step", self.h, float(dt), int(step), C.c_void_p(U.data_ptr()),
                    C.c_void_p(lo.data_ptr()), C.c_void_p(li.data_ptr()), C.c_void_p(dparams.data_ptr()))
            self._keep = (U, lo)
        else:
            U1 = self._dev(first_sweep)
            _d.call("dimp_adjoint_step_kept", self.h, float(dt), int(step), C.c_void_p(U.data_ptr()),
                    C.c_void_p(U1.data_ptr()), C.c_void_p(lo.data_ptr()), C.c_void_p(li.data_ptr()),
                    C.c_void_p(dparams.data_ptr()))
            self._keep = (U, U1, lo)
        return li

    def adjoint_params(self, dparams) -> np.ndarray:
        """(2, 4) array: dJ/d(gamma or Gamma0, p_inf, G0, sigma_Y) per material"""
        raw = np.ascontiguousarray(
            dparams.detach().cpu().numpy() if isinstance(dparams, torch.Tensor) else dparams, dtype=np.float64)
        g = np.zeros(8)
        _d.call("dimp_adjoint_params", self.h, raw.ctypes.data_as(C.POINTER(C.c_double)),
                g.ctypes.data_as(C.POINTER(C.c_double)))
        return g.reshape(2, 4)

    def check_state(self) -> int:
        n = C.c_int64()
        rc = _d.lib.dimp_check_state(self.h, C.byref(n))
        if rc not in (_d.OK, _d.ENONPHYSICAL):
            raise _d.DimpError(rc, "dimp_check_state", _d.lib.dimp_last_error().decode())
        return n.value


GHOST = 2


def patch_offsets(sizes) -> np.ndarray:
    """start of every patch in the stored element order (npatch + 1 entries)"""
    sizes = np.asarray(sizes, dtype=np.int64).reshape(-1, 2)
    return np.concatenate([[0], np.cumsum((sizes[:, 0] + 2 * GHOST) * (sizes[:, 1] + 2 * GHOST))])


def pack_patches(F: int, sizes, prims) -> np.ndarray:
    """global (F, E) array from per-patch interior arrays (F, ny, nx), the
    ghost layers filled with the images of the boundary cells"""
    offs = patch_offsets(sizes)
    out = np.empty((F, int(offs[-1])), dtype=np.float64)
    for p, ((nx, ny), W) in enumerate(zip(np.asarray(sizes).reshape(-1, 2), prims)):
        W = np.asarray(W, dtype=np.float64)
        if W.shape != (F, ny, nx):
            raise ValueError(f"patch {p}: expected shape {(F, int(ny), int(nx))}, got {W.shape}")
        padded = np.pad(W, ((0, 0), (GHOST, GHOST), (GHOST, GHOST)), mode="edge")
        out[:, offs[p]:offs[p + 1]] = padded.reshape(F, -1)
    return out


def patch_problem(pbc, box):
    """the problem of the grid that stores a ratio-2 patch over coarse cells
    [i0, i1) x [j0, j1) of pbc with 4 ghost layers (the sizes dimp_amr_create
    asks for), transmissive at its own edges"""
    i0, j0, i1, j1 = [int(v) for v in box]
    G = 4
    dx = (pbc.dx[0] / 2, pbc.dx[1] / 2, pbc.dx[2])
    lo = (pbc.lo[0] + i0 * pbc.dx[0] - G * dx[0], pbc.lo[1] + j0 * pbc.dx[1] - G * dx[1], pbc.lo[2])
    return pbc.replace(n=(2 * (i1 - i0) + 2 * G, 2 * (j1 - j0) + 2 * G, 1), dx=dx, lo=lo,
                       bc=(_p.BC_TRANSMISSIVE,) * 3)


def patch_prim(pbc, W, box):
    """a patch grid's initial primitive state: every fine cell takes its
    coarse parent's (host arrays)"""
    import numpy as np

    pbf = patch_problem(pbc, box)
    G = 4
    I = np.clip(int(box[0]) + np.floor_divide(np.arange(pbf.n[0]) - G, 2), 0, pbc.n[0] - 1)
    J = np.clip(int(box[1]) + np.floor_divide(np.arange(pbf.n[1]) - G, 2), 0, pbc.n[1] - 1)
    return pbf, np.ascontiguousarray(W[:, J[:, None], I[None, :]])


class Hierarchy:
    """Two-level subcycled refinement (Sec. 3): a coarse Grid and one refined
    patch Grid over coarse cells [i0, i1) x [j0, j1) at ratio 2, stored with 4
    ghost layers (dimp_amr_create states the sizes).  The grids stay usable
    on their own; the hierarchy must be closed before them."""

    def __init__(self, coarse: Grid, fine: Grid, box):
        self.coarse, self.fine = coarse, fine
        h = C.c_void_p()
        b = (C.c_int64 * 4)(*[int(v) for v in box])
        nb = C.c_size_t()
        _d.call("dimp_amr_workspace_bytes", coarse.h, b, C.byref(nb))
        with torch.cuda.device(coarse.device):
            self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=coarse.device)
        _d.call("dimp_amr_create", coarse.h, fine.h, b, C.c_void_p(self.ws.data_ptr()), nb, C.byref(h))
        self.h = h
        self._box = tuple(int(v) for v in box)

    def dt(self, cfl: float | None = None) -> float:
        """fills the fine ghost cells from the coarse level; min(coarse CFL
        step, twice the fine one)"""
        cfl = self.coarse.pb.cfl if cfl is None else cfl
        out = C.c_double()
        _d.call("dimp_amr_dt", self.h, float(cfl), C.byref(out))
        return out.value

    def advance(self, dt: float) -> None:
        """one coarse step of dt with two fine steps of dt/2 (through the
        nested hierarchy when there is one)"""
        _d.call("dimp_amr_advance", self.h, float(dt))

    def nest(self, inner: "Hierarchy") -> None:
        """refine this hierarchy's fine grid with inner (whose coarse grid it
        is): a stack of three or more levels stepped through this one; close
        the outer hierarchy first"""
        _d.call("dimp_amr_nest", self.h, inner.h)
        self.inner = inner

    def group(self, member: "Hierarchy") -> None:
        """step member (a hierarchy over the same coarse grid, its patch
        sharing no coarse cell with the others; touching patches exchange
        their fine data, split integrator only) together with this one: a
        level of several patches, advanced through this hierarchy"""
        _d.call("dimp_amr_group", self.h, member.h)
        self.members = getattr(self, "members", []) + [member]

    def prolong(self) -> None:
        """every fine cell from the current coarse state"""
        _d.call("dimp_amr_prolong", self.h)

    def box(self):
        return tuple(self._box)

    def regrid(self, box) -> "Hierarchy":
        """a hierarchy over a new patch box: a new fine grid whose cells are
        prolonged from the coarse level (which holds the averaged fine
        solution); this hierarchy is closed"""
        i0, j0, i1, j1 = [int(v) for v in box]
        pbf = patch_problem(self.coarse.pb, box)
        fine = Grid(pbf, device=str(self.coarse.device), stream=self.coarse.stream)
        self.close()
        h = Hierarchy(self.coarse, fine, (i0, j0, i1, j1))
        h.prolong()
        return h

    def close(self):
        if getattr(self, "h", None):
            _d.lib.dimp_amr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def amr_tag(grid: Grid, threshold: float):
    """the Sec. 4.2 refinement criterion on a 2-D grid's current state:
    (tags as a uint8 tensor of the field shape, tagged extent (i0, j0, i1,
    j1), all 0 when none)"""
    prim = grid.primitive()
    return amr_tag_prim(grid, prim, threshold)


def amr_tag_prim(grid: Grid, prim: torch.Tensor, threshold: float):
    """the criterion on a given primitive state (device, the grid's layout)"""
    prim = prim.contiguous()
    tags = torch.empty(grid.pb.shape, dtype=torch.uint8, device=grid.device)
    bbox = (C.c_int64 * 4)()
    _d.call("dimp_amr_tag", grid.h, C.c_void_p(prim.data_ptr()), float(threshold), C.c_void_p(tags.data_ptr()),
            bbox)
    return tags, tuple(int(v) for v in bbox)


def cluster_tags(tags, margin: int, n):
    """patch boxes (i0, j0, i1, j1) for a level of several patches from a
    host array of tags (ny, nx): the tags grown by margin cells in each
    direction (a square neighbourhood), one box per 8-connected region of
    the grown set, each kept 3 cells inside the grid, and boxes that touch or
    overlap merged until every two are at least one cell apart (the spacing
    dimp_amr_group asks for); sorted by (j0, i0)"""
    t = np.asarray(tags).astype(bool)
    ny, nx = t.shape
    grown = t.copy()
    for _ in range(int(margin)):  # one cell of the square neighbourhood per pass
        g = grown.copy()
        g[1:, :] |= grown[:-1, :]
        g[:-1, :] |= grown[1:, :]
        grown = g
        g = grown.copy()
        g[:, 1:] |= grown[:, :-1]
        g[:, :-1] |= grown[:, 1:]
        grown = g
    # connected regions: every grown cell repeatedly takes the smallest label
    # of its 3 x 3 neighbourhood until nothing changes
    big = ny * nx
    lab = np.where(grown, np.arange(big).reshape(ny, nx), big)
    while True:
        pad = np.full((ny + 2, nx + 2), big)
        pad[1:-1, 1:-1] = lab
        m = lab.copy()
        for dj in (0, 1, 2):
            for di in (0, 1, 2):
                m = np.minimum(m, pad[dj:dj + ny, di:di + nx])
        m = np.where(grown, m, big)
        if np.array_equal(m, lab):
            break
        lab = m
    boxes = []
    for v in np.unique(lab[grown]):
        jj, ii = np.nonzero(lab == v)
        b = (max(int(ii.min()), 3), max(int(jj.min()), 3), min(int(ii.max()) + 1, n[0] - 3),
             min(int(jj.max()) + 1, n[1] - 3))
        if b[2] > b[0] and b[3] > b[1]:
            boxes.append(b)

    def apart(a, b):
        return a[2] < b[0] or b[2] < a[0] or a[3] < b[1] or b[3] < a[1]

    done = False
    while not done:
        done = True
        for x in range(len(boxes)):
            for y in range(x + 1, len(boxes)):
                if not apart(boxes[x], boxes[y]):
                    a, b = boxes[x], boxes.pop(y)
                    boxes[x] = (min(a[0], b[0]), min(a[1], b[1]), max(a[2], b[2]), max(a[3], b[3]))
                    done = False
                    break
            if not done:
                break
    return sorted(boxes, key=lambda b: (b[1], b[0]))


def regrid_patches(coarse: Grid, old, boxes):
    """a level of several patches over new boxes: the old hierarchies (a
    group, head first) are closed, and one new patch grid per box is
    prolonged from the coarse level (which holds the averaged fine solution)
    and grouped under the first; returns the new hierarchies, head first"""
    for h in old:
        h.close()
    hs = []
    for b in boxes:
        fine = Grid(patch_problem(coarse.pb, b), device=str(coarse.device), stream=coarse.stream)
        h = Hierarchy(coarse, fine, b)
        h.prolong()
        hs.append(h)
    for h in hs[1:]:
        hs[0].group(h)
    return hs


class PatchSet(Grid):
    """Independent 2-D patches (interior sizes (npatch, 2) as (nx, ny)) sharing
    the template's materials, options and cell widths; stored with GHOST
    layers around every patch in one structure-of-arrays buffer."""

    def __init__(self, tmpl: _p.Problem, sizes, device: str = "cuda", stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the diffuse-interface solver needs a ROCm GPU (no CPU path)")
        self.pb = tmpl
        self.device = torch.device(device)
        self.sizes = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32).reshape(-1, 2))
        self.npatch = len(self.sizes)
        h = C.c_void_p()
        dx = (C.c_double * 2)(float(tmpl.dx[0]), float(tmpl.dx[1]))
        with torch.cuda.device(self.device):
            _d.call("dimp_create_patch_set", self.npatch,
                    self.sizes.ctypes.data_as(C.POINTER(C.c_int32)), dx, C.byref(h))
        self.h = h
        mats = (_d.dimp_material * tmpl.nmat)(*[_d.material(m) for m in tmpl.materials])
        rx = _d.reactive(tmpl.reactive)
        _d.call("dimp_set_materials", h, tmpl.nmat, mats, C.byref(rx))
        opt = _d.options(tmpl)
        _d.call("dimp_set_options", h, C.byref(opt))
        nf, nc = C.c_int(), C.c_int64()
        _d.call("dimp_nfields", h, C.byref(nf), C.byref(nc))
        self.F, self.ncell = nf.value, nc.value
        offs = (C.c_int64 * (self.npatch + 1))()
        _d.call("dimp_patch_offsets", h, offs)
        self.offsets = np.array(offs[:], dtype=np.int64)
        if not np.array_equal(self.offsets, patch_offsets(self.sizes)):
            raise RuntimeError("patch offsets of the library and of the binding disagree")
        with torch.cuda.device(self.device):
            self.bufs = [torch.zeros((self.F, self.ncell), dtype=torch.float64, device=self.device) for _ in range(2)]
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws_purposes = 0
        self._bind(0)

    @property
    def interior_cells(self) -> int:
        return int(np.sum(self.sizes[:, 0].astype(np.int64) * self.sizes[:, 1]))

    def pack(self, prims) -> np.ndarray:
        return pack_patches(self.F, self.sizes, prims)

    def _dev(self, a) -> torch.Tensor:
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        a = a.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(a.shape) != (self.F, self.ncell):
            raise ValueError(f"expected shape {(self.F, self.ncell)}, got {tuple(a.shape)}")
        return a

    def set_primitive(self, prims) -> None:
        if isinstance(prims, (list, tuple)):
            prims = self.pack(prims)
        super().set_primitive(prims)

    def patch(self, p: int, interior: bool = False) -> torch.Tensor:
        nx, ny = (int(v) for v in self.sizes[p])
        a = self.state[:, self.offsets[p]:self.offsets[p + 1]].reshape(self.F, ny + 2 * GHOST, nx + 2 * GHOST)
        return a[:, GHOST:-GHOST, GHOST:-GHOST] if interior else a

    def set_launch(self, per_patch: bool = False, row_waves: int = 4, tile_columns: int = 4) -> None:
        _d.call("dimp_set_patch_launch", self.h, int(per_patch), int(row_waves), int(tile_columns))

    def autotune(self, nsteps: int = 2, cfl: float | None = None):
        cfl = self.pb.cfl if cfl is None else cfl
        best = (C.c_int * 2)()
        snap = torch.empty_like(self.state)
        _d.call("dimp_autotune", self.h, int(nsteps), float(cfl), C.c_void_p(snap.data_ptr()), best)
        return tuple(best)
