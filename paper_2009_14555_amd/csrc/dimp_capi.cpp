// dimp_capi.cpp -- C-ABI of the diffuse-interface step (see include/dimp.h).
//
// Host side only: argument validation, parameter packing, buffer ping-pong
// and kernel launches on the bound stream.  No call synchronises except the
// ones documented to do so (wave speed to host, state check).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dimp.h"
#include "dimp_amr.hpp"
#include "dimp_internal.hpp"

namespace {

thread_local std::string g_err;

dimp_status fail(dimp_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
dimp_status fail(dimp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

dimp_status hip_fail(hipError_t e, const char* what) {
  return fail(DIMP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHECK(call, what)                 \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

}  // namespace

struct dimp_ctx {
  int ndim = 0;
  int64_t n[3] = {1, 1, 1};
  double dx[3] = {1, 1, 1};
  int32_t bc[3] = {0, 0, 0};
  int nmat = 0;
  dimp_material mats[4];
  dimp_reactive rx;
  bool mats_set = false;
  dimp_options opt;
  double* buf[2] = {nullptr, nullptr};
  int cur = 0;
  hipStream_t stream = nullptr;
  bool bound = false;
  // caller-owned workspace (dimp_workspace_bytes / dimp_bind), carved into
  // the regions below; the library allocates no device memory after bind
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  int ws_purposes = 0;
  unsigned long long* dsmax = nullptr;  // [0..2] wave speeds as bit patterns, [3] bad-cell count, [4] dt,
                                        // [5] status: 1 = a device CFL step was not finite
  // a device CFL step asked of the next fused sweep's reduction (dt set), and
  // whether a reduction served it
  dimp::DtReq req;
  bool req_served = false;
  unsigned long long* dtag = nullptr;   // tagged extent of the refinement criterion (4 values)
  double* dpart = nullptr;              // per-wave wave-speed slots of the fused sweep (3 doubles each)
  int64_t part_cap = 0;
  bool smax_valid = false;
  int64_t step = 0;
  dimp::Params P;
  // patch set (2-D, independent patches with PATCH_GHOST ghost layers)
  bool patches = false;
  int64_t npatch = 0;
  std::vector<int32_t> pnx, pny;
  std::vector<int64_t> poff;
  dimp::PatchGeo* d_geo = nullptr;
  // packed work lists: x rows and y column chunks (for both tile widths),
  // batched (patches share waves) and per patch (every patch starts a new
  // work item); uploaded when the patch set is created
  struct List {
    int4* d_seg = nullptr;
    int32_t* d_beg = nullptr;
    int64_t nwork = 0;
    std::vector<int64_t> pwork;  // first work item of each patch (per-patch lists), npatch + 1 entries
  };
  List lx, lx_pp, ly[2], ly_pp[2];  // ly[0]: 4 tile columns, ly[1]: 8
  int per_patch = 0;                       // 1: one launch per patch and sweep
  int cw = 4;                              // tile columns of the y tasks
  int row_wpb = 4;                         // waves per block of the x sweep
  // adjoint workspace region: two recomputed states, one adjoint buffer, the
  // interface-normal transfer buffers and the per-block parameter partials
  double* aw = nullptr;
  // hyperbolic integrator and the SSP-RK3 workspace region: the stage state
  // q3 and the partial sums of D(q) (one buffer per direction before x)
  int integrator = DIMP_INTEGRATOR_SPLIT;
  int geom = DIMP_GEOMETRY_CARTESIAN;
  double r_lo = 0.0;  // cylindrical: radius of the low x face
  double* rkw = nullptr;
  // captured two-step graph (device dt)
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  double graph_cfl = -1.0;
  int graph_sig = -1;
  // optional per-launch timing of the sweeps with HIP events
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;  // one entry per recorded (start, stop) pair
  size_t ev_used = 0;
  int64_t ncell() const { return n[0] * n[1] * n[2]; }
  bool reactive() const { return rx.mat >= 0; }
  // the Johnson-Cook material (its plastic strain fills the history slot), or -1
  int jc_mat() const {
    for (int l = 0; l < nmat; ++l)
      if (mats[l].plast == DIMP_PLAST_JOHNSON_COOK) return l;
    return -1;
  }
  // the RX layouts (history slot present)
  bool hist() const { return reactive() || jc_mat() >= 0; }
  // the RX instance of the kernels: 0 no history slot, 1 a history slot, 2
  // a reactive mixture with a JWL component
  int rxk() const { return !hist() ? 0 : (P.rx.gen ? 2 : 1); }
  int nfields() const {
    const int nv = ndim == 1 ? 3 : ndim == 2 ? 5 : 9;
    return (nmat - 1) + nmat + (hist() ? 1 : 0) + ndim + 1 + nv;
  }
  const List& ylist(bool pp) const { return pp ? ly_pp[cw == 8] : ly[cw == 8]; }
};

namespace {

void default_options(dimp_options* o) {
  o->limiter = DIMP_LIMITER_MINMOD;
  o->thinc = 0;
  o->beta0 = 2.5;
  o->delta = 1e-5;
  o->eps = 1e-20;
  const double vs[6] = {1.0, 1e3, 1.0, 1e3, 1e9, 1.0};
  for (int i = 0; i < 6; ++i) o->va_scale[i] = vs[i];
}

dimp::MatP pack_material(const dimp_material& m) {
  dimp::MatP q;
  std::memset(&q, 0, sizeof q);
  q.eos = m.eos;
  q.plast = m.plast;
  q.cv = m.cv;
  if (m.eos == DIMP_EOS_ROMENSKII) {
    q.Gam = m.Gamma0;
    q.inv_rho0 = 1.0 / m.rho0;
    q.abar = m.abar;
    q.bbar = m.bbar;
    q.K0a = m.K0 / m.abar;
    q.ec_coef = m.K0 / (2.0 * m.rho0 * m.abar * m.abar);
    q.dpc_coef = m.K0 / (m.abar * m.rho0);
    q.G0 = m.G0;
    q.abar_one = (m.abar == 1.0);
    q.bbar_three = (m.bbar == 3.0);
    q.shear = (m.G0 > 0.0);
    q.yield_s6 = m.yield / std::sqrt(6.0);
    if (m.plast == DIMP_PLAST_JOHNSON_COOK) {
      q.jc_c1 = m.jc[0];
      q.jc_c2 = m.jc[1];
      q.jc_inv_c3 = 1.0 / m.jc[2];
      q.jc_n = m.jc[3];
      q.jc_m = m.jc[4];
      q.jc_inv_dT = 1.0 / m.jc[5];
      q.jc_chi0 = m.jc[6];
    }
  } else if (m.eos == DIMP_EOS_JWL) {
    q.Gam = m.Gamma0;  // reference curves carried by the reactive parameters
  } else {
    q.Gam = m.gamma - 1.0;
    q.pref0 = (m.eos == DIMP_EOS_STIFFENED) ? -m.gamma * m.pinf : 0.0;
    q.eref0 = (m.eos == DIMP_EOS_STIFFENED) ? m.eref : 0.0;
  }
  q.invGam = 1.0 / q.Gam;
  return q;
}

dimp_status check_material(const dimp_material& m, const char* what) {
  if (m.eos == DIMP_EOS_IDEAL || m.eos == DIMP_EOS_STIFFENED) {
    if (!(m.gamma > 1.0) || !std::isfinite(m.gamma)) return fail(DIMP_EINVAL, "%s: gamma must be > 1", what);
    if (!std::isfinite(m.pinf) || !std::isfinite(m.eref)) return fail(DIMP_EINVAL, "%s: non-finite p_inf/e_ref", what);
  } else if (m.eos == DIMP_EOS_ROMENSKII) {
    if (!(m.rho0 > 0) || !(m.K0 > 0) || !(m.G0 >= 0) || !(m.abar > 0) || !(m.Gamma0 > 0) || !std::isfinite(m.bbar))
      return fail(DIMP_EINVAL, "%s: Romenskii needs rho0, K0, abar, Gamma0 > 0 and G0 >= 0", what);
    if (m.plast == DIMP_PLAST_PERFECT && !(m.yield > 0))
      return fail(DIMP_EINVAL, "%s: perfect plasticity needs yield > 0", what);
    if (m.plast == DIMP_PLAST_JOHNSON_COOK &&
        !(m.G0 > 0 && m.cv > 0 && m.jc[0] > 0 && m.jc[1] >= 0 && m.jc[2] > 0 && m.jc[3] > 0 && m.jc[4] > 0 &&
          m.jc[5] > 0 && m.jc[6] > 0))
      return fail(DIMP_EINVAL, "%s: Johnson-Cook needs G0, cv, c1, c3, n, m, Tmelt - T0, chi0 > 0 and c2 >= 0", what);
  } else if (m.eos == DIMP_EOS_JWL) {
    if (!(m.rho0 > 0) || !(m.Gamma0 > 0) || !(m.jwl[2] > 0) || !(m.jwl[3] > 0) || !std::isfinite(m.jwl[0]) ||
        !std::isfinite(m.jwl[1]) || !std::isfinite(m.rho0))
      return fail(DIMP_EINVAL, "%s: JWL needs rho0, Gamma0, R1, R2 > 0 and finite A, B", what);
    if (m.plast != DIMP_PLAST_NONE) return fail(DIMP_EINVAL, "%s: a JWL material has no plasticity", what);
  } else {
    return fail(DIMP_EINVAL, "%s: unknown equation of state %d", what, m.eos);
  }
  if (m.plast != DIMP_PLAST_NONE && m.plast != DIMP_PLAST_PERFECT && m.plast != DIMP_PLAST_JOHNSON_COOK)
    return fail(DIMP_EINVAL, "%s: unknown plasticity model %d", what, m.plast);
  if (m.plast == DIMP_PLAST_JOHNSON_COOK && m.eos != DIMP_EOS_ROMENSKII)
    return fail(DIMP_EINVAL, "%s: Johnson-Cook plasticity needs a Romenskii solid", what);
  return DIMP_OK;
}

void rebuild_params(dimp_ctx* h) {
  dimp::Params& P = h->P;
  std::memset(&P, 0, sizeof P);
  for (int d = 0; d < 3; ++d) {
    P.n[d] = h->n[d];
    P.dx[d] = h->dx[d];
    P.bc[d] = h->bc[d];
  }
  P.ncell = h->ncell();
  P.limiter = h->opt.limiter;
  P.thinc = h->opt.thinc;
  P.beta0 = h->opt.beta0;
  P.delta = h->opt.delta;
  P.eps = h->opt.eps;
  for (int i = 0; i < 6; ++i) {
    const double e = 1e-6 * h->opt.va_scale[i];
    P.va_e2[i] = e * e;
  }
  P.geom = h->geom;
  P.r_lo = h->r_lo;
  P.any_shear = 0;
  P.nmat = h->nmat;
  for (int l = 0; l < h->nmat && l < dimp::MAXMAT; ++l) {
    P.mat[l] = pack_material(h->mats[l]);
    if (P.mat[l].shear && !(h->reactive() && h->rx.mat == l)) P.any_shear = 1;
  }
  P.rx.mat = h->rx.mat;
  P.rx.kind = dimp::RXK_MIX;
  if (h->jc_mat() >= 0) {
    P.rx.mat = h->jc_mat();
    P.rx.kind = dimp::RXK_EPS;
  }
  if (h->reactive()) {
    const dimp::MatP a = pack_material(h->rx.reactant), b = pack_material(h->rx.product);
    P.rx.Ga = a.Gam;
    P.rx.invGa = a.invGam;
    P.rx.pa = a.pref0;
    P.rx.ea = a.eref0;
    P.rx.cva = h->rx.reactant.cv;
    P.rx.Gb = b.Gam;
    P.rx.invGb = b.invGam;
    P.rx.pb = b.pref0;
    P.rx.eb = b.eref0 - h->rx.Q;
    P.rx.cvb = h->rx.product.cv;
    P.rx.k = h->rx.k;
    P.rx.n = h->rx.n;
    P.rx.n_is2 = (h->rx.n == 2.0);
    P.rx.inv_pref = 1.0 / h->rx.pref;
    P.rx.law = h->rx.law;
    P.rx.gen = 0;
    const dimp_material* comp[2] = {&h->rx.reactant, &h->rx.product};
    for (int c = 0; c < 2; ++c) {
      const dimp_material& m = *comp[c];
      P.rx.jwl[c] = (m.eos == DIMP_EOS_JWL);
      if (!P.rx.jwl[c]) continue;
      P.rx.gen = 1;
      P.rx.jA[c] = m.jwl[0];
      P.rx.jB[c] = m.jwl[1];
      P.rx.jR1[c] = m.jwl[2] * m.rho0;
      P.rx.jR2[c] = m.jwl[3] * m.rho0;
      P.rx.jiR1[c] = 1.0 / (m.jwl[2] * m.rho0);
      P.rx.jiR2[c] = 1.0 / (m.jwl[3] * m.rho0);
    }
    const double* g = h->rx.ig;
    P.rx.igI = g[0];
    P.rx.igG1 = g[1];
    P.rx.igG2 = g[2];
    P.rx.ig_a = g[3];
    P.rx.ig_b = g[4];
    P.rx.ig_c = g[5];
    P.rx.ig_d = g[6];
    P.rx.ig_e = g[7];
    P.rx.ig_g = g[8];
    P.rx.ig_x = g[9];
    P.rx.ig_y = g[10];
    P.rx.ig_z = g[11];
    P.rx.igFig = g[12];
    P.rx.igFG1 = g[13];
    P.rx.igFG2 = g[14];
    P.rx.ig_rho0 = g[15];
    P.rx.ig_punit = g[16];
  }
}

dimp_status need_bound(dimp_ctx* h) {
  if (!h) return fail(DIMP_EINVAL, "null handle");
  if (!h->mats_set) return fail(DIMP_ESTATE, "materials not set");
  if (!h->bound) return fail(DIMP_ESTATE, "no state bound");
  return DIMP_OK;
}

// bound, with a workspace (the calls that reduce, count or keep stage states)
dimp_status need_ws(dimp_ctx* h) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (!h->ws) return fail(DIMP_ESTATE, "no workspace bound (see dimp_workspace_bytes)");
  return DIMP_OK;
}

// wave-speed slots a fused sweep along dir writes
int64_t sweep_slot_count(const dimp_ctx* h, int dir) {
  if (!h->patches) return dimp::sweep_slots(h->P, h->ndim, dir);
  const dimp_ctx::List& L = dir == 0 ? (h->per_patch ? h->lx_pp : h->lx) : h->ylist(h->per_patch);
  return dir == 0 ? L.nwork : L.nwork * h->cw;
}

// slots the handle's fused sweeps may write (any direction, either tile
// width and launch mode of a patch set)
int64_t slot_need(const dimp_ctx* h) {
  int64_t need = 1;
  if (!h->patches) {
    for (int d = 0; d < h->ndim; ++d) need = std::max(need, dimp::sweep_slots(h->P, h->ndim, d));
  } else {
    need = std::max({need, h->lx.nwork, h->lx_pp.nwork, h->ly[0].nwork * 4, h->ly_pp[0].nwork * 4,
                     h->ly[1].nwork * 8, h->ly_pp[1].nwork * 8});
  }
  return need;
}

// Workspace regions (byte offsets from the workspace base, each 256-byte
// aligned): the reduction words, the refinement-tag extent, the wave-speed
// slots with their first reduction stage, then the RK3 stage buffers
// (purpose DIMP_WS_RK3) and the adjoint buffers (DIMP_WS_ADJOINT).
struct WsLayout {
  size_t smax, tag, part, rk, adj, total;
  int64_t part_cap;
};

constexpr size_t ws_align(size_t b) { return (b + 255) & ~size_t(255); }

// parameter partial sums of one step adjoint: the plastic step's blocks,
// then the two sweeps' (kept apart, totalled once)
int64_t adjoint_blocks(const dimp_ctx* h) {
  return dimp::adjoint_sweep_blocks(h->P, 0) + dimp::adjoint_sweep_blocks(h->P, 1) + dimp::adjoint_cell_blocks(h->P);
}

WsLayout ws_layout(const dimp_ctx* h, int purposes) {
  WsLayout L{};
  size_t off = 0;
  L.smax = off;
  off += ws_align(8 * sizeof(unsigned long long));
  L.tag = off;
  off += ws_align(4 * sizeof(unsigned long long));
  L.part_cap = slot_need(h);
  L.part = off;
  off += ws_align((size_t)(L.part_cap + dimp::reduce_smax_blocks(L.part_cap)) * 3 * sizeof(double));
  const size_t S = (size_t)h->nfields() * (size_t)h->ncell();
  L.rk = off;
  if (purposes & DIMP_WS_RK3) off += ws_align((size_t)h->ndim * S * sizeof(double));
  L.adj = off;
  if (purposes & DIMP_WS_ADJOINT)
    off += ws_align(((size_t)(3 * h->nfields() + 2) * (size_t)h->ncell() + (size_t)adjoint_blocks(h) * 12) *
                    sizeof(double));
  L.total = off;
  return L;
}

// the purposes a handle's workspace may serve
dimp_status check_purposes(const dimp_ctx* h, int purposes) {
  if (purposes & ~(DIMP_WS_RK3 | DIMP_WS_ADJOINT)) return fail(DIMP_EINVAL, "unknown workspace purpose bits");
  if (h->patches && purposes) return fail(DIMP_EUNSUPPORTED, "patch sets step the split integrator only");
  return DIMP_OK;
}

// launch one sweep, bracketed by HIP events when timing is on
dimp_status sweep_launch(dimp_ctx* h, double dt, const double* dtp, int dir, bool fuse) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->timing) {
    while (h->ev_pool.size() < 2 * (h->ev_used + 1)) {
      hipEvent_t e;
      HIPCHECK(hipEventCreate(&e), "event create");
      h->ev_pool.push_back(e);
    }
    e0 = h->ev_pool[2 * h->ev_used];
    e1 = h->ev_pool[2 * h->ev_used + 1];
    HIPCHECK(hipEventRecord(e0, h->stream), "event record");
  }
  if (!h->patches) {
    HIPCHECK(dimp::launch_sweep(h->P, h->ndim, h->rxk(), h->buf[h->cur], h->buf[h->cur ^ 1], dt, dtp, dir,
                                fuse, h->dpart, dimp::COL_SEGMENT, h->stream),
             "sweep");
  } else if (!h->per_patch) {
    const dimp_ctx::List& L = dir == 0 ? h->lx : h->ylist(false);
    HIPCHECK(dimp::launch_patch_sweep(h->P, h->rxk(), h->d_geo, {L.d_seg, L.d_beg}, 0, L.nwork, h->buf[h->cur],
                                      h->buf[h->cur ^ 1], dt, dtp, dir, fuse, h->dpart, h->row_wpb, h->cw,
                                      h->stream),
             "patch sweep");
  } else {
    const dimp_ctx::List& L = dir == 0 ? h->lx_pp : h->ylist(true);
    for (int64_t p = 0; p < h->npatch; ++p)
      HIPCHECK(dimp::launch_patch_sweep(h->P, h->rxk(), h->d_geo, {L.d_seg, L.d_beg}, L.pwork[p],
                                        L.pwork[p + 1] - L.pwork[p], h->buf[h->cur], h->buf[h->cur ^ 1], dt, dtp,
                                        dir, fuse, h->dpart, h->row_wpb, h->cw, h->stream),
               "patch sweep (per patch)");
  }
  if (fuse) {
    const dimp::DtReq* rq = h->req.dt ? &h->req : nullptr;
    HIPCHECK(dimp::launch_reduce_smax(h->dpart, sweep_slot_count(h, dir), h->ndim, h->dpart + 3 * h->part_cap,
                                      h->dsmax, h->stream, rq),
             "wave-speed reduction");
    h->req_served = h->req_served || rq;
  }
  if (h->timing) {
    HIPCHECK(hipEventRecord(e1, h->stream), "event record");
    h->ev_kind.push_back(2 * dir + (fuse ? 1 : 0));
    h->ev_used += 1;
  }
  h->cur ^= 1;
  return DIMP_OK;
}

void free_list(dimp_ctx::List& L) {
  if (L.d_seg) (void)hipFree(L.d_seg);
  if (L.d_beg) (void)hipFree(L.d_beg);
  L.d_seg = nullptr;
  L.d_beg = nullptr;
  L.nwork = 0;
}

dimp_status upload_list(dimp_ctx::List& L, const std::vector<dimp::Line>& lines, int64_t npatch, bool per_patch) {
  static_assert(sizeof(dimp::Seg) == sizeof(int4), "a segment is read as an int4");
  std::vector<dimp::Seg> seg;
  std::vector<int64_t> beg64;
  free_list(L);
  dimp::pack_lines(lines, npatch, per_patch, seg, beg64, L.pwork);
  if (seg.size() >= (size_t(1) << 31)) return fail(DIMP_EINVAL, "patch set too large for one work list");
  const std::vector<int32_t> beg(beg64.begin(), beg64.end());
  void* a = nullptr;
  void* b = nullptr;
  hipError_t e = hipMalloc(&a, seg.size() * sizeof(int4));
  if (e == hipSuccess) e = hipMalloc(&b, beg.size() * sizeof(int32_t));
  if (e != hipSuccess) {
    if (a) (void)hipFree(a);
    return fail(DIMP_ENOMEM, "work list: %s", hipGetErrorString(e));
  }
  L.d_seg = static_cast<int4*>(a);
  L.d_beg = static_cast<int32_t*>(b);
  L.nwork = (int64_t)beg.size() - 1;
  HIPCHECK(hipMemcpy(L.d_seg, seg.data(), seg.size() * sizeof(int4), hipMemcpyHostToDevice), "work list upload");
  HIPCHECK(hipMemcpy(L.d_beg, beg.data(), beg.size() * sizeof(int32_t), hipMemcpyHostToDevice), "work list upload");
  return DIMP_OK;
}

// x lists: every interior row of every patch
dimp_status build_x_lists(dimp_ctx* h) {
  std::vector<dimp::Line> lines;
  for (int64_t p = 0; p < h->npatch; ++p)
    for (int j = 0; j < h->pny[p]; ++j) lines.push_back({(int32_t)p, j, h->pnx[p]});
  dimp_status s = upload_list(h->lx, lines, h->npatch, false);
  return s ? s : upload_list(h->lx_pp, lines, h->npatch, true);
}

// y lists for both tile widths: every chunk of 4 (8) columns of every patch
dimp_status build_y_lists(dimp_ctx* h) {
  for (int k = 0; k < 2; ++k) {
    const int cw = k ? 8 : 4;
    std::vector<dimp::Line> lines;
    for (int64_t p = 0; p < h->npatch; ++p)
      for (int x0 = 0; x0 < h->pnx[p]; x0 += cw) lines.push_back({(int32_t)p, x0, h->pny[p]});
    dimp_status s = upload_list(h->ly[k], lines, h->npatch, false);
    if (!s) s = upload_list(h->ly_pp[k], lines, h->npatch, true);
    if (s) return s;
  }
  return DIMP_OK;
}

void drop_graph(dimp_ctx* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
  h->graph_sig = -1;
}

// one launch of the RK3 step, bracketed by HIP events when timing is on
// (kinds as the split sweeps: 2*dir + 1 for the fused last launch)
dimp_status rk_launch(dimp_ctx* h, int dir, int mode, int stage, bool fuse, const double* in, double* out,
                      const double* Rin, const double* qn, double dt, const double* dtp) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->timing) {
    while (h->ev_pool.size() < 2 * (h->ev_used + 1)) {
      hipEvent_t e;
      HIPCHECK(hipEventCreate(&e), "event create");
      h->ev_pool.push_back(e);
    }
    e0 = h->ev_pool[2 * h->ev_used];
    e1 = h->ev_pool[2 * h->ev_used + 1];
    HIPCHECK(hipEventRecord(e0, h->stream), "event record");
  }
  HIPCHECK(dimp::launch_rk_sweep(h->P, h->ndim, h->rxk(), dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp,
                                 h->dpart, h->stream),
           "RK3 pass");
  if (fuse) {
    const dimp::DtReq* rq = h->req.dt ? &h->req : nullptr;
    HIPCHECK(dimp::launch_reduce_smax(h->dpart, dimp::sweep_slots(h->P, h->ndim, 0), h->ndim,
                                      h->dpart + 3 * h->part_cap, h->dsmax, h->stream, rq),
             "wave-speed reduction");
    h->req_served = h->req_served || rq;
  }
  if (h->timing) {
    HIPCHECK(hipEventRecord(e1, h->stream), "event record");
    h->ev_kind.push_back(2 * dir + (fuse ? 1 : 0));
    h->ev_used += 1;
  }
  return DIMP_OK;
}

// The fractional source steps as their own pass (plastic, reaction, and the
// cylindrical geometric source, which needs the cell's radius) and the wave
// speed of the result, where they are not fused into the last sweep
dimp_status unfused_sources(dimp_ctx* h, double dt, const double* dtp) {
  HIPCHECK(dimp::launch_sources(h->P, h->ndim, h->rxk(), h->buf[h->cur], dt, dtp, h->stream), "sources");
  HIPCHECK(dimp::launch_wavespeed(h->P, h->ndim, h->rxk(), h->buf[h->cur], h->dsmax, h->stream), "wavespeed");
  return DIMP_OK;
}

// One SSP-RK3 step (Sec. 3.1, eq. (rk)): per stage, the y pass writes the
// partial stage a qn + b (q - dt D_y(q)) (R0), z subtracts b dt D_z (R1) and
// the x pass b dt D_x, writing the stage result.  qn stays in buf[cur] until
// the third stage overwrites it cell by cell.
// Faces whose fluxes a 2-D step records (a refined patch's coarse/fine
// boundary on one level), per sweep axis, and where they go (for the RK3,
// the stages' fluxes weighted 1/6, 1/6, 2/3 and summed).  The flux
// kernels are a few waves each and latency-bound, so they run on a stream of
// their own beside the sweeps: kernel k starts when the state sweep k reads
// is ready (ready[k]) and sweep k + 1, which overwrites that state, waits for
// it (done[k]); the caller waits for done[1] before using the fluxes or
// writing the state again.
struct FluxTap {
  dimp::FaceSet fs[2];
  double* out[2];
  hipStream_t side = nullptr;
  hipEvent_t ready[2]{}, done[2]{};
};

// The ghost-ring refill of a patch's RK3 stage inputs from the level above
// (its states before and after its step, and the patch's substep): q^(1) at
// the fine step's end, q^(3) at its middle
struct RkHook {
  const dimp::AmrBox* box;
  const double* cold;
  const double* cnew;
  int sub;
};

dimp_status rk3_step(dimp_ctx* h, double dt, const double* dtp, const FluxTap* const* taps = nullptr, int ntap = 0,
                     const RkHook* hook = nullptr) {
  const int D = h->ndim;
  const double wst[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
  const size_t S = (size_t)h->nfields() * h->ncell();
  double* qn = h->buf[h->cur];
  double* q1 = h->buf[h->cur ^ 1];
  double* q3 = h->rkw;
  double* R0 = h->rkw + S;
  double* R1 = h->rkw + 2 * S;
  const double* stage_in[3] = {qn, q1, q3};
  double* stage_out[3] = {q1, q3, qn};
  for (int st = 0; st < 3; ++st) {
    const double* q = stage_in[st];
    const double* R = nullptr;
    if (hook && st > 0)
      HIPCHECK(dimp::launch_amr_fill(*hook->box, hook->cold, hook->cnew, 0.5 * (hook->sub + (st == 1 ? 1.0 : 0.5)),
                                     const_cast<double*>(q), h->stream),
               "amr stage fill");
    // the stage's boundary fluxes beside its passes (which do not write q)
    for (int i = 0; i < ntap; ++i) {
      const FluxTap* t = taps[i];
      if (!t) continue;
      HIPCHECK(hipEventRecord(t->ready[st & 1], h->stream), "event record");
      HIPCHECK(hipStreamWaitEvent(t->side, t->ready[st & 1], 0), "stream wait");
      for (int dir = 0; dir < D; ++dir)
        HIPCHECK(dimp::launch_amr_flux(h->P, h->rxk(), dir, t->fs[dir], q, dt, t->out[dir], t->side, true, wst[st],
                                       st > 0),
                 "boundary fluxes");
      HIPCHECK(hipEventRecord(t->done[st & 1], t->side), "event record");
    }
    if (D >= 2) {
      dimp_status s = rk_launch(h, 1, 1, st + 1, false, q, R0, nullptr, qn, dt, dtp);
      if (s) return s;
      R = R0;
    }
    if (D == 3) {
      dimp_status s = rk_launch(h, 2, 2, st + 1, false, q, R1, R0, qn, dt, dtp);
      if (s) return s;
      R = R1;
    }
    dimp_status s = rk_launch(h, 0, 3, st + 1, st == 2 && !h->geom, q, stage_out[st], R, qn, dt, dtp);
    if (s) return s;
    for (int i = 0; i < ntap; ++i)
      if (taps[i]) HIPCHECK(hipStreamWaitEvent(h->stream, taps[i]->done[st & 1], 0), "stream wait");
  }
  if (h->geom) {
    dimp_status s = unfused_sources(h, dt, dtp);
    if (s) return s;
  }
  h->step += 1;
  h->smax_valid = true;
  return DIMP_OK;
}

// one full step; dt on the host, or read by the kernels from dtp (device);
// with taps (2-D, dt on the host), the fluxes of each sweep (or RK3 stage)
// through the tapped faces are recorded from the state it reads (one per
// patch the grid holds, and one more for the patch it is in a nested
// hierarchy); hook: the RK3 stage refills of a patch grid
dimp_status step_once(dimp_ctx* h, double dt, const double* dtp, const FluxTap* const* taps = nullptr,
                      int ntap = 0, const RkHook* hook = nullptr) {
  if (h->integrator == DIMP_INTEGRATOR_RK3) return rk3_step(h, dt, dtp, taps, ntap, hook);
  const int D = h->ndim;
  for (int k = 0; k < D; ++k) {
    const int dir = (h->step % 2 == 0) ? k : D - 1 - k;
    for (int i = 0; i < ntap; ++i) {
      const FluxTap* t = taps[i];
      if (!t) continue;
      HIPCHECK(hipEventRecord(t->ready[k], h->stream), "event record");
      HIPCHECK(hipStreamWaitEvent(t->side, t->ready[k], 0), "stream wait");
      HIPCHECK(dimp::launch_amr_flux(h->P, h->rxk(), dir, t->fs[dir], h->buf[h->cur], dt, t->out[dir], t->side),
               "boundary fluxes");
      HIPCHECK(hipEventRecord(t->done[k], t->side), "event record");
    }
    for (int i = 0; i < ntap; ++i)
      if (taps[i] && k > 0) HIPCHECK(hipStreamWaitEvent(h->stream, taps[i]->done[k - 1], 0), "stream wait");
    dimp_status s = sweep_launch(h, dt, dtp, dir, k == D - 1 && !h->geom);
    if (s) return s;
  }
  if (h->geom) {
    dimp_status s = unfused_sources(h, dt, dtp);
    if (s) return s;
  }
  h->step += 1;
  h->smax_valid = true;
  return DIMP_OK;
}

}  // namespace

extern "C" {

const char* dimp_last_error(void) { return g_err.c_str(); }

dimp_status dimp_create_grid(int ndim, const int64_t n[3], const double dx[3], const int32_t bc[3],
                             dimp_handle* out) {
  if (!out || !n || !dx || !bc) return fail(DIMP_EINVAL, "null argument");
  *out = nullptr;
  if (ndim < 1 || ndim > 3) return fail(DIMP_EINVAL, "ndim must be 1..3 (got %d)", ndim);
  auto* h = new (std::nothrow) dimp_ctx();
  if (!h) return fail(DIMP_ENOMEM, "host allocation failed");
  h->ndim = ndim;
  for (int d = 0; d < ndim; ++d) {
    if (n[d] < 1 || n[d] > (int64_t(1) << 31)) {
      delete h;
      return fail(DIMP_EINVAL, "n[%d] = %lld out of range", d, (long long)n[d]);
    }
    if (!(dx[d] > 0.0) || !std::isfinite(dx[d])) {
      delete h;
      return fail(DIMP_EINVAL, "dx[%d] must be positive", d);
    }
    if (bc[d] < DIMP_BC_TRANSMISSIVE || bc[d] > DIMP_BC_AXIS) {
      delete h;
      return fail(DIMP_EINVAL, "bc[%d] = %d unknown", d, bc[d]);
    }
    h->n[d] = n[d];
    h->dx[d] = dx[d];
    h->bc[d] = bc[d];
  }
  if (h->ncell() > (int64_t(1) << 34)) {
    delete h;
    return fail(DIMP_EINVAL, "grid too large");
  }
  h->rx.mat = -1;
  default_options(&h->opt);
  *out = h;
  return DIMP_OK;
}

dimp_status dimp_create_patch_set(int64_t npatch, const int32_t* sizes, const double dx[2], dimp_handle* out) {
  if (!out || !sizes || !dx) return fail(DIMP_EINVAL, "null argument");
  *out = nullptr;
  if (npatch < 1 || npatch > (int64_t(1) << 24)) return fail(DIMP_EINVAL, "npatch out of range");
  if (!(dx[0] > 0.0) || !(dx[1] > 0.0) || !std::isfinite(dx[0]) || !std::isfinite(dx[1]))
    return fail(DIMP_EINVAL, "dx must be positive");
  auto* h = new (std::nothrow) dimp_ctx();
  if (!h) return fail(DIMP_ENOMEM, "host allocation failed");
  h->ndim = 2;
  h->patches = true;
  h->npatch = npatch;
  h->pnx.resize(npatch);
  h->pny.resize(npatch);
  h->poff.resize(npatch + 1);
  const int G = dimp::PATCH_GHOST;
  int64_t off = 0;
  std::vector<dimp::PatchGeo> geo(npatch);
  for (int64_t p = 0; p < npatch; ++p) {
    const int32_t nx = sizes[2 * p], ny = sizes[2 * p + 1];
    if (nx < 1 || ny < 1 || nx > 65536 || ny > 65536) {
      delete h;
      return fail(DIMP_EINVAL, "patch %lld has size %d x %d", (long long)p, nx, ny);
    }
    h->pnx[p] = nx;
    h->pny[p] = ny;
    h->poff[p] = off;
    geo[p].off = off;
    geo[p].nx = nx;
    geo[p].ny = ny;
    off += (int64_t)(nx + 2 * G) * (ny + 2 * G);
  }
  h->poff[npatch] = off;
  if (off > (int64_t(1) << 34)) {
    delete h;
    return fail(DIMP_EINVAL, "patch set too large");
  }
  h->n[0] = off;  // pointwise kernels run over every stored element, ghosts included
  h->n[1] = h->n[2] = 1;
  h->dx[0] = dx[0];
  h->dx[1] = dx[1];
  h->rx.mat = -1;
  default_options(&h->opt);
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, npatch * sizeof(dimp::PatchGeo));
  if (e == hipSuccess) {
    h->d_geo = static_cast<dimp::PatchGeo*>(q);
    e = hipMemcpy(h->d_geo, geo.data(), npatch * sizeof(dimp::PatchGeo), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    dimp_destroy(h);
    return fail(DIMP_EHIP, "patch set upload: %s", hipGetErrorString(e));
  }
  dimp_status st = build_x_lists(h);
  if (!st) st = build_y_lists(h);
  if (st) {
    const std::string msg = g_err;
    dimp_destroy(h);
    g_err = msg;
    return st;
  }
  *out = h;
  return DIMP_OK;
}

dimp_status dimp_patch_offsets(dimp_handle h, int64_t* offsets) {
  if (!h || !offsets) return fail(DIMP_EINVAL, "null argument");
  if (!h->patches) return fail(DIMP_EINVAL, "not a patch set");
  for (int64_t p = 0; p <= h->npatch; ++p) offsets[p] = h->poff[p];
  return DIMP_OK;
}

dimp_status dimp_set_patch_launch(dimp_handle h, int per_patch, int row_waves, int tile_columns) {
  if (!h) return fail(DIMP_EINVAL, "null handle");
  if (!h->patches) return fail(DIMP_EINVAL, "not a patch set");
  if (per_patch != 0 && per_patch != 1) return fail(DIMP_EINVAL, "per_patch must be 0 or 1");
  if (row_waves != 1 && row_waves != 2 && row_waves != 4) return fail(DIMP_EINVAL, "row_waves must be 1, 2 or 4");
  if (tile_columns != 4 && tile_columns != 8) return fail(DIMP_EINVAL, "tile_columns must be 4 or 8");
  h->per_patch = per_patch;
  h->row_wpb = row_waves;
  h->cw = tile_columns;  // both widths' lists exist, and the slots cover both
  drop_graph(h);
  return DIMP_OK;
}

dimp_status dimp_set_materials(dimp_handle h, int nmat, const dimp_material* mats, const dimp_reactive* rx) {
  if (!h || !mats) return fail(DIMP_EINVAL, "null argument");
  if (nmat < 1 || nmat > 4) return fail(DIMP_EINVAL, "nmat must be 1..4 (got %d)", nmat);
  if (nmat == 1 || nmat > dimp::MAXMAT)
    return fail(DIMP_EUNSUPPORTED, "the GPU kernels are built for 2 or 3 materials (got %d)", nmat);
  if (nmat == 3 && h->ndim == 3) return fail(DIMP_EUNSUPPORTED, "three materials are built for 1-D and 2-D grids");
  for (int l = 0; l < nmat; ++l) {
    char what[32];
    snprintf(what, sizeof what, "material %d", l);
    dimp_status s = check_material(mats[l], what);
    if (s) return s;
    if (mats[l].eos == DIMP_EOS_JWL && !(rx && rx->mat == l))
      return fail(DIMP_EUNSUPPORTED, "%s: JWL is supported for reactive components only", what);
  }
  dimp_reactive r;
  std::memset(&r, 0, sizeof r);
  r.mat = -1;
  if (rx && rx->mat >= 0) {
    if (rx->mat >= nmat) return fail(DIMP_EINVAL, "reactive material index %d out of range", rx->mat);
    for (const dimp_material* c : {&rx->reactant, &rx->product}) {
      dimp_status s = check_material(*c, "reactive component");
      if (s) return s;
      if (c->eos == DIMP_EOS_ROMENSKII)
        return fail(DIMP_EUNSUPPORTED, "reactive components must be ideal or stiffened gases or JWL on the GPU");
      if (!(c->cv > 0)) return fail(DIMP_EINVAL, "reactive components need cv > 0");
    }
    if (!std::isfinite(rx->Q)) return fail(DIMP_EINVAL, "reaction needs a finite Q");
    if (rx->law == DIMP_RATE_POWER) {
      if (!(rx->pref > 0) || !(rx->k >= 0) || !(rx->n >= 0))
        return fail(DIMP_EINVAL, "the power rate needs pref > 0, k >= 0, n >= 0");
    } else if (rx->law == DIMP_RATE_IGNITION_GROWTH) {
      const double* g = rx->ig;
      bool ok = g[15] > 0 && g[16] > 0;  // rho0, pressure unit
      for (int i = 0; i < 3; ++i) ok = ok && g[i] >= 0 && std::isfinite(g[i]);   // I, G1, G2
      for (int i = 4; i < 12; ++i) ok = ok && g[i] >= 0 && std::isfinite(g[i]);  // exponents
      ok = ok && g[6] > 0 && g[8] > 0;  // F^d, F^g vanish at F = 0
      for (int i : {3, 12, 13, 14}) ok = ok && std::isfinite(g[i]);
      if (!ok)
        return fail(DIMP_EINVAL,
                    "ignition and growth needs rho0, punit, d, g > 0, finite thresholds and non-negative rates "
                    "and exponents");
    } else {
      return fail(DIMP_EINVAL, "unknown rate law %d", rx->law);
    }
    r = *rx;
  }
  int njc = 0;
  for (int l = 0; l < nmat; ++l) njc += (mats[l].plast == DIMP_PLAST_JOHNSON_COOK) ? 1 : 0;
  if (njc > 1) return fail(DIMP_EUNSUPPORTED, "at most one Johnson-Cook material (one history slot)");
  if (njc && r.mat >= 0) return fail(DIMP_EUNSUPPORTED, "a Johnson-Cook solid and a reactive mixture share one slot");
  if (h->bound && (h->nmat != nmat || h->rx.mat != r.mat || (h->jc_mat() >= 0) != (njc > 0)))
    return fail(DIMP_ESTATE, "cannot change the field count while a state is bound");
  h->nmat = nmat;
  for (int l = 0; l < nmat; ++l) h->mats[l] = mats[l];
  h->rx = r;
  h->mats_set = true;
  rebuild_params(h);
  h->smax_valid = false;
  drop_graph(h);
  return DIMP_OK;
}

dimp_status dimp_set_options(dimp_handle h, const dimp_options* o) {
  if (!h || !o) return fail(DIMP_EINVAL, "null argument");
  if (o->limiter != DIMP_LIMITER_MINMOD && o->limiter != DIMP_LIMITER_VANALBADA)
    return fail(DIMP_EINVAL, "unknown limiter %d", o->limiter);
  if (o->thinc != 0 && o->thinc != 1) return fail(DIMP_EINVAL, "thinc must be 0 or 1");
  if (!(o->beta0 > 0) || !(o->delta > 0 && o->delta < 0.5) || !(o->eps >= 0))
    return fail(DIMP_EINVAL, "need beta0 > 0, 0 < delta < 0.5, eps >= 0");
  for (int i = 0; i < 6; ++i)
    if (!(o->va_scale[i] > 0)) return fail(DIMP_EINVAL, "va_scale[%d] must be > 0", i);
  h->opt = *o;
  rebuild_params(h);
  h->smax_valid = false;
  drop_graph(h);
  return DIMP_OK;
}

dimp_status dimp_nfields(dimp_handle h, int* nfields, int64_t* ncell) {
  if (!h || !nfields || !ncell) return fail(DIMP_EINVAL, "null argument");
  if (!h->mats_set) return fail(DIMP_ESTATE, "materials not set");
  *nfields = h->nfields();
  *ncell = h->ncell();
  return DIMP_OK;
}

dimp_status dimp_workspace_bytes(dimp_handle h, int purposes, size_t* bytes) {
  if (!h || !bytes) return fail(DIMP_EINVAL, "null argument");
  if (!h->mats_set) return fail(DIMP_ESTATE, "materials not set");
  dimp_status s = check_purposes(h, purposes);
  if (s) return s;
  if (!h->patches) rebuild_params(h);
  *bytes = ws_layout(h, purposes).total;
  return DIMP_OK;
}

dimp_status dimp_bind(dimp_handle h, double* buf0, double* buf1, void* workspace, size_t ws_bytes, int purposes,
                      void* stream) {
  if (!h || !buf0 || !buf1) return fail(DIMP_EINVAL, "null argument");
  if (buf0 == buf1) return fail(DIMP_EINVAL, "the two state buffers must differ");
  if (!h->mats_set) return fail(DIMP_ESTATE, "materials not set");
  dimp_status s = check_purposes(h, purposes);
  if (s) return s;
  if (!h->patches) rebuild_params(h);  // grid sizes for the slot count
  const WsLayout W = ws_layout(h, purposes);
  if (workspace) {
    if (ws_bytes < W.total)
      return fail(DIMP_EINVAL, "workspace of %zu bytes is too small (%zu needed for purposes %d)", ws_bytes, W.total,
                  purposes);
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
      return fail(DIMP_EINVAL, "the workspace must be 256-byte aligned");
  } else if (ws_bytes || purposes) {
    return fail(DIMP_EINVAL, "no workspace given for %zu bytes / purposes %d", ws_bytes, purposes);
  }
  if (h->integrator == DIMP_INTEGRATOR_RK3 && !(purposes & DIMP_WS_RK3) && workspace)
    return fail(DIMP_EINVAL, "the RK3 integrator is set: bind a workspace with DIMP_WS_RK3");
  if (workspace)  // clear the reduction words (status, counters) before first use
    HIPCHECK(dimp::launch_zero_u64(reinterpret_cast<unsigned long long*>(static_cast<unsigned char*>(workspace) + W.smax),
                                   8, static_cast<hipStream_t>(stream)),
             "workspace init");
  h->ws = static_cast<unsigned char*>(workspace);
  h->ws_bytes = workspace ? ws_bytes : 0;
  h->ws_purposes = workspace ? purposes : 0;
  h->dsmax = workspace ? reinterpret_cast<unsigned long long*>(h->ws + W.smax) : nullptr;
  h->dtag = workspace ? reinterpret_cast<unsigned long long*>(h->ws + W.tag) : nullptr;
  h->dpart = workspace ? reinterpret_cast<double*>(h->ws + W.part) : nullptr;
  h->part_cap = workspace ? W.part_cap : 0;
  h->rkw = (purposes & DIMP_WS_RK3) ? reinterpret_cast<double*>(h->ws + W.rk) : nullptr;
  h->aw = (purposes & DIMP_WS_ADJOINT) ? reinterpret_cast<double*>(h->ws + W.adj) : nullptr;
  h->buf[0] = buf0;
  h->buf[1] = buf1;
  h->cur = 0;
  h->stream = static_cast<hipStream_t>(stream);
  h->bound = true;
  h->smax_valid = false;
  drop_graph(h);
  return DIMP_OK;
}

dimp_status dimp_current(dimp_handle h, int* which) {
  if (!h || !which) return fail(DIMP_EINVAL, "null argument");
  *which = h->cur;
  return DIMP_OK;
}

dimp_status dimp_prim_to_cons(dimp_handle h, const double* prim) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (!prim) return fail(DIMP_EINVAL, "null primitive array");
  HIPCHECK(dimp::launch_prim_to_cons(h->P, h->ndim, h->rxk(), prim, h->buf[h->cur], h->stream), "prim_to_cons");
  h->step = 0;
  h->smax_valid = false;
  return DIMP_OK;
}

dimp_status dimp_set_conserved(dimp_handle h, const double* cons_dev) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (!cons_dev) return fail(DIMP_EINVAL, "null conserved array");
  double* dst = h->buf[h->cur];
  if (cons_dev != dst)
    HIPCHECK(hipMemcpyAsync(dst, cons_dev, sizeof(double) * (size_t)h->nfields() * (size_t)h->ncell(),
                            hipMemcpyDeviceToDevice, h->stream),
             "set_conserved copy");
  h->smax_valid = false;
  return DIMP_OK;
}

dimp_status dimp_cons_to_prim(dimp_handle h, double* prim) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (!prim) return fail(DIMP_EINVAL, "null primitive array");
  HIPCHECK(dimp::launch_cons_to_prim(h->P, h->ndim, h->rxk(), h->buf[h->cur], prim, h->stream), "cons_to_prim");
  return DIMP_OK;
}

dimp_status dimp_sweep(dimp_handle h, double dt, int dir) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DIMP_EINVAL, "dt must be positive and finite");
  if (dir < 0 || dir >= h->ndim) return fail(DIMP_EINVAL, "dir %d out of range", dir);
  s = sweep_launch(h, dt, nullptr, dir, false);
  if (s) return s;
  h->smax_valid = false;
  return DIMP_OK;
}

dimp_status dimp_sources(dimp_handle h, double dt) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(DIMP_EINVAL, "dt must be non-negative and finite");
  HIPCHECK(dimp::launch_sources(h->P, h->ndim, h->rxk(), h->buf[h->cur], dt, nullptr, h->stream), "sources");
  h->smax_valid = false;
  return DIMP_OK;
}

dimp_status dimp_advance(dimp_handle h, double dt) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DIMP_EINVAL, "dt must be positive and finite");
  return step_once(h, dt, nullptr);
}

static dimp_status ensure_smax(dimp_handle h);

// One step of dt read from dtp; with next_cfl > 0 the step's wave-speed
// reduction also writes the next step's dt to dtp (and log[idx]) where its
// last sweep is fused: *served tells whether it did (else the caller
// launches the dt kernel before the next step).
static dimp_status step_with_next_dt(dimp_handle h, double* dtp, double next_cfl, double* log, int64_t idx,
                                     bool* served) {
  h->req = dimp::DtReq{};
  if (next_cfl > 0.0) h->req = dimp::DtReq{next_cfl, h->P.dx[0], h->P.dx[1], h->P.dx[2], dtp, log, idx};
  h->req_served = false;
  const dimp_status s = step_once(h, 0.0, dtp);
  *served = h->req_served && next_cfl > 0.0;
  h->req = dimp::DtReq{};
  h->req_served = false;
  return s;
}

dimp_status dimp_advance_cfl(dimp_handle h, double cfl, int nsteps, double* dt_log_dev) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(DIMP_EINVAL, "cfl must be positive and finite");
  if (nsteps < 0) return fail(DIMP_EINVAL, "nsteps must be >= 0");
  s = ensure_smax(h);
  if (s) return s;
  double* dtp = reinterpret_cast<double*>(h->dsmax + 4);
  bool have_dt = false;  // the previous step's reduction wrote this step's dt
  for (int i = 0; i < nsteps; ++i) {
    if (!have_dt)
      HIPCHECK(dimp::launch_cfl_dt(h->P, h->ndim, h->dsmax, cfl, dtp, dt_log_dev, i, h->stream), "advance_cfl: dt");
    s = step_with_next_dt(h, dtp, i + 1 < nsteps ? cfl : 0.0, dt_log_dev, i + 1, &have_dt);
    if (s) return s;
  }
  return DIMP_OK;
}

dimp_status dimp_advance_graph(dimp_handle h, double cfl, int nsteps) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(DIMP_EINVAL, "cfl must be positive and finite");
  if (nsteps < 0) return fail(DIMP_EINVAL, "nsteps must be >= 0");
  if (h->timing) return fail(DIMP_ESTATE, "kernel timing is on; graphs are replayed without it");
  s = ensure_smax(h);
  if (s) return s;
  if (nsteps > 0 && (h->step % 2) != 0) {  // the graph starts on an even step
    s = dimp_advance_cfl(h, cfl, 1, nullptr);
    if (s) return s;
    nsteps -= 1;
  }
  const int pairs = nsteps / 2;
  const int sig = h->cur;  // the graph bakes in which buffer holds the state
  if (pairs > 0 && (!h->gexec || h->graph_cfl != cfl || h->graph_sig != sig)) {
    drop_graph(h);
    if (!h->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "capture stream");
    hipStream_t keep = h->stream;
    const int cur0 = h->cur;
    const int64_t step0 = h->step;
    h->stream = h->cap_stream;
    HIPCHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    double* dtp = reinterpret_cast<double*>(h->dsmax + 4);
    dimp_status cs = DIMP_OK;
    bool have_dt = false;  // the first step's reduction writes the second step's dt
    for (int i = 0; i < 2 && cs == DIMP_OK; ++i) {
      hipError_t e =
          have_dt ? hipSuccess : dimp::launch_cfl_dt(h->P, h->ndim, h->dsmax, cfl, dtp, nullptr, 0, h->stream);
      cs = (e == hipSuccess) ? step_with_next_dt(h, dtp, i == 0 ? cfl : 0.0, nullptr, 0, &have_dt)
                             : hip_fail(e, "capture dt");
    }
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(h->cap_stream, &graph);
    h->stream = keep;
    h->cur = cur0;
    h->step = step0;
    if (cs) {
      if (graph) (void)hipGraphDestroy(graph);
      return cs;
    }
    if (ee != hipSuccess) return hip_fail(ee, "end capture");
    hipError_t ie = hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      h->gexec = nullptr;
      return hip_fail(ie, "graph instantiate");
    }
    h->graph_cfl = cfl;
    h->graph_sig = sig;
  }
  for (int i = 0; i < pairs; ++i) HIPCHECK(hipGraphLaunch(h->gexec, h->stream), "graph launch");
  h->step += 2 * pairs;
  if (pairs > 0) h->smax_valid = true;
  if (nsteps % 2) {
    s = dimp_advance_cfl(h, cfl, 1, nullptr);
    if (s) return s;
  }
  return DIMP_OK;
}

namespace {

// one autotune trial: restore the snapshot, warm up one step, time nsteps
dimp_status autotune_trial(dimp_ctx* h, const void* snap, size_t bytes, int cur0, int64_t step0, int nsteps,
                           double cfl, hipEvent_t e0, hipEvent_t e1, float* ms) {
  h->cur = cur0;
  h->step = step0;
  HIPCHECK(hipMemcpyAsync(h->buf[h->cur], snap, bytes, hipMemcpyDeviceToDevice, h->stream), "autotune restore");
  h->smax_valid = false;
  dimp_status s = ensure_smax(h);
  if (!s) s = dimp_advance_cfl(h, cfl, 1, nullptr);
  if (s) return s;
  HIPCHECK(hipEventRecord(e0, h->stream), "event record");
  s = dimp_advance_cfl(h, cfl, nsteps, nullptr);
  if (s) return s;
  HIPCHECK(hipEventRecord(e1, h->stream), "event record");
  HIPCHECK(hipEventSynchronize(e1), "event sync");
  HIPCHECK(hipEventElapsedTime(ms, e0, e1), "event time");
  return DIMP_OK;
}

}  // namespace

dimp_status dimp_autotune(dimp_handle h, int nsteps, double cfl, double* snapshot_dev, int* best) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (!h->patches) return fail(DIMP_EINVAL, "autotune applies to patch sets");
  if (nsteps < 1) return fail(DIMP_EINVAL, "nsteps must be >= 1");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(DIMP_EINVAL, "cfl must be positive and finite");
  if (!snapshot_dev) return fail(DIMP_EINVAL, "null snapshot buffer");
  if (snapshot_dev == h->buf[0] || snapshot_dev == h->buf[1])
    return fail(DIMP_EINVAL, "the snapshot buffer must not be a bound state buffer");
  if (h->timing) return fail(DIMP_ESTATE, "kernel timing is on");
  // snapshot of the state; every trial starts from it and it is restored at the end
  const size_t bytes = (size_t)h->nfields() * (size_t)h->ncell() * sizeof(double);
  void* snap = snapshot_dev;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int cur0 = h->cur;
  const int64_t step0 = h->step;
  const int per_patch0 = h->per_patch, wpb0 = h->row_wpb, cw0 = h->cw;
  const int wpbs[3] = {1, 2, 4}, cws[2] = {4, 8};
  float best_ms = 3.0e38f;
  int best_cfg[2] = {wpb0, cw0};
  hipError_t e = hipMemcpyAsync(snap, h->buf[h->cur], bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) s = hip_fail(e, "autotune set-up");
  for (int c = 0; c < 2 && !s; ++c)
    for (int a = 0; a < 3 && !s; ++a) {
      s = dimp_set_patch_launch(h, 0, wpbs[a], cws[c]);
      float ms = 0.0f;
      if (!s) s = autotune_trial(h, snap, bytes, cur0, step0, nsteps, cfl, e0, e1, &ms);
      if (!s && ms < best_ms) {
        best_ms = ms;
        best_cfg[0] = wpbs[a];
        best_cfg[1] = cws[c];
      }
    }
  // keep the winner (or the previous shape after a failure); restore the state
  const dimp_status s2 = s ? dimp_set_patch_launch(h, per_patch0, wpb0, cw0)
                           : dimp_set_patch_launch(h, per_patch0, best_cfg[0], best_cfg[1]);
  h->cur = cur0;
  h->step = step0;
  hipError_t re = hipMemcpyAsync(h->buf[h->cur], snap, bytes, hipMemcpyDeviceToDevice, h->stream);
  if (re == hipSuccess) re = hipStreamSynchronize(h->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->smax_valid = false;
  if (s) return s;
  if (s2) return s2;
  if (re != hipSuccess) return hip_fail(re, "autotune restore");
  if (best) {
    best[0] = best_cfg[0];
    best[1] = best_cfg[1];
  }
  return DIMP_OK;
}

namespace {

// configuration checks of the adjoint and its workspace (allocated on first use)
dimp_status need_adjoint(dimp_ctx* h) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (h->patches) return fail(DIMP_EUNSUPPORTED, "the adjoint runs on single grids");
  if (h->integrator != DIMP_INTEGRATOR_SPLIT) return fail(DIMP_ESTATE, "the adjoint reverses the split integrator");
  if (h->ndim != 2 || h->nmat != 2 || h->hist())
    return fail(DIMP_EUNSUPPORTED, "the adjoint is built for 2-D, two materials, no reactive mixture");
  if (h->opt.limiter != DIMP_LIMITER_VANALBADA)
    return fail(DIMP_EUNSUPPORTED, "the adjoint needs the van Albada limiter (smooth slopes)");
  for (int d = 0; d < 2; ++d) {
    if (h->bc[d] == DIMP_BC_PERIODIC && h->n[d] < 6)
      return fail(DIMP_EUNSUPPORTED, "the adjoint needs >= 6 cells along a periodic axis");
    if (h->bc[d] == DIMP_BC_REFLECTIVE || h->bc[d] == DIMP_BC_AXIS)
      return fail(DIMP_EUNSUPPORTED, "the adjoint is built for transmissive and periodic boundaries");
  }
  if (h->geom) return fail(DIMP_EUNSUPPORTED, "the adjoint is built for Cartesian grids");
  if (!h->aw) return fail(DIMP_ESTATE, "the bound workspace has no adjoint region: bind one sized for DIMP_WS_ADJOINT");
  return DIMP_OK;
}

double* aw_state(dimp_ctx* h, int k) { return h->aw + (size_t)k * h->nfields() * h->ncell(); }
double* aw_tang(dimp_ctx* h) { return h->aw + (size_t)3 * h->nfields() * h->ncell(); }
double* aw_part(dimp_ctx* h) { return aw_tang(h) + (size_t)2 * h->ncell(); }

dimp_status adjoint_args(const double* a, const double* b, const double* c, const double* dp) {
  if (!a || !b || !c || !dp) return fail(DIMP_EINVAL, "null argument");
  if (c == a || c == b) return fail(DIMP_EINVAL, "the output adjoint must not alias an input");
  return DIMP_OK;
}

}  // namespace

dimp_status dimp_adjoint_sweep(dimp_handle h, double dt, int dir, const double* state_in, const double* adj_out,
                               double* adj_in, double* dparams) {
  dimp_status s = need_adjoint(h);
  if (s) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DIMP_EINVAL, "dt must be positive and finite");
  if (dir < 0 || dir > 1) return fail(DIMP_EINVAL, "dir %d out of range", dir);
  s = adjoint_args(state_in, adj_out, adj_in, dparams);
  if (s) return s;
  HIPCHECK(dimp::launch_sweep_adjoint(h->P, dir, state_in, adj_out, adj_in, aw_tang(h), aw_part(h), dparams, dt,
                                      h->stream),
           "sweep adjoint");
  return DIMP_OK;
}

dimp_status dimp_adjoint_plastic(dimp_handle h, const double* state_in, const double* adj_out, double* adj_in,
                                 double* dparams) {
  dimp_status s = need_adjoint(h);
  if (s) return s;
  s = adjoint_args(state_in, adj_out, adj_in, dparams);
  if (s) return s;
  HIPCHECK(dimp::launch_plastic_adjoint(h->P, state_in, adj_out, adj_in, aw_part(h), dparams, h->stream),
           "plastic adjoint");
  return DIMP_OK;
}

dimp_status dimp_adjoint_step(dimp_handle h, double dt, int64_t step_index, const double* state_in,
                              const double* adj_out, double* adj_in, double* dparams) {
  return dimp_adjoint_step_kept(h, dt, step_index, state_in, nullptr, adj_out, adj_in, dparams);
}

dimp_status dimp_adjoint_step_kept(dimp_handle h, double dt, int64_t step_index, const double* state_in,
                                   const double* first_sweep, const double* adj_out, double* adj_in,
                                   double* dparams) {
  dimp_status s = need_adjoint(h);
  if (s) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DIMP_EINVAL, "dt must be positive and finite");
  if (step_index < 0) return fail(DIMP_EINVAL, "step index must be >= 0");
  s = adjoint_args(state_in, adj_out, adj_in, dparams);
  if (s) return s;
  if (first_sweep && first_sweep == adj_in) return fail(DIMP_EINVAL, "the output adjoint must not alias an input");
  const int d1 = (step_index % 2 == 0) ? 0 : 1, d2 = 1 - d1;
  const double* U1 = first_sweep;
  double* U2 = aw_state(h, 1);
  double* tmp = aw_state(h, 2);
  // recompute the intermediate states of the step (the sweeps of the
  // forward); a caller that kept the first sweep's output passes it
  if (!U1) {
    HIPCHECK(dimp::launch_sweep(h->P, 2, false, state_in, aw_state(h, 0), dt, nullptr, d1, false, h->dpart,
                                dimp::COL_SEGMENT, h->stream),
             "adjoint: recompute sweep");
    U1 = aw_state(h, 0);
  }
  HIPCHECK(dimp::launch_sweep(h->P, 2, false, U1, U2, dt, nullptr, d2, false, h->dpart, dimp::COL_SEGMENT,
                              h->stream),
           "adjoint: recompute sweep");
  // reverse: plastic relaxation, second sweep, first sweep
  // the three parameter partial-sum sets side by side, totalled once
  const int64_t nc = dimp::adjoint_cell_blocks(h->P), n2 = dimp::adjoint_sweep_blocks(h->P, d2);
  double* part = aw_part(h);
  HIPCHECK(dimp::launch_plastic_adjoint(h->P, U2, adj_out, tmp, part, nullptr, h->stream), "plastic adjoint");
  HIPCHECK(dimp::launch_sweep_adjoint(h->P, d2, U1, tmp, U2, aw_tang(h), part + 12 * nc, nullptr, dt, h->stream),
           "sweep adjoint");
  HIPCHECK(dimp::launch_sweep_adjoint(h->P, d1, state_in, U2, adj_in, aw_tang(h), part + 12 * (nc + n2), nullptr, dt,
                                      h->stream),
           "sweep adjoint");
  HIPCHECK(dimp::launch_param_total(part, adjoint_blocks(h), dparams, h->stream), "parameter total");
  return DIMP_OK;
}

dimp_status dimp_adjoint_params(dimp_handle h, const double raw[12], double grad[8]) {
  if (!h || !raw || !grad) return fail(DIMP_EINVAL, "null argument");
  if (!h->mats_set) return fail(DIMP_ESTATE, "materials not set");
  if (h->nmat != 2) return fail(DIMP_EUNSUPPORTED, "the adjoint is built for two materials");
  for (int l = 0; l < 2; ++l) {
    const dimp_material& m = h->mats[l];
    const dimp::MatP q = pack_material(m);
    const double* r = raw + 6 * l;
    double* g = grad + 4 * l;
    // gamma (or Gamma0): Gamma = gamma - 1 (Gamma0), 1/Gamma, and p_ref = -gamma p_inf
    g[0] = r[0] - r[1] / (q.Gam * q.Gam);
    g[1] = 0.0;
    if (m.eos == DIMP_EOS_STIFFENED) {
      g[0] += r[2] * (-m.pinf);
      g[1] = r[2] * (-m.gamma);
    }
    g[2] = (m.eos == DIMP_EOS_ROMENSKII) ? r[4] : 0.0;
    g[3] = (m.eos == DIMP_EOS_ROMENSKII) ? r[5] / std::sqrt(6.0) : 0.0;
  }
  return DIMP_OK;
}

dimp_status dimp_with_velocity(dimp_handle h, const double* rest_dev, const double* vel_dev, double* out_dev) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (h->patches) return fail(DIMP_EUNSUPPORTED, "velocity fields are set on grids");
  if (h->nmat != 2) return fail(DIMP_EUNSUPPORTED, "velocity fields are built for two materials");
  if (!rest_dev || !vel_dev || !out_dev) return fail(DIMP_EINVAL, "null argument");
  if (out_dev == vel_dev) return fail(DIMP_EINVAL, "the output must not alias the velocity");
  HIPCHECK(dimp::launch_with_velocity(h->ndim, h->hist(), h->ncell(), rest_dev, vel_dev, out_dev, h->stream),
           "with_velocity");
  return DIMP_OK;
}

dimp_status dimp_with_velocity_adjoint(dimp_handle h, const double* rest_dev, const double* vel_dev,
                                       const double* adj_out_dev, double* adj_rest_dev, double* adj_vel_dev) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (h->patches) return fail(DIMP_EUNSUPPORTED, "velocity fields are set on grids");
  if (h->nmat != 2) return fail(DIMP_EUNSUPPORTED, "velocity fields are built for two materials");
  if (!rest_dev || !vel_dev || !adj_out_dev || !adj_rest_dev || !adj_vel_dev) return fail(DIMP_EINVAL, "null argument");
  for (const double* o : {static_cast<const double*>(adj_rest_dev), static_cast<const double*>(adj_vel_dev)})
    if (o == rest_dev || o == vel_dev || o == adj_out_dev)
      return fail(DIMP_EINVAL, "the output adjoints must not alias an input");
  if (adj_rest_dev == adj_vel_dev) return fail(DIMP_EINVAL, "the two output adjoints must differ");
  HIPCHECK(dimp::launch_with_velocity_adj(h->ndim, h->hist(), h->ncell(), rest_dev, vel_dev, adj_out_dev,
                                          adj_rest_dev, adj_vel_dev, h->stream),
           "with_velocity adjoint");
  return DIMP_OK;
}

}  // extern "C"

// ------------------------------------------------------ no-allocation step
// Scratch memory of dimp_advance_static: the reduction words (first 256
// bytes), then the wave-speed slots of the fused sweep and the first stage of
// their reduction.  One array per GPU, held until the process ends; every
// call on a GPU shares it.  In host code `scratch` names a host-side stand-in:
// kernels and copies take the device address from hipGetSymbolAddress, taken
// once per device with that device current.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[MAX_DEVICES] = {};

dimp_status static_scratch(unsigned char** out) {
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(DIMP_EUNSUPPORTED, "device %d beyond the static scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "static scratch address");
    g_scratch_dev[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_dev[dev];
  return DIMP_OK;
}

}  // namespace

extern "C" {

dimp_status dimp_advance_static(dimp_handle h, double dt, double* smax_dev) {
  dimp_status s = need_bound(h);
  if (s) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DIMP_EINVAL, "dt must be positive and finite");
  if (!smax_dev) return fail(DIMP_EINVAL, "null wave-speed output");
  if (h->integrator != DIMP_INTEGRATOR_SPLIT)
    return fail(DIMP_EUNSUPPORTED, "the no-allocation step runs the split integrator (the RK3 needs stage states)");
  const int64_t cap = slot_need(h);
  const size_t need = 256 + (size_t)(cap + dimp::reduce_smax_blocks(cap)) * 3 * sizeof(double);
  if (need > STATIC_SCRATCH_BYTES)
    return fail(DIMP_EINVAL, "this grid needs %zu bytes of static scratch; the limit is %zu (use dimp_advance)", need,
                STATIC_SCRATCH_BYTES);
  unsigned char* base = nullptr;
  s = static_scratch(&base);
  if (s) return s;
  // the step's kernels take the static words and slots in place of the
  // workspace's; the handle's own are restored afterwards
  unsigned long long* keep_smax = h->dsmax;
  double* keep_part = h->dpart;
  const int64_t keep_cap = h->part_cap;
  h->dsmax = reinterpret_cast<unsigned long long*>(base);
  h->dpart = reinterpret_cast<double*>(base + 256);
  h->part_cap = cap;
  s = step_once(h, dt, nullptr);
  hipError_t e = hipSuccess;
  if (!s) e = dimp::launch_u64_to_f64(h->dsmax, smax_dev, 3, h->stream);
  h->dsmax = keep_smax;
  h->dpart = keep_part;
  h->part_cap = keep_cap;
  h->smax_valid = false;  // the handle's words do not hold this state's wave speed
  if (s) return s;
  if (e != hipSuccess) return hip_fail(e, "wave-speed copy");
  return DIMP_OK;
}

dimp_status dimp_set_integrator(dimp_handle h, int integrator) {
  if (!h) return fail(DIMP_EINVAL, "null handle");
  if (integrator != DIMP_INTEGRATOR_SPLIT && integrator != DIMP_INTEGRATOR_RK3)
    return fail(DIMP_EINVAL, "unknown integrator %d", integrator);
  if (integrator == DIMP_INTEGRATOR_RK3 && h->patches)
    return fail(DIMP_EUNSUPPORTED, "the RK3 integrator is built for grids, not patch sets");
  if (integrator == DIMP_INTEGRATOR_RK3 && h->bound && !h->rkw)
    return fail(DIMP_ESTATE, "the bound workspace has no RK3 region: bind one sized for DIMP_WS_RK3");
  h->integrator = integrator;
  drop_graph(h);
  h->smax_valid = false;
  return DIMP_OK;
}

dimp_status dimp_set_geometry(dimp_handle h, int geometry, double r_lo) {
  if (!h) return fail(DIMP_EINVAL, "null handle");
  if (geometry != DIMP_GEOMETRY_CARTESIAN && geometry != DIMP_GEOMETRY_CYLINDRICAL)
    return fail(DIMP_EINVAL, "unknown geometry %d", geometry);
  if (geometry == DIMP_GEOMETRY_CYLINDRICAL) {
    if (h->patches) return fail(DIMP_EUNSUPPORTED, "patch sets are built Cartesian");
    if (h->ndim != 2) return fail(DIMP_EUNSUPPORTED, "the cylindrical form is 2-D (x = r, y = z)");
    if (!(r_lo >= 0.0) || !std::isfinite(r_lo)) return fail(DIMP_EINVAL, "r_lo must be >= 0 and finite");
  }
  h->geom = geometry;
  h->r_lo = (geometry == DIMP_GEOMETRY_CYLINDRICAL) ? r_lo : 0.0;
  rebuild_params(h);
  drop_graph(h);
  h->smax_valid = false;
  return DIMP_OK;
}

dimp_status dimp_set_step_index(dimp_handle h, int64_t step) {
  if (!h) return fail(DIMP_EINVAL, "null handle");
  if (step < 0) return fail(DIMP_EINVAL, "step index must be >= 0");
  h->step = step;
  return DIMP_OK;
}

static dimp_status ensure_smax(dimp_handle h) {
  if (!h->smax_valid) {
    HIPCHECK(dimp::launch_wavespeed(h->P, h->ndim, h->rxk(), h->buf[h->cur], h->dsmax, h->stream), "wavespeed");
    h->smax_valid = true;
  }
  return DIMP_OK;
}

dimp_status dimp_max_wavespeed(dimp_handle h, double smax[3]) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (!smax) return fail(DIMP_EINVAL, "null output");
  s = ensure_smax(h);
  if (s) return s;
  unsigned long long bits[3] = {0, 0, 0};
  HIPCHECK(hipMemcpyAsync(bits, h->dsmax, sizeof bits, hipMemcpyDeviceToHost, h->stream), "wavespeed copy");
  HIPCHECK(hipStreamSynchronize(h->stream), "wavespeed sync");
  for (int d = 0; d < 3; ++d) {
    double v;
    std::memcpy(&v, &bits[d], sizeof v);
    smax[d] = d < h->ndim ? v : 0.0;
  }
  return DIMP_OK;
}

dimp_status dimp_max_wavespeed_device(dimp_handle h, double* smax_dev) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (!smax_dev) return fail(DIMP_EINVAL, "null output");
  s = ensure_smax(h);
  if (s) return s;
  HIPCHECK(dimp::launch_u64_to_f64(h->dsmax, smax_dev, 3, h->stream), "wavespeed convert");
  return DIMP_OK;
}

dimp_status dimp_check_state(dimp_handle h, int64_t* nbad) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (!nbad) return fail(DIMP_EINVAL, "null output");
  HIPCHECK(dimp::launch_check(h->P, h->ndim, h->rxk(), h->buf[h->cur], h->dsmax + 3, h->stream), "check");
  unsigned long long v[3] = {0, 0, 0};  // bad cells, dt, status
  HIPCHECK(hipMemcpyAsync(v, h->dsmax + 3, sizeof v, hipMemcpyDeviceToHost, h->stream), "check copy");
  HIPCHECK(hipStreamSynchronize(h->stream), "check sync");
  *nbad = (int64_t)v[0];
  if (v[2]) {  // reported once
    HIPCHECK(dimp::launch_zero_u64(h->dsmax + 5, 1, h->stream), "status clear");
    return fail(DIMP_ENONPHYSICAL, "a device CFL time step was not finite and positive (that step ran with dt = 0); "
                "%llu non-physical cells", v[0]);
  }
  if (v[0]) return fail(DIMP_ENONPHYSICAL, "%llu non-physical cells", v[0]);
  return DIMP_OK;
}

dimp_status dimp_set_kernel_timing(dimp_handle h, int enable) {
  if (!h) return fail(DIMP_EINVAL, "null handle");
  h->timing = enable != 0;
  h->ev_used = 0;
  h->ev_kind.clear();
  return DIMP_OK;
}

dimp_status dimp_kernel_times(dimp_handle h, double ms[6], int64_t counts[6]) {
  if (!h || !ms || !counts) return fail(DIMP_EINVAL, "null argument");
  for (int k = 0; k < 6; ++k) {
    ms[k] = 0.0;
    counts[k] = 0;
  }
  if (h->ev_used) HIPCHECK(hipStreamSynchronize(h->stream), "timing sync");
  for (size_t i = 0; i < h->ev_used; ++i) {
    float t = 0.0f;
    HIPCHECK(hipEventElapsedTime(&t, h->ev_pool[2 * i], h->ev_pool[2 * i + 1]), "event elapsed");
    ms[h->ev_kind[i]] += t;
    counts[h->ev_kind[i]] += 1;
  }
  h->ev_used = 0;
  h->ev_kind.clear();
  return DIMP_OK;
}

// ------------------------------------------------------------ refinement
struct dimp_amr_ctx {
  dimp_ctx* coarse = nullptr;
  dimp_ctx* fine = nullptr;
  dimp::AmrBox box{};
  // caller-owned workspace (dimp_amr_workspace_bytes): the coarse state
  // before its step (time interpolation), then the fluxes through the
  // coarse/fine boundary ([F][2][len] per set): the coarse step's, then the
  // two fine steps'
  double* cold = nullptr;
  double* flux = nullptr;
  FluxTap tap[3]{};
  hipStream_t side = nullptr;  // the flux kernels' stream (default priority)
  // nesting: `inner` refines this hierarchy's fine grid (its coarse grid is
  // our fine one) and is advanced in place of stepping that grid; `outer` is
  // the hierarchy this one is nested in
  dimp_amr_ctx* inner = nullptr;
  dimp_amr_ctx* outer = nullptr;
  // several patches on one level: hierarchies over the same coarse grid,
  // listed from the head (head == nullptr for the head or a lone one), are
  // stepped together through the head
  dimp_amr_ctx* head = nullptr;
  dimp_amr_ctx* next = nullptr;
};

static void amr_release(dimp_amr_ctx* a) {
  if (a->inner) a->inner->outer = nullptr;
  if (a->outer) a->outer->inner = nullptr;
  if (a->head) {  // a member leaves its group
    dimp_amr_ctx* q = a->head;
    while (q->next != a) q = q->next;
    q->next = a->next;
  } else {  // a head's members become lone hierarchies
    for (dimp_amr_ctx* q = a->next; q;) {
      dimp_amr_ctx* n = q->next;
      q->head = nullptr;
      q->next = nullptr;
      q = n;
    }
  }
  for (FluxTap& t : a->tap)
    for (int k = 0; k < 2; ++k) {
      if (t.ready[k]) (void)hipEventDestroy(t.ready[k]);
      if (t.done[k]) (void)hipEventDestroy(t.done[k]);
    }
  if (a->side) (void)hipStreamDestroy(a->side);
  delete a;
}

// the hierarchy's workspace: the coarse state before its step, then the
// boundary fluxes ([F][2][len] per face set: the coarse step's and the two
// fine steps')
static size_t amr_ws_cold(const dimp_ctx* c) { return ws_align(sizeof(double) * (size_t)c->nfields() * c->ncell()); }
static size_t amr_ws_flux(const dimp_ctx* c, const int64_t box[4]) {
  return ws_align(sizeof(double) * (size_t)(c->nfields() * 2 * ((box[2] - box[0]) + (box[3] - box[1])) * 5));
}

dimp_status dimp_amr_workspace_bytes(dimp_handle coarse, const int64_t box[4], size_t* bytes) {
  if (!coarse || !box || !bytes) return fail(DIMP_EINVAL, "null argument");
  if (!coarse->mats_set) return fail(DIMP_ESTATE, "materials not set");
  if (box[2] <= box[0] || box[3] <= box[1]) return fail(DIMP_EINVAL, "empty box");
  *bytes = amr_ws_cold(coarse) + amr_ws_flux(coarse, box);
  return DIMP_OK;
}

dimp_status dimp_amr_create(dimp_handle coarse, dimp_handle fine, const int64_t box[4], void* workspace,
                            size_t ws_bytes, dimp_amr* out) {
  if (!coarse || !fine || !box || !out || !workspace) return fail(DIMP_EINVAL, "null argument");
  *out = nullptr;
  for (dimp_ctx* h : {coarse, fine}) {
    dimp_status s = need_ws(h);
    if (s) return s;
    if (h->patches) return fail(DIMP_EUNSUPPORTED, "refinement levels are grids, not patch sets");
    if (h->ndim != 2) return fail(DIMP_EUNSUPPORTED, "refinement is built for 2-D grids");
  }
  if (coarse == fine) return fail(DIMP_EINVAL, "the two levels must be different grids");
  if (coarse->nfields() != fine->nfields() || coarse->nmat != fine->nmat || coarse->rx.mat != fine->rx.mat ||
      coarse->rxk() != fine->rxk())
    return fail(DIMP_EINVAL, "the two levels must carry the same fields");
  if (coarse->stream != fine->stream) return fail(DIMP_EINVAL, "the two levels must be bound on one stream");
  const int64_t i0 = box[0], j0 = box[1], i1 = box[2], j1 = box[3];
  const int G = 4;
  if (!(i0 >= 3 && j0 >= 3 && i1 > i0 && j1 > j0 && i1 <= coarse->n[0] - 3 && j1 <= coarse->n[1] - 3))
    return fail(DIMP_EINVAL, "the patch must lie at least 3 coarse cells inside the coarse grid");
  if (fine->n[0] != 2 * (i1 - i0) + 2 * G || fine->n[1] != 2 * (j1 - j0) + 2 * G)
    return fail(DIMP_EINVAL, "the fine grid must be %lld x %lld (the patch at ratio 2 with %d ghost layers)",
                (long long)(2 * (i1 - i0) + 2 * G), (long long)(2 * (j1 - j0) + 2 * G), G);
  for (int d = 0; d < 2; ++d)
    if (std::fabs(2.0 * fine->dx[d] - coarse->dx[d]) > 1e-12 * coarse->dx[d])
      return fail(DIMP_EINVAL, "the fine cell widths must be half the coarse ones");
  const size_t need = amr_ws_cold(coarse) + amr_ws_flux(coarse, box);
  if (ws_bytes < need) return fail(DIMP_EINVAL, "hierarchy workspace of %zu bytes is too small (%zu needed)", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(DIMP_EINVAL, "the workspace must be 256-byte aligned");
  auto* a = new (std::nothrow) dimp_amr_ctx();
  if (!a) return fail(DIMP_ENOMEM, "host allocation failed");
  a->coarse = coarse;
  a->fine = fine;
  a->box = dimp::AmrBox{i0, j0, i1, j1, coarse->n[0], coarse->n[1], fine->n[0], fine->n[1], G, coarse->nfields()};
  a->cold = static_cast<double*>(workspace);
  a->flux = reinterpret_cast<double*>(static_cast<unsigned char*>(workspace) + amr_ws_cold(coarse));
  const int64_t pw = i1 - i0, ph = j1 - j0, F = coarse->nfields();
  hipError_t e = hipStreamCreateWithFlags(&a->side, hipStreamNonBlocking);
  for (FluxTap& t : a->tap)
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
      e = hipEventCreateWithFlags(&t.ready[k], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&t.done[k], hipEventDisableTiming);
    }
  if (e != hipSuccess) {
    amr_release(a);
    return hip_fail(e, "amr stream and events");
  }
  for (FluxTap& t : a->tap) t.side = a->side;
  // coarse faces i0, i1 (rows j0..j1-1) and j0, j1 (columns i0..i1-1); on
  // the fine level the same faces, G cells in from its edges
  a->tap[0].fs[0] = dimp::FaceSet{{i0, i1}, j0, ph};
  a->tap[0].fs[1] = dimp::FaceSet{{j0, j1}, i0, pw};
  a->tap[0].out[0] = a->flux;
  a->tap[0].out[1] = a->flux + F * 2 * ph;
  for (int s = 1; s < 3; ++s) {
    double* base = a->flux + F * 2 * (pw + ph) * (1 + 2 * (s - 1));
    a->tap[s].fs[0] = dimp::FaceSet{{G, fine->n[0] - G}, G, 2 * ph};
    a->tap[s].fs[1] = dimp::FaceSet{{G, fine->n[1] - G}, G, 2 * pw};
    a->tap[s].out[0] = base;
    a->tap[s].out[1] = base + F * 2 * 2 * ph;
  }
  fine->step = 2 * coarse->step;
  *out = a;
  return DIMP_OK;
}

// whether two patches of the head's group touch (their boxes are disjoint;
// touching ones share a face or a corner)
static bool group_touches(const dimp_amr_ctx* a) {
  for (const dimp_amr_ctx* p = a; p; p = p->next)
    for (const dimp_amr_ctx* q = p->next; q; q = q->next) {
      const dimp::AmrBox &u = p->box, &v = q->box;
      if (u.i0 <= v.i1 && v.i0 <= u.i1 && u.j0 <= v.j1 && v.j0 <= u.j1) return true;
    }
  return false;
}

// fine-to-fine exchange among the patches of the head's group (split
// integrator): every patch's stored cells inside another patch's interior <-
// that patch's state (after the coarse fills, before any patch steps; the
// ghost layers reach two coarse cells, so patches one cell apart exchange too)
static dimp_status group_exchange(dimp_amr_ctx* a) {
  for (dimp_amr_ctx* p = a; p; p = p->next)
    for (dimp_amr_ctx* q = a; q; q = q->next)
      if (q != p)
        HIPCHECK(dimp::launch_amr_exchange(p->box, q->box, q->fine->buf[q->fine->cur], p->fine->buf[p->fine->cur],
                                           a->coarse->stream),
                 "amr exchange");
  return DIMP_OK;
}

// dt of the hierarchy's coarse level: min(coarse CFL step, 2 x the finer
// levels' dt), each finer level after a ghost fill from the level above (and
// the exchange among touching patches)
static dimp_status amr_dt(dimp_amr_ctx* a, double cfl, double* dt) {
  dimp_ctx* c = a->coarse;
  const double* cu = c->buf[c->cur];
  double sc[3];
  dimp_status s = dimp_max_wavespeed(c, sc);
  if (s) return s;
  double dc = INFINITY, df = INFINITY;
  for (int d = 0; d < 2; ++d) dc = std::min(dc, cfl * (c->dx[d] / sc[d]));
  for (dimp_amr_ctx* q = a; q; q = q->next) {  // every patch of the level
    HIPCHECK(dimp::launch_amr_fill(q->box, cu, cu, 0.0, q->fine->buf[q->fine->cur], c->stream), "amr fill");
    q->fine->smax_valid = false;
  }
  if (a->next && c->integrator != DIMP_INTEGRATOR_RK3) {
    s = group_exchange(a);
    if (s) return s;
  }
  for (dimp_amr_ctx* q = a; q; q = q->next) {
    dimp_ctx* f = q->fine;
    if (q->inner) {
      double di;
      s = amr_dt(q->inner, cfl, &di);
      if (s) return s;
      df = std::min(df, di);
    } else {
      double sf[3];
      s = dimp_max_wavespeed(f, sf);
      if (s) return s;
      for (int d = 0; d < 2; ++d) df = std::min(df, cfl * (f->dx[d] / sf[d]));
    }
  }
  *dt = std::min(dc, 2.0 * df);
  return DIMP_OK;
}

// One coarse step of dt with the finer levels subcycled, for every patch of
// the head's group; outer_tap: the faces of the patch the coarse grid is in a
// nested stack (its fluxes are recorded for the level above's correction)
static dimp_status amr_advance(dimp_amr_ctx* a, double dt, const FluxTap* outer_tap,
                               const RkHook* outer_hook = nullptr) {
  dimp_ctx* c = a->coarse;
  const bool rk3 = c->integrator == DIMP_INTEGRATOR_RK3;
  if (rk3 && group_touches(a)) return fail(DIMP_EUNSUPPORTED, "touching patches step the split integrator only");
  std::vector<const FluxTap*> taps;
  for (dimp_amr_ctx* q = a; q; q = q->next) {
    if (q->fine->integrator != c->integrator)
      return fail(DIMP_EINVAL, "the levels of a hierarchy must step the same integrator");
    taps.push_back(&q->tap[0]);
  }
  if (outer_tap) taps.push_back(outer_tap);
  const size_t bytes = sizeof(double) * (size_t)c->nfields() * c->ncell();
  HIPCHECK(hipMemcpyAsync(a->cold, c->buf[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream), "amr save");
  dimp_status s = step_once(c, dt, nullptr, taps.data(), (int)taps.size(), outer_hook);
  if (s) return s;
  for (dimp_amr_ctx* q = a; q; q = q->next)
    HIPCHECK(hipStreamWaitEvent(c->stream, q->tap[0].done[1], 0), "stream wait");
  // per substep: every patch's coarse fill, the exchange among the patches
  // (split integrator), then every patch's step
  for (int sub = 0; sub < 2; ++sub) {
    for (dimp_amr_ctx* q = a; q; q = q->next)
      HIPCHECK(dimp::launch_amr_fill(q->box, a->cold, c->buf[c->cur], 0.5 * sub, q->fine->buf[q->fine->cur],
                                     c->stream),
               "amr fill");
    if (a->next && !rk3) {
      s = group_exchange(a);
      if (s) return s;
    }
    for (dimp_amr_ctx* q = a; q; q = q->next) {
      const FluxTap* t = &q->tap[1 + sub];
      const RkHook hk{&q->box, a->cold, c->buf[c->cur], sub};
      s = q->inner ? amr_advance(q->inner, 0.5 * dt, t, &hk) : step_once(q->fine, 0.5 * dt, nullptr, &t, 1, &hk);
      if (s) return s;
      HIPCHECK(hipStreamWaitEvent(c->stream, t->done[1], 0), "stream wait");
    }
  }
  // the flux correction of the conserved fields (partial densities, history
  // slot, momentum, energy; the volume fractions and Vbar, whose sweeps carry
  // non-conservative terms, are left), then the averaging down: a corrected
  // cell that another patch covers takes that patch's average
  const int c0 = c->nmat - 1, c1 = c->nfields() - 5;
  const double lam[2] = {dt / c->dx[0], dt / c->dx[1]};
  for (dimp_amr_ctx* q = a; q; q = q->next) {
    HIPCHECK(dimp::launch_amr_reflux(q->box, c0, c1, lam, q->tap[0].out, q->tap[1].out, q->tap[2].out,
                                     c->buf[c->cur], c->stream),
             "amr reflux");
    q->fine->smax_valid = false;
  }
  for (dimp_amr_ctx* q = a; q; q = q->next)
    HIPCHECK(dimp::launch_amr_average(q->box, q->fine->buf[q->fine->cur], c->buf[c->cur], c->stream),
             "amr average");
  c->smax_valid = false;
  return DIMP_OK;
}

dimp_status dimp_amr_dt(dimp_amr a, double cfl, double* dt) {
  if (!a || !dt) return fail(DIMP_EINVAL, "null argument");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(DIMP_EINVAL, "cfl must be positive");
  if (a->outer) return fail(DIMP_ESTATE, "a nested hierarchy is stepped through the one it is nested in");
  if (a->head) return fail(DIMP_ESTATE, "a grouped hierarchy is stepped through its group's head");
  return amr_dt(a, cfl, dt);
}

dimp_status dimp_amr_advance(dimp_amr a, double dt) {
  if (!a) return fail(DIMP_EINVAL, "null handle");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DIMP_EINVAL, "dt must be positive and finite");
  if (a->outer) return fail(DIMP_ESTATE, "a nested hierarchy is stepped through the one it is nested in");
  if (a->head) return fail(DIMP_ESTATE, "a grouped hierarchy is stepped through its group's head");
  return amr_advance(a, dt, nullptr);
}

dimp_status dimp_amr_group(dimp_amr head, dimp_amr member) {
  if (!head || !member) return fail(DIMP_EINVAL, "null handle");
  if (head == member || head->coarse != member->coarse)
    return fail(DIMP_EINVAL, "the hierarchies of a group share their coarse grid");
  if (head->head || member->head || member->next || member->outer)
    return fail(DIMP_ESTATE, "group a lone hierarchy under a head that is not a member");
  if (head->outer) {  // a nested group: every patch 7 cells inside the outer fine grid
    const dimp::AmrBox& b = member->box;
    const int64_t m = head->outer->box.G + 3;
    if (b.i0 < m || b.j0 < m || b.i1 > b.nxc - m || b.j1 > b.nyc - m)
      return fail(DIMP_EINVAL, "the patch must lie at least %lld cells inside the outer fine grid", (long long)m);
  }
  for (dimp_amr_ctx* q = head; q; q = q->next) {
    const dimp::AmrBox &p = q->box, &b = member->box;
    if (p.i0 < b.i1 && b.i0 < p.i1 && p.j0 < b.j1 && b.j0 < p.j1)
      return fail(DIMP_EINVAL, "patches of a group must not share a coarse cell");
  }
  dimp_amr_ctx* q = head;
  while (q->next) q = q->next;
  q->next = member;
  member->head = head;
  return DIMP_OK;
}

dimp_status dimp_amr_nest(dimp_amr outer, dimp_amr inner) {
  if (!outer || !inner) return fail(DIMP_EINVAL, "null handle");
  if (outer == inner || inner->coarse != outer->fine)
    return fail(DIMP_EINVAL, "the inner hierarchy's coarse grid must be the outer one's fine grid");
  if (outer->inner || inner->outer) return fail(DIMP_ESTATE, "a hierarchy nests at most one and in at most one");
  if (inner->head) return fail(DIMP_ESTATE, "nest the head of a group");
  {  // every fine grid of inner's tree (its group, and what each nests)
    std::vector<dimp_amr_ctx*> todo{inner};
    while (!todo.empty()) {
      dimp_amr_ctx* q = todo.back();
      todo.pop_back();
      for (; q; q = q->next) {
        if (q->fine == outer->coarse) return fail(DIMP_EINVAL, "nesting would form a cycle");
        if (q->inner) todo.push_back(q->inner);
      }
    }
  }
  // the inner patch's ghost fill reads its parents and their neighbours,
  // which must be interior cells of the outer fine grid
  const int64_t m = outer->box.G + 3;
  for (dimp_amr_ctx* q = inner; q; q = q->next) {  // every patch of the inner group
    const dimp::AmrBox& b = q->box;
    if (b.i0 < m || b.j0 < m || b.i1 > b.nxc - m || b.j1 > b.nyc - m)
      return fail(DIMP_EINVAL, "the inner patch must lie at least %lld cells inside the outer fine grid", (long long)m);
  }
  outer->inner = inner;
  inner->outer = outer;
  inner->fine->step = 2 * inner->coarse->step;
  return DIMP_OK;
}

dimp_status dimp_amr_prolong(dimp_amr a) {
  if (!a) return fail(DIMP_EINVAL, "null handle");
  dimp_ctx* c = a->coarse;
  dimp_ctx* f = a->fine;
  const double* cu = c->buf[c->cur];
  HIPCHECK(dimp::launch_amr_fill(a->box, cu, cu, 0.0, f->buf[f->cur], c->stream, true), "amr prolong");
  f->smax_valid = false;
  return DIMP_OK;
}

dimp_status dimp_amr_tag(dimp_handle h, const double* prim, double threshold, uint8_t* tags, int64_t bbox[4]) {
  dimp_status s = need_ws(h);
  if (s) return s;
  if (!prim || !tags || !bbox) return fail(DIMP_EINVAL, "null argument");
  if (h->patches || h->ndim != 2) return fail(DIMP_EUNSUPPORTED, "the refinement criterion is built for 2-D grids");
  if (!(threshold > 0.0) || !std::isfinite(threshold)) return fail(DIMP_EINVAL, "threshold must be positive");
  const int N = h->nmat;
  dimp::TagLayout t;
  t.nphi = N - 1;
  t.rho0 = N - 1;
  t.nmat = N;
  t.u0 = 2 * N - 1 + (h->hist() ? 1 : 0);
  t.ndim = 2;
  t.p = t.u0 + 2;
  t.nx = h->n[0];
  t.ny = h->n[1];
  t.floor_phi = 1e-6 * h->opt.va_scale[0];
  t.floor_rho = 1e-6 * h->opt.va_scale[1];
  t.floor_u = 1e-6 * h->opt.va_scale[3];
  t.floor_p = 1e-6 * h->opt.va_scale[4];
  const unsigned long long init[4] = {~0ULL, ~0ULL, 0ULL, 0ULL};
  HIPCHECK(hipMemcpyAsync(h->dtag, init, sizeof init, hipMemcpyHostToDevice, h->stream), "tag init");
  HIPCHECK(dimp::launch_amr_tag(t, prim, threshold, tags, h->dtag, h->stream), "amr tag");
  unsigned long long out[4];
  HIPCHECK(hipMemcpyAsync(out, h->dtag, sizeof out, hipMemcpyDeviceToHost, h->stream), "tag read");
  HIPCHECK(hipStreamSynchronize(h->stream), "tag sync");
  if (out[0] == ~0ULL) {
    for (int k = 0; k < 4; ++k) bbox[k] = 0;
  } else {
    bbox[0] = (int64_t)out[0];
    bbox[1] = (int64_t)out[1];
    bbox[2] = (int64_t)out[2] + 1;
    bbox[3] = (int64_t)out[3] + 1;
  }
  return DIMP_OK;
}

dimp_status dimp_amr_destroy(dimp_amr a) {
  if (!a) return DIMP_OK;
  amr_release(a);
  return DIMP_OK;
}

dimp_status dimp_destroy(dimp_handle h) {
  if (!h) return DIMP_OK;
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  drop_graph(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->d_geo) (void)hipFree(h->d_geo);
  free_list(h->lx);
  free_list(h->lx_pp);
  for (int k = 0; k < 2; ++k) {
    free_list(h->ly[k]);
    free_list(h->ly_pp[k]);
  }
  delete h;
  return DIMP_OK;
}

}  // extern "C"
