/*
 * dimp.h -- C-ABI of the MI355X diffuse-interface multiphysics step.
 *
 * The library advances the single hyperbolic system of Wallis, Barton &
 * Nikiforakis (arXiv 2009.14555, Sec. 2.1 and the vector form of Sec. 3) for
 * N materials -- ideal gases, stiffened gases and Romenskii elastoplastic
 * solids (Sec. 2.3), plus at most one reactive two-component mixture (Sec.
 * 2.3.1, Appendix B) -- on a regular Cartesian grid of 1, 2 or 3 dimensions,
 * with one explicit step per call: dimensionally split MUSCL-Hancock sweeps
 * on primitive variables (Sec. 3.1), THINC/BVD steepening of the volume
 * fractions (Appendix A), an HLLC-type flux with the non-conservative terms of
 * phi and Vbar, then the plastic (Sec. 3.2) and reactive (Sec. 3.3)
 * fractional steps, and the CFL wave-speed reduction.
 *
 * Conventions shared by every entry point:
 *  - Every call returns dimp_status: 0 = DIMP_OK, negative = error.  No C++
 *    exception crosses the ABI.  dimp_last_error() returns a thread-local,
 *    NUL-terminated message for the last failing call of this thread.
 *  - Pointers named *_dev are device (HBM) pointers; the caller owns them and
 *    keeps them alive while they are bound.  Host pointers are read during the
 *    call only.
 *  - All floating point is IEEE binary64.  The state is structure-of-arrays,
 *    field-major: field f of cell (i,j,k) is at
 *        f*ncell + i + n0*(j + n1*k),   ncell = n0*n1*n2,
 *    with field order
 *        phi_1..phi_{N-1} | m_1..m_N | [m_lambda] | rho u_1..rho u_D | rho E | Vbar
 *    where m_l = phi_l rho_l, m_lambda = phi_y rho_y lambda of the reactive
 *    material y, and the Vbar entries are 11,22,33 (D=1), 11,12,21,22,33
 *    (D=2, plane strain) or all nine row-major (D=3).  Primitive arrays use the
 *    same slots: phi_l, rho_l (phasic), lambda, u_k, p, Vbar.
 *  - Kernels are enqueued on the stream given to dimp_bind (NULL = the null
 *    stream) and never synchronise, except where a call says it does.
 *  - Handles are not thread-safe; concurrent calls on one handle race.
 */
#ifndef DIMP_H
#define DIMP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DIMP_OK = 0,
  DIMP_EINVAL = -1,        /* bad argument (null pointer, size, value) */
  DIMP_EUNSUPPORTED = -2,  /* valid but not built (e.g. nmat != 2 on the GPU) */
  DIMP_EHIP = -3,          /* a HIP runtime call failed */
  DIMP_ENOMEM = -4,        /* device allocation failed */
  DIMP_ENONPHYSICAL = -5,  /* state check found non-physical cells */
  DIMP_ESTATE = -6         /* call out of order (e.g. advance before bind) */
} dimp_status;

typedef struct dimp_ctx* dimp_handle;

/* Boundary rule per dimension: transmissive (zero-gradient copy of the
   boundary cell), periodic (wrap), reflective walls at both ends (ghost cells
   are mirror images: the normal momentum and the stretch-tensor entries with
   exactly one normal index change sign), or AXIS: reflective at the low end
   (the symmetry axis r = 0 of the cylindrical form) and transmissive at the
   high end.  Every rule applies along any axis of 1-D, 2-D and 3-D grids. */
enum { DIMP_BC_TRANSMISSIVE = 0, DIMP_BC_PERIODIC = 1, DIMP_BC_REFLECTIVE = 2, DIMP_BC_AXIS = 3 };
enum { DIMP_EOS_IDEAL = 0, DIMP_EOS_STIFFENED = 1, DIMP_EOS_ROMENSKII = 2, DIMP_EOS_JWL = 3 };
enum { DIMP_RATE_POWER = 0, DIMP_RATE_IGNITION_GROWTH = 1 };
enum { DIMP_PLAST_NONE = 0, DIMP_PLAST_PERFECT = 1, DIMP_PLAST_JOHNSON_COOK = 2 };
enum { DIMP_LIMITER_MINMOD = 0, DIMP_LIMITER_VANALBADA = 1 };

/* One Mie-Grueneisen material, p = p_ref(rho) + rho Gamma (e - e_ref(rho))
   (Sec. 2.3).  Ideal: gamma.  Stiffened: gamma, pinf, eref (p_ref = -gamma
   pinf, e_ref = eref).  Romenskii: rho0, K0, G0, abar, bbar, Gamma0 with cold
   energy K0 (x^abar - 1)^2/(2 rho0 abar^2), x = rho/rho0, and shear modulus
   G0 x^(bbar+1).  plast/yield: ideal (perfect) plasticity with yield stress
   sigma_Y (Sec. 2.3.2), applied as an instantaneous return to the yield
   surface.  DIMP_PLAST_JOHNSON_COOK (a Romenskii solid; Sec. 2.3.2 rate
   law, Sec. 3.2 relaxation): plastic rate chi = jc[6] exp((s - 1)/jc[2]), s =
   sqrt(3/2)|dev sigma| / sigma_Y, sigma_Y = (jc[0] + jc[1] eps_p^jc[3])(1 -
   theta^jc[4]), theta = (T - T0)/(jc[5] - T0) in [0, 1] with T - T0 = (p -
   p_ref)/(rho Gamma cv); its plastic strain eps_p is stored (phi rho eps_p)
   in the history slot of the layout (see dimp_nfields), so a Johnson-Cook
   solid and a reactive mixture cannot be set together; the relaxation
   residual of Sec. 3.2 is solved per cell by safeguarded Newton steps
   inside a bisection bracket (the paper bisects; same root to rounding).  cv: specific heat (reactive
   components, Johnson-Cook softening).  JWL (Sec. 2.3, Table 3; reactive
   components only): rho0, Gamma0 and jwl = {A, B, R1, R2} with p_ref =
   A exp(-R1 rho0/rho) + B exp(-R2 rho0/rho), e_ref = A/(R1 rho0)
   exp(-R1 rho0/rho) + B/(R2 rho0) exp(-R2 rho0/rho). */
typedef struct {
  int32_t eos;
  int32_t plast;
  double gamma, pinf, eref;
  double rho0, K0, G0, abar, bbar, Gamma0;
  double cv;
  double yield;
  double jc[7]; /* Johnson-Cook: c1, c2, c3, n, m, T_melt - T0, chi0 */
  double jwl[4]; /* JWL: A, B (Pa), R1, R2 */
} dimp_material;

/* The reactive mixture (Sec. 2.3.1): material index `mat` of the list is a
   physical mixture of `reactant` (lambda = 1) and `product` (lambda = 0) at
   equal pressure and temperature; the product's reference energy is lowered
   by Q.  Components: ideal, stiffened or JWL; the split of Appendix B is
   solved in closed form for two gases and by safeguarded Newton steps on
   the temperature equality otherwise.  Rate (paper convention, lambda = 1
   unreacted), integrated by RK4 (Sec. 3.3):
     law DIMP_RATE_POWER: dlambda/dt = -k lambda (max(p,0)/pref)^n;
     law DIMP_RATE_IGNITION_GROWTH (Sec. 4.2, Table 4), F = 1 - lambda,
       rho the mixture material's own density, p in units of punit:
       dlambda/dt = -[ I (1-F)^b max(rho/rho0 - 1 - a, 0)^x H(F_ig - F)
                     + G1 (1-F)^c F^d p^y H(F_G1 - F)
                     + G2 (1-F)^e F^g p^z H(F - F_G2) ],  H(x) = [x > 0],
       with ig = {I, G1, G2, a, b, c, d, e, g, x, y, z, F_ig, F_G1, F_G2,
       rho0, punit}. */
typedef struct {
  int32_t mat; /* -1: no reactive material */
  int32_t law; /* DIMP_RATE_* */
  dimp_material reactant;
  dimp_material product;
  double Q, k, n, pref;
  double ig[17];
} dimp_reactive;

/* Numerical options.  limiter: DIMP_LIMITER_*; thinc: 1 = THINC/BVD on the
   volume fraction (Appendix A) with steepness beta0 |n_d| + 0.01, mixed-cell
   threshold delta and epsilon eps; va_scale: the van Albada epsilon is
   1e-6 times the scale of the field kind (phi, rho, lambda, u, p, Vbar). */
typedef struct {
  int32_t limiter;
  int32_t thinc;
  double beta0, delta, eps;
  double va_scale[6];
} dimp_options;

/* Create a grid of ndim (1..3) dimensions with n[d] >= 1 interior cells and
   cell widths dx[d] > 0; bc[d] is the boundary rule of dimension d
   (transmissive = zero-gradient, periodic = wrap).  Entries beyond ndim are
   ignored.  *out receives a new handle (release with dimp_destroy). */
dimp_status dimp_create_grid(int ndim, const int64_t n[3], const double dx[3], const int32_t bc[3],
                             dimp_handle* out);

/* Create a set of npatch independent 2-D patches (the patches of one AMR
   level, Sec. 3: the update runs over every patch of a level), sizes[2p],
   sizes[2p+1] = interior cells of patch p along x and y (1..65536), cell
   widths dx[0], dx[1] shared by all patches.  Every patch is stored with 2
   ghost layers: field f of cell (i, j) of patch p, -2 <= i < nx+2,
   -2 <= j < ny+2, is at  f*E + off[p] + (j+2)*(nx+4) + (i+2)  with off[] from
   dimp_patch_offsets and E = off[npatch] = the ncell of dimp_nfields.
   Boundaries are transmissive per patch (stencils clamp into the patch, so
   stored ghost values are never read); every sweep writes the ghost images of
   the boundary cells it updates, for consumers of the stored arrays.  All
   patches share one dt.  2-D, two or three materials, with or without a
   history slot (a reactive mixture, gas or JWL, or a Johnson-Cook solid). */
dimp_status dimp_create_patch_set(int64_t npatch, const int32_t* sizes, const double dx[2], dimp_handle* out);

/* Element offsets of the patches (npatch + 1 values, ghosts included). */
dimp_status dimp_patch_offsets(dimp_handle h, int64_t* offsets);

/* How a patch set is launched: per_patch = 0 runs one kernel per sweep over a
   task list of all patches (x sweep: one wave per row segment of 58 cells,
   row_waves = 1, 2 or 4 waves per block; y sweep: one block per tile of
   tile_columns = 4 or 8 columns by 58 rows); per_patch = 1 launches the same
   kernels once per patch and sweep (the baseline the batched mode is measured
   against; bitwise identical results). */
dimp_status dimp_set_patch_launch(dimp_handle h, int per_patch, int row_waves, int tile_columns);

/* Time each (row_waves, tile_columns) pair on the bound patch-set state for
   nsteps steps and keep the fastest (per_patch is left as it was); the state
   and the step counter are restored afterwards through snapshot_dev, a
   caller-owned device buffer of nfields*ncell doubles (not a bound state
   buffer).  best (nullable) receives {row_waves, tile_columns}.
   Synchronises. */
dimp_status dimp_autotune(dimp_handle h, int nsteps, double cfl, double* snapshot_dev, int best[2]);

/* ---------------------------------------------------------------- adjoint
   Vector-Jacobian products of the step (Sec. 3: split sweeps, then the
   plastic relaxation of Sec. 3.2) for calibrating material parameters: given
   the adjoint adj_out = dJ/dU of the state after an operation, they return
   adj_in = dJ/dU of the state before it and add the parameter adjoints to
   dparams.  The time step is a frozen input (no adjoint flows through dt).
   Built for 2-D grids (not patch sets), two materials, no reactive mixture
   and the van Albada limiter (DIMP_EUNSUPPORTED otherwise; periodic axes
   need >= 6 cells); min/max, clamps, the Riemann branch, the BVD choice,
   the THINC mixed-cell test and the yield min are differentiated along the
   branch the forward takes.
   All arrays are device pointers in the state layout (F fields of ncell
   doubles); adj_in must not alias state_in or adj_out.  dparams is a device
   array of 12 doubles, per material l at 6*l: the adjoints of Gamma, 1/Gamma,
   p_ref, e_ref (ideal/stiffened constants), G0 and sigma_Y/sqrt(6), summed in
   a fixed order (deterministic); map them with dimp_adjoint_params.  Work is
   queued on the bound stream; the recomputed states live in the adjoint
   region of the bound workspace (DIMP_WS_ADJOINT; DIMP_ESTATE without). */

/* One sweep along dir (0 = x, 1 = y) of size dt from state_in. */
dimp_status dimp_adjoint_sweep(dimp_handle h, double dt, int dir, const double* state_in, const double* adj_out,
                               double* adj_in, double* dparams);

/* The plastic relaxation applied to state_in (the state after the sweeps). */
dimp_status dimp_adjoint_plastic(dimp_handle h, const double* state_in, const double* adj_out, double* adj_in,
                                 double* dparams);

/* One whole step (as dimp_advance with the same dt and step index) from
   state_in: recomputes the intermediate states, then reverses the plastic
   relaxation and both sweeps. */
dimp_status dimp_adjoint_step(dimp_handle h, double dt, int64_t step_index, const double* state_in,
                              const double* adj_out, double* adj_in, double* dparams);

/* dimp_adjoint_step with the step's first sweep kept by the caller:
   first_sweep (device, the layout of state_in) is the unfused sweep along
   x (even step_index) or y (odd) of size dt from state_in, as dimp_sweep
   writes it; only the second sweep is recomputed.  After dimp_advance of this
   configuration (2-D, split integrator, Cartesian single grid) the bound
   buffer that does not hold the state holds exactly that sweep, so a caller
   replaying the forward can copy it from there.  NULL first_sweep is
   dimp_adjoint_step.  first_sweep is read only and must not alias adj_in
   (DIMP_EINVAL); the other arguments and errors are dimp_adjoint_step's. */
dimp_status dimp_adjoint_step_kept(dimp_handle h, double dt, int64_t step_index, const double* state_in,
                                   const double* first_sweep, const double* adj_out, double* adj_in,
                                   double* dparams);

/* Host: map the 12 packed parameter adjoints (raw, host copy of dparams) to
   grad[4*l + k] = dJ/d(gamma or Gamma0, p_inf, G0, sigma_Y) of material l
   (zero where the material has no such parameter). */
dimp_status dimp_adjoint_params(dimp_handle h, const double raw[12], double grad[8]);

/* A state at rest given a velocity field (the initial velocity the
   calibration differentiates with respect to): out = rest_dev with the
   momentum rho u_k = rho vel_k and the total energy E_rest + rho |vel|^2 / 2
   (E = e + |u|^2 / 2, Sec. 2.2; rho = sum_l phi_l rho_l of rest_dev), every
   other field copied.  vel_dev holds ndim fields of ncell doubles; all
   pointers are device arrays in the handle's layout, out_dev may alias
   rest_dev but not vel_dev.  dimp_with_velocity_adjoint: given adj_out =
   dJ/d(out), writes adj_rest = dJ/d(rest) (zero in the momentum fields,
   which out overwrites) and adj_vel = dJ/d(vel); outputs alias no input.
   Grids only (DIMP_EUNSUPPORTED for a patch set); bound handle; queued on
   the bound stream. */
dimp_status dimp_with_velocity(dimp_handle h, const double* rest_dev, const double* vel_dev, double* out_dev);
dimp_status dimp_with_velocity_adjoint(dimp_handle h, const double* rest_dev, const double* vel_dev,
                                       const double* adj_out_dev, double* adj_rest_dev, double* adj_vel_dev);

/* Set the materials and the optional reactive mixture (NULL or mat = -1
   for none).  nmat in 1..4 is accepted as input; the GPU kernels are built
   for two materials and, except on 3-D grids, for three, and return
   DIMP_EUNSUPPORTED otherwise.  One history slot: at most
   one Johnson-Cook solid or one reactive mixture, not both
   (DIMP_EUNSUPPORTED); JWL only as a reactive component.  Copied; may be
   called again (not to another field count while a state is bound:
   DIMP_ESTATE). */
dimp_status dimp_set_materials(dimp_handle h, int nmat, const dimp_material* mats,
                               const dimp_reactive* rx);

/* Numerical options (copied).  Defaults: minmod, THINC off, beta0 2.5,
   delta 1e-5, eps 1e-20, va_scale {1,1e3,1,1e3,1e9,1}. */
dimp_status dimp_set_options(dimp_handle h, const dimp_options* opt);

/* Number of stored fields and cells per field for the current materials:
   (N - 1) volume fractions, N partial densities, the history slot when there
   is a reactive mixture (phi rho lambda) or a Johnson-Cook solid (phi rho
   eps_p), D momenta, the total energy and the stretch tensor (3, 5 or 9). */
dimp_status dimp_nfields(dimp_handle h, int* nfields, int64_t* ncell);

/* Device workspace.  The library keeps no device memory of its own for a
   grid's steps: the reduction words, the refinement-tag extent and the
   wave-speed slots of the fused sweeps always, the stage buffers of the
   SSP-RK3 (purpose DIMP_WS_RK3: ndim states) and the adjoint's recomputed
   states and partial sums (DIMP_WS_ADJOINT: about 3 states) when asked for,
   live in one caller-owned device buffer.  dimp_workspace_bytes returns its
   size for the current grid, materials and purposes (materials must be
   set; patch sets accept purposes = 0 only: DIMP_EUNSUPPORTED).  The size
   depends on the grid, the field count and the purposes only. */
enum { DIMP_WS_RK3 = 1, DIMP_WS_ADJOINT = 2 };
dimp_status dimp_workspace_bytes(dimp_handle h, int purposes, size_t* bytes);

/* Bind two caller-owned device buffers of nfields*ncell doubles each, the
   workspace (256-byte aligned device memory of at least
   dimp_workspace_bytes(h, purposes) bytes, caller-owned, not to be shared
   with another bound handle) and the stream (a hipStream_t, NULL for the
   null stream).  Sweeps ping-pong between the two buffers; dimp_current tells
   which one holds the state.  buf0 holds the state right after binding.
   Binding again replaces the buffers, the workspace and the stream (the step
   counter is kept).  workspace may be NULL with ws_bytes = 0 and purposes =
   0: then only the calls that need no scratch memory work (conversions,
   single sweeps, the sources, and dimp_advance_static); the others return
   DIMP_ESTATE.  The RK3 integrator needs DIMP_WS_RK3 and the adjoint entry
   points DIMP_WS_ADJOINT (DIMP_EINVAL from binding an RK3 handle without
   it, DIMP_ESTATE from the calls).  The bind enqueues the clearing of the
   workspace's reduction words on the stream.  Errors: DIMP_EINVAL (null or
   equal buffers, a workspace too small or misaligned, unknown purpose bits),
   DIMP_ESTATE (materials not set), DIMP_EHIP. */
dimp_status dimp_bind(dimp_handle h, double* buf0_dev, double* buf1_dev, void* workspace_dev, size_t ws_bytes,
                      int purposes, void* stream);

/* Index (0 or 1) of the bound buffer that holds the current state. */
dimp_status dimp_current(dimp_handle h, int* which);

/* Convert a device array of primitive variables (same layout) into the
   current conserved state (Sec. 2.2 mixture rules; Appendix B primitive
   branch for the reactive mixture).  Resets the step counter to 0. */
dimp_status dimp_prim_to_cons(dimp_handle h, const double* prim_dev);

/* Copy a device array of conserved variables (same layout) into the
   current state buffer on the bound stream (cons_dev may be that buffer:
   then nothing is copied), and mark the state as changed, so that the next
   wave-speed query or device CFL step reduces it afresh.  Any write to the
   bound buffers that bypasses the library must be announced this way.  The
   step counter is kept. */
dimp_status dimp_set_conserved(dimp_handle h, const double* cons_dev);

/* Write the primitive variables of the current state into prim_dev. */
dimp_status dimp_cons_to_prim(dimp_handle h, double* prim_dev);

/* One dimensionally split sweep in direction dir with time step dt (no
   source terms); the state moves to the other buffer. */
dimp_status dimp_sweep(dimp_handle h, double dt, int dir);

/* The plastic and reactive fractional steps alone (and the geometric step of
   a cylindrical grid, see dimp_set_geometry), in place. */
dimp_status dimp_sources(dimp_handle h, double dt);

/* One full step of size dt > 0: the D sweeps (x..z on even step indices,
   z..x on odd ones), then plastic relaxation and the reaction, and the
   per-direction max wave speed of the new state (kept on the device).
   Asynchronous.  Increments the step counter. */
dimp_status dimp_advance(dimp_handle h, double dt);

/* nsteps full steps with the CFL time step computed on the device before
   each one: dt = cfl * min_d dx_d / smax_d from the wave speed of the
   current state (the value fused into the previous step, or a standalone
   reduction for the first).  Asynchronous: no host synchronisation.  If
   dt_log_dev is not NULL it receives the nsteps time steps (device doubles).
   A step that would not be finite and positive runs with dt = 0 and is
   reported by the next dimp_check_state. */
dimp_status dimp_advance_cfl(dimp_handle h, double cfl, int nsteps, double* dt_log_dev);

/* Same as dimp_advance_cfl, with pairs of steps replayed from a captured HIP
   graph (captured on first use for this cfl and buffer parity and kept until
   the materials, options, binding or launch shape change).  An odd step at
   either end runs without the graph.  Asynchronous. */
dimp_status dimp_advance_graph(dimp_handle h, double cfl, int nsteps);

/* Hyperbolic integrator of the advancing calls (dimp_advance, _cfl, _graph).
   DIMP_INTEGRATOR_SPLIT (the default): dimensionally split MUSCL-Hancock
   sweeps.  DIMP_INTEGRATOR_RK3: the paper's own (Sec. 3.1): the unsplit
   spatial operator D(q) of eq. (spat_op) -- per direction the MUSCL / THINC /
   BVD edges without a predictor, the HLLC-type fluxes, the flux difference
   minus the non-conservative sources, over dx; summed over the directions --
   advanced by the three-stage SSP Runge-Kutta of eq. (rk), then the plastic
   and reactive steps and the wave speed as in the split step.  The state
   stays in the same bound buffer (dimp_current does not change); the RK3
   needs one (1-D), two (2-D) or three (3-D) more state-sized device buffers:
   the RK3 region of the bound workspace (DIMP_WS_RK3; DIMP_ESTATE when a
   state is bound with a workspace that lacks it).  Grids only: a
   patch set returns DIMP_EUNSUPPORTED; the adjoint entry points need the
   split integrator (DIMP_ESTATE otherwise).  integrator outside the two
   values: DIMP_EINVAL. */
enum { DIMP_INTEGRATOR_SPLIT = 0, DIMP_INTEGRATOR_RK3 = 1 };
dimp_status dimp_set_integrator(dimp_handle h, int integrator);

/* Two-level subcycled refinement (Sec. 3: each level advanced by the
   single-grid update, the finer one taking two steps of dt/2 per coarse step
   of dt; refinement ratio 2).  `coarse` and `fine` are bound 2-D grids with
   the same materials, fields and stream; the refined patch covers coarse
   cells [box[0], box[2]) x [box[1], box[3]), at least 3 coarse cells inside
   the coarse grid, and `fine` stores it with 4 ghost layers: fine n =
   (2 (box[2] - box[0]) + 8, 2 (box[3] - box[1]) + 8), fine dx = coarse dx / 2,
   fine cell (i, j) centred over coarse position box[0] + (i - 4 + 1/2)/2.
   The hierarchy does not own the grids (destroy it first); it sets the fine
   grid's step index to twice the coarse one.
   dimp_amr_advance: one coarse step of dt, then two fine steps of dt/2, each
   after a ghost fill: the coarse state linear in time between before and
   after its step (weights 0 and 1/2) and linear in space inside each coarse
   parent with minmod-limited slopes of the conserved variables; then every
   covered coarse cell becomes the mean of its four fine children; last, the
   flux correction: each coarse cell outside the patch that shares a face
   with it takes, through that face, the mean of the fluxes of the face's two
   fine faces over the two fine steps in place of its coarse flux (the
   fluxes each split sweep computes from the state it reads), for the
   partial densities, the history slot, the momentum and the energy, so
   these are conserved over the composite grid (the volume fractions and
   Vbar, whose sweeps carry non-conservative terms, are left).  Both levels
   step the same integrator (DIMP_EINVAL otherwise): with the SSP-RK3 the
   fine grid's stage inputs q(1) and q(3) take their ghost rings from the
   coarse level at the fine step's end and middle, and the correction uses
   each face's fluxes over the stages weighted 1/6, 1/6, 2/3.
   dimp_amr_dt: fills the fine ghost cells from the current coarse state and
   returns min(coarse CFL step, 2 x fine CFL step) for the Courant number
   cfl (both over all their cells).
   Workspace: the hierarchy keeps the coarse state before its step and the
   boundary fluxes in a caller-owned, 256-byte aligned device buffer of
   dimp_amr_workspace_bytes(coarse, box) bytes (it must outlive the
   hierarchy and serve no other).
   Errors: DIMP_EINVAL (sizes, box, cell widths, fields, streams that do not
   match, a workspace too small), DIMP_EUNSUPPORTED (not 2-D grids),
   DIMP_ESTATE (a grid not bound with a workspace), DIMP_EHIP. */
typedef struct dimp_amr_ctx* dimp_amr;
dimp_status dimp_amr_workspace_bytes(dimp_handle coarse, const int64_t box[4], size_t* bytes);
dimp_status dimp_amr_create(dimp_handle coarse, dimp_handle fine, const int64_t box[4], void* workspace_dev,
                            size_t ws_bytes, dimp_amr* out);
dimp_status dimp_amr_dt(dimp_amr a, double cfl, double* dt);
dimp_status dimp_amr_advance(dimp_amr a, double dt);
/* More than two levels (Sec. 3 recursively; Berger-Colella): `inner` is a
   hierarchy whose coarse grid is `outer`'s fine grid, its patch at least 7
   cells (4 ghost layers + 3) inside that grid, so that its ghost fill reads
   only the interior of the level above.  From then on dimp_amr_advance(outer)
   advances `inner` (with dt/2, twice) wherever it would step the fine grid:
   each level's ghost ring is filled from the level above at that level's
   old and new times, and after its substeps every level is averaged down into
   the level above and that level's cells beside the patch are
   flux-corrected; dimp_amr_dt(outer) returns min over the levels of 2^l x the
   level's CFL step (each finer level after a ghost fill).  A nested hierarchy
   is stepped only through the outer one (DIMP_ESTATE from its own dt and
   advance); destroying either ends the nesting.  Errors: DIMP_EINVAL (grids
   that do not chain, a cycle, the patch too near the edge), DIMP_ESTATE (either
   hierarchy already nested). */
dimp_status dimp_amr_nest(dimp_amr outer, dimp_amr inner);
/* Several patches on one level (Sec. 3: a level is a set of patches):
   `member`, a hierarchy over the same coarse grid as `head`, joins head's
   group; its patch must share no coarse cell with any patch of the group
   (patches may touch: share a face or a corner).  dimp_amr_advance(head)
   then takes one coarse step with every patch's boundary fluxes recorded and
   two fine substeps, each filling every patch's ghost ring from the coarse
   level, then (split integrator) copying every patch's interior into the
   stored cells of the others that it covers (fine-to-fine exchange; the 4
   ghost layers reach 2 coarse cells), then stepping every patch; then it
   corrects the coarse cells beside every patch and averages every patch
   down (a corrected cell another patch covers takes that patch's average).
   With the RK3 every ghost ring comes from the coarse level only and
   touching patches are refused (DIMP_EUNSUPPORTED from the advance).
   dimp_amr_dt(head) takes the minimum over the coarse grid and all patches
   (after the same fills and exchange).  Members are stepped only through the head
   (DIMP_ESTATE from their own dt and advance); destroying a member removes
   it from the group, destroying the head dissolves the group.  Groups and
   nesting combine into a refinement tree: a member may nest a hierarchy of
   its own, and a head may be nested (the whole group then refines the outer
   fine grid, every patch at least 7 cells inside it).  Errors: DIMP_EINVAL
   (different coarse grids, patches sharing a coarse cell, a nested group's
   patch too near the outer grid's edge), DIMP_ESTATE (head is a member,
   member already grouped or nested). */
dimp_status dimp_amr_group(dimp_amr head, dimp_amr member);
dimp_status dimp_amr_destroy(dimp_amr a);
/* Every fine cell (interior and ghosts) takes the conserved state of its
   coarse parent (a new or regridded patch: exactly conservative, no new
   states; the ghost ring is refilled by the linear fill before each fine
   step). */
dimp_status dimp_amr_prolong(dimp_amr a);

/* Refinement criterion of Sec. 4.2 on a bound 2-D grid: cell (i, j) is
   tagged (tags_dev[j n0 + i] = 1, else 0; device, ncell bytes) when one of
   the refinement variables -- the stored volume fractions, phi_l rho_l of
   every material, u_x, u_y and p -- changes to a face neighbour (across the
   grid's edge there is none) by more than threshold as a fraction:
   |q_n - q_c| > threshold max(|q_c|, |q_n|, floor), the floor 1e-6 times the
   option's va_scale of the variable's kind (phi; rho for phi_l rho_l; u; p).
   prim_dev holds the primitive state (dimp_cons_to_prim).  bbox (host)
   receives the tagged cells' extent [i0, j0, i1, j1) (all 0 when none is
   tagged).  Errors: DIMP_EINVAL, DIMP_EUNSUPPORTED (not a 2-D grid). */
dimp_status dimp_amr_tag(dimp_handle h, const double* prim_dev, double threshold, uint8_t* tags_dev,
                         int64_t bbox[4]);

/* Geometry of a 2-D grid (Sec. 3).  DIMP_GEOMETRY_CYLINDRICAL: axisymmetric
   form with x = r, y = z; r_lo >= 0 is the radius of the grid's low x face
   (cell i is centred at r_lo + (i + 1/2) dx[0]).  After the plastic and
   reactive steps every step (and dimp_sources) adds the geometric source
   s_g = -(1/r) (0, m_l u_r, m_hist u_r, rho u_r^2 - sig_rr + sig_tt,
   rho u_z u_r - sig_rz, rho E u_r - (u_r sig_rr + u_z sig_zr),
   (1/3 - delta_{i theta}) Vbar_ij u_r) as a fractional step by Heun's method;
   with r_lo = 0 use DIMP_BC_AXIS along x.  These steps then run as their own
   pass after the last sweep (not fused into it).  Errors: DIMP_EINVAL (an
   unknown geometry, r_lo < 0), DIMP_EUNSUPPORTED (not 2-D; a patch set).
   The adjoint entry points reject a cylindrical grid. */
enum { DIMP_GEOMETRY_CARTESIAN = 0, DIMP_GEOMETRY_CYLINDRICAL = 1 };
dimp_status dimp_set_geometry(dimp_handle h, int geometry, double r_lo);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): one step
   as dimp_advance with the split integrator, whose scratch memory -- the
   wave-speed slots of the fused last sweep, their reduction and the
   reduction words -- is a static device array of the library (8 MiB, one
   per GPU, held until the process ends) instead of the bound workspace, so
   the handle may be bound without one.  The caller passes the bound state
   buffers (dimp_bind) and smax_dev, a device array of 3 doubles that
   receives the per-direction max wave speed of the new state (entries
   beyond ndim are 0).  Calls no allocating routine.  Every call on one GPU
   shares the static array: calls that overlap on one GPU (two streams, two
   threads) race and must be serialised by the caller.  The handle's own
   wave-speed words are not updated (dimp_max_wavespeed recomputes).
   Errors: DIMP_EINVAL (dt not positive and finite, null smax_dev, a grid or
   patch set whose wave-speed slots need more than the static array holds:
   348 000 slots of 58 cells along x, about 20 M cells for wide grids, 256^3
   included), DIMP_EUNSUPPORTED (the RK3 integrator),
   DIMP_ESTATE (nothing bound), DIMP_EHIP. */
dimp_status dimp_advance_static(dimp_handle h, double dt, double* smax_dev);

/* Set the step counter (selects the sweep order of the next step). */
dimp_status dimp_set_step_index(dimp_handle h, int64_t step);

/* Per-direction max over cells of |u_d| + c_L of the current state, where
   c_L^2 = c^2 + 4 G / (3 rho).  Synchronises the stream and copies
   smax[0..ndim-1] to the host.  Reuses the value fused into the last advance
   when the state has not changed since. */
dimp_status dimp_max_wavespeed(dimp_handle h, double smax[3]);

/* Same, asynchronous: writes three doubles to smax_dev on the bound stream. */
dimp_status dimp_max_wavespeed_device(dimp_handle h, double* smax_dev);

/* Count cells with a non-finite field, a volume fraction outside [0,1], a
   non-positive phasic density or a non-positive squared sound speed.
   Synchronises.  Returns DIMP_ENONPHYSICAL when *nbad > 0, and also (once)
   when a device CFL step since the last check was not finite and positive
   (a zero or non-finite wave speed; that step ran with dt = 0 and the
   dt log holds 0). */
dimp_status dimp_check_state(dimp_handle h, int64_t* nbad);

/* Measurement hook: when enabled, every sweep launch is bracketed by HIP
   events recorded on the bound stream.  dimp_kernel_times synchronises and
   returns, for each kind k = 2*dir + (1 if the launch carried the fused
   source/wave-speed epilogue), the summed milliseconds and launch count since
   the last query or enable, then clears them.  Off by default. */
dimp_status dimp_set_kernel_timing(dimp_handle h, int enable);
dimp_status dimp_kernel_times(dimp_handle h, double ms[6], int64_t counts[6]);

/* Thread-local message of the last failing call ("" if none). */
const char* dimp_last_error(void);

/* Release the handle and the library's own device memory (not the bound
   buffers).  NULL is accepted. */
dimp_status dimp_destroy(dimp_handle h);

#ifdef __cplusplus
}
#endif
#endif
