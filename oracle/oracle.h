/*
 * oracle.h -- C interface of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, double-precision CPU
 * implementation of the explicit diffuse-interface finite-volume step of
 * Wallis, Barton & Nikiforakis, "A Diffuse Interface Model of Reactive-fluids
 * and Solid-dynamics" (arXiv 2009.14555).  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  The GPU library
 * shares no code, header, table or helper with it.
 *
 * State layout (structure of arrays, field-major, x fastest):
 *   field f of cell (i,j,k) lives at  f*ncell + i + n0*(j + n1*k).
 * Field order for N materials, D dimensions, optional reactive mixture:
 *   phi_1..phi_{N-1}          volume fractions (phi_N = 1 - sum)
 *   m_1..m_N                  partial densities phi_l*rho_l
 *   [m_lam]                   phi_y*rho_y*lambda of the reactive material y, or
 *   [m_eps]                   phi_s*rho_s*eps_p of the Johnson-Cook material s
 *                             (at most one of the two: a reactive mixture and a
 *                             Johnson-Cook solid do not coexist)
 *   rho*u_1..rho*u_D          momentum
 *   rho*E                     total energy
 *   Vbar components           D=1: 11,22,33  D=2: 11,12,21,22,33  D=3: all 9
 * Primitive vectors use the same slots: phi_l, rho_l, lambda or eps_p, u_k, p, Vbar.
 *
 * Every function returns 0 on success and a negative value on a bad argument.
 */
#ifndef DIMP_ORACLE_H
#define DIMP_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { OR_EOS_IDEAL = 0, OR_EOS_STIFFENED = 1, OR_EOS_ROMENSKII = 2, OR_EOS_JWL = 3 };
enum { OR_RATE_POWER = 0, OR_RATE_IG = 1 };
enum { OR_PLAST_NONE = 0, OR_PLAST_PERFECT = 1, OR_PLAST_JC = 2 };
/* boundary rule per dimension: transmissive (zero-gradient copy), periodic,
   reflective walls at both ends (ghost cells are mirror images with the normal
   momentum and the stretch-tensor entries with exactly one normal index
   negated), or AXIS: reflective at the low end (the symmetry axis r = 0 of
   the cylindrical form) and transmissive at the high end */
enum { OR_BC_TRANSMISSIVE = 0, OR_BC_PERIODIC = 1, OR_BC_REFLECTIVE = 2, OR_BC_AXIS = 3 };
enum { OR_GEOM_CARTESIAN = 0, OR_GEOM_CYLINDRICAL = 1 };
enum { OR_LIM_MINMOD = 0, OR_LIM_VANALBADA = 1 };
#define OR_MAXMAT 4

typedef struct {
  int32_t eos;      /* OR_EOS_* */
  int32_t plast;    /* OR_PLAST_*; only meaningful when the shear modulus is non-zero */
  double gamma;     /* ideal / stiffened: adiabatic index */
  double pinf;      /* stiffened: p_inf */
  double eref;      /* stiffened: e_inf (reference energy) */
  double rho0, K0, G0, abar, bbar, Gamma0;  /* Romenskii */
  double cv;        /* specific heat: reactive temperature equilibrium, Johnson-Cook softening */
  double yield;     /* perfect plasticity yield stress */
  /* Johnson-Cook (Sec. 2.3.2): sigma_Y = (c1 + c2 eps_p^n)(1 - theta^m), theta
     = (T - T0)/(Tmelt - T0) clipped to [0, 1]; plastic rate chi = chi0 exp((s -
     1)/c3), s = sqrt(3/2) |dev sigma| / sigma_Y */
  double jc_c1, jc_c2, jc_c3, jc_n, jc_m, jc_tmelt, jc_t0, jc_chi0;
  /* JWL (Sec. 2.3, Table 3): p_ref = A exp(-R1 rho0/rho) + B exp(-R2 rho0/rho),
     e_ref = A/(R1 rho0) exp(-R1 rho0/rho) + B/(R2 rho0) exp(-R2 rho0/rho),
     constant Gamma0; uses rho0 and Gamma0 above */
  double jwl_A, jwl_B, jwl_R1, jwl_R2;
} or_mat;

typedef struct {
  int32_t mat;      /* index of the reactive mixture material, or -1 */
  int32_t law;      /* OR_RATE_POWER or OR_RATE_IG */
  or_mat reactant;  /* component alpha (lambda = 1) */
  or_mat product;   /* component beta  (lambda = 0); its reference energy is shifted by -Q */
  double Q, k, n, pref;  /* OR_RATE_POWER: dlambda/dt = -k lambda (max(p,0)/pref)^n */
  /* OR_RATE_IG, the three-term ignition-and-growth law (Sec. 4.2, Table 4) with
     F = 1 - lambda the reacted fraction and rho the mixture material's own
     density rho_y:
       dF/dt = I (1-F)^b (rho/rho0 - 1 - a)^x H(F_ig - F)
             + G1 (1-F)^c F^d p^y H(F_G1 - F) + G2 (1-F)^e F^g p^z H(F - F_G2),
     dlambda/dt = -dF/dt; p in units of ig_punit (Pa), clipped at 0; the
     compression term clipped at 0; H(x) = 1 for x > 0, else 0 */
  double ig_I, ig_G1, ig_G2, ig_a, ig_b, ig_c, ig_d, ig_e, ig_g, ig_x, ig_y, ig_z;
  double ig_Fig, ig_FG1, ig_FG2, ig_rho0, ig_punit;
} or_rx;

typedef struct {
  int32_t ndim, nmat;
  int64_t n[3];
  double dx[3];
  int32_t bc[3];
  int32_t limiter;
  int32_t thinc;
  int32_t pad;
  double beta0, delta, eps;
  double va_scale[6];  /* van Albada epsilon scales: phi, rho, lambda, u, p, Vbar */
  or_mat mat[OR_MAXMAT];
  or_rx rx;
  double lo[3];     /* coordinate of the low face of the grid per dimension */
  int32_t geom;     /* OR_GEOM_*; cylindrical: 2-D, x = r (lo[0] + dx[0]/2 > 0), y = z */
  int32_t pad2;
} or_config;

int or_nfields(const or_config* c);
void or_set_threads(int nthreads);
int or_get_threads(void);

/* whole-grid operations */
int or_prim_to_cons(const or_config* c, const double* prim, double* cons);
int or_cons_to_prim(const or_config* c, const double* cons, double* prim);
int or_sweep(const or_config* c, double* cons, double dt, int dir);
/* or_sweep that also writes the numerical face fluxes it used: flux is the
   grid's shape with n_dir + 1 faces along dir (x fastest), F components
   each; face f along dir sits between cells f - 1 and f.  The conserved
   components (partial densities, history slot, momentum, energy) update as
   U_i - dt/dx (flux_{i+1} - flux_i); the volume fractions and Vbar carry
   non-conservative terms besides. */
int or_sweep_flux(const or_config* c, double* cons, double dt, int dir, double* flux);
int or_plastic(const or_config* c, double* cons);
/* the plastic step with a time step (the Johnson-Cook rate integrates over
   dt; or_plastic is this with dt = 0, which leaves a Johnson-Cook solid
   unrelaxed) */
int or_plastic_dt(const or_config* c, double* cons, double dt);
int or_reaction(const or_config* c, double* cons, double dt);
/* the cylindrical geometric source of Sec. 3 (s_g, r = x) as a fractional
   step over dt by Heun's method; a no-op on a Cartesian grid.  or_step and
   or_step_rk3 apply it after the reaction. */
int or_geometric(const or_config* c, double* cons, double dt);
int or_step(const or_config* c, double* cons, double dt, int64_t step_index);
int or_max_wavespeed(const or_config* c, const double* cons, double* smax /* [3] */);

/* The paper's own hyperbolic integrator (Sec. 3.1): or_rhs evaluates the
   unsplit spatial operator D(q) of eq. (spat_op) (per direction: MUSCL /
   THINC / BVD edges without a predictor, HLLC-type fluxes, flux differences
   minus the non-conservative sources, over dx; summed x, y, z) into rhs
   (F x ncell); or_step_rk3 advances cons by the SSP-RK3 of eq. (rk) on D,
   then applies the plastic and reactive fractional steps. */
int or_rhs(const or_config* c, const double* cons, double* rhs);
int or_step_rk3(const or_config* c, double* cons, double dt);
/* Direction dir's part of D(cons) added into rhs (zeroed by the caller) and
   that direction's face fluxes written to flux (the grid's shape with one
   more face along dir, component-major): all directions in order give
   or_rhs's result bit for bit (refluxing of a refined RK3 step). */
int or_rhs_dir_flux(const or_config* c, const double* cons, int dir, double* rhs, double* flux);

/* One whole step (as or_step) on forward-mode dual numbers: the exact tangent
   of the discrete step in K <= OR_DUAL_K directions.  cons (F x ncell) is
   advanced in place; tan (K x F x ncell) holds the state tangents of the K
   directions and is advanced with it; par_tan (K x nmat x 4) seeds the
   tangents of each material's (gamma, p_inf, G0, yield).  dt carries no
   tangent.  Non-smooth operations follow the branch of the value. */
#define OR_DUAL_K 6
int or_step_dual(const or_config* c, double* cons, double* tan, const double* par_tan, double dt,
                 int64_t step_index, int K);
/* one stage of it: stage = d < ndim is the sweep along d alone, stage = ndim
   the plastic (and reactive) fractional steps alone, -1 the whole step */
int or_stage_dual(const or_config* c, double* cons, double* tan, const double* par_tan, double dt,
                  int64_t step_index, int K, int stage);

/* One whole step (as or_step) on operation-counting scalars: cons is
   advanced in place (bit for bit as by or_step) and counts, (ndim + 2) x 6,
   receives the operations of each phase summed over the grid: rows 0..ndim-1
   the sweep along each axis, row ndim the plastic (and reactive) steps, row
   ndim + 1 the wave speed of the result; columns add, mul, div, sqrt,
   transcendental, comparison.  Operations on structural zeros (the constant
   0, e.g. the unused entries of a 3x3 tensor below 3-D) are not counted. */
int or_step_flops(const or_config* c, double* cons, double dt, int64_t step_index, double* counts);
/* The same for one step of or_step_rk3: counts is (ndim + 3) x 6: rows
   0..ndim-1 one evaluation of each direction's part of D(q), row ndim the
   three stage combinations, then the sources and the wave speed. */
int or_step_rk3_flops(const or_config* c, double* cons, double dt, double* counts);
/* the counting rules on fixed expressions, three rows of 6 (for tests) */
int or_flops_selftest(double* out /* 18 */);

/* pointwise pieces, exposed so tests can pin them */
int or_eos(const or_mat* m, double rho, double J2, double* out /* Gamma,pref,eref,dpref,deref,G */);
int or_thinc(double qm, double q0, double qp, double beta, double eps, double delta,
             double* out /* qL, qR, C, mixed */);
int or_youngs_beta(const or_config* c, const double* cons, int64_t cell, int dir, double* beta);
/* BVD choice of Appendix A from the edge candidates cand = {MUSCL right of
   i-1, THINC right of i-1, MUSCL left of i, MUSCL right of i, THINC left of
   i, THINC right of i, MUSCL left of i+1, THINC left of i+1}: returns 1 when
   THINC is chosen for cell i, 0 for MUSCL; v receives the four boundary
   variations (MUSCL|MUSCL, THINC|THINC, MUSCL|THINC, THINC|MUSCL
   neighbours) for P = MUSCL, then for P = THINC */
int or_bvd_thinc(const double cand[8], double v[8]);
/* the root rx_solve takes for a conserved cell (t = 1: a pure cell, no split) */
int or_rx_split(const or_config* c, const double* U, double* t);
/* the reactive split's residual at the conserved cell U for n values t[i] of
   t = rho_alpha / (rho_alpha + rho_beta): out[4 i ..] = T_beta - T_alpha, the
   pressure of the Appendix B pressure function, T_alpha, T_beta */
int or_rx_residual(const or_config* c, const double* U, int n, const double* t, double* out);
/* the volume-fraction edges of cell i as the sweep forms them, from the
   stencil q = phi_{i-2..i+2} and the steepness beta of cells i-1, i, i+1
   (the config's limiter, thinc, eps and delta): out = {left edge, right edge,
   the 8 variations of or_bvd_thinc, 1 if THINC was chosen, MUSCL left,
   MUSCL right, THINC left, THINC right (the MUSCL edges where the cell is
   not mixed), 0} */
int or_phi_edges(const or_config* c, const double q[5], const double beta[3], double out[16]);
int or_strain(const double* V /* 3x3 row-major */, double* H /* 3x3 */, double* J2);
int or_pade_exp(const double* H, double* V);
/* cell diagnostics from a conserved cell vector:
   out = p, c2, cL2, Gmix, rho, s, rho_a, rho_b, T_a, T_b, xi, J2 */
int or_cell_diag(const or_config* c, const double* U, double* out);
/* cell diagnostics from a primitive cell vector (same outputs, and U) */
int or_cell_diag_prim(const or_config* c, const double* W, double* out, double* U);
/* HLLC-type face flux between primitive states WL | WR in direction dir.
   flux has nfields entries (the phi entries hold phi_K * u_star),
   extra = u_star, Vbar*_{n1}, Vbar*_{n2}, Vbar*_{n3} */
int or_face_flux(const or_config* c, int dir, const double* WL, const double* WR,
                 double* flux, double* extra);

#ifdef __cplusplus
}
#endif
#endif
