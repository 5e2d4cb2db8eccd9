/*
 * CPU oracle for the method-of-lines hot path of Palenzuela et al.,
 * "A Simflowny-based finite-difference code for high-performance computing
 * in Relativity" (arXiv:1806.04182).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, single-threaded, FP64 C that follows the
 * paper's formulas in the paper's order.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library; the product
 * path never does.  It shares no code, header or table with the HIP library.
 *
 * Array convention used by every entry point here ("patch array"):
 *   a patch with interior size n = (nx, ny, nz) is stored with a ghost layer of
 *   ORC_G = 3 points on every side, i.e. over (nx+6) x (ny+6) x (nz+6) points,
 *   x fastest, then y, then z, then field:
 *       U[((f*(nz+6) + k)*(ny+6) + j)*(nx+6) + i]
 *   interior points are i in [3, nx+3), etc.  Right-hand sides are written on
 *   interior points only.
 *
 * Parity status of every function is listed in the oracle section of the
 * project's design notes; functions without an independent pin carry the
 * words "parity unpinned" in their comment below.
 */
#ifndef MOLAMR_ORACLE_H
#define MOLAMR_ORACLE_H

#include <stdint.h>

#define ORC_G 3

/* Physical / numerical parameters of every system (one struct for all). */
typedef struct {
    double sigma;      /* Kreiss-Oliger strength (Sec. II.B.1, KO operator) */
    /* Newtonian MHD (Sec. IV.B) */
    double gamma_ad;   /* ideal-gas adiabatic index */
    double weno_eps;   /* WENO epsilon; <= 0 selects dx^4 of the sweep direction (App. B) */
    double weno_q;     /* WENO-Z exponent q (App. B) */
    /* CCZ4 (Sec. V) */
    double kappa_z;    /* constraint damping kappa_z */
    double kappa_c;    /* conformal-constraint damping kappa_c */
    double bm_f0;      /* Bona-Masso f = bm_f0 + bm_f1/alpha */
    double bm_f1;
    double gd_g;       /* Gamma-driver g */
    double gd_eta;     /* Gamma-driver eta */
    double upwind;     /* 1: lop-sided advection stencils; 0: centred */
    /* MHD variants (Sec. II.B.2, App. A, App. B) */
    double mhd_recon;  /* 0: WENO5-Z, 1: WENO5-JS, 2: WENO3 */
    double mhd_riemann; /* 0: local Lax-Friedrichs (eq. LLF), 1: HLL, 2: LLF flux splitting
                           (reading R2: reconstruct (F +- alpha U)/2) */
    double mhd_ch;     /* divergence cleaning (Sec. IV.B, 9-field system): speed c_h */
    double mhd_kpsi;   /* and damping kappa_psi */
} orc_params;

enum { ORC_WAVE = 0, ORC_MHD = 1, ORC_CCZ4 = 2, ORC_MHD_GLM = 3 };
enum { ORC_RK4 = 0, ORC_SSPRK3 = 1 };

int orc_nfields(int system);

/* ---- one-dimensional stencils (Sec. II.B.1), applied to u[0] with stride s ---- */
double orc_d1(const double* u, long s, double h);
double orc_d2(const double* u, long s, double h);
double orc_adv(const double* u, long s, double h, double beta);
double orc_ko(const double* u, long s, double h, double sigma);
double orc_dmix(const double* u, long sa, double ha, long sb, double hb);

/* ---- ghost fill of a single periodic patch (every ghost point) ---- */
void orc_fill_periodic(double* U, int nf, int nx, int ny, int nz);

/* ---- right-hand sides L(U) + Q_d(U) on the interior ---- */
void orc_wave_rhs(const double* U, double* R, int nx, int ny, int nz,
                  const double h[3], const orc_params* p);
/* nine fields (ORC_MHD_GLM): the cleaning scalar psi last */
void orc_mhd_glm_rhs(const double* U, double* R, int nx, int ny, int nz,
                     const double h[3], const orc_params* p);
void orc_mhd_rhs(const double* U, double* R, int nx, int ny, int nz,
                 const double h[3], const orc_params* p);
void orc_ccz4_rhs(const double* U, double* R, int nx, int ny, int nz,
                  const double h[3], const orc_params* p);
void orc_rhs(int system, const double* U, double* R, int nx, int ny, int nz,
             const double h[3], const orc_params* p);

/* ---- constraint and dissipation monitors (Sec. V; Sec. II.B.1) ---- */
/* CCZ4, at every interior point, into five fields of M (patch-array layout):
 * Theta, gamma_ij Z^i Z^j, H_Z (the bracket of the Theta equation), ln det gt,
 * tr At, each as the right-hand side evaluates it. */
void orc_ccz4_monitor(const double* U, double* M, int nx, int ny, int nz,
                      const double h[3], const orc_params* p);
/* any system: M[c] = sum_f (sum_d KO_d U_f)^2 at every interior point, the
 * square of the dissipation term's magnitude over all nf fields */
void orc_ko_monitor(int system, const double* U, double* M, int nx, int ny, int nz,
                    const double h[3], const orc_params* p);

/* WENO5-Z reconstruction of the left state at i+1/2 from u[-2..2] and the right
 * state at i-1/2 from u[-2..2] (App. B); exposed for the pins. */
double orc_weno5z_left(const double* u, double eps, double q);
double orc_weno5z_right(const double* u, double eps, double q);
/* WENO5-JS variants (App. B, generic weights of Sec. II.B.2) */
double orc_weno5js_left(const double* u, double eps);
double orc_weno5js_right(const double* u, double eps);
/* WENO3 (App. A): U^L_{i+1/2} from u[-1..1] and U^R_{i-1/2} from u[-1..1] */
double orc_weno3_left(const double* u, double eps);
double orc_weno3_right(const double* u, double eps);
/* Interface flux between the reconstructed states UL, UR (8 fields) along
 * axis d: LLF (riemann 0) or HLL (riemann 1) */
void orc_mhd_interface_flux(const double UL[8], const double UR[8], int d, double gam, int riemann,
                            double F[8]);
/* fast magnetosonic speed c_f of the state U along axis d */
double orc_mhd_fast_speed(const double U[8], int d, double gam);

/* ---- explicit Runge-Kutta (eq. eRK) on one periodic patch ---- */
/* nsteps full steps with periodic ghost fill before every stage. */
void orc_rk_run(int system, int scheme, double* U, int nx, int ny, int nz,
                const double h[3], double dt, int nsteps, const orc_params* p);
/* one-step amplification factor of a scheme on u' = z u (complex z) */
void orc_rk_scalar(int scheme, double zr, double zi, double* outr, double* outi);

/* ---- dense output (App. C) and BOR (App. D) ---- */
/* b_j(theta) and its m-th theta-derivative for RK4, j = 0..3 */
double orc_dense_rk4(int j, int m, double theta);
/* BOR fine-stage state from coarse U^n and k_1..k_4 (App. D, RK4):
 * out[i] = state of fine step r (0..R-1), fine stage s (1..4) for i < n. */
void orc_bor_rk4(int R, int r, int s, double dt, const double* Un,
                 const double* const* k, double* out, long n);
/* the same for SSP-RK(3,3): its dense output (App. C, j = 0..2) and BOR
 * (App. D) from U^n and k_1..k_3, fine stage s = 1..3 */
double orc_dense_ssp3(int j, int m, double theta);
void orc_bor_ssp3(int R, int r, int s, double dt, const double* Un,
                  const double* const* k, double* out, long n);

/* ---- Lagrange prolongation (Sec. III.A) ---- */
/* weights of the 6-point Lagrange polynomial through nodes -2..3 at xi */
void orc_lagrange6(double xi, double w[6]);

/* ---- hierarchy (Sec. III): boxes in level index space, vertex-centred ---- */
typedef struct orc_hier orc_hier;
/* nlev levels; ratio[l] is the ratio of level l to level l-1 (ratio[0] unused);
 * the domain is periodic with N0 level-0 points per axis (N0 * R_1 * .. * R_l
 * on level l); boxes are (lo,hi) inclusive,
 * six ints per patch, npatch[l] patches on level l, concatenated. */
orc_hier* orc_hier_create(int system, int nlev, const int* ratio, const int N0[3],
                          const double xlo[3], double dx0, const int* npatch,
                          const int* boxes);
void orc_hier_destroy(orc_hier* H);
int orc_hier_npatch(const orc_hier* H, int l);
/* copy one patch (whole ghosted array) in/out */
void orc_hier_set(orc_hier* H, int l, int p, const double* src);
void orc_hier_get(const orc_hier* H, int l, int p, double* dst);
/* ghost points of level l that have a same-level source (periodic images
 * included): copy it.  Acts on the current state. */
void orc_hier_fill_same(orc_hier* H, int l);
/* one sub-cycled coarse step (RK4 or SSP-RK3) with prolongation and injection */
void orc_hier_step(orc_hier* H, double dt0, const orc_params* p);
/* time refinement of the sub-cycled step (Sec. III.B); BOR by default */
enum { ORC_TIME_BOR = 0, ORC_TIME_BO = 1, ORC_TIME_BO1 = 2, ORC_TIME_NOSUB = 3 };
void orc_hier_set_time_mode(orc_hier* H, int mode);
void orc_time_state(int mode, int R, int r, int s, double dt, const double* Un,
                    const double* const* k, double* out, long n);
void orc_time_state_ssp3(int mode, int R, int r, int s, double dt, const double* Un,
                         const double* const* k, double* out, long n);
/* integrator of the sub-cycled step: ORC_RK4 (default) or ORC_SSPRK3 */
void orc_hier_set_scheme(orc_hier* H, int scheme);
/* Open (non-periodic) domain with radiative boundaries (Sec. V): level 0 is a
 * single patch and each of its ghost points evolves by
 *   d_t U = -v (x^i / r) d_i U - v (U - U_inf) / r
 * (v and U_inf per field, r the distance to the coordinate origin), d_i
 * centred where both neighbours are in the ghosted array, one-sided (2nd
 * order) at its edge. */
void orc_hier_set_open(orc_hier* H, const double* v, const double* uinf);
/* the pieces, for the unit checks: prolong into level l (>0) at fine step r,
 * stage s, from the parent's saved U^n and k's (set with orc_hier_set_parent) */
void orc_hier_set_parent_data(orc_hier* H, int l, int p, const double* Un,
                              const double* k1, const double* k2,
                              const double* k3, const double* k4);
void orc_hier_prolong(orc_hier* H, int l, int r, int s, double dt_parent);
void orc_hier_restrict(orc_hier* H, int l);
/* Regrid at a synchronised time (Sec. III.A): Hn has the same system, level-0
 * boxes, level count and ratios as Ho.  Level 0 is copied; on each level
 * l >= 1 (in increasing l) every interior point of Hn takes Ho's value where an
 * Ho patch of that level holds it, and otherwise the tensor-product 6-point
 * Lagrange interpolant of Hn's level l-1 (nodes i0-2..i0+3 on the axes where
 * the point is between parent nodes).  Ghost points of Hn are not set. */
void orc_hier_regrid(orc_hier* Hn, const orc_hier* Ho);

/* ---- wave adjoint (vector-Jacobian product of the RHS, scatter form) ---- */
void orc_wave_rhs_adjoint(const double* lam, double* lamU, int nx, int ny, int nz,
                          const double h[3], const orc_params* p);
/* adjoint of the periodic ghost fill: add ghost entries to their owners, zero ghosts */
void orc_fill_periodic_adjoint(double* A, int nf, int nx, int ny, int nz);
/* gradient of J = sum_{|x|<rad} phi dx^3 at final time w.r.t. the initial
 * state (phi, Pi) after nsteps RK4 steps of the periodic wave: lam0 receives
 * dJ/dU0 on the interior (ghosts zero) */
void orc_wave_adjoint_run(double* lam0, int nx, int ny, int nz, const double h[3],
                          const double xlo[3], double dt, int nsteps, double rad,
                          const orc_params* p);

/* ---- norms (Sec. IV, convergence factor and relative error) ---- */
double orc_sphere_integral(const double* U, int field, int nx, int ny, int nz,
                           const double xlo[3], const double h[3], double rad,
                           double shift);

#endif
