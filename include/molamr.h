/*
 * molamr — method-of-lines hot path on SAMRAI-style patches for gfx950.
 *
 * C ABI of the HIP library libmolamr.so.  The operations follow Palenzuela
 * et al., "A Simflowny-based finite-difference code for high-performance
 * computing in Relativity" (arXiv:1806.04182); each entry point names the
 * section or equation that defines it.
 *
 * Conventions (all entry points):
 *  - Ownership.  A patchset owns its host metadata and its device tables
 *    (allocated in mol_create_patchset, freed in mol_destroy_patchset).  The
 *    caller owns every field buffer: device memory holding float64 values in
 *    the layout reported by mol_level_layout.  Input buffers are not written.
 *  - Streams.  Every call that takes a `stream` (a hipStream_t; NULL is the
 *    default stream) only enqueues work on it: no call synchronises, and none
 *    allocates device memory after mol_create_patchset, so sequences of calls
 *    can be captured in a HIP graph.
 *  - Errors.  Every int-returning call returns 0 on success or a negative
 *    code; mol_last_error() returns a message for the calling thread's last
 *    failure.  Argument errors are detected on the host before any work is
 *    enqueued.  Faults inside kernels surface at the caller's next
 *    synchronisation.  No C++ exception crosses this interface.
 *  - Threading.  Calls on different patchsets are independent; concurrent
 *    calls that write the same buffers race.
 *
 * Geometry (Sec. III).  Grids are vertex centred: level l has spacing
 * dx0 / (R_1 ... R_l), and fine point R*i coincides with coarse point i for
 * any integer ratio R (which makes injection a copy for R = 2 and R = 3).
 * The domain is periodic with N0 level-0 points per axis (N0 R_1 ... R_l on
 * level l).  Boxes are inclusive (lo, hi) index ranges in level index space.
 * Every patch carries a ghost layer of 3 points (MOL_GHOST).
 *
 * Field layout of a level buffer: patch p starts at patch_offsets[p]; from
 * there, field f starts at f * fstride_p, and point (i, j, k) of the ghosted
 * box (0 <= i < nx+6, ...) is at (k * (ny+6) + j) * px_p + i, where the row
 * pitch px_p = nx+6 rounded up to a multiple of 8 doubles (of 16 when
 * nx+6 >= 256) and fstride_p = px_p (ny+6)(nz+6) rounded up to a multiple of
 * 32 doubles.  Patch offsets are 5 (13 when px_p is rounded to 16) more than
 * a multiple of 32 doubles, so that every interior row (i = 3) starts on a
 * 64-byte (128-byte) boundary, for a buffer that itself starts on one; the
 * doubles between rows are padding that no call reads as data.
 */
#ifndef MOLAMR_H
#define MOLAMR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOL_GHOST 3
#define MOL_MAX_LEVELS 8

/* error codes */
#define MOL_OK 0
#define MOL_EINVAL (-1)
#define MOL_ENOMEM (-2)
#define MOL_EHIP (-3)
#define MOL_EUNSUPPORTED (-4)
#define MOL_ESTATE (-5)

/* systems */
#define MOL_WAVE 0 /* scalar wave, Sec. IV.A: fields phi, Pi */
#define MOL_MHD 1  /* Newtonian ideal MHD, Sec. IV.B: rho, S_x, S_y, S_z, E, B^x, B^y, B^z */
#define MOL_CCZ4 2 /* CCZ4, Sec. V: chi, gt_ij(6), trKhat, At_ij(6), Ghat^i(3), Theta,
                      alpha, beta^i(3), B^i(3); symmetric pairs ordered xx xy xz yy yz zz */
#define MOL_MHD_GLM 3 /* MHD with the divergence-cleaning scalar (Sec. IV.B): the eight MHD
                         fields and psi; B^i flux + delta^{di} psi, psi flux c_h^2 B^d, source
                         -kappa_psi psi; the cleaning speeds -c_h, +c_h enter LLF and HLL */

/* MHD reconstruction of the evolved fields (App. A, App. B) and interface
 * flux (Sec. II.B.2) */
#define MOL_RECON_WENO5Z 0  /* WENO5-Z, q and epsilon as below (default) */
#define MOL_RECON_WENO5JS 1 /* WENO5-JS, alpha_r = d_r / (eps + beta_r)^2 */
#define MOL_RECON_WENO3 2   /* WENO3 (k = 2); epsilon defaults to dx^2 */
#define MOL_FLUX_LLF 0      /* local Lax-Friedrichs, eq. LLF (default) */
#define MOL_FLUX_HLL 1      /* HLL with S^L = min(v_d - c_f), S^R = max(v_d + c_f) over the two
                               states, clamped to S^L <= 0 <= S^R */
#define MOL_FLUX_SPLIT 2    /* LLF flux splitting: the reconstruction acts on (F +- alpha U)/2
                               cell by cell, alpha the largest |v_d| + c_f over the stencil */

/* time integrators */
#define MOL_RK4 0    /* Table RK44 */
#define MOL_SSPRK3 1 /* SSP-RK(3,3) of App. D (stage 3 = U^n + k1/4 + k2/4, weights (1,1,4)/6) */

typedef struct {
    int nlevels;          /* 1 .. MOL_MAX_LEVELS */
    int N0[3];            /* level-0 points per axis (periodic domain) */
    double xlo[3];        /* coordinate of index 0 on every level */
    double dx0;           /* level-0 spacing */
    const int* ratio;     /* [nlevels]; ratio[l] = dx_{l-1}/dx_l in {2,3,4}; ratio[0] ignored */
    const int* npatch;    /* [nlevels] */
    const int* boxes;     /* 6 ints per patch (lo x y z, hi x y z), levels concatenated */
    int open;             /* 0: periodic level 0; 1: open domain with radiative outer
                             boundaries (level 0 one patch; see mol_set_radiative) */
} mol_hierarchy_desc;

typedef struct {
    int system;           /* MOL_WAVE, MOL_MHD or MOL_CCZ4 */
    int upwind;           /* CCZ4: 1 = lop-sided advection stencils (Sec. II.B.1), 0 = centred */
    double sigma;         /* Kreiss-Oliger strength (Sec. II.B.1); wave and CCZ4 */
    double gamma_ad;      /* MHD ideal-gas index (Sec. IV.B) */
    double weno_eps;      /* MHD WENO epsilon; <= 0 means dx^4 (dx^2 for WENO3) (App. A, B) */
    double weno_q;        /* MHD WENO-Z exponent q (App. B); 2 */
    double kappa_z;       /* CCZ4 damping (Sec. V) */
    double kappa_c;
    double bm_f0;         /* CCZ4 Bona-Masso f = bm_f0 + bm_f1 / alpha (1+log: 0, 2) */
    double bm_f1;
    double gd_g;          /* CCZ4 Gamma-driver g and eta */
    double gd_eta;
    int mhd_recon;        /* MOL_RECON_* */
    int mhd_flux;         /* MOL_FLUX_* */
    double mhd_ch;        /* MOL_MHD_GLM: cleaning speed c_h (>= 0) */
    double mhd_kpsi;      /* MOL_MHD_GLM: damping kappa_psi (>= 0) */
} mol_system_desc;

typedef struct mol_patchset mol_patchset;

/* Build a patchset: validates the hierarchy (boxes inside the level's
 * periodic domain and non-overlapping, level 0 tiling the domain, every
 * prolongation stencil node inside the interior of a parent patch -- a margin
 * of 6 parent points between a fine level's region and the boundary of its
 * parent level's region suffices) and builds the
 * device tables: same-level/periodic ghost lists, coarse-fine ghost lists
 * (Sec. III.A), injection lists and per-level tile work lists.
 * Returns MOL_EINVAL on a bad description, MOL_EHIP/MOL_ENOMEM on device
 * failure. */
int mol_create_patchset(const mol_hierarchy_desc* h, const mol_system_desc* s,
                        mol_patchset** out);
/* As mol_create_patchset, for a hierarchy that shares its leading levels
 * with `prev` (a regrid, Sec. III.A): the levels 0..k-1 that have the same
 * ratios and boxes (in the same order) as prev's, for the same system, domain
 * and boundary, take prev's schedules (copied on the device) instead of being
 * built again; the others are built.  prev is only read and may be destroyed
 * afterwards.  Errors as mol_create_patchset; MOL_EINVAL for a null prev. */
int mol_create_patchset_from(const mol_hierarchy_desc* h, const mol_system_desc* s, const mol_patchset* prev,
                             mol_patchset** out);
/* Waits for the device to go idle, then frees the patchset. */
void mol_destroy_patchset(mol_patchset* ps);
const char* mol_last_error(void);

/* Number of fields of the patchset's system. */
int mol_nfields(const mol_patchset* ps);

/* Layout of a level buffer (pure host query).  nelems receives the number of
 * doubles of one level buffer (all fields); patch_offsets[np] (nullable) the
 * start of each patch; patch_dims[3*np] (nullable) the interior size of each
 * patch; fstrides[np] (nullable) the field stride of each patch; row_pitch[np]
 * (nullable) the row pitch px of each patch. */
int mol_level_layout(const mol_patchset* ps, int level, int64_t* nelems,
                     int64_t* patch_offsets, int32_t* patch_dims, int64_t* fstrides,
                     int32_t* row_pitch);
int mol_level_npatch(const mol_patchset* ps, int level);

/* Ghost fill of level `level`, same-level and periodic sources only (the
 * "level synchronization" of the Sec. III skeleton): every ghost point
 * (faces, edges and corners of the 3-point layer) that lies in the interior
 * of a patch of the same level, modulo the period, takes that value.  nf
 * fields of U are filled (nf = 0 means all fields of the system). */
int mol_fill_ghosts(mol_patchset* ps, int level, double* U, int nf, void* stream);

/* Right-hand side L(U) + Q_d(U) (eq. semidiscrete) on the interior of every
 * patch of the level: wave Sec. IV.A; MHD eq. conservative_discretization
 * with WENO5-Z reconstruction of the evolved fields (App. B) and the LLF flux
 * (eq. LLF); CCZ4 eqs. syseq1 .. syseq2 with the gauge of Sec. V.  U must
 * have filled ghosts.  dUdt ghosts are not written. */
int mol_rhs(mol_patchset* ps, int level, const double* U, double* dUdt, void* stream);

/* One Runge-Kutta stage (eq. eRK) fused with the right-hand side:
 * k = dt (L + Q_d)(Us) on the interior, then
 *  RK4 (Table RK44), stage s = 1..4:
 *    s = 1: Acc = k/6,  Uout = Un + k/2     s = 2: Acc += k/3, Uout = Un + k/2
 *    s = 3: Acc += k/3, Uout = Un + k       s = 4: Uout = Un + (Acc + k/6)
 *  SSP-RK3, stage s = 1..3 (Acc unused, may be NULL):
 *    s = 1: Uout = Un + k;  s = 2: Uout = 3/4 Un + 1/4 (Us + k);
 *    s = 3: Uout = 1/3 Un + 2/3 (Us + k)
 * k_store (nullable) receives k on the interior.  Us must have filled
 * ghosts and must not alias Uout; Un may alias Us; Uout may alias Un only for
 * the last stage.  Ghosts of Uout are not written, except on a CCZ4 level
 * that is one periodic patch of at least 6 points per axis: there every
 * ghost point of Uout receives the value of the interior point it is the
 * periodic image of (what mol_fill_ghosts would write), so the next stage
 * needs no fill. */
int mol_rk_stage(mol_patchset* ps, int level, int scheme, int stage, double dt,
                 const double* Un, const double* Us, double* Acc, double* Uout,
                 double* k_store, void* stream);

/* Coarse-fine ghost fill of fine level `fine_level` (>= 1) with Berger-Oliger
 * without order reduction (App. D, RK4) and quintic Lagrange interpolation
 * (Sec. III.A): for fine step r (0 <= r < R) inside the parent step and fine
 * stage s (1..4), every ghost point of the level that has no same-level
 * source takes
 *   sum_{a,b,c} L_a(xi_x) L_b(xi_y) L_c(xi_z) [Un_c + sum_j w_j(R,r,s) k_c[j]]
 * over the parent nodes around it (6 per axis, or the coincident node when
 * the fine index is a multiple of R), with w_j from the RK4 dense output and
 * the App. D fine increments.  Un_c and the k_c[4] are parent-level buffers;
 * only their interior values are read (each parent node is taken from the
 * patch whose interior owns it).  The parent stage state
 * is staged in a band buffer owned by the patchset: mol_prolong calls on one
 * patchset must not overlap in time. */
int mol_prolong(mol_patchset* ps, int fine_level, int r, int stage,
                const double* Un_c, const double* const* k_c, double* U_f, void* stream);

/* BOR weights w_1..w_4 used by mol_prolong (host query). */
int mol_bor_weights(int R, int r, int stage, double w[4]);

/* Time-refinement strategies of the sub-cycled step (Sec. III.B), or-ed into
 * the mode of mol_advance.  Each fixes the parent state U^n + sum_j w_j k_j
 * that is prolonged into the ghosts of fine step r (0 <= r < R), stage s:
 *   MOL_TIME_BOR    App. D fine increments (mol_bor_weights), order 4;
 *   MOL_TIME_BO     Berger-Oliger with the RK4 dense output b_j(theta) at
 *                   the stage time theta = (r + c_s)/R, c = (0, 1/2, 1/2, 1);
 *   MOL_TIME_BO1    linear Berger-Oliger, theta (1, 2, 2, 1)/6;
 *   MOL_TIME_NOSUB  no sub-cycling: every level steps with the parent's dt
 *                   (R = 1 in time) and stage s reads the parent's own stage
 *                   state, w = 0, (1/2,0,0,0), (0,1/2,0,0), (0,0,1,0). */
#define MOL_TIME_BOR 0
#define MOL_TIME_BO 16
#define MOL_TIME_BO1 32
#define MOL_TIME_NOSUB 48
/* Or-ed into the mode of mol_advance (and into tmode of mol_time_weights):
 * SSP-RK3 steps (App. D scheme, three stages) instead of RK4; the parent state
 * of fine step r, stage s (1..3) is then built from the SSP-RK3 increments
 * k_1..k_3 with the SSP dense output of App. C: BOR as in App. D (fine
 * k_1 = dt_F U', k_2 = dt_F U' + dt_F^2 U''; stage states U, U + k_1,
 * U + (k_1 + k_2)/4), BO at the stage time theta = (r + c_s)/R with
 * c = (0, 1, 1/2), BO1 theta (1, 1, 4)/6, no sub-cycling the parent's stage
 * states. */
#define MOL_ADV_SSPRK3 64

/* Weights w_1..w_4 of strategy `tmode` (one of MOL_TIME_*, optionally or-ed
 * with MOL_ADV_SSPRK3: then stage <= 3 and w_4 = 0), host query; for
 * MOL_TIME_NOSUB only R = 1 is valid.  MOL_EINVAL on bad arguments. */
int mol_time_weights(int tmode, int R, int r, int stage, double w[4]);

/* Radiative outer boundary of an open domain (Sec. V): every ghost point of
 * the level-0 patch evolves, in the same Runge-Kutta stages as the interior,
 * by d_t U = -v (x^i / r) d_i U - v (U - U_inf) / r, with r the distance to
 * the coordinate origin and d_i the 2nd-order centred difference where both
 * neighbours lie in the ghosted array, one-sided (2nd order, inward) at its
 * edge.  v[nf] and uinf[nf] are host arrays (defaults: v = 1, U_inf = 0).
 * MOL_EUNSUPPORTED for a periodic patchset.  The first refined level must
 * keep 6 level-0 points from the outer boundary.  The ghost shell of level 0
 * is then part of the evolved state: callers set it with the initial data. */
int mol_set_radiative(mol_patchset* ps, const double* v, const double* uinf);

/* Injection (Sec. III.A): every interior point of the parent level that
 * coincides with an interior point of `fine_level` takes the fine value. */
int mol_restrict(mol_patchset* ps, int fine_level, const double* U_f, double* U_c,
                 void* stream);

/* Vector-Jacobian product of the right-hand side (project addition; wave
 * and CCZ4 systems): lamU = (d(L + Q_d)/dU)^T lam at the state U, over the
 * ghosted box of every patch, with lam read on interior points only (its
 * ghost values are ignored).  Ghost entries of lamU receive the
 * contributions of the stencil reads; fold them back with
 * mol_fill_ghosts_adjoint.  U (ghosts filled) is read by the CCZ4 system;
 * the wave operator is linear and ignores it.  work: device memory of
 * mol_adjoint_workspace(ps, level) doubles (NULL when that is 0), overwritten.
 * The sign branch of the lop-sided advection stencils is taken at U.
 * MOL_EUNSUPPORTED for MHD. */
int mol_rhs_adjoint(mol_patchset* ps, int level, const double* U, const double* lam,
                    double* lamU, double* work, void* stream);
/* Doubles of workspace mol_rhs_adjoint needs on `level` (0 for the wave;
 * CCZ4: 299 per interior point, rows padded to 16 doubles: 139
 * stencil-input adjoints, 103 stored forward values, 57 adjoints handed
 * between its kernels); negative on error. */
int64_t mol_adjoint_workspace(const mol_patchset* ps, int level);
/* mol_rhs_adjoint without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The CCZ4 workspace lives in a static
 * device array of MOL_ADJOINT_SCRATCH_BYTES that each GPU the library runs
 * on holds until the process ends; the wave needs none.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); its device
 * address is looked up once per device on the first call made with that
 * device current.  Levels whose workspace (mol_adjoint_workspace) exceeds
 * the array are rejected with MOL_EINVAL (use mol_rhs_adjoint there): a CCZ4
 * patch of up to about 29^3 interior points fits.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other threads) race; calls ordered on one stream do not.  No
 * slot has to start at zero: every slot a call reads was written by that
 * call.  Same arguments, results and errors as mol_rhs_adjoint otherwise. */
#define MOL_ADJOINT_SCRATCH_BYTES (64ll << 20)
int mol_rhs_adjoint_noalloc(mol_patchset* ps, int level, const double* U, const double* lam,
                            double* lamU, void* stream);
/* Transpose of mol_fill_ghosts: every source point adds the ghost entries
 * that copy it, then those ghost entries are zeroed (owner gather, no atomics). */
int mol_fill_ghosts_adjoint(mol_patchset* ps, int level, double* lamU, void* stream);
/* Reverse of one RK4 step (Table RK44) on one periodic level:
 * lam <- (dU^{n+1}/dU^n)^T lam on interior points, where U^n is the state at
 * the start of the step (ghosts filled; read by the CCZ4 system, which
 * recomputes the stage states from it with the forward stage kernel; NULL
 * allowed for the wave).  w[0..5]: work buffers of the level's size (the wave
 * uses w[0..2] only); work: as for mol_rhs_adjoint.  Ghost entries of lam are
 * ignored and left unchanged. */
int mol_rk4_adjoint_step(mol_patchset* ps, int level, double dt, const double* Un, double* lam,
                         double* const w[6], double* work, void* stream);
/* The same reverse RK4 step from stage states the caller kept (project
 * addition): Ust[0..3] = U_1 = U^n, U_2 = U^n + k_1/2, U_3 = U^n + k_2/2,
 * U_4 = U^n + k_3 with k_s = dt L(U_s), ghosts filled, exactly as the forward
 * stages of mol_rk_stage produce them; read by the CCZ4 system (Ust may be
 * NULL for the wave).  Needs no forward recomputation, so a caller that
 * stores the stage states while it recomputes a checkpoint segment saves
 * three stage launches per reverse step.  w[0..2]: work buffers of the
 * level's size; work: as for mol_rhs_adjoint.  The stage states must not
 * alias lam, w or work (MOL_EINVAL). */
int mol_rk4_adjoint_step_stages(mol_patchset* ps, int level, double dt, const double* const Ust[4], double* lam,
                                double* const w[3], double* work, void* stream);

/* Reductions over the interior of every patch of the level, for
 * v = U[field] - shift: out_dev[0] = sum |v| dV, [1] = sum v^2 dV,
 * [2] = max |v|, [3] = sum over points with |x| < radius of v dV,
 * [4] = number of non-finite values.  out_dev is device memory (5 doubles).
 * The summation order is fixed (deterministic). */
int mol_norms(mol_patchset* ps, int level, const double* U, int field, double shift,
              double radius, double* out_dev, void* stream);

/* The same reductions restricted to the interior points whose coordinates lie
 * in the closed box lo[d] <= x_d <= hi[d] (infinite bounds allowed), with
 * out_dev[3] = sum over the box of v dV.  For a channel one point thick in y
 * and z, out_dev[0] / dx^2 is the line integral of |v| over [lo[0], hi[0]],
 * the reflection integral Q of the FMR wave test (Sec. IV.A).  MOL_EINVAL for
 * a NaN bound. */
int mol_box_norms(mol_patchset* ps, int level, const double* U, int field, double shift,
                  const double lo[3], const double hi[3], double* out_dev, void* stream);

/* Constraint and dissipation monitors (Sec. V, Sec. II.B.1) over the
 * interior of every patch of the level; U needs filled ghosts.  Bits of
 * `which`, and the quantity v evaluated at each interior point:
 *   MOL_MON_THETA  Theta (CCZ4)
 *   MOL_MON_Z      |Z| = sqrt(gamma_ij Z^i Z^j), Z^i = chi (Ghat^i - Gt^i)/2,
 *                  gamma_ij = gt_ij / chi (CCZ4)
 *   MOL_MON_HZ     H_Z = R + 2 nabla_i Z^i + 2/3 trKhat^2
 *                  + 2/3 Theta (trKhat - 2 Theta) - At_ij At^ij, the bracket
 *                  of the Theta equation (with Theta = Z = 0 the Hamiltonian
 *                  constraint); R + 2 nabla_i Z^i is the trace
 *                  chi gt^ij (Rhat_ij + Rhat^chi_ij) (CCZ4)
 *   MOL_MON_LNDET  ln det gt, the first conformal constraint (CCZ4)
 *   MOL_MON_TRA    tr At = gt^ij At_ij, the second (CCZ4)
 *   MOL_MON_KO     sqrt(sum_f (Q_d U_f)^2), the size of the KO term of the
 *                  right-hand side over all fields (every system)
 * out_dev (device memory, MOL_MON_OUT doubles): for monitor q (bit q),
 * out_dev[3q] = sum |v| dV, [3q+1] = sum v^2 dV, [3q+2] = max |v|, over the
 * points where v is finite (0 for monitors not requested);
 * out_dev[3 MOL_MON_COUNT] = number of non-finite values among all fields of
 * U at interior points.  The summation order is fixed (deterministic).
 * pointwise (device memory in the level layout, or NULL): the k-th
 * requested monitor (in bit order) is written to field k at every interior
 * point.  MOL_EINVAL for an empty or unknown mask, MOL_EUNSUPPORTED for a
 * CCZ4 monitor on another system. */
#define MOL_MON_THETA (1u << 0)
#define MOL_MON_Z (1u << 1)
#define MOL_MON_HZ (1u << 2)
#define MOL_MON_LNDET (1u << 3)
#define MOL_MON_TRA (1u << 4)
#define MOL_MON_KO (1u << 5)
#define MOL_MON_COUNT 6
#define MOL_MON_ALL 0x3fu
#define MOL_MON_OUT (3 * MOL_MON_COUNT + 1)
int mol_monitor(mol_patchset* ps, int level, const double* U, uint32_t which, double* pointwise,
                double* out_dev, void* stream);

/* Puncture initial data of Sec. V for the CCZ4 system on every patch of
 * `level`: the conformal factor psi = 1 + sum_A m_A / (2 r_A)
 * (eq. conformal_factor; Brill-Lindquist), chi = psi^-4, gt_ij = delta_ij,
 * alpha = psi^-2, At_ij = psi^-6 times the sum over the holes of the
 * Bowen-York solution for the hole's momentum P and spin S, and zero for
 * trKhat, Theta, Ghat^i, beta^i, B^i.  holes: nholes (1..MOL_MAX_HOLES)
 * records of 10 doubles on the host, (m, c_x, c_y, c_z, P_x, P_y, P_z, S_x,
 * S_y, S_z), with m > 0.  whole = 0 writes the interior points, 1 the whole
 * ghosted boxes (for the outer shell of an open level 0, which is evolved
 * state).  U: device level buffer.  No grid point may coincide with a
 * puncture (the data are infinite there; not checked).  MOL_EUNSUPPORTED
 * for other systems, MOL_EINVAL for bad arguments. */
#define MOL_MAX_HOLES 8
int mol_ccz4_puncture(mol_patchset* ps, int level, int nholes, const double* holes, int whole, double* U,
                      void* stream);

/* Transpose of the sphere integral of mol_norms (out_dev[3]): lam[field] =
 * scale * dV at interior points with |x| < radius, 0 at the other interior
 * points; the other fields are set to 0 on interior points; ghost entries
 * are not written. */
int mol_sphere_adjoint(mol_patchset* ps, int level, int field, double radius, double scale,
                       double* lam, void* stream);

/* Wave initial data phi = A exp(-|x-c|^2/w^2) (minimum image), Pi = 0, with
 * prm = {A, w, cx, cy, cz}; and its vector-Jacobian product
 * grad_dev[i] = sum_points lam_phi d phi / d prm_i (interior points). */
int mol_wave_gaussian(mol_patchset* ps, int level, const double prm[5], double* U,
                      void* stream);
int mol_wave_gaussian_vjp(mol_patchset* ps, int level, const double prm[5],
                          const double* lam, double* grad_dev, void* stream);
/* CCZ4 lapse pulse (a pure-gauge perturbation of flat space, Sec. V
 * variables): chi = 1, gt_ij = delta_ij, alpha = 1 + A exp(-|x-c|^2/w^2)
 * (minimum image), every other field 0, with prm = {A, w, cx, cy, cz}; and
 * its vector-Jacobian product grad_dev[i] = sum_points lam_alpha
 * d alpha / d prm_i (interior points). */
int mol_ccz4_lapse_pulse(mol_patchset* ps, int level, const double prm[5], double* U,
                         void* stream);
int mol_ccz4_lapse_pulse_vjp(mol_patchset* ps, int level, const double prm[5],
                             const double* lam, double* grad_dev, void* stream);

/* ---- sub-cycled driver (Sec. III skeleton, BOR sub-cycling) ---- */
typedef struct {
    double* U;    /* state; holds U^n on entry and U^{n+1} on return (ghosts filled) */
    double* S0;   /* stage-state work buffers */
    double* S1;
    double* acc;  /* RK4 accumulator */
    double* k[4]; /* stage increments; required on levels that have a finer level */
} mol_level_state;

#define MOL_BATCHED 0 /* one launch per level and operation (work list over all patches) */
#define MOL_PLAIN 1   /* one launch per patch and operation */

/* One RK4 (or, with MOL_ADV_SSPRK3, SSP-RK3) step of size dt0 on level 0
 * with sub-cycling of the finer levels (each level steps with dt / R of its
 * parent), prolongation of the parent state into the fine ghosts at every
 * stage and injection; states[nlevels].  mode = MOL_BATCHED or MOL_PLAIN,
 * or-ed with one MOL_TIME_* strategy (MOL_TIME_BOR when none is given) and
 * optionally MOL_ADV_SSPRK3.  MOL_EINVAL on an unknown mode. */
int mol_advance(mol_patchset* ps, const mol_level_state* states, double dt0, int mode,
                void* stream);
/* nsteps >= 1 consecutive mol_advance steps.  Every step leaves level 0's U
 * with filled ghosts, so the steps after the first skip the ghost fill of U
 * before their first stage; on a wave level that is one periodic patch, whose
 * stages read periodic images instead of ghosts, only the last step fills
 * U's ghosts.  The results are those of nsteps mol_advance calls bit for bit
 * (ghost cells of the end state included).  MOL_EINVAL when nsteps < 1. */
int mol_advance_steps(mol_patchset* ps, const mol_level_state* states, double dt0, int nsteps, int mode,
                      void* stream);

/* ---- adaptive refinement (Sec. III.A): tagging, boxes, regrid ---- */

/* flags_dev[(gz * P_y + gy) * P_x + gx] = 1 at every interior point of
 * `level` where |U[field]| >= threshold, P the level's index extent (the
 * level-0 point counts times the ratios); other entries are not written (the
 * caller clears the array).  MOL_EINVAL for a bad level or field. */
int mol_tag(mol_patchset* ps, int level, const double* U, int field, double threshold,
            uint8_t* flags_dev, void* stream);

/* Boxes that cover the tagged points of a level: the host flags
 * (dims[0] x dims[1] x dims[2], x fastest) are dilated by `buffer` points
 * (periodically), grouped into face-connected components (not across the
 * domain edges, so no box wraps), and each component's bounding box is taken;
 * boxes that overlap are merged.  boxes_out: 6 ints per box (lo x y z, hi x y
 * z), at most max_boxes; *nboxes receives the count (0 when nothing is
 * tagged).  MOL_EINVAL when more than max_boxes boxes result. */
int mol_cluster(const uint8_t* flags, const int dims[3], int buffer, int max_boxes, int* boxes_out,
                int* nboxes);

typedef struct mol_regrid mol_regrid;
/* Transfer plan between two patchsets of the same system with the same level-0
 * boxes, level count and ratios (a regrid at a synchronised time): level 0 is
 * copied; on level l >= 1 each interior point takes the old level-l value
 * where an old patch owned it, otherwise the quintic Lagrange interpolant
 * (Sec. III.A) of the new level l-1.  Built once (host lists, device
 * memory); MOL_EINVAL when the two patchsets do not match or a new point's
 * stencil leaves the new parent level. */
int mol_regrid_create(mol_patchset* ps_new, const mol_patchset* ps_old, mol_regrid** out);
/* Apply the plan: U_old[l], U_new[l] are level buffers of the old and new
 * patchsets; the ghosts of U_new[l-1] are filled before level l is
 * interpolated.  Allocates nothing. */
int mol_regrid_apply(mol_regrid* r, const double* const* U_old, double* const* U_new, void* stream);
/* Waits for the device to go idle, then frees the plan. */
void mol_regrid_destroy(mol_regrid* r);

/* ---- autotuning of the stage launches ---- */
typedef struct {
    int tdim[3]; /* launch shape: thread tile, or 64 x 8 (wave) / 15 x 15 (MHD) columns and a z-chunk length */
    int order;   /* tiles in the launch: 0 patches as listed, x fastest within a patch;
                    1 largest interior first; 2 as 0 with the tiles of each patch in
                    columns along z (z fastest); 3 as 2 with columns in blocks of 2 x 2 */
    double ms;   /* measured time of one stage launch (mol_autotune) */
} mol_tiling;
/* Time the batched stage kernel of `level` under every candidate launch shape
 * of the system (wave: z-chunks 4..512 of the z-marching kernel and five
 * thread tiles of the point-wise one; MHD: z-chunks 4..32; CCZ4: tiles
 * 8 x 8 x 4, 8 x 8 x 8 and 8 x 4 x 8) and tile orders (0 and 1; CCZ4 also 2
 * and 3), `reps` launches each (RK4 stage 2 with U as
 * U^n, S0 as stage state, acc and S1 overwritten; the kernel variant the
 * driver launches on the level: periodic stencil reads on a wave level that is
 * one periodic patch, ghost-image stores on such a CCZ4 level), and keep the fastest for
 * the level's later stage launches; *best (nullable) receives it.  The
 * results of a stage do not depend on the tiling.  Synchronises the stream;
 * graphs created before keep the tiling they captured. */
int mol_autotune(mol_patchset* ps, int level, const mol_level_state* st, double dt, int reps, mol_tiling* best,
                 void* stream);
/* Use a known tiling (one mol_autotune found earlier); MOL_EINVAL when tdim
 * is not a launch shape of the system's stage kernel or order is not 0..3. */
int mol_set_tiling(mol_patchset* ps, int level, const mol_tiling* t);

typedef struct mol_graph mol_graph;
/* Capture mol_advance(ps, states, dt0, MOL_BATCHED) into a HIP graph and
 * instantiate it (the states' buffers are baked in). */
int mol_graph_create(mol_patchset* ps, const mol_level_state* states, double dt0,
                     mol_graph** out);
/* The same for mol_advance_steps(ps, states, dt0, nsteps, MOL_BATCHED): one
 * graph whose launch takes nsteps steps. */
int mol_graph_create_steps(mol_patchset* ps, const mol_level_state* states, double dt0, int nsteps,
                           mol_graph** out);
int mol_graph_launch(mol_graph* g, void* stream);
void mol_graph_destroy(mol_graph* g);

#ifdef __cplusplus
}
#endif

#endif
