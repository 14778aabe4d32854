/*
 * fftevp.h — C ABI of the MI355X FFT-EVP fixed-point solve.
 *
 * The library solves, at every strain increment, the small-strain
 * elasto-viscoplastic problem of Zhao, Low, Wang & Niezgoda (Sec. 2.1):
 *   - implicit Euler Hooke law  sigma = C(x):[eps - epsp_t - epsdot_p(sigma) dt]  (Eq. 1),
 *   - plastic strain rate as a sum over slip systems  epsdot_p = sum_a m_a gdot_a  (Eq. 2),
 *   - stress equilibrium and strain compatibility on a periodic voxel grid,
 *     solved spectrally (FFT + Green operator of an isotropic reference medium)
 *     with an augmented-Lagrangian treatment of the nonlinear local law (Sec. 2.1),
 * with a power-law flow rule over the 12 FCC {111}<110> slip systems and a
 * Kocks-Mecking law for one dislocation density per voxel (the storage and
 * athermal-recovery terms of Eq. 6, Taylor hardening as in the passing stress
 * of Eq. 3). Inputs follow the paper's statement of the problem: a periodic
 * voxel grid, a lattice orientation and a dislocation density per voxel,
 * cubic elastic constants, an applied macroscopic strain rate with
 * stress-free lateral faces (simple compression, Sec. 3), and a time
 * increment.
 *
 * Conventions
 *   - Units: MPa, s, m, m^-2.
 *   - Symmetric tensors at this boundary are plain components in the order
 *     [11, 22, 33, 23, 13, 12] (tensor strain, not engineering shear).
 *   - Fields are device pointers, FP64, component-major and voxel-minor:
 *     element (c, z, y, x) at c*V + (z*n1 + y)*n0 + x, V = n0*n1*n2.
 *   - Quaternions (w, x, y, z), unit, rotate crystal -> sample (active).
 *   - Every call is enqueued on the stream given to fftevp_create; calls that
 *     return host scalars synchronise that stream.
 *   - The caller owns every pointer it passes; fftevp_set_* copy their input.
 *     The context owns its device workspaces.
 *   - One context per host thread at a time; contexts are independent.
 *   - The library never aborts: failures return a negative status and set
 *     the text returned by fftevp_last_error.
 */
#ifndef FFTEVP_H
#define FFTEVP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFTEVP_OK = 0,
  FFTEVP_NOT_CONVERGED = 1, /* result reported, state NOT committed           */
  FFTEVP_EINVAL = -1,       /* bad argument; nothing was changed               */
  FFTEVP_ENOMEM = -2,       /* device allocation failed                        */
  FFTEVP_EHIP = -3,         /* a HIP runtime call failed                       */
  FFTEVP_ENONFINITE = -4,   /* residual or average not finite; not committed   */
  FFTEVP_ELOCAL = -5,       /* a voxel's Newton solve did not converge         */
  FFTEVP_ESTATE = -6        /* call out of order (e.g. step before set_*)      */
} fftevp_status;

typedef enum { FFTEVP_FP64 = 0, FFTEVP_MIXED = 1 } fftevp_precision;

typedef enum {
  FFTEVP_FIELD_SIGMA = 0,       /* committed stress, 6 comps                      */
  FFTEVP_FIELD_STRAIN = 1,      /* committed compatible strain e, 6 comps         */
  FFTEVP_FIELD_EPS_P = 2,       /* plastic strain, 6 comps                        */
  FFTEVP_FIELD_RHO = 3,         /* dislocation density, 1 comp                    */
  FFTEVP_FIELD_SIGMA_ITER = 4,  /* stress of the latest iteration, 6 comps        */
  FFTEVP_FIELD_STRAIN_ITER = 5, /* compatible strain after the latest iteration   */
  FFTEVP_FIELD_GDOT = 6,        /* slip rates of the 12 systems, 1/s (see below)  */
  FFTEVP_FIELD_RHO_GNDS = 7,    /* screw GND density per system, 12 comps, m^-2   */
  FFTEVP_FIELD_RHO_GNDET = 8,   /* edge GND density per system, 12 comps, m^-2    */
  FFTEVP_FIELD_RHO_SSD = 9,     /* SSD density per system (paper's law), 12 comps */
  FFTEVP_FIELD_KAPPA = 10,      /* DRX nucleation strength, m^-2                  */
  FFTEVP_FIELD_GRAIN = 11,      /* grain ids (as doubles; nuclei negative)        */
  FFTEVP_FIELD_QUAT = 12        /* orientation quaternions (w,x,y,z), 4 comps      */
} fftevp_field;

typedef struct fftevp_ctx fftevp_ctx;

/* Cubic elastic constants in the crystal frame (MPa). Eq. 1's C(x) is this
 * tensor rotated by the voxel orientation. Requires C11 > |C12|,
 * C11 + 2 C12 > 0, C44 > 0. */
typedef struct { double C11, C12, C44; } fftevp_cubic;

/* Flow and hardening parameters.
 *   gdot_a = gdot0 |tau_a / tauc|^n sign(tau_a),   tau_a = m_a : sigma
 *   tauc   = tau0 + alpha mu b sqrt(rho)
 *   d rho / dt = (k1 sqrt(rho) - k2 rho) sum_a |gdot_a|
 * (tau0, k1, k2, n) are the parameters the adjoint differentiates.
 * Requires n >= 1, gdot0 >= 0, tau0 > 0, alpha, mu, b >= 0, k1, k2 >= 0. */
typedef struct {
  double tau0, k1, k2, n;       /* MPa, 1/m, -, -  */
  double gdot0, alpha, mu, b;   /* 1/s, -, MPa, m  */
} fftevp_flow;

/* Macroscopic loading for the next increments. Component c is strain
 * controlled when strain_ctrl[c] != 0 (its mean strain advances by
 * Edot[c]*dt per increment), otherwise stress controlled (mean stress held
 * at Sigma[c]). At least one component must be strain controlled. dt > 0. */
typedef struct {
  double Edot[6];
  double Sigma[6];
  int strain_ctrl[6];
  double dt;
} fftevp_loading;

/* Solver options. A zero field selects the default shown.
 *   tol        stop when err_c < tol and err_bc < tol          (1e-6)
 *   max_iter   fixed-point iterations per increment            (1000)
 *   newton_max Newton iterations per voxel and iteration       (50)
 *   c0_lambda, c0_mu  isotropic reference medium (MPa). Default: bulk
 *              modulus of the crystal, shear modulus 1/16 of the crystal's
 *              Voigt average. Both must be given together. */
typedef struct {
  double tol;
  int max_iter;
  int newton_max;
  double c0_lambda, c0_mu;
} fftevp_opts;

/* Per-increment report.
 *   err_c   rms_x |e - eps| / |E|   (compatibility vs. constitutive strain)
 *   err_bc  |(Sigma* - <sigma>)_s| / |<sigma>| over stress-controlled comps
 *   Sigma   volume-averaged stress of the last iterate, E the mean strain
 *   rho_mean mean density after the state update (unchanged if not committed)
 *   newton_mean, linesearch_mean  Newton iterations and line-search halvings
 *           per voxel in the last iteration */
typedef struct {
  int iters, newton_max_seen, newton_failed;
  double err_c, err_bc, Sigma[6], E[6], rho_mean;
  double newton_mean, linesearch_mean;
  double l_eff; /* effective length after the increment (m); 0 without GND */
} fftevp_report;

/* Create a context for an n0 x n1 x n2 grid (x, y, z), each a power of two
 * in [8, 512]. hip_stream is a hipStream_t (NULL: the null stream).
 * On success *out owns all device workspaces. */
fftevp_status fftevp_create(int n0, int n1, int n2, fftevp_precision precision,
                            void* hip_stream, fftevp_ctx** out);
fftevp_status fftevp_destroy(fftevp_ctx* ctx);

/* Elastic constants and flow/hardening parameters (Eq. 1-3, 6 roles above).
 * May be called again between increments (e.g. to change the parameters). */
fftevp_status fftevp_set_material(fftevp_ctx* ctx, const fftevp_cubic* cubic,
                                  const fftevp_flow* flow);

/* Per-voxel orientation and density (device, FP64): quat [4][V], rho [V].
 * Validates: quaternions finite with |q| within 1e-6 of 1, rho finite and
 * > 0; EINVAL otherwise. Resets the mechanical state (stress, strain,
 * plastic strain, mean strain, time) to zero. */
fftevp_status fftevp_set_microstructure(fftevp_ctx* ctx, const double* quat_dev,
                                        const double* rho_dev);

fftevp_status fftevp_set_loading(fftevp_ctx* ctx, const fftevp_loading* loading);

/* Geometrically necessary dislocation densities (Sec. 2.2, Eq. 7-8). From
 * this call on, every committed increment adds dt times the rates
 *   screw: -(1/b) grad(gdot_a) . t_a,   edge: (1/b) grad(gdot_a) . d_a
 * per slip system a (t = n x d, rotated to the sample frame; gdot_a the
 * increment's converged slip rates, density from the increment's start) to
 * two per-system density fields that start at zero, then multiplies the
 * effective length l_eff (the gradient's grid spacing, initially l0) by
 * (1 + eps_vm / xi), eps_vm the von Mises equivalent of the new mean strain.
 * The gradient is a finite difference on the periodic grid: central where
 * both neighbours along an axis belong to the voxel's grain, one-sided
 * towards the one that does, zero where neither does. grain_dev: device
 * int32 [V], one grain id per voxel, copied. l0, xi: finite, > 0 (EINVAL).
 * Calling it again restarts the densities and l_eff. Snapshots taken while
 * GND is tracked hold the densities and l_eff and load only into a context
 * that tracks GND too. The densities do not act back on the solve. */
fftevp_status fftevp_set_gnd(fftevp_ctx* ctx, const int* grain_dev, double l0, double xi);

/* Constants of the paper's dislocation-based law (Sec. 2.2, Eq. 3-6; Table 1
 * for Q_slip, Q_bulk, c1..c8). mu and b come from fftevp_flow. */
typedef struct {
  double T;               /* temperature, K */
  double Q_slip, Q_bulk;  /* activation energies, J */
  double c1, c2, c3;      /* passing stress, jump width, obstacle width */
  double c4;              /* lock forming, 1/m */
  double c5;              /* athermal annihilation */
  double c6;              /* dipole forming, 1/m */
  double c7;              /* thermal annihilation, m^5 s^(c8-1) */
  double c8;              /* climb exponent */
  double nu_D;            /* attempt frequency, 1/s */
  double poisson;         /* Poisson's ratio */
} fftevp_mr;

/* Select the flow rule and hardening law. law 0: the power law with the
 * Kocks-Mecking density above (default). law 1: the paper's law: per slip
 * system, gdot = gdot_0 exp(-Q_slip/kB T) sinh((|tau| - tau_pass)/tau_cut)
 * sign(tau) above the passing stress (Eq. 3), with tau_pass = c1 mu b
 * sqrt(rho_P), tau_cut = Q_slip/(c2 c3 b^2) sqrt(rho_F), gdot_0 = 2 kB T
 * nu_D sqrt(rho_P)/(c1 c3 mu b^2); forest/parallel densities from the
 * per-system SSD densities and, when tracked, the GND densities (Eq. 4-5);
 * SSD evolution (Eq. 6) with the mobile density 2 kB T sqrt(rho_P rho_F)/
 * (c1 c2 c3 mu b^3), the dipole distance sqrt3 mu b/(16 pi (1-nu) |tau|),
 * the voxel's von Mises stress and equivalent plastic rate. The parameters
 * are frozen over an increment (densities of its start) and the densities
 * advance explicitly from the converged slip rates. law 1 needs
 * set_material and set_microstructure first (ESTATE) and splits each
 * voxel's density equally over the 12 systems; set_microstructure repeats
 * that split. p: constants (EINVAL if missing or out of range; ignored for
 * law 0). The voxel density field (FFTEVP_FIELD_RHO, report rho_mean) is
 * then the sum of the 12 SSD densities. The adjoint covers law 0 only
 * (EINVAL otherwise); snapshots record the law and load only into a
 * context with the same law. */
fftevp_status fftevp_set_law(fftevp_ctx* ctx, int law, const fftevp_mr* p);

/* DRX nucleation parameters (Table 2): characteristic density kc (m^-2),
 * Weibull exponent q, kc factor s_nucl for strengths drawn after a
 * nucleation, fraction s_soften of the GND densities a nucleus keeps. */
typedef struct {
  double kc, q, s_nucl, s_soften;
} fftevp_drx;

/* Enable DRX nucleation (Sec. 2.3, 2.5): draws the nucleation strength of
 * every voxel by inverting the Weibull law P(kappa < k) = 1 - exp(-(k/kc)^q)
 * (Eq. 9-10) at the caller's uniform numbers u_dev (device, FP64 [V], each
 * in [0, 1), EINVAL otherwise; nothing is changed then). Needs GND tracking,
 * whose grain ids define the grain-boundary sites (ESTATE otherwise).
 * EINVAL unless kc, q, s_nucl > 0 and 0 <= s_soften <= 1. */
fftevp_status fftevp_set_drx(fftevp_ctx* ctx, const fftevp_drx* p, const double* u_dev);

/* One nucleation test on the committed state (call after fftevp_step). A
 * voxel with a face neighbour of another grain (periodic) nucleates when its
 * total dislocation density (Eq. 11: per system, SSD + mobile + GND, the GND
 * density being sqrt(screw^2 + edge^2); with the power law, which has one
 * density and no mobile density, the voxel density + the GND densities)
 * exceeds its strength. All sites are tested on the same state, then every
 * nucleus becomes a single-voxel grain (id -(index + 1)), keeps s_soften of
 * its GND densities (Eq. 16; SSD densities and orientation unchanged) and
 * draws a new strength with s_nucl kc at u_dev (device, FP64 [V] in [0, 1),
 * checked first: EINVAL changes nothing). The number of nuclei goes to
 * *n_nuclei (may be NULL). The stress is then out of balance with the
 * softened nuclei (their slip resistances drop with the paper's law):
 * fftevp_redistribute computes the new equilibrium. */
fftevp_status fftevp_drx_nucleate(fftevp_ctx* ctx, const double* u_dev, long long* n_nuclei);

/* Stress redistribution after the DRX microstructure update (Sec. 2.5: the
 * equilibrium stress is computed again, with the pre-DRX strain rate
 * prescribed, before further loading). Repeats the last increment's solve
 * from the mechanical state stored in state_before_dev (a snapshot, from
 * fftevp_save_state, taken just before that increment: its plastic strain,
 * stress, compatible strain and mean strain), with the same loading (the
 * same prescribed macroscopic strain increment over the same dt) and the
 * current microstructure: densities, GND densities, grains and orientations
 * as the increment, fftevp_drx_nucleate and fftevp_drx_grow left them, so
 * the slip resistances of the softened points. Commits the new stress,
 * compatible strain, mean strain and the plastic strain of the repeated
 * increment (start value + dt times the rate at the new stress); densities,
 * effective length, orientations and time are not advanced again. With the
 * power law and a density that did not change the result is the committed
 * state itself. Needs fftevp_set_drx (ESTATE). EINVAL if the snapshot does
 * not belong to this context or is not from exactly one increment before
 * the current time. NOT_CONVERGED / ENONFINITE change nothing; ELOCAL as for
 * fftevp_step. out may be NULL. */
fftevp_status fftevp_redistribute(fftevp_ctx* ctx, const void* state_before_dev, const fftevp_opts* opts,
                                  fftevp_report* out);

/* Lattice rotation (reading of the orientation change of Sec. 2.5; the
 * paper gives no equation): on = 1 turns, after every committed increment
 * (after the GND update), each voxel's lattice by exp(dw - dt Omega_p) with
 * Omega_p = sum_a gdot_a skew(d_a (x) n_a) (the increment's slip rates, the
 * sample-frame unit slip direction d_a and plane normal n_a) and dw the
 * local rigid rotation of the increment: the antisymmetric part of the
 * gradient of the periodic displacement fluctuation whose symmetric part is
 * the increment's compatible strain change, computed spectrally (axial
 * vector n x (e n) per wave direction n; none at the mean and at Nyquist
 * frequencies). The imposed macroscopic spin is zero. Orientations then
 * enter snapshots; the adjoint is unavailable (EINVAL). on = 0 (default)
 * keeps them fixed. EINVAL unless on is 0 or 1. */
fftevp_status fftevp_set_rotation(fftevp_ctx* ctx, int on);

/* One strain increment: the fixed-point solve, then the explicit update of
 * plastic strain and density at the converged stress (Eq. 1 first-order
 * update; hardening law above). Returns OK, NOT_CONVERGED (max_iter reached:
 * state kept from before the call), ENONFINITE, or ELOCAL (converged but
 * some voxel Newton solves hit newton_max; state committed). out may be NULL. */
fftevp_status fftevp_step(fftevp_ctx* ctx, const fftevp_opts* opts, fftevp_report* out);

/* fftevp_step without any allocation, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc). Same
 * increment, same kernels and bit-identical results as fftevp_step; the
 * increment's scratch (per-block partial sums, first-stage sums, control
 * block, reduction pair: about 12.6 MB) lives in a static device array of
 * the library instead of the context, one copy per device, held until the
 * process ends. The context must have been created (fftevp_create allocates
 * its fields as before); the call itself allocates nothing, device or
 * host. Limits: at most 2^24 voxels (EINVAL otherwise, nothing changed).
 * Calls that overlap on one device (two host threads, or two contexts on
 * different streams of the same device) share that array and race: the
 * caller serialises them. Kernel timing (fftevp_set_profiling) is not
 * recorded for this call. Returns as fftevp_step. */
fftevp_status fftevp_step_noalloc(fftevp_ctx* ctx, const fftevp_opts* opts, fftevp_report* out);

/* Copy a field (fftevp_field) into dst_dev (device, FP64, [ncomp][V]).
 * FFTEVP_FIELD_GDOT: the flow rule (Eq. 2 with the power law above) evaluated
 * at the committed stress and the current density, one rate per slip system
 * in the order of the system list (planes (111), (-111), (1-11), (11-1),
 * three <110> directions each), [12][V]; needs set_material and
 * set_microstructure (ESTATE otherwise). */
fftevp_status fftevp_get_field(fftevp_ctx* ctx, int field, double* dst_dev);

/* Opaque device snapshot of the committed state (plastic strain, density,
 * stress, compatible strain, mean strain, time). Buffers are device memory of
 * fftevp_state_bytes() bytes owned by the caller. Loading a snapshot makes
 * the following increments bit-identical to those run after the save. */
size_t fftevp_state_bytes(const fftevp_ctx* ctx);
fftevp_status fftevp_save_state(fftevp_ctx* ctx, void* dst_dev);
fftevp_status fftevp_load_state(fftevp_ctx* ctx, const void* src_dev);

/* Adjoint of one increment (reverse mode through the converged fixed point).
 * state_before / state_after: snapshots taken before and after the increment
 * (same loading and parameters as when it ran). dL_dSigma_mean: derivative of
 * the loss w.r.t. the increment's volume-averaged stress (plain comps; only
 * strain-controlled components matter, the others are fixed by the loading).
 * adj_state_dev (device, caller-owned, fftevp_adjoint_bytes() bytes, zero it
 * before the last increment): adjoint of the state after the increment on
 * entry, adjoint of the state before it on return. It also keeps the
 * converged solution of the implicit linear problem, from which the next
 * call (the increment before) starts its iteration: pass the same workspace
 * through the whole reverse walk, whatever the checkpoint schedule (each
 * call then starts from its successor's solution, so schedules give
 * bit-identical gradients). dL_dtheta[4] (host,
 * d/d(tau0, k1, k2, n)) is accumulated. The implicit linear problem is
 * solved with the same spectral iteration, to opts->tol; in MIXED precision
 * to max(opts->tol, 1e-5), since FP32 fields stall the tangent residual
 * near that level once the adjoint state has accumulated over many
 * increments (the gradient is then within ~1e-5 of the FP64 one). Its
 * boundary residual (stress-controlled mean components) is measured against
 * the stress scale 2 mu0 |strain| of the problem's right-hand side. The call
 * allocates nothing: it reuses the context's state buffers, so load a
 * snapshot before the next fftevp_step (ESTATE otherwise). */
size_t fftevp_adjoint_bytes(const fftevp_ctx* ctx);
fftevp_status fftevp_adjoint_increment(fftevp_ctx* ctx, const fftevp_opts* opts,
                                       const void* state_before_dev,
                                       const void* state_after_dev,
                                       const double dL_dSigma_mean[6],
                                       void* adj_state_dev, double dL_dtheta[4]);

/* Kernel timing (diagnostics). Bit k of class_mask brackets every launch of
 * kernel class k with HIP events on the context's stream: 0 local solve +
 * x-FFTs, 1 lattice rotation, 2 forward y-FFT + first reduction stage, 3 z-FFT +
 * Green operator + stop test, 4 inverse y-FFT, 5 end-of-increment update,
 * 6 adjoint set-up and reverse update, 7 GND update. Durations of launches
 * that did work (not those skipped after convergence) are summed per class.
 * fftevp_get_profile copies the sums (ms) and launch counts into caller
 * arrays of FFTEVP_NPROF entries and, if reset != 0, clears them. Each timed
 * launch adds about 4 us of event overhead to the stream. */
#define FFTEVP_NPROF 8
fftevp_status fftevp_set_profiling(fftevp_ctx* ctx, int class_mask);
fftevp_status fftevp_get_profile(fftevp_ctx* ctx, double* ms, long long* launches, int reset);

const char* fftevp_status_string(fftevp_status status);
const char* fftevp_last_error(const fftevp_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* FFTEVP_H */
