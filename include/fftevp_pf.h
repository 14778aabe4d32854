/*
 * fftevp_pf.h — C ABI of the phase-field growth of recrystallised grains.
 *
 * Grain boundary migration after DRX nucleation (Sec. 2.4): every grain i
 * carries two order parameters, eta_rex,i (recrystallised) and eta_def,i
 * (deformed). The free energy (Eq. 12) is the multi-well grain-boundary
 * energy of Eq. 13 with its gradient term plus the stored energy of Eq. 14,
 *   f_def = E_store sum_i eta_def,i^2 / sum_i (eta_rex,i^2 + eta_def,i^2),
 * and each order parameter follows the Allen-Cahn equation (Eq. 15) with the
 * kinetic coefficient 4 M_gb / (3 l_gb). A point keeps at most K order
 * parameters (the sparse storage the paper adopts to bound the number of
 * equations per point).
 *
 * Units and discretisation. The solver works in the units of the
 * quantitative parameter choice quoted in Sec. 2.4: grid spacing dx = 1,
 * l_gb = sqrt(9.6), omega_gb = l_gb / 6, M_gb dt = 0.0375 l_gb with one step
 * dt = 1. Hence the well height 6 omega/l = 1, the gradient coefficient
 * 3 omega l / 4 = 1.2 and the kinetic coefficient 4 M / (3 l) = 0.05. Energy
 * densities are in units of 6 omega_gb / l_gb (SI: 6 omega_gb /
 * (sqrt(9.6) dx_SI)), so a stored energy E_store = rho_tot zeta mu b^2 enters
 * as E_store / (6 omega_gb / (sqrt(9.6) dx_SI)). One step lasts
 * 0.225 omega_gb / M_gb seconds (Sec. 2.4), and an increment Delta t of the
 * mechanical solve allows floor(Delta t / that) steps.
 * Explicit Euler, 7-point Laplacian, periodic grid.
 *
 * Grids. The PF grid refines the mechanical grid 2:1 per axis (Sec. 2.4):
 * mechanical point i = (x, y, z) of an n0 x n1 x n2 grid covers PF points
 * 2i + a, a in {0, 1}^3, of the (2 n0) x (2 n1) x (2 n2) grid. Fields are
 * device pointers, voxel order [z][y][x] (x fastest); a slot-major array
 * holds element (j, p) at j * Vf + p, Vf = 8 n0 n1 n2.
 *
 * Order parameter keys: grain id g (int32) maps to key 2 g for eta_def and
 * 2 g + 1 for eta_rex; grains with negative ids (DRX nuclei) start
 * recrystallised, all others deformed. The grain of a key is key >> 1
 * (arithmetic shift, i.e. floor(key / 2)).
 *
 * Truncation: after every step a point keeps its order parameters above the
 * threshold, at most K of them, the largest first; equal values keep the
 * smaller key. A key absent from a point is zero there; it reappears when a
 * neighbour's value diffuses in.
 *
 * Every call is enqueued on the stream given to fftevp_pf_create; calls that
 * return a status found on the device synchronise it. The caller owns every
 * pointer it passes; the context owns its device buffers. Failures return a
 * negative fftevp_status and set fftevp_pf_last_error; nothing is changed
 * then.
 */
#ifndef FFTEVP_PF_H
#define FFTEVP_PF_H

#include "fftevp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fftevp_pf fftevp_pf;

#define FFTEVP_PF_KMAX 6

/* Create a phase-field context for the PF grid refining an n0 x n1 x n2
 * mechanical grid (each >= 1; EINVAL if 8 n0 n1 n2 >= 2^31). K: order
 * parameters kept per point, 1..FFTEVP_PF_KMAX. threshold: values <= it are
 * dropped, 0 <= threshold < 1. precision FFTEVP_FP64 keeps and updates the
 * order parameters and stored energy in FP64, FFTEVP_MIXED in FP32.
 * stream: a hipStream_t (NULL: the default stream). ENOMEM if the device
 * buffers (2 x (1 + 4 K + s K) + s bytes per PF point, s = 8 or 4) cannot
 * be allocated. */
fftevp_status fftevp_pf_create(int n0, int n1, int n2, int K, double threshold, int precision,
                               void* stream, fftevp_pf** out);
fftevp_status fftevp_pf_destroy(fftevp_pf* pf);

/* Start from a sharp grain map (Sec. 2.4): grain_dev (int32 [V], mechanical
 * grid) is refined by giving every PF point the grain of its mechanical
 * point, where it takes its one order parameter (value 1). estore_dev
 * (FP64 [V], the stored energy in the units above, finite) is refined by
 * trilinear interpolation between the mechanical points i and i + 1 along
 * each axis (periodic): a PF point 2i + a takes the mean of the two
 * neighbours for a = 1, applied along z, then y, then x. EINVAL if a value
 * is not finite or a grain id lies outside [-2^30, 2^30). */
fftevp_status fftevp_pf_refine(fftevp_pf* pf, const int* grain_dev, const double* estore_dev);

/* Replace the state by a given one on the PF grid: keys_dev (int32) and
 * vals_dev (FP64), slot-major [kin][Vf], kin in 1..64; a slot whose value,
 * rounded to the context's precision, is <= threshold is unused (its key is
 * ignored). Each point keeps its K largest values (truncation above).
 * estore_dev: FP64 [Vf], finite. EINVAL if a point holds a key twice among
 * its used slots, a used key is INT32_MIN, or a value is not finite. */
fftevp_status fftevp_pf_import(fftevp_pf* pf, const int* keys_dev, const double* vals_dev, int kin,
                               const double* estore_dev);

/* Advance nsteps >= 0 explicit steps of Eq. 15 (ESTATE before a state was
 * set by refine or import). */
fftevp_status fftevp_pf_steps(fftevp_pf* pf, int nsteps);

/* The state, slot-major [K][Vf]: keys (int32) and values (FP64), the slots
 * of a point in decreasing value (equal values: smaller key first); unused
 * slots hold key INT32_MIN and value 0. */
fftevp_status fftevp_pf_export(fftevp_pf* pf, int* keys_dev, double* vals_dev);

/* Grain map back on the mechanical grid (Sec. 2.4): mechanical point i takes
 * the grain of the largest order parameter at PF point 2i (equal values:
 * smaller key), or keeps grain_before_dev[i] if that point holds none.
 * grain_before_dev, grain_out_dev: int32 [V]; they may be the same buffer. */
fftevp_status fftevp_pf_grains(fftevp_pf* pf, const int* grain_before_dev, int* grain_out_dev);

/* The mechanical grid the context refines (host ints). */
fftevp_status fftevp_pf_dims(const fftevp_pf* pf, int* n0, int* n1, int* n2);

/* Number of PF steps that fit in a mechanical increment dt (s):
 * floor(dt / (0.225 omega_gb / M_gb)) (Sec. 2.4), omega_gb in J/m^2, M_gb in
 * m^4/(J s); -1 if an argument is not finite and positive or the count
 * exceeds 2^31 - 1. */
int fftevp_pf_step_count(double dt, double omega_gb, double mobility);

/* Grain growth after nucleation, on the mechanical solver's committed state
 * (Sec. 2.4-2.5): the stored energy E_store = rho_tot zeta mu b^2 of every
 * voxel (rho_tot as in fftevp_drx_nucleate, Eq. 11; mu and b of
 * fftevp_set_material, MPa and m) in units of 6 omega_gb / (sqrt(9.6) dx),
 * refinement of it and of the grain map onto pf (fftevp_pf_refine), nsteps
 * steps, and the grain map read back (fftevp_pf_grains). Voxels whose grain
 * changed to a recrystallised one (negative id) keep s_soften of their GND
 * densities (Eq. 16, as points of a new grain; SSD densities, orientation
 * and nucleation strength unchanged). With orientations inherited the
 * elastic moduli do not change, so the stress needs no re-solve here.
 * n_changed (may be NULL): voxels whose grain changed; n_rex (may be NULL):
 * of those, the ones now recrystallised. ESTATE unless DRX nucleation is
 * enabled on ctx; EINVAL if pf refines another grid, zeta, omega_gb or dx
 * is not finite and positive, or nsteps < 0. */
typedef struct {
  double zeta;      /* stored-energy constant (Table 2)            */
  double omega_gb;  /* grain-boundary energy, J/m^2 (Table 2)      */
  double dx;        /* PF grid spacing, m (half the voxel size)    */
} fftevp_grow;
fftevp_status fftevp_drx_grow(fftevp_ctx* ctx, fftevp_pf* pf, const fftevp_grow* p, int nsteps,
                              long long* n_changed, long long* n_rex);

const char* fftevp_pf_last_error(const fftevp_pf* pf);

#ifdef __cplusplus
}
#endif
#endif /* FFTEVP_PF_H */
