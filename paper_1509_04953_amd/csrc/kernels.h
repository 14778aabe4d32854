// Launch interface between the C-ABI layer and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "device_math.h"
#include "fft_lds.h"

namespace fftevp {

enum { MODE_NEWTON = 0, MODE_TANGENT = 1, MODE_EXPORT = 2 };

// per-block partial sums of the local kernel, stored [NPART][blocks]:
// [0] sum |e - eps|^2, [1..6] sum sigma, [7] Newton failures,
// [8] sum Newton iterations, [9] sum line-search halvings,
// [10] max Newton iterations (reduced by max)
constexpr int NPART = 11;

// Voxels per block of the local kernel (min(256, voxels) threads, one voxel
// per thread up to 256) and x-lines per block for a line length n0 (every
// power of two in [8, 512] divides the planes n1 * n2 >= 64). At 128 a block
// is one 128-point line: 3.7 % (FP64) and 4 % (FP32) faster local kernels at
// 128^3 than with 256 (more, shorter blocks per CU overlap their load, FFT
// and Newton phases better).
#ifndef FFTEVP_LOCAL_VPB
#define FFTEVP_LOCAL_VPB 128
#endif
static_assert(FFTEVP_LOCAL_VPB >= 128 && FFTEVP_LOCAL_VPB <= 512 &&
                  (FFTEVP_LOCAL_VPB & (FFTEVP_LOCAL_VPB - 1)) == 0,
              "local block size: a power of two in [128, 512] voxels");
__host__ __device__ constexpr int local_lines_per_block(int n0) {
  return n0 >= FFTEVP_LOCAL_VPB ? 1 : FFTEVP_LOCAL_VPB / n0;
}


// Device-resident control block of one increment.
struct Ctl {
  double E[6];      // macroscopic strain (Mandel) used by the next spectral update
  double Sigma[6];  // mean stress of the latest iterate (Mandel)
  double err_c, err_bc, nfail, nmax, nsum, lssum;
  int done;         // 0 running, 1 converged, 2 non-finite
  int iters;        // completed local solves
};

struct FinArgs {
  const double* partial;  // [NPART][blocks]
  int nblocks;
  double nvox, tol;
  double enorm;        // > 0: normalises err_c instead of |E|
  double sscale;       // > 0: normalises err_bc instead of |Sigma| (the adjoint's stress scale)
  int strain_ctrl[6];
  double sig_star[6];  // Mandel
  double css[36];      // [(C0)_ss]^-1 embedded in 6x6 (Mandel), zero elsewhere
  Ctl* ctl;
};

template <typename T>
// The iteration works on the increment's strain change: the spectra hold
// de = e - e_t (a compatible field of mean E - E_t), each voxel carries the
// offset q = e_t - epsp_t, and the local right-hand side is
// b = C0^-1 lam + de + q, the polarisation tau = sigma - C0 (de - C0^-1
// (sigma - lam)). In exact arithmetic this is the plain iteration on e (the
// Green operator maps C0 e_t to e_t - E_t); in floating point it never
// subtracts the total strains (0.1-0.4 late in a path) to form the elastic
// strain (1e-3), which in FP32 would cost five digits.
struct LocalArgs {
  const cx<T>* e_main;  // x-half-spectrum of de (export: of the field exported), [6][n2][n1][n0/2]
  const T* e_nyq;       // x-Nyquist plane of de, [6][n2][n1]
  cx<T>* t_main;        // out: x-half-spectrum of tau
  T* e_nyq_next;        // out: x-Nyquist plane of the next de
  const T* lam;         // multiplier (previous stress), [6][V] Mandel
  T* sig;               // out: stress, [6][V] Mandel
  const T* q;           // strain offset of b: e_t - epsp_t (tangent mode: -eigenstrain), [6][V]
  int zero_in;          // de is zero (the first iterate): the spectra are not read
  T* out_t;             // export mode: Mandel components in T, [6][V] (instead of out)
  const T* rho;         // density, [V]
  const T* quat;        // orientation, [4][V]
  const T* sig_t;       // tangent mode: stress the tangent is taken at
  const T* sysp;        // paper's flow rule: per-system parameters [3][12][V]; null: power law
  double* partial;      // [NPART][blocks]
  const Ctl* ctl;
  const cx<T>* tw;      // twiddles for n0
  double* out;          // export mode: plain-component strain, [6][V] FP64
  int nout;             // export mode: components written (0: all six)
  double dE[6];
  int add_dE;
  int n1, n2;
  Mat m;
};

template <typename T>
struct YArgs {
  const cx<T>* src;
  cx<T>* dst;
  const cx<T>* tw;
  const Ctl* ctl;
  int h;  // n0 / 2
  // forward pass only: first-stage reduction of the local kernel's partials
  // by an extra row of blocks, [NPART][n_stage1] out
  const double* partial;
  int nb_local;
  double* stage1;
  int no_reduce;  // forward pass without the reduction row (the local-rotation transform)
};

template <typename T>
struct ZArgs {
  cx<T>* buf;
  const cx<T>* tw;
  Ctl* ctl;
  const double* stage1;  // [NPART][n_stage1] partial sums from the y pass
  int n_stage1;
  FinArgs fin;           // stop test and mixed-BC update, done by the block holding xi = 0
  int h, n1;
  double inv_n0, inv_n1, inv_n2, inv_ntot;
  double c0l, c0m, ci_d, ci_o, ci_s;
  double E0[6];          // mean strain at the start of the increment (Mandel): the mean of de is E - E0
};

// GND update (Sec. 2.2, Eq. 7-8)
template <typename T>
struct GndArgs {
  const T* quat;      // [4][V]
  const int* grain;   // [V] grain ids
  const T* gd;        // slip rates of the increment (written by k_state), [12][V]
  T* rs;              // screw GND density per system (in/out), [12][V]
  T* ret;             // edge GND density per system (in/out), [12][V]
  size_t V;
  int n0, n1, n2;
  double dt, inv_b, inv_h;  // increment, 1/b (1/m), 1/l_eff (1/m)
};

// Constants of the paper's law (Sec. 2.2, Eq. 3-6), SI with stresses in MPa:
//   tau_pass = tp_c sqrt(rho_P), tau_cut = tc_c sqrt(rho_F), A = a_c sqrt(rho_P),
//   rho_M = rhom_c sqrt(rho_P rho_F), d_dipole = dd_c / |tau|,
//   climb term = climb_c sigma_vm rho_SSD^2 gdot_vm^c8.
struct MrConst {
  double tp_c, tc_c, a_c;
  double c4, c5, c6, c8;
  double rhom_c, dd_c, climb_c;
};

// DRX nucleation test (Sec. 2.3, 2.5)
template <typename T>
struct DrxArgs {
  const int* grain;   // [V] in
  int* grain_out;     // [V] out
  T* gs;              // screw GND densities [12][V] (in/out)
  T* ge;              // edge GND densities [12][V] (in/out)
  const T* ssd;       // paper's law: per-system SSD [12][V]
  const T* rho;       // power law: voxel density [V]
  T* kappa;           // nucleation strength [V] (in/out)
  const double* u;    // uniforms for the redraws [V]
  double* partial;    // [blocks][2]: nuclei count
  size_t V;
  int n0, n1, n2;
  double rhom_c, s_soften, kc_new, iq;
};

template <typename T>
struct StateArgs {
  const T* sig;
  const T* quat;
  T* epsp;
  T* rho;
  double* partial;  // [blocks][2]: sum rho_new, sum sum_a |gdot_a|
  T* gd;            // optional out: slip rates of the increment, [12][V] (GND update)
  int dens;         // 1: advance the densities too; 0: plastic strain only
  T* q;             // offset e - epsp (in/out): += de - dt epsdot_p, [6][V] Mandel
  const T* de;      // the increment's strain change, [6][V] Mandel; null: uniform dEu
  double dEu[6];
  size_t nvox;
  double dt, gdot0, k1, k2;
  Mat m;
  // paper's law: per-system SSD densities (in/out) and frozen parameters;
  // GND densities enter the forest/parallel projections when tracked
  T* ssd;             // [12][V]
  const T* sysp;      // [3][12][V]
  const T* gnds;      // [12][V] or null
  const T* gndet;     // [12][V] or null
  MrConst mr;
};

// scalar parameters of the adjoint kernels
struct AdjArgsBase {
  double dt, gdot0, n, tau0, taylor, k1, k2;
  int n_int;
};

template <typename T>
struct AdjArgs {
  const T* sig_t;   // converged stress of the increment, [6][V] Mandel
  const T* rho0;    // density at the start of the increment, [V]
  const T* quat;
  T* a_eps;         // adjoint of the plastic strain (in/out), [6][V] Mandel
  T* a_rho;         // adjoint of the density (in/out), [V]
  T* eta;           // out (setup): eigenstrain of the adjoint linear problem
  const T* z;       // in (update): stress solving the adjoint linear problem
  double* partial;
  size_t nvox;
  AdjArgsBase b;
};

struct Shift6 {
  double v[6];
};

template <typename T, int MODE>
hipError_t launch_local(int n0, const LocalArgs<T>& a, hipStream_t s);
template <typename T>
int local_blocks(int n0, int n1, int n2);
template <typename T>
int ypass_tiles(int n1, int h);
template <typename T, bool INV>
hipError_t launch_ypass(int n1, int n2, const YArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_zgamma(int n2, const ZArgs<T>& a, hipStream_t s);
// local rotation of a strain increment: forward z-FFT, w = n x (e n) per
// frequency (zero at xi = 0 and Nyquist) into components 0..2, scaled by
// a.inv_ntot, inverse z-FFT; a.ctl unused
template <typename T>
hipError_t launch_zspin(int n2, const ZArgs<T>& a, hipStream_t s);
// out = a + b, n complex values (out may alias a or b)
template <typename T>
hipError_t launch_cadd(const cx<T>* a, const cx<T>* b, cx<T>* out, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_state(const StateArgs<T>& a, int nblocks, double* out2, hipStream_t s);
template <typename T>
hipError_t launch_gdot(const T* sig, const T* quat, const T* rho, double* out, size_t V, const Mat& m,
                       double gdot0, hipStream_t s);
template <typename T>
hipError_t launch_gnd(const GndArgs<T>& a, hipStream_t s);
// paper's law: end-of-increment update, per-system parameters, slip rates
template <typename T>
hipError_t launch_state_mr(const StateArgs<T>& a, int nblocks, double* out2, hipStream_t s);
template <typename T>
hipError_t launch_split12(const T* rho, T* ssd, size_t V, hipStream_t s);
template <typename T>
hipError_t launch_kappa(const double* u, T* kappa, size_t V, double kc, double q, double* partial, int nblocks,
                        double* out2, hipStream_t s);
template <typename T>
hipError_t launch_drx(const DrxArgs<T>& a, bool mr, int nblocks, double* out2, hipStream_t s);
// lattice rotation by minus the plastic spin of the slip rates gd [12][V] over dt
template <typename T>
hipError_t launch_rotate(T* quat, const T* gd, const double* spin, size_t V, double dt, hipStream_t s);
// scale x total dislocation density (Eq. 11) of every voxel into out [V]
template <typename T>
hipError_t launch_rho_tot(const DrxArgs<T>& a, bool mr, double scale, double* out, hipStream_t s);
// grain ids a.grain (before) vs a.grain_out (after growth): counts of changed
// voxels and of those now in recrystallised grains into out2, GND softening
template <typename T>
hipError_t launch_sweep(const DrxArgs<T>& a, int nblocks, double* out2, hipStream_t s);
hipError_t launch_export_int(const int* src, double* dst, size_t V, hipStream_t s);
template <typename T>
hipError_t launch_mr_params(const T* ssd, const T* gnds, const T* gndet, T* sysp, size_t V, const MrConst& c,
                            hipStream_t s);
template <typename T>
hipError_t launch_gdot_mr(const T* sig, const T* quat, const T* sysp, double* out, size_t V, hipStream_t s);
template <typename T>
hipError_t launch_ingest(const double* q, const double* rho, T* qo, T* ro, size_t V, double* partial,
                         int nblocks, double* out2, hipStream_t s);
template <typename T>
hipError_t launch_export(const T* src, double* dst, size_t V, int ncomp, int mandel, hipStream_t s);
template <typename T>
hipError_t launch_shift_dc(cx<T>* main, size_t planes, int h, const double dE[6], hipStream_t s);
template <typename T>
hipError_t launch_fill(T* p, size_t n, T v, hipStream_t s);
template <typename T>
hipError_t launch_adj_setup(const AdjArgs<T>& a, int nblocks, double* out, hipStream_t s);
template <typename T>
hipError_t launch_adj_update(const AdjArgs<T>& a, int nblocks, double* out, hipStream_t s);

}  // namespace fftevp
