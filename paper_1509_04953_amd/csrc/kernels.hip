// FFT-EVP fixed-point iteration kernels for gfx950.
//
// One iteration of the augmented-Lagrangian scheme (Sec. 2.1, Eq. 1-2) is
// four passes over HBM:
//   k_local    per x-line: inverse real FFT along x of the compatible strain
//              (LDS), local Newton solve per voxel (registers), polarisation
//              tau = sigma - C0:eps, forward real FFT along x (LDS); FP64
//              partial sums of the residual and the mean stress.
//   k_ypass    forward FFT along y (tiles of x-frequencies, LDS); an extra
//              row of blocks reduces the partial sums (first stage, fixed
//              order) at the same time.
//   k_zgamma   forward FFT along z, Green operator per frequency, inverse
//              FFT along z, for all six components at once (LDS). The block
//              holding xi = 0 first finishes the reduction, tests for
//              convergence and updates the macroscopic strain of the
//              stress-controlled components (mixed boundary conditions).
//   k_ypass    inverse FFT along y into the next strain buffer.
// The x-Nyquist plane never needs y/z transforms: there the Green operator
// is the constant C0^-1, so k_local writes the next strain's Nyquist plane
// directly. Every kernel first reads the device stop flag and exits if the
// iteration has converged, so the host can enqueue iterations ahead.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "fft_lds.h"
#include "kernels.h"

namespace fftevp {

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block of 256 threads: reduce NP values (the last NMAX of them by max) and
// write them to out[k * stride], k < NP. Deterministic order.
template <int NP, int NMAX>
__device__ __forceinline__ void block_reduce(double (&v)[NP], double* __restrict__ out, size_t stride = 1) {
  __shared__ double red[4][NP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double r = (k >= NP - NMAX) ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == 0) red[wv][k] = r;
  }
  __syncthreads();
  if (threadIdx.x < NP) {
    const int k = threadIdx.x;
    double r = red[0][k];
    for (int w = 1; w < 4; ++w) r = (k >= NP - NMAX) ? fmax(r, red[w][k]) : r + red[w][k];
    out[k * stride] = r;
  }
}

// Block of NT threads (128 or 256), reduction through LDS (scratch:
// NP * (NT + 32) doubles): every thread stores its NP values; C threads per
// value (16, or 8 when 16 NP exceeds NT) combine NT / C entries each (thread
// c takes entries c, c + C, ...); one thread per value combines those C
// results. The last NMAX values are reduced by max. Fixed order.
template <int NP, int NMAX, int NT>
__device__ __forceinline__ void block_reduce_lds(const double (&v)[NP], double* red,
                                                 double* __restrict__ out, size_t stride) {
  constexpr int C = NP * 16 <= NT ? 16 : 8;
  static_assert(NT % C == 0 && NP * C <= NT, "one thread per (value, column)");
  constexpr int RS = NT + 16;  // row stride: rows of adjacent values fall on other banks
  double* red2 = red + NP * RS;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NP; ++k) red[k * RS + t] = v[k];
  __syncthreads();
  if (t < NP * C) {
    const int k = t / C, c = t % C;
    const double* row = red + k * RS + c;
    double r = row[0];
    if (k >= NP - NMAX) {
#pragma unroll
      for (int i = 1; i < NT / C; ++i) r = fmax(r, row[C * i]);
    } else {
#pragma unroll
      for (int i = 1; i < NT / C; ++i) r += row[C * i];
    }
    red2[t] = r;
  }
  __syncthreads();
  if (t < NP) {
    double r = red2[C * t];
    if (t >= NP - NMAX) {
#pragma unroll
      for (int i = 1; i < C; ++i) r = fmax(r, red2[C * t + i]);
    } else {
#pragma unroll
      for (int i = 1; i < C; ++i) r += red2[C * t + i];
    }
    out[t * stride] = r;
  }
}

// ---------------------------------------------------------------------------
// local kernel
// ---------------------------------------------------------------------------
template <typename T, int N0>
struct LocalShape {
  static constexpr int LPB = local_lines_per_block(N0);  // x-lines per block
  static constexpr int NT = LPB * N0 < 256 ? LPB * N0 : 256;
  static constexpr int VPT = LPB * N0 / NT;              // voxels per thread
  static constexpr int LS = N0 + 1;                    // LDS line stride
  static constexpr int H = N0 / 2;
};

// Load the x-half-spectra of the six strain components of this block's lines
// and pack them pairwise as Z = Xa + i Xb over the full length N0 (Hermitian
// extension), ready for one inverse complex FFT per pair. Spectra are stored
// with the six components innermost, so a line is one contiguous block.
template <typename T, int N0>
__device__ __forceinline__ void load_packed(const cx<T>* __restrict__ main, const T* __restrict__ nyq,
                                            size_t line0, cx<T>* sh) {
  using S = LocalShape<T, N0>;
  constexpr int PER_LINE = S::H + 1;
  // spectra are [line][k][component]: thread idx takes pair p of (l, k).
  // All loads of the thread are issued before the first LDS store.
  constexpr int TOT = 3 * S::LPB * PER_LINE, PER = (TOT + S::NT - 1) / S::NT;
  cx<T> xa[PER], xb[PER];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + b * S::NT;
    if (idx < TOT) {
      const int l = idx / (3 * PER_LINE);
      const int rem = idx - l * (3 * PER_LINE);
      const int k = rem / 3, p = rem - (rem / 3) * 3;
      const size_t line = line0 + l;
      if (k < S::H) {
        const cx<T>* src = main + (line * S::H + k) * 6 + 2 * p;
        xa[b] = src[0];
        xb[b] = src[1];
      } else {
        xa[b] = {nyq[line * 6 + 2 * p], T(0)};
        xb[b] = {nyq[line * 6 + 2 * p + 1], T(0)};
      }
    }
  }
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + b * S::NT;
    if (idx < TOT) {
      const int l = idx / (3 * PER_LINE);
      const int rem = idx - l * (3 * PER_LINE);
      const int k = rem / 3, p = rem - (rem / 3) * 3;
      if (k == 0) {
        xa[b].y = T(0);
        xb[b].y = T(0);
      }
      cx<T>* Z = sh + (p * S::LPB + l) * S::LS;
      Z[k] = {xa[b].x - xb[b].y, xa[b].y + xb[b].x};
      if (k > 0 && k < S::H) Z[N0 - k] = {xa[b].x + xb[b].y, xb[b].x - xa[b].y};
    }
  }
}

#ifndef FFTEVP_LOCAL_WAVES
#define FFTEVP_LOCAL_WAVES 1
#endif
#ifndef FFTEVP_LOCAL_WAVES_F32
#define FFTEVP_LOCAL_WAVES_F32 4
#endif
// the paper's flow rule, with its per-system parameters staged in LDS: two
// waves per SIMD in FP64 (256 VGPRs with 10 spilled in 128-thread blocks),
// four in FP32 (122)
#ifndef FFTEVP_MR_WAVES
#define FFTEVP_MR_WAVES 2
#endif
#ifndef FFTEVP_MR_WAVES_F32
#define FFTEVP_MR_WAVES_F32 4
#endif

// waves per SIMD the local kernel is compiled for; with two voxels per
// thread (lines of 512 points) the targets at which it does not spill (one
// wave FP64, three FP32)
template <typename T, int N0, int FLOW>
__host__ __device__ constexpr int local_waves() {
  if (LocalShape<T, N0>::VPT > 1) return sizeof(T) == 8 ? 1 : 3;
  if (FLOW == FLOW_MR) return sizeof(T) == 8 ? FFTEVP_MR_WAVES : FFTEVP_MR_WAVES_F32;
  return sizeof(T) == 8 ? FFTEVP_LOCAL_WAVES : FFTEVP_LOCAL_WAVES_F32;
}

// FLOW: the flow rule (FLOW_POWER, FLOW_POWER_INT when the rate exponent is
// a positive integer, FLOW_MR for the paper's law; the host picks the
// instance).
template <typename T, int N0, int MODE, int FLOW>
__global__ __launch_bounds__((LocalShape<T, N0>::NT), (local_waves<T, N0, FLOW>())) void k_local(
    LocalArgs<T> a) {
  using S = LocalShape<T, N0>;
  if (a.ctl && a.ctl->done) return;
  // LDS: the six strain/polarisation lines (complex pairs), later reused by
  // the block reduction
  constexpr int SH_BYTES = 3 * S::LPB * S::LS * (int)sizeof(cx<T>);
  constexpr int RED_BYTES = NPART * (S::NT + 32) * (int)sizeof(double);
  // the paper's law: per-system parameters of the thread's voxel staged in
  // LDS after the lines, MRQ rows (the reduction reuses the space). FP32 in
  // 128-thread blocks: all 36. FP64 in 128-thread blocks (HYB): tau_pass and
  // A, with 1/tau_cut in 24 registers, so that four blocks fit a CU (31 KB
  // each; all 36 rows, 43 KB, fit three: 12 % slower). 256-thread blocks:
  // tau_pass and 1/tau_cut, A read from cache (36 FP64 rows, 74 KB, would
  // leave one block per CU)
  constexpr bool HYB = FLOW == FLOW_MR && sizeof(T) == 8 && S::NT <= 128;
  constexpr int MRQ = FLOW != FLOW_MR ? 0 : (HYB ? 24 : (S::NT <= 128 ? 36 : 24));
  constexpr bool STAGE = MRQ > 0;
  constexpr int MRP_BYTES = MRQ * S::NT * (int)sizeof(T);
  constexpr int LDS_BYTES = SH_BYTES + MRP_BYTES > RED_BYTES ? SH_BYTES + MRP_BYTES : RED_BYTES;
  __shared__ __align__(16) unsigned char lds[LDS_BYTES];
  cx<T>* sh = reinterpret_cast<cx<T>*>(lds);
  T* mrp = reinterpret_cast<T*>(lds + SH_BYTES);
  const size_t planes = (size_t)a.n1 * a.n2;
  const size_t vox = planes * N0;
  const size_t line0 = (size_t)blockIdx.x * S::LPB;
  const Mat& M = a.m;

  // per-voxel inputs of the thread's first voxel, requested before the x-FFT
  // so that their latency overlaps it (later voxels load in the loop)
  T pq[4], plam[6], poff[6], prho;
  auto fetch = [&](size_t g) {
#pragma unroll
    for (int k = 0; k < 4; ++k) pq[k] = a.quat[(size_t)k * vox + g];
#pragma unroll
    for (int k = 0; k < 6; ++k) plam[k] = a.lam[(size_t)k * vox + g];
#pragma unroll
    for (int k = 0; k < 6; ++k) poff[k] = a.q[(size_t)k * vox + g];
    prho = a.rho[g];
  };
  if constexpr (MODE != MODE_EXPORT) {
    const int l = threadIdx.x / N0, x = threadIdx.x - (threadIdx.x / N0) * N0;
    fetch((line0 + l) * N0 + x);
  }

  const bool zero_in = MODE != MODE_EXPORT && a.zero_in;
  if (!zero_in) {
    load_packed<T, N0>(a.e_main, a.e_nyq, line0, sh);
    __syncthreads();
    fft_lines<T, N0, true, 3 * S::LPB, S::LS, S::NT>(sh, a.tw);
  }

  if constexpr (MODE == MODE_EXPORT) {
    // write the real field: plain components in FP64, or Mandel in T
#pragma unroll
    for (int v = 0; v < S::VPT; ++v) {
      const int t = threadIdx.x + v * S::NT;
      const int l = t / N0, x = t - (t / N0) * N0;
      const size_t g = (line0 + l) * N0 + x;
      if (a.out_t) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const cx<T> z = sh[(p * S::LPB + l) * S::LS + x];
          a.out_t[(size_t)(2 * p) * vox + g] = z.x;
          a.out_t[(size_t)(2 * p + 1) * vox + g] = z.y;
        }
        continue;
      }
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const cx<T> z = sh[(p * S::LPB + l) * S::LS + x];
        const double f0 = (2 * p >= 3) ? kIR2 : 1.0;
        const double f1 = (2 * p + 1 >= 3) ? kIR2 : 1.0;
        const int nout = a.nout > 0 ? a.nout : 6;
        if (2 * p < nout) a.out[(size_t)(2 * p) * vox + g] = f0 * (double)z.x;
        if (2 * p + 1 < nout) a.out[(size_t)(2 * p + 1) * vox + g] = f1 * (double)z.y;
      }
    }
    return;
  }

  double part[NPART];
#pragma unroll
  for (int k = 0; k < NPART; ++k) part[k] = 0.0;

  const T ci_d = T(M.ci_d), ci_o = T(M.ci_o), ci_s = T(M.ci_s);
  const T c0l = T(M.c0l), c0m2 = T(2.0 * M.c0m);

#pragma unroll 1
  for (int v = 0; v < S::VPT; ++v) {
    const int t = threadIdx.x + v * S::NT;
    const int l = t / N0, x = t - (t / N0) * N0;
    const size_t g = (line0 + l) * N0 + x;
    auto load_e = [&](T (&e)[6]) {
      if (zero_in) {
#pragma unroll
        for (int k = 0; k < 6; ++k) e[k] = T(0);
      } else {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const cx<T> z = sh[(p * S::LPB + l) * S::LS + x];
          e[2 * p] = z.x;
          e[2 * p + 1] = z.y;
        }
      }
      if (a.add_dE) {
#pragma unroll
        for (int k = 0; k < 6; ++k) e[k] += T(a.dE[k]);
      }
    };
    if (v > 0) fetch(g);
    if constexpr (STAGE) {
      // each thread reads back only its own column: no barrier
#pragma unroll
      for (int q = 0; q < MRQ; ++q)
        mrp[q * S::NT + threadIdx.x] = a.sysp[(size_t)(HYB && q >= 12 ? q + 12 : q) * vox + g];
    }
    const T tauc = T(M.tau0) + T(M.taylor) * sqrt(prho);
    const T itauc = T(1) / tauc;

    // b = C0^-1 lam + de + q in the crystal frame; start from lam
    T b[6], sc[6];
    {
      T R[9], e[6], bs[6];
      quat_rot(pq[0], pq[1], pq[2], pq[3], R);
      load_e(e);
      cubic_mul(ci_d, ci_o, ci_s, plam, bs);
#pragma unroll
      for (int k = 0; k < 6; ++k) bs[k] += e[k] + poff[k];
      to_crystal(R, bs, b);
      if constexpr (MODE == MODE_NEWTON) to_crystal(R, plam, sc);
    }

    int nit = 0, fail = 0, nls = 0;
    if constexpr (MODE == MODE_NEWTON) {
      // Damped Newton on the convex potential, written around one evaluation
      // of the residual: each pass evaluates the candidate, then either
      // halves the step (line search) or accepts it and computes the next
      // Newton direction from the accepted point's tangent.
      float w[12], r[6], d[6];
      T phi = T(0);
      float slope = 0.f, rn2 = 0.f;
      T step = T(0);
      const float cj = FLOW == FLOW_MR ? float(M.dt) : float(T(M.c1) * T(M.n) * itauc);
      const SysParams<T> sp{a.sysp, vox, g};
      T itcr[12];
      if constexpr (HYB) {
#pragma unroll
        for (int q = 0; q < 12; ++q) itcr[q] = sp.itc(q);
      }
      const T ntol2 = T(M.ntol) * T(M.ntol), qtol2 = T(M.qtol) * T(M.qtol);
      bool conv = false, first = true;
#pragma unroll
      for (int k = 0; k < 6; ++k) d[k] = 0.f;
#pragma unroll 1
      for (int pass = 0; pass < 64 * M.newton_max; ++pass) {
        T phi1, cand[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) cand[k] = sc[k] + step * T(d[k]);
        if constexpr (STAGE) {
          // the per-system parameters are re-read at every evaluation (from
          // LDS; 1/tau_cut from registers in FP64 128-thread blocks, A from
          // cache in 256-thread blocks) through a column index and a pointer
          // made opaque per pass, instead of being hoisted out of the loop
          // into 36 (FP32) or 72 (FP64) live registers: at 128^3 the local
          // kernel takes 29 % (FP32) and 44 % (FP64) less time than with the
          // parameters in registers (FP32) or re-read from cache (FP64)
          uint64_t pp = reinterpret_cast<uint64_t>(sp.p);
          int col = threadIdx.x;
          asm volatile("" : "+s"(pp), "+v"(col));
          if constexpr (HYB) {
            const SysParamsHybrid<T> spp{mrp, S::NT, col, itcr};
            local_residual<FLOW>(M, cand, b, tauc, itauc, w, r, phi1, spp);
          } else {
            const SysParamsStaged<T, MRQ> spp{reinterpret_cast<const T*>(pp), sp.V, sp.g, mrp, S::NT, col};
            local_residual<FLOW>(M, cand, b, tauc, itauc, w, r, phi1, spp);
          }
        } else {
          local_residual<FLOW>(M, cand, b, tauc, itauc, w, r, phi1, sp);
        }
        float rn1 = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) rn1 += r[k] * r[k];
        if (!first) {
          const bool ok = isfinite(phi1) && (phi1 <= phi + T(1e-4) * step * T(slope) || rn1 <= 0.25f * rn2);
          if (!ok && step > T(1e-12)) {
            step *= T(0.5);
            ++nls;
            continue;
          }
          T dn2 = T(0), sn2 = T(0);
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            const T dk = step * T(d[k]);
            dn2 += dk * dk;
            sc[k] = cand[k];
            sn2 += cand[k] * cand[k];
          }
          ++nit;
          const T sc2 = fmax(sn2, T(1));
          if (dn2 <= ntol2 * sc2) {
            conv = true;
            break;
          }
          if (nit >= M.newton_max) break;
        }
        first = false;
        phi = phi1;
        rn2 = rn1;
        {
          // Newton direction in FP32: the residual, line search and stop
          // test stay in T, so the converged stress is the T-precision root
          float J[21], mr[6];
          local_jacobian<float>(M, w, cj, J);
#pragma unroll
          for (int k = 0; k < 6; ++k) mr[k] = -r[k];
          ldl_solve(J, mr, d);
        }
        // a full step this small is in the quadratic regime: take it without
        // evaluating the candidate (its error is of the step's square)
        {
          T dn2 = T(0), sn2 = T(0);
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            dn2 += T(d[k]) * T(d[k]);
            sn2 += sc[k] * sc[k];
          }
          if (dn2 <= qtol2 * fmax(sn2, T(1))) {
#pragma unroll
            for (int k = 0; k < 6; ++k) sc[k] += T(d[k]);
            ++nit;
            conv = true;
            break;
          }
        }
        slope = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) slope += r[k] * d[k];
        step = T(1);
      }
      fail = conv ? 0 : 1;
    } else {  // MODE_TANGENT: linear solve with the tangent at the given stress
      T R[9], st[6], stc[6], w[12], g6[6], visc, asum, J[21];  // full precision tangent
      quat_rot(pq[0], pq[1], pq[2], pq[3], R);
#pragma unroll
      for (int k = 0; k < 6; ++k) st[k] = a.sig_t[(size_t)k * vox + g];
      to_crystal(R, st, stc);
      static_assert(FLOW != FLOW_MR, "tangent solves use the power law");
      flow_eval<FLOW == FLOW_POWER_INT>(stc, itauc, T(M.n), M.n_int, w, g6, visc, asum);
      local_jacobian<T>(M, w, T(M.c1) * T(M.n) * itauc, J);
      ldl_solve(J, b, sc);
      nit = 1;
    }

    // back to the sample frame; eps - e_t = de - C0^-1 (sigma - lam); tau = sigma - C0 (eps - e_t)
    T sig[6], err[6], e[6];
    {
      T R[9], dsl[6];
      quat_rot(pq[0], pq[1], pq[2], pq[3], R);
      to_sample(R, sc, sig);
#pragma unroll
      for (int k = 0; k < 6; ++k) dsl[k] = sig[k] - plam[k];
      cubic_mul(ci_d, ci_o, ci_s, dsl, err);
    }
    // re-read e from LDS rather than keeping it live through the Newton loop
    asm volatile("" ::: "memory");
    load_e(e);
    T tr = T(0), eps[6], tau[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      eps[k] = e[k] - err[k];
      if (k < 3) tr += eps[k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) tau[k] = sig[k] - c0m2 * eps[k] - (k < 3 ? c0l * tr : T(0));
#pragma unroll
    for (int k = 0; k < 6; ++k) a.sig[(size_t)k * vox + g] = sig[k];
#pragma unroll
    for (int p = 0; p < 3; ++p) sh[(p * S::LPB + l) * S::LS + x] = {tau[2 * p], tau[2 * p + 1]};

    double e2 = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      e2 += (double)err[k] * (double)err[k];
      part[1 + k] += (double)sig[k];
    }
    part[0] += e2;
    part[7] += (double)fail;
    part[8] += (double)nit;
    part[9] += (double)nls;
    part[10] = fmax(part[10], (double)nit);
  }
  __syncthreads();
  fft_lines<T, N0, false, 3 * S::LPB, S::LS, S::NT>(sh, a.tw);

  // unpack: Xa[k] = (Z[k] + conj Z[N-k]) / 2, Xb[k] = (Z[k] - conj Z[N-k]) / 2i
  constexpr int UPER = (3 * S::LPB * S::H + S::NT - 1) / S::NT;
#pragma unroll
  for (int ub = 0; ub < UPER; ++ub) {
    const int idx = threadIdx.x + ub * S::NT;
    if (idx >= 3 * S::LPB * S::H) break;
    const int l = idx / (3 * S::H);
    const int rem = idx - l * (3 * S::H);
    const int k = rem / 3, p = rem - (rem / 3) * 3;
    const cx<T>* Z = sh + (p * S::LPB + l) * S::LS;
    const cx<T> zk = Z[k], zm = Z[(N0 - k) & (N0 - 1)];
    const cx<T> xa = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    const cx<T> xb = {T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
    cx<T>* dst = a.t_main + ((line0 + l) * S::H + k) * 6 + 2 * p;
    dst[0] = xa;
    dst[1] = xb;
  }
  // x-Nyquist plane of the next strain: e = -C0^-1 tau_hat / n0 (real)
  if (threadIdx.x < S::LPB) {
    const int l = threadIdx.x;
    T tn[6], en[6];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const cx<T> z = sh[(p * S::LPB + l) * S::LS + S::H];
      tn[2 * p] = z.x;
      tn[2 * p + 1] = z.y;
    }
    cubic_mul(ci_d, ci_o, ci_s, tn, en);
    const T s = -T(M.inv_n0);
#pragma unroll
    for (int k = 0; k < 6; ++k) a.e_nyq_next[(line0 + l) * 6 + k] = s * en[k];
  }
  __syncthreads();  // the line buffer is reused below
  block_reduce_lds<NPART, 1, S::NT>(part, reinterpret_cast<double*>(lds), a.partial + blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// y pass: FFT along y of tiles of TX consecutive x-frequencies
// ---------------------------------------------------------------------------
// LDS budget of the y and z passes; the tile width TX (x-frequencies per
// block, six components each) is the largest power of two that fits.
#ifndef FFTEVP_SPEC_LDS_KB
#define FFTEVP_SPEC_LDS_KB 25
#endif
#ifndef FFTEVP_Y_LDS_KB
#define FFTEVP_Y_LDS_KB 25
#endif

// FP64 lines of 256 points or more get twice the budget: with 25 KB a tile
// holds one x-frequency, whose 96-byte row segments straddle cache lines
// that neighbouring tiles complete (measured at 256^3: the y passes wrote
// 1.3x their bytes); two x-frequencies (49 KB, three blocks per CU) ran the
// FP64 y and z passes 23-27 % faster there. Shorter lines measured fastest
// at 25 KB.
#ifndef FFTEVP_SPEC_LDS_KB_F64_LONG
#define FFTEVP_SPEC_LDS_KB_F64_LONG 50
#endif
// FP32 lines of 256+ points: the z pass and the inverse y pass take 50 KB
// tiles too (four x-frequencies, rows of 192 B instead of 96 B that two
// tiles share a cache line of): 20 % and 11 % faster at 256^3; the forward
// y pass, which also reduces the local kernel's partials, measured 7 %
// slower with them and keeps 25 KB.
#ifndef FFTEVP_SPEC_LDS_KB_F32_LONG
#define FFTEVP_SPEC_LDS_KB_F32_LONG 50
#endif
#ifndef FFTEVP_Y_FWD_WIDE32
#define FFTEVP_Y_FWD_WIDE32 0
#endif
template <typename T>
__host__ __device__ constexpr int spec_budget_kb(int n, int kb, bool wide32) {
  if (n < 256) return kb;
  return sizeof(T) == 8 ? FFTEVP_SPEC_LDS_KB_F64_LONG : (wide32 ? FFTEVP_SPEC_LDS_KB_F32_LONG : kb);
}
template <typename T>
__host__ __device__ constexpr int spec_tile(int n, int kb = FFTEVP_SPEC_LDS_KB, bool wide32 = true) {
  int tx = 16;
  const int budget = spec_budget_kb<T>(n, kb, wide32);
  while (tx > 1 && 6 * tx * (n + 1) * 2 * (int)sizeof(T) > budget * 1024) tx /= 2;
  return tx;
}
template <typename T, bool INV>
__host__ __device__ constexpr int y_tile(int n) {
  return spec_tile<T>(n, FFTEVP_Y_LDS_KB, INV || FFTEVP_Y_FWD_WIDE32);
}

// Workgroups are dealt round-robin to the eight XCDs, each with its own L2.
// The y and z passes renumber them so that every XCD takes a contiguous range
// of tiles: neighbouring tiles, whose rows share cache lines, then meet in
// the same L2 instead of fetching those lines twice.
#ifndef FFTEVP_XCD_REMAP
#define FFTEVP_XCD_REMAP 1
#endif
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int nx = gridDim.x, total = gridDim.x * gridDim.y;
  int id = blockIdx.x + nx * blockIdx.y;
  if (FFTEVP_XCD_REMAP && total % 8 == 0) id = (id % 8) * (total / 8) + id / 8;
  bx = id % nx;
  by = id / nx;
}

// Rows of W = 6 TX contiguous complex values (row stride rs) <-> W lines of
// length N in LDS (line stride N + 1).
template <typename T, int N, int W>
__device__ __forceinline__ void rows_to_lines(const cx<T>* __restrict__ src, size_t rs, cx<T>* sh) {
  if constexpr (sizeof(T) == 4 && W % 2 == 0) {
    // FP32: two complex values per 16-byte load (rows, strides and bases
    // hold an even number of complex values, so every pair is aligned)
    constexpr int TOT = N * W / 2, PER = (TOT + 255) / 256;
    float4 v[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int idx = threadIdx.x + 256 * b;
      if (TOT % 256 == 0 || idx < TOT) {
        const int e = 2 * idx, r = e / W, w = e - (e / W) * W;
        v[b] = *reinterpret_cast<const float4*>(src + (size_t)r * rs + w);
      }
    }
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int idx = threadIdx.x + 256 * b;
      if (TOT % 256 == 0 || idx < TOT) {
        const int e = 2 * idx, r = e / W, w = e - (e / W) * W;
        sh[w * (N + 1) + r] = {v[b].x, v[b].y};
        sh[(w + 1) * (N + 1) + r] = {v[b].z, v[b].w};
      }
    }
    return;
  }
  // every load of the thread is issued before the first LDS store, so the
  // HBM latencies overlap instead of adding up
  constexpr int TOT = N * W, PER = (TOT + 255) / 256;
  cx<T> v[PER];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + 256 * b;
    if (TOT % 256 == 0 || idx < TOT) {
      const int r = idx / W, w = idx - (idx / W) * W;
      v[b] = src[(size_t)r * rs + w];
    }
  }
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + 256 * b;
    if (TOT % 256 == 0 || idx < TOT) {
      const int r = idx / W, w = idx - (idx / W) * W;
      sh[w * (N + 1) + r] = v[b];
    }
  }
}
template <typename T, int N, int W>
__device__ __forceinline__ void lines_to_rows(const cx<T>* sh, cx<T>* __restrict__ dst, size_t rs) {
  if constexpr (sizeof(T) == 4 && W % 2 == 0) {
    constexpr int TOT = N * W / 2, PER = (TOT + 255) / 256;
    float4 v[PER];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int idx = threadIdx.x + 256 * b;
      if (TOT % 256 == 0 || idx < TOT) {
        const int e = 2 * idx, r = e / W, w = e - (e / W) * W;
        const cx<T> z0 = sh[w * (N + 1) + r], z1 = sh[(w + 1) * (N + 1) + r];
        v[b] = make_float4(z0.x, z0.y, z1.x, z1.y);
      }
    }
#pragma unroll
    for (int b = 0; b < PER; ++b) {
      const int idx = threadIdx.x + 256 * b;
      if (TOT % 256 == 0 || idx < TOT) {
        const int e = 2 * idx, r = e / W, w = e - (e / W) * W;
        *reinterpret_cast<float4*>(dst + (size_t)r * rs + w) = v[b];
      }
    }
    return;
  }
  constexpr int TOT = N * W, PER = (TOT + 255) / 256;
  cx<T> v[PER];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + 256 * b;
    if (TOT % 256 == 0 || idx < TOT) {
      const int r = idx / W, w = idx - (idx / W) * W;
      v[b] = sh[w * (N + 1) + r];
    }
  }
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + 256 * b;
    if (TOT % 256 == 0 || idx < TOT) {
      const int r = idx / W, w = idx - (idx / W) * W;
      dst[(size_t)r * rs + w] = v[b];
    }
  }
}

// Transforms of a tile's W lines between global rows and LDS. With FUSE the
// first stage of the plan reads the rows itself and the last one writes
// them, so a two-stage line (32 to 256 points) passes through LDS once
// instead of three times, with one barrier instead of five. The z pass
// (forward, Green operator, inverse in one block) gained 4-11 % from it at
// 128^3 and 256^3 and the y passes 2-8 % on lines of 128 points; on lines of
// 256 points the y passes ran 5-11 % slower (fewer threads issue the row
// accesses), so they keep the row copies there.
#ifndef FFTEVP_FUSED_EDGE
#define FFTEVP_FUSED_EDGE 1
#endif
#ifndef FFTEVP_FUSED_Y_MAX
#define FFTEVP_FUSED_Y_MAX 128
#endif
// lines per thread at the edges: FP32 lines of 256+ points move in pairs as
// one 16-byte access (z pass 8 % faster at 256^3), shorter ones singly (z
// pass 8 % faster at 128^3, where a tile has twice the lines)
#ifndef FFTEVP_ROW_PACK32_MIN_N
#define FFTEVP_ROW_PACK32_MIN_N 256
#endif
template <typename T, int N>
constexpr int row_pack = (sizeof(T) == 4 && N >= FFTEVP_ROW_PACK32_MIN_N) ? 2 : 1;

// rows -> LDS, all stages of the plan but the last (ends with a barrier)
template <typename T, int N, int W, bool INV, int LS, bool FUSE>
__device__ __forceinline__ void fft_head(const cx<T>* __restrict__ src, size_t rs, cx<T>* sh,
                                         const cx<T>* __restrict__ tw) {
  constexpr int NSL = last_stage_ns(N);
  if constexpr (FUSE && NSL > 1) {
    first_stage_from_rows<T, N, W, INV, LS, 256, row_pack<T, N>>(src, rs, sh);
    fft_stages<T, N, radix_at(N, 1), NSL, INV, W, LS, 256>(sh, tw);
  } else {
    static_assert(LS == N + 1, "row copies use line stride N + 1");
    rows_to_lines<T, N, W>(src, rs, sh);
    __syncthreads();
    fft_stages<T, N, 1, NSL, INV, W, LS, 256>(sh, tw);
  }
}
// the plan's last stage, LDS -> rows
template <typename T, int N, int W, bool INV, int LS, bool FUSE>
__device__ __forceinline__ void fft_tail(const cx<T>* sh, const cx<T>* __restrict__ tw,
                                         cx<T>* __restrict__ dst, size_t rs) {
  if constexpr (FUSE) {
    last_stage_to_rows<T, N, W, INV, LS, 256, row_pack<T, N>>(sh, tw, dst, rs);
  } else {
    constexpr int NSL = last_stage_ns(N);
    fft_stages<T, N, NSL, N, INV, W, LS, 256>(const_cast<cx<T>*>(sh), tw);
    lines_to_rows<T, N, W>(sh, dst, rs);
  }
}

// FFT along y of TX x-frequencies x 6 components. The forward pass has one
// extra row of blocks (blockIdx.y == 0): block b of that row reduces a
// contiguous share of the local kernel's per-block partial sums, in a fixed
// order, while the other rows transform.
// waves per SIMD the y and z passes are compiled for (register budget)
#ifndef FFTEVP_SPEC_WAVES
#define FFTEVP_SPEC_WAVES 1
#endif


template <typename T, int N1, int TX, bool INV>
__global__ __launch_bounds__(256, FFTEVP_SPEC_WAVES) void k_ypass(YArgs<T> a) {
  if (a.ctl && a.ctl->done) return;
  int bx, by;
  xcd_tile(bx, by);
  const bool red_row = !INV && !a.no_reduce;
  if constexpr (!INV) {
    if (red_row && by == 0) {
      const int ns = gridDim.x, nb = a.nb_local;
      const int chunk = (nb + ns - 1) / ns;
      const int b0 = bx * chunk, b1 = min(nb, b0 + chunk);
      double v[NPART];
#pragma unroll
      for (int k = 0; k < NPART; ++k) v[k] = 0.0;
      for (int b = b0 + threadIdx.x; b < b1; b += 256) {
#pragma unroll
        for (int k = 0; k < NPART - 1; ++k) v[k] += a.partial[(size_t)k * nb + b];
        v[NPART - 1] = fmax(v[NPART - 1], a.partial[(size_t)(NPART - 1) * nb + b]);
      }
      block_reduce<NPART, 1>(v, a.stage1 + bx, ns);
      return;
    }
  }
  constexpr int W = 6 * TX;
  __shared__ cx<T> sh[W * (N1 + 1)];
  const size_t rs = (size_t)a.h * 6;  // y stride
  const size_t z = red_row ? by - 1 : by;
  const size_t base = z * N1 * rs + (size_t)bx * W;
  constexpr bool FUSE = FFTEVP_FUSED_EDGE && N1 <= FFTEVP_FUSED_Y_MAX;
  fft_head<T, N1, W, INV, N1 + 1, FUSE>(a.src + base, rs, sh, a.tw);
  fft_tail<T, N1, W, INV, N1 + 1, FUSE>(sh, a.tw, a.dst + base, rs);
}

// ---------------------------------------------------------------------------
// z pass with the Green operator of the isotropic reference medium
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void apply_gamma(cx<T> (&t)[6], T nx, T ny, T nz, T c_mu, T c_ratio) {
  // v = tau n;  w = (v - ratio (n.v) n) / mu0;  e = -sym(n (x) w)   (Mandel)
  const T h = T(kIR2);
  cx<T> v[3];
  // tensor components: T11=t0, T22=t1, T33=t2, T23=h t3, T13=h t4, T12=h t5
  v[0] = {t[0].x * nx + h * (t[5].x * ny + t[4].x * nz), t[0].y * nx + h * (t[5].y * ny + t[4].y * nz)};
  v[1] = {h * t[5].x * nx + t[1].x * ny + h * t[3].x * nz, h * t[5].y * nx + t[1].y * ny + h * t[3].y * nz};
  v[2] = {h * (t[4].x * nx + t[3].x * ny) + t[2].x * nz, h * (t[4].y * nx + t[3].y * ny) + t[2].y * nz};
  const cx<T> nv = {v[0].x * nx + v[1].x * ny + v[2].x * nz, v[0].y * nx + v[1].y * ny + v[2].y * nz};
  const T nn[3] = {nx, ny, nz};
  cx<T> w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    w[i] = {c_mu * (v[i].x - c_ratio * nv.x * nn[i]), c_mu * (v[i].y - c_ratio * nv.y * nn[i])};
  const T r2 = T(kR2) * T(0.5);
  t[0] = {-nx * w[0].x, -nx * w[0].y};
  t[1] = {-ny * w[1].x, -ny * w[1].y};
  t[2] = {-nz * w[2].x, -nz * w[2].y};
  t[3] = {-r2 * (ny * w[2].x + nz * w[1].x), -r2 * (ny * w[2].y + nz * w[1].y)};
  t[4] = {-r2 * (nx * w[2].x + nz * w[0].x), -r2 * (nx * w[2].y + nz * w[0].y)};
  t[5] = {-r2 * (nx * w[1].x + ny * w[0].x), -r2 * (nx * w[1].y + ny * w[0].y)};
}

template <typename T, int N2, int TX>
__global__ __launch_bounds__(256, FFTEVP_SPEC_WAVES) void k_zgamma(ZArgs<T> a) {
  if (a.ctl->done) return;
  constexpr int LS = N2 + 1;
  constexpr int W = 6 * TX;
  __shared__ cx<T> sh[W * LS];
  __shared__ double E_sh[6];
  int bx, by;
  xcd_tile(bx, by);
  // the block holding xi = 0 finishes the reduction, tests for convergence
  // and updates the macroscopic strain before using it
  if (bx == 0 && by == 0) {
    __shared__ double tot[NPART];
    if (threadIdx.x < NPART) {
      const int k = threadIdx.x;
      double r = a.stage1[(size_t)k * a.n_stage1];
      for (int b = 1; b < a.n_stage1; ++b) {
        const double x = a.stage1[(size_t)k * a.n_stage1 + b];
        r = (k == NPART - 1) ? fmax(r, x) : r + x;
      }
      tot[k] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      finalize_sums(a.fin, a.ctl, tot);
      for (int k = 0; k < 6; ++k) E_sh[k] = a.ctl->E[k] - a.E0[k];
    }
    __syncthreads();
  }
  const int H = a.h, n1 = a.n1;
  const int ky = by, kx0 = bx * TX;
  const size_t zs = (size_t)n1 * H * 6;  // z stride
  cx<T>* __restrict__ buf = a.buf + ((size_t)ky * H + kx0) * 6;
  fft_head<T, N2, W, false, LS, FFTEVP_FUSED_EDGE>(buf, zs, sh, a.tw);
  fft_stages<T, N2, last_stage_ns(N2), N2, false, W, LS, 256>(sh, a.tw);

  const T inv_n = T(a.inv_ntot);
  const T c_mu = T(1.0 / a.c0m), c_ratio = T((a.c0l + a.c0m) / (a.c0l + 2.0 * a.c0m));
  const T ci_d = T(a.ci_d), ci_o = T(a.ci_o), ci_s = T(a.ci_s);
  const int ky_s = ky < n1 / 2 ? ky : ky - n1;
  const bool nyq_y = (2 * ky == n1);
  for (int idx = threadIdx.x; idx < N2 * TX; idx += 256) {
    const int z = idx / TX, kx = idx - (idx / TX) * TX;
    const int kz_s = z < N2 / 2 ? z : z - N2;
    cx<T> t[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) t[c] = sh[(kx * 6 + c) * LS + z];
    const int kxg = kx0 + kx;
    if (kxg == 0 && ky == 0 && z == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) t[c] = {T(E_sh[c]), T(0)};
    } else if (nyq_y || 2 * z == N2) {
      cx<T> o[6];
      T re[6], im[6], ro[6], io[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        re[c] = t[c].x;
        im[c] = t[c].y;
      }
      cubic_mul(ci_d, ci_o, ci_s, re, ro);
      cubic_mul(ci_d, ci_o, ci_s, im, io);
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = {-inv_n * ro[c], -inv_n * io[c]};
#pragma unroll
      for (int c = 0; c < 6; ++c) t[c] = o[c];
    } else {
      const T fx = T(kxg) * T(a.inv_n0), fy = T(ky_s) * T(a.inv_n1), fz = T(kz_s) * T(a.inv_n2);
      const T in = T(1) / sqrt(fx * fx + fy * fy + fz * fz);
      apply_gamma(t, fx * in, fy * in, fz * in, c_mu, c_ratio);
#pragma unroll
      for (int c = 0; c < 6; ++c) t[c] = {inv_n * t[c].x, inv_n * t[c].y};
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) sh[(kx * 6 + c) * LS + z] = t[c];
  }
  __syncthreads();
  fft_stages<T, N2, 1, last_stage_ns(N2), true, W, LS, 256>(sh, a.tw);
  fft_tail<T, N2, W, true, LS, FFTEVP_FUSED_EDGE>(sh, a.tw, buf, zs);
}

// ---------------------------------------------------------------------------
// z pass of the local rotation of a compatible strain increment
// ---------------------------------------------------------------------------
// For a compatible mode e(xi) = sym(i xi (x) u), the antisymmetric part of
// i xi (x) u has the axial vector w = n x (e n), n = xi / |xi| (no frequency
// scale enters). Forward z-FFT of the six components, w into components
// 0..2 (zero elsewhere, and at xi = 0 and every Nyquist index, where the
// solver's strain is not a gradient), times a.inv_ntot, inverse z-FFT.
template <typename T, int N2, int TX>
__global__ __launch_bounds__(256, FFTEVP_SPEC_WAVES) void k_zspin(ZArgs<T> a) {
  constexpr int LS = N2 + 1;
  constexpr int W = 6 * TX;
  __shared__ cx<T> sh[W * LS];
  int bx, by;
  xcd_tile(bx, by);
  const int H = a.h, n1 = a.n1;
  const int ky = by, kx0 = bx * TX;
  const size_t zs = (size_t)n1 * H * 6;
  cx<T>* __restrict__ buf = a.buf + ((size_t)ky * H + kx0) * 6;
  fft_head<T, N2, W, false, LS, FFTEVP_FUSED_EDGE>(buf, zs, sh, a.tw);
  fft_stages<T, N2, last_stage_ns(N2), N2, false, W, LS, 256>(sh, a.tw);
  const T scale = T(a.inv_ntot), h = T(kIR2);
  const int ky_s = ky < n1 / 2 ? ky : ky - n1;
  const bool nyq_y = (2 * ky == n1);
  for (int idx = threadIdx.x; idx < N2 * TX; idx += 256) {
    const int z = idx / TX, kx = idx - (idx / TX) * TX;
    const int kz_s = z < N2 / 2 ? z : z - N2;
    const int kxg = kx0 + kx;
    cx<T> w[3] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
    if (!(kxg == 0 && ky == 0 && z == 0) && !nyq_y && 2 * z != N2) {
      cx<T> t[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) t[c] = sh[(kx * 6 + c) * LS + z];
      const T fx = T(kxg) * T(a.inv_n0), fy = T(ky_s) * T(a.inv_n1), fz = T(kz_s) * T(a.inv_n2);
      const T in = T(1) / sqrt(fx * fx + fy * fy + fz * fz);
      const T nx = fx * in, ny = fy * in, nz = fz * in;
      // v = e n (Mandel: e23 = h t3, e13 = h t4, e12 = h t5)
      const cx<T> v0 = {t[0].x * nx + h * (t[5].x * ny + t[4].x * nz), t[0].y * nx + h * (t[5].y * ny + t[4].y * nz)};
      const cx<T> v1 = {h * t[5].x * nx + t[1].x * ny + h * t[3].x * nz, h * t[5].y * nx + t[1].y * ny + h * t[3].y * nz};
      const cx<T> v2 = {h * (t[4].x * nx + t[3].x * ny) + t[2].x * nz, h * (t[4].y * nx + t[3].y * ny) + t[2].y * nz};
      w[0] = {scale * (ny * v2.x - nz * v1.x), scale * (ny * v2.y - nz * v1.y)};
      w[1] = {scale * (nz * v0.x - nx * v2.x), scale * (nz * v0.y - nx * v2.y)};
      w[2] = {scale * (nx * v1.x - ny * v0.x), scale * (nx * v1.y - ny * v0.y)};
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[(kx * 6 + c) * LS + z] = w[c];
#pragma unroll
    for (int c = 3; c < 6; ++c) sh[(kx * 6 + c) * LS + z] = {T(0), T(0)};
  }
  __syncthreads();
  fft_stages<T, N2, 1, last_stage_ns(N2), true, W, LS, 256>(sh, a.tw);
  fft_tail<T, N2, W, true, LS, FFTEVP_FUSED_EDGE>(sh, a.tw, buf, zs);
}

template <typename T>
__global__ __launch_bounds__(256) void k_cadd(const cx<T>* a, const cx<T>* b, cx<T>* out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const cx<T> x = a[i], y = b[i];
    out[i] = {x.x + y.x, x.y + y.y};
  }
}

// ---------------------------------------------------------------------------
// stop test and mixed-BC update from the reduced sums (one thread)
// ---------------------------------------------------------------------------
__device__ void finalize_sums(const FinArgs& a, Ctl* ctl, const double (&tot)[NPART]) {
  const double iv = 1.0 / a.nvox;
  double Sig[6], nE = 0.0, nS = 0.0, nbc = 0.0, dS[6];
  for (int k = 0; k < 6; ++k) {
    Sig[k] = tot[1 + k] * iv;
    nE += ctl->E[k] * ctl->E[k];
    nS += Sig[k] * Sig[k];
    dS[k] = a.strain_ctrl[k] ? 0.0 : (a.sig_star[k] - Sig[k]);
    nbc += dS[k] * dS[k];
  }
  const double err_c = sqrt(tot[0] * iv) / (a.enorm > 0.0 ? a.enorm : sqrt(nE));
  const double err_bc = a.sscale > 0.0 ? sqrt(nbc) / a.sscale
                                       : (nS > 0.0 ? sqrt(nbc / nS) : (nbc == 0.0 ? 0.0 : INFINITY));
  for (int k = 0; k < 6; ++k) ctl->Sigma[k] = Sig[k];
  ctl->err_c = err_c;
  ctl->err_bc = err_bc;
  ctl->nfail = tot[7];
  ctl->nsum = tot[8];
  ctl->lssum = tot[9];
  ctl->nmax = tot[10];
  ctl->iters += 1;
  if (!isfinite(err_c) || isnan(err_bc) || !isfinite(nS)) {
    ctl->done = 2;
  } else if (err_c < a.tol && err_bc < a.tol) {
    ctl->done = 1;
  } else {
    for (int i = 0; i < 6; ++i) {
      if (a.strain_ctrl[i]) continue;
      double s = 0.0;
      for (int j = 0; j < 6; ++j) s += a.css[6 * i + j] * dS[j];
      ctl->E[i] += s;
    }
  }
}

// ---------------------------------------------------------------------------
// end-of-increment state update (FP64 arithmetic in both precisions)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_state(StateArgs<T> a) {
  const size_t V = a.nvox;
  double part[2] = {0.0, 0.0};
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    double R[9], s[6], sc[6];
    quat_rot<double>(a.quat[g], a.quat[V + g], a.quat[2 * V + g], a.quat[3 * V + g], R);
    for (int k = 0; k < 6; ++k) s[k] = a.sig[k * V + g];
    to_crystal(R, s, sc);
    const double rho = a.rho[g];
    const double tauc = a.m.tau0 + a.m.taylor * sqrt(rho);
    double w[12], gk[6], visc, asum;
    if (a.m.n_int > 0) flow_eval<true>(sc, 1.0 / tauc, a.m.n, a.m.n_int, w, gk, visc, asum);
    else flow_eval<false>(sc, 1.0 / tauc, a.m.n, a.m.n_int, w, gk, visc, asum);
    double dpc[6], dp[6];
    for (int k = 0; k < 6; ++k) dpc[k] = a.gdot0 * (k < 3 ? kUN : kUS) * gk[k];
    to_sample(R, dpc, dp);
    for (int k = 0; k < 6; ++k) {
      a.epsp[k * V + g] = (T)((double)a.epsp[k * V + g] + a.dt * dp[k]);
      const double dek = a.de ? (double)a.de[k * V + g] : a.dEu[k];
      a.q[k * V + g] = (T)((double)a.q[k * V + g] + dek - a.dt * dp[k]);
    }
    const double rn = a.dens ? rho + a.dt * (a.k1 * sqrt(rho) - a.k2 * rho) * a.gdot0 * asum : rho;
    if (a.dens) a.rho[g] = (T)rn;
    if (a.gd) {
      // the increment's slip rates for the GND update: gdot0 |x|^(n-1) x
      const double itauc = 1.0 / tauc;
      static_for<0, 12>([&](auto ac) {
        constexpr int A = decltype(ac)::value;
        a.gd[(size_t)A * V + g] = (T)(a.gdot0 * w[A] * (resolved<A>(sc) * itauc));
      });
    }
    part[0] += (double)(T)rn;
    part[1] += a.gdot0 * asum;
  }
  block_reduce<2, 0>(part, a.partial + (size_t)blockIdx.x * 2);
}

// Slip rates gdot_a = gdot0 |tau_a / tauc|^n sign(tau_a) of the 12 systems at
// a stress field (crystal-frame resolved shears), FP64 out, [12][V].
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_gdot(const T* __restrict__ sig, const T* __restrict__ quat,
                                              const T* __restrict__ rho, TO* __restrict__ out,
                                              size_t V, Mat m, double gdot0) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    double R[9], s[6], sc[6];
    quat_rot<double>(quat[g], quat[V + g], quat[2 * V + g], quat[3 * V + g], R);
    for (int k = 0; k < 6; ++k) s[k] = sig[k * V + g];
    to_crystal(R, s, sc);
    const double itauc = 1.0 / (m.tau0 + m.taylor * sqrt((double)rho[g]));
    static_for<0, 12>([&](auto ac) {
      constexpr int A = decltype(ac)::value;
      const double x = resolved<A>(sc) * itauc;
      const double ax = fabs(x);
      double p;
      if (m.n_int > 0) {
        double b = ax;
        p = 1.0;
        for (int e = m.n_int; e != 0; e >>= 1) {
          if (e & 1) p *= b;
          b *= b;
        }
      } else {
        p = ax > 0.0 ? exp(m.n * log(ax)) : 0.0;
      }
      out[(size_t)A * V + g] = (TO)(x < 0.0 ? -gdot0 * p : gdot0 * p);
    });
  }
}

// Crystal-frame slip plane normals and directions of the 12 systems (the
// same list as the Schmid sign table: unnormalised integer vectors, |n| =
// sqrt3, |d| = sqrt2), and the check that sym(d x n) reproduces the table.
constexpr int kN[12][3] = {{1, 1, 1},  {1, 1, 1},  {1, 1, 1},  {-1, 1, 1}, {-1, 1, 1}, {-1, 1, 1},
                           {1, -1, 1}, {1, -1, 1}, {1, -1, 1}, {1, 1, -1}, {1, 1, -1}, {1, 1, -1}};
constexpr int kD[12][3] = {{0, 1, -1}, {1, 0, -1}, {1, -1, 0}, {0, 1, -1}, {1, 0, 1}, {1, 1, 0},
                           {0, 1, 1},  {1, 0, -1}, {1, 1, 0},  {0, 1, 1},  {1, 0, 1}, {1, -1, 0}};
__host__ __device__ constexpr bool nd_match_sign_table() {
  const int pi[3] = {1, 0, 0}, pj[3] = {2, 2, 1};  // Mandel shear slots 23, 13, 12
  for (int a = 0; a < 12; ++a) {
    for (int i = 0; i < 3; ++i)
      if (kD[a][i] * kN[a][i] != kSign[a][i]) return false;
    for (int k = 0; k < 3; ++k)
      if (kD[a][pi[k]] * kN[a][pj[k]] + kD[a][pj[k]] * kN[a][pi[k]] != kSign[a][3 + k]) return false;
    if (kN[a][0] * kD[a][0] + kN[a][1] * kD[a][1] + kN[a][2] * kD[a][2] != 0) return false;
  }
  return true;
}
static_assert(nd_match_sign_table(), "slip normals/directions disagree with the Schmid sign table");
// t = n x d in integers (|t| = sqrt6)
struct IntVec12 {
  int v[12][3];
};
__host__ __device__ constexpr IntVec12 cross_nd() {
  IntVec12 r{};
  for (int a = 0; a < 12; ++a) {
    r.v[a][0] = kN[a][1] * kD[a][2] - kN[a][2] * kD[a][1];
    r.v[a][1] = kN[a][2] * kD[a][0] - kN[a][0] * kD[a][2];
    r.v[a][2] = kN[a][0] * kD[a][1] - kN[a][1] * kD[a][0];
  }
  return r;
}
constexpr IntVec12 kTv = cross_nd();
#define kT kTv.v

// GND densities (Sec. 2.2, Eq. 7-8): per system, rates -(1/b) grad(gdot).t
// (screw) and (1/b) grad(gdot).d (edge), t = n x d, rotated to the sample
// frame; the gradient is a finite difference with spacing l_eff, central
// where both neighbours along an axis share the voxel's grain, one-sided
// towards the one that does, zero if neither does; periodic grid. One
// thread per voxel; workgroups renumbered so each XCD takes a contiguous
// range of voxels (neighbours along y and z then share its L2).
#ifndef FFTEVP_GND_GROUP
#define FFTEVP_GND_GROUP 3
#endif
constexpr int GND_GROUP = FFTEVP_GND_GROUP;
static_assert(12 % GND_GROUP == 0, "GND system groups must divide 12");

// Density rates of system al from the sample-frame gradient D of its slip
// rate: (R v) . D = v . (R^T D) for the integer crystal-frame vectors d
// (|d| = sqrt2) and t = n x d (|t| = sqrt6).
template <typename T>
__device__ __forceinline__ void gnd_system(int al, const double (&D)[3], const double (&R)[9], double cs_t,
                                           double cs_d, T rv, T ev, T* rs_out, T* ret_out) {
  double u[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) u[j] = R[j] * D[0] + R[3 + j] * D[1] + R[6 + j] * D[2];
  double gd_ = 0.0, gt = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (kD[al][j] > 0) gd_ += u[j];
    else if (kD[al][j] < 0) gd_ -= u[j];
    if (kT[al][j] != 0) gt += kT[al][j] * u[j];
  }
  *rs_out = (T)((double)rv - cs_t * gt);
  *ret_out = (T)((double)ev + cs_d * gd_);
}

// stencil weights along one axis: D = wp f(+) + wc f(0) + wm f(-)
__device__ __forceinline__ void gnd_weights(bool p, bool m, double& wp, double& wc, double& wm) {
  wp = p ? (m ? 0.5 : 1.0) : 0.0;
  wm = m ? (p ? -0.5 : -1.0) : 0.0;
  wc = (p && !m) ? -1.0 : ((m && !p) ? 1.0 : 0.0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gnd(GndArgs<T> a) {
  const int nb = gridDim.x;
  int b = blockIdx.x;
  if (FFTEVP_XCD_REMAP && nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
  const size_t g = (size_t)b * 256 + threadIdx.x;
  if (g >= a.V) return;
  const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
  const int x = (int)(g % n0), y = (int)((g / n0) % n1), z = (int)(g / ((size_t)n0 * n1));
  // neighbour offsets and stencil weights per axis: D = wp f(+) + wc f(0) + wm f(-)
  const size_t sx = 1, sy = (size_t)n0, sz = (size_t)n0 * n1;
  const size_t gp[3] = {x + 1 < n0 ? g + sx : g + sx - (size_t)n0 * sx,
                        y + 1 < n1 ? g + sy : g + sy - (size_t)n1 * sy,
                        z + 1 < n2 ? g + sz : g + sz - (size_t)n2 * sz};
  const size_t gm[3] = {x > 0 ? g - sx : g - sx + (size_t)n0 * sx, y > 0 ? g - sy : g - sy + (size_t)n1 * sy,
                        z > 0 ? g - sz : g - sz + (size_t)n2 * sz};
  const T* __restrict__ gdv = a.gd;
  T* __restrict__ rsv = a.rs;
  T* __restrict__ retv = a.ret;
  const int me = a.grain[g];
  double wp[3], wc[3], wm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gnd_weights(a.grain[gp[k]] == me, a.grain[gm[k]] == me, wp[k], wc[k], wm[k]);
  double R[9];
  quat_rot<double>(a.quat[g], a.quat[a.V + g], a.quat[2 * a.V + g], a.quat[3 * a.V + g], R);
  const double cs = a.dt * a.inv_b * a.inv_h;
  const double cs_d = cs * kIR2, cs_t = cs * 0.40824829046386301637;  // 1/sqrt2, 1/sqrt6
  // systems in groups: every load of a group is issued before its arithmetic
  // and stores, so the latencies overlap
#pragma unroll
  for (int grp = 0; grp < 12 / GND_GROUP; ++grp) {
    T fv[GND_GROUP][7], rv[GND_GROUP], ev[GND_GROUP];
#pragma unroll
    for (int q = 0; q < GND_GROUP; ++q) {
      const T* __restrict__ f = gdv + (size_t)(GND_GROUP * grp + q) * a.V;
      fv[q][0] = f[g];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        fv[q][1 + k] = f[gp[k]];
        fv[q][4 + k] = f[gm[k]];
      }
      rv[q] = rsv[(size_t)(GND_GROUP * grp + q) * a.V + g];
      ev[q] = retv[(size_t)(GND_GROUP * grp + q) * a.V + g];
    }
#pragma unroll
    for (int q = 0; q < GND_GROUP; ++q) {
      const int al = GND_GROUP * grp + q;
      double D[3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        D[k] = wp[k] * (double)fv[q][1 + k] + wc[k] * (double)fv[q][0] + wm[k] * (double)fv[q][4 + k];
      gnd_system<T>(al, D, R, cs_t, cs_d, rv[q], ev[q], rsv + (size_t)al * a.V + g, retv + (size_t)al * a.V + g);
    }
  }
}

// The same update marching along z: block (tile, chunk) takes 256
// consecutive voxels of an xy-plane and walks ZC planes. The slip rates of
// planes z-1, z and z+1 at its voxels stay in registers, so each plane of
// slip rates is fetched once per chunk (plus two planes of halo) instead of
// three times; the x and y neighbours are read while the neighbouring
// threads, and the blocks of the neighbouring tiles running on the same XCD,
// read them as their own. Needs n0 n1 a multiple of 256 and n2 of ZC.
#ifndef FFTEVP_GND_MARCH
#define FFTEVP_GND_MARCH 1
#endif
#ifndef FFTEVP_GND_WAVES
#define FFTEVP_GND_WAVES 1
#endif
template <typename T, int ZC>
__global__ __launch_bounds__(256, FFTEVP_GND_WAVES) void k_gnd_z(GndArgs<T> a) {
  const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
  const size_t P = (size_t)n0 * n1, V = a.V;
  const int ntile = (int)(P / 256), nb = gridDim.x;
  int b = blockIdx.x;
  if (FFTEVP_XCD_REMAP && nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
  const int tile = b % ntile, z0 = (b / ntile) * ZC;
  const size_t p = (size_t)tile * 256 + threadIdx.x;
  const int x = (int)(p % n0), y = (int)(p / n0);
  const size_t pxp = x + 1 < n0 ? p + 1 : p + 1 - n0, pxm = x > 0 ? p - 1 : p - 1 + n0;
  const size_t pyp = y + 1 < n1 ? p + n0 : p + n0 - P, pym = y > 0 ? p - n0 : p - n0 + P;
  const T* __restrict__ gdv = a.gd;
  T* __restrict__ rsv = a.rs;
  T* __restrict__ retv = a.ret;
  const size_t zm = (size_t)(z0 > 0 ? z0 - 1 : n2 - 1) * P, zc0 = (size_t)z0 * P;
  T f[12][3];  // slip rates of this column at z-1, z, z+1
  int gz[3];   // grain ids at z-1, z, z+1
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    f[al][0] = gdv[(size_t)al * V + zm + p];
    f[al][1] = gdv[(size_t)al * V + zc0 + p];
  }
  gz[0] = a.grain[zm + p];
  gz[1] = a.grain[zc0 + p];
  const double cs = a.dt * a.inv_b * a.inv_h;
  const double cs_d = cs * kIR2, cs_t = cs * 0.40824829046386301637;  // 1/sqrt2, 1/sqrt6
#pragma unroll
  for (int st = 0; st < ZC; ++st) {
    const int z = z0 + st;
    const size_t bz = (size_t)z * P, bp = (size_t)(z + 1 < n2 ? z + 1 : 0) * P;
    const size_t g = bz + p;
#pragma unroll
    for (int al = 0; al < 12; ++al) f[al][2] = gdv[(size_t)al * V + bp + p];
    gz[2] = a.grain[bp + p];
    const int me = gz[1];
    double wp[3], wc[3], wm[3];
    gnd_weights(a.grain[bz + pxp] == me, a.grain[bz + pxm] == me, wp[0], wc[0], wm[0]);
    gnd_weights(a.grain[bz + pyp] == me, a.grain[bz + pym] == me, wp[1], wc[1], wm[1]);
    gnd_weights(gz[2] == me, gz[0] == me, wp[2], wc[2], wm[2]);
    double R[9];
    quat_rot<double>(a.quat[g], a.quat[V + g], a.quat[2 * V + g], a.quat[3 * V + g], R);
#pragma unroll
    for (int grp = 0; grp < 12 / GND_GROUP; ++grp) {
      T nv[GND_GROUP][4], rv[GND_GROUP], ev[GND_GROUP];  // x+, y+, x-, y- neighbours
#pragma unroll
      for (int q = 0; q < GND_GROUP; ++q) {
        const T* __restrict__ fa = gdv + (size_t)(GND_GROUP * grp + q) * V + bz;
        nv[q][0] = fa[pxp];
        nv[q][1] = fa[pyp];
        nv[q][2] = fa[pxm];
        nv[q][3] = fa[pym];
        rv[q] = rsv[(size_t)(GND_GROUP * grp + q) * V + g];
        ev[q] = retv[(size_t)(GND_GROUP * grp + q) * V + g];
      }
#pragma unroll
      for (int q = 0; q < GND_GROUP; ++q) {
        const int al = GND_GROUP * grp + q;
        const double c = (double)f[al][1];
        double D[3];
        D[0] = wp[0] * (double)nv[q][0] + wc[0] * c + wm[0] * (double)nv[q][2];
        D[1] = wp[1] * (double)nv[q][1] + wc[1] * c + wm[1] * (double)nv[q][3];
        D[2] = wp[2] * (double)f[al][2] + wc[2] * c + wm[2] * (double)f[al][0];
        gnd_system<T>(al, D, R, cs_t, cs_d, rv[q], ev[q], rsv + (size_t)al * V + g, retv + (size_t)al * V + g);
      }
    }
#pragma unroll
    for (int al = 0; al < 12; ++al) {
      f[al][0] = f[al][1];
      f[al][1] = f[al][2];
    }
    gz[0] = gz[1];
    gz[1] = gz[2];
  }
}

// Lattice rotation after an increment (reading of Sec. 2.5): the lattice spins
// with minus the plastic spin, Omega_e = -sum_a gdot_a skew(d_a (x) n_a) (no
// imposed spin), whose axial vector is -1/2 sum_a gdot_a R t_a with the unit
// sense vector t = n x d = (integer n x integer d) / sqrt6; the orientation
// turns by exp(dt Omega_e): q <- (cos(|th|/2), sin(|th|/2) th/|th|) q with
// th = dt times that axial vector, renormalised, w >= 0.
template <typename T>
__global__ __launch_bounds__(256) void k_rotate(T* __restrict__ quat, const T* __restrict__ gd,
                                                const double* __restrict__ spin, size_t V, double dt) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    const double q0 = quat[g], q1 = quat[V + g], q2 = quat[2 * V + g], q3 = quat[3 * V + g];
    double u[3] = {0.0, 0.0, 0.0};  // sum_a gdot_a (integer n x d), crystal frame
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      const double r = gd[(size_t)a * V + g];
#pragma unroll
      for (int j = 0; j < 3; ++j) u[j] += r * (double)kT[a][j];
    }
    double R[9];
    quat_rot<double>(q0, q1, q2, q3, R);
    const double c = -0.5 * dt * 0.40824829046386301637;  // -dt / (2 sqrt6)
    double th[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) th[i] = c * (R[3 * i] * u[0] + R[3 * i + 1] * u[1] + R[3 * i + 2] * u[2]);
    // plus the local rotation of the increment (axial vector, sample frame)
    if (spin) {
#pragma unroll
      for (int i = 0; i < 3; ++i) th[i] += spin[(size_t)i * V + g];
    }
    const double ang = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    double a0 = 1.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (ang > 0.0) {
      const double sh = sin(0.5 * ang) / ang;
      a0 = cos(0.5 * ang);
      a1 = sh * th[0];
      a2 = sh * th[1];
      a3 = sh * th[2];
    }
    // Hamilton product (a0, a) (q0, q)
    double w = a0 * q0 - a1 * q1 - a2 * q2 - a3 * q3;
    double x = a0 * q1 + a1 * q0 + a2 * q3 - a3 * q2;
    double y = a0 * q2 - a1 * q3 + a2 * q0 + a3 * q1;
    double z = a0 * q3 + a1 * q2 - a2 * q1 + a3 * q0;
    const double inv = (w < 0.0 ? -1.0 : 1.0) / sqrt(w * w + x * x + y * y + z * z);
    quat[g] = (T)(w * inv);
    quat[V + g] = (T)(x * inv);
    quat[2 * V + g] = (T)(y * inv);
    quat[3 * V + g] = (T)(z * inv);
  }
}

// ---------------------------------------------------------------------------
// the paper's dislocation-based law (Sec. 2.2, Eq. 3-6)
// ---------------------------------------------------------------------------
// |cos| and |sin| of the angles (n_a, t_b) and (n_a, d_b) from the integer
// vectors: |n.t| = k / sqrt18 (k <= 4), |n.d| = k / sqrt6 (k <= 2).
struct ProjTab {
  double cnt[12][12], snt[12][12], cnd[12][12], snd[12][12];
};
__host__ __device__ constexpr ProjTab make_proj_tab() {
  // k / sqrt18 and sqrt(18 - k^2) / sqrt18, k = 0..4
  const double c18[5] = {0.0, 0.23570226039551584147, 0.47140452079103168293, 0.70710678118654752440,
                         0.94280904158206336587};
  const double s18[5] = {1.0, 0.97182531580755005857, 0.88191710368819698821, 0.70710678118654752440,
                         0.33333333333333333333};
  // k / sqrt6 and sqrt(6 - k^2) / sqrt6, k = 0..2
  const double c6[3] = {0.0, 0.40824829046386301637, 0.81649658092772603273};
  const double s6[3] = {1.0, 0.91287092917527685576, 0.57735026918962576451};
  ProjTab t{};
  for (int a = 0; a < 12; ++a)
    for (int b = 0; b < 12; ++b) {
      int nt = kN[a][0] * kT[b][0] + kN[a][1] * kT[b][1] + kN[a][2] * kT[b][2];
      int nd = kN[a][0] * kD[b][0] + kN[a][1] * kD[b][1] + kN[a][2] * kD[b][2];
      nt = nt < 0 ? -nt : nt;
      nd = nd < 0 ? -nd : nd;
      t.cnt[a][b] = c18[nt];
      t.snt[a][b] = s18[nt];
      t.cnd[a][b] = c6[nd];
      t.snd[a][b] = s6[nd];
    }
  return t;
}
__device__ constexpr ProjTab kProj = make_proj_tab();

// forest and parallel densities (Eq. 4-5) of the 12 systems of voxel g
template <typename T>
__device__ __forceinline__ void mr_projections(const T* __restrict__ ssd, const T* __restrict__ gs,
                                               const T* __restrict__ ge, size_t V, size_t g, double (&F)[12],
                                               double (&P)[12]) {
  double r[12], rs[12], re[12];
#pragma unroll
  for (int b = 0; b < 12; ++b) {
    r[b] = ssd[(size_t)b * V + g];
    rs[b] = gs ? fabs((double)gs[(size_t)b * V + g]) : 0.0;
    re[b] = ge ? fabs((double)ge[(size_t)b * V + g]) : 0.0;
  }
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    double f = 0.0, p = 0.0;
#pragma unroll
    for (int b = 0; b < 12; ++b) {
      f += (r[b] + re[b]) * kProj.cnt[a][b] + rs[b] * kProj.cnd[a][b];
      p += (r[b] + re[b]) * kProj.snt[a][b] + rs[b] * kProj.snd[a][b];
    }
    F[a] = f;
    P[a] = p;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mr_params(const T* __restrict__ ssd, const T* __restrict__ gs,
                                                   const T* __restrict__ ge, T* __restrict__ sysp, size_t V,
                                                   MrConst c) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    double F[12], P[12];
    mr_projections(ssd, gs, ge, V, g, F, P);
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      const double sp = sqrt(P[a]), tc = c.tc_c * sqrt(F[a]), amp = c.a_c * sp;
      sysp[(size_t)a * V + g] = (T)(c.tp_c * sp);
      sysp[(size_t)(12 + a) * V + g] = (T)(1.0 / tc);
      sysp[(size_t)(24 + a) * V + g] = (T)amp;
    }
  }
}

// slip rate of system a at resolved shear tau (FP64)
template <typename T>
__device__ __forceinline__ double mr_rate(const SysParams<T>& sp, int a, double tau) {
  const double xx = (fabs(tau) - (double)sp.tp(a)) * (double)sp.itc(a);
  if (!(xx > 0.0)) return 0.0;
  const double ex = exp(xx);
  const double r = (double)sp.amp(a) * 0.5 * (ex - 1.0 / ex);
  return tau < 0.0 ? -r : r;
}

// end of an increment with the paper's law: slip rates at the converged
// stress (parameters of the increment's start), plastic strain, SSD
// densities (Eq. 6, explicit), their sum as the voxel density
template <typename T>
__global__ __launch_bounds__(256) void k_state_mr(StateArgs<T> a) {
  const size_t V = a.nvox;
  double part[2] = {0.0, 0.0};
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    double R[9], s[6], sc[6];
    quat_rot<double>(a.quat[g], a.quat[V + g], a.quat[2 * V + g], a.quat[3 * V + g], R);
    for (int k = 0; k < 6; ++k) s[k] = a.sig[k * V + g];
    to_crystal(R, s, sc);
    const SysParams<T> sp{a.sysp, V, g};
    double tau[12], gd[12], gk[6] = {0, 0, 0, 0, 0, 0}, gsum = 0.0;
    static_for<0, 12>([&](auto ac) {
      constexpr int A = decltype(ac)::value;
      tau[A] = resolved<A>(sc);
      gd[A] = mr_rate(sp, A, tau[A]);
      gsum += fabs(gd[A]);
      static_for<0, 6>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        acc_sign<kSign[A][K]>(gk[K], gd[A]);
      });
    });
    double dpc[6], dp[6], ep2 = 0.0;
    for (int k = 0; k < 6; ++k) {
      dpc[k] = (k < 3 ? kUN : kUS) * gk[k];
      ep2 += dpc[k] * dpc[k];
    }
    to_sample(R, dpc, dp);
    for (int k = 0; k < 6; ++k) {
      a.epsp[k * V + g] = (T)((double)a.epsp[k * V + g] + a.dt * dp[k]);
      const double dek = a.de ? (double)a.de[k * V + g] : a.dEu[k];
      a.q[k * V + g] = (T)((double)a.q[k * V + g] + dek - a.dt * dp[k]);
    }
    // von Mises stress and equivalent plastic rate (frame invariant)
    const double tr = (sc[0] + sc[1] + sc[2]) / 3.0;
    double s2 = 0.0;
    for (int k = 0; k < 6; ++k) {
      const double dv = sc[k] - (k < 3 ? tr : 0.0);
      s2 += dv * dv;
    }
    const double svm = sqrt(1.5 * s2), gvm = sqrt(2.0 / 3.0 * ep2);
    const double climb_f = a.mr.climb_c * svm * (gvm > 0.0 ? pow(gvm, a.mr.c8) : 0.0);
    double F[12], P[12];
    mr_projections(a.ssd, a.gnds, a.gndet, V, g, F, P);
    double tot = 0.0;
#pragma unroll
    for (int al = 0; al < 12; ++al) {
      const double rho = a.ssd[(size_t)al * V + g];
      const double ag = fabs(gd[al]);
      const double rhom = a.mr.rhom_c * sqrt(P[al] * F[al]);
      const double ddip = ag > 0.0 ? a.mr.dd_c / fabs(tau[al]) : 0.0;
      const double rate = a.mr.c4 * sqrt(F[al]) * ag + a.mr.c6 * ddip * rhom * ag - a.mr.c5 * rho * ag -
                          climb_f * rho * rho;
      const double rn = a.dens ? rho + a.dt * rate : rho;
      if (a.dens) a.ssd[(size_t)al * V + g] = (T)rn;
      tot += (double)(T)rn;
      if (a.gd) a.gd[(size_t)al * V + g] = (T)gd[al];
    }
    if (a.dens) a.rho[g] = (T)tot;
    part[0] += (double)(T)tot;
    part[1] += gsum;
  }
  block_reduce<2, 0>(part, a.partial + (size_t)blockIdx.x * 2);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gdot_mr(const T* __restrict__ sig, const T* __restrict__ quat,
                                                 const T* __restrict__ sysp, double* __restrict__ out, size_t V) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    double R[9], s[6], sc[6];
    quat_rot<double>(quat[g], quat[V + g], quat[2 * V + g], quat[3 * V + g], R);
    for (int k = 0; k < 6; ++k) s[k] = sig[k * V + g];
    to_crystal(R, s, sc);
    const SysParams<T> sp{sysp, V, g};
    static_for<0, 12>([&](auto ac) {
      constexpr int A = decltype(ac)::value;
      out[(size_t)A * V + g] = mr_rate(sp, A, resolved<A>(sc));
    });
  }
}

// ---------------------------------------------------------------------------
// DRX nucleation (Sec. 2.3, 2.5)
// ---------------------------------------------------------------------------
// nucleation strength kappa = kc (-ln(1 - u))^(1/q) (inverse of the Weibull
// law of Eq. 9-10); counts the uniforms outside [0, 1)
template <typename T>
__global__ __launch_bounds__(256) void k_kappa(const double* __restrict__ u, T* __restrict__ kappa, size_t V,
                                               double kc, double iq, double* partial) {
  double bad[2] = {0.0, 0.0};
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    const double x = u[g];
    if (!(x >= 0.0 && x < 1.0)) {
      bad[0] += 1.0;
      continue;
    }
    if (kappa) kappa[g] = (T)(kc * pow(-log1p(-x), iq));
  }
  block_reduce<2, 0>(bad, partial + (size_t)blockIdx.x * 2);
}

// Total dislocation density of voxel g (Eq. 11): per-system SSD + GND (sqrt
// of screw^2 + edge^2) + mobile for the paper's law; the voxel density + GND
// for the power law.
template <typename T, bool MRLAW>
__device__ __forceinline__ double drx_total_density(const DrxArgs<T>& a, size_t g) {
  const size_t V = a.V;
  double k = 0.0;
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    const double gs = a.gs[(size_t)al * V + g], ge = a.ge[(size_t)al * V + g];
    k += sqrt(gs * gs + ge * ge);
  }
  if constexpr (MRLAW) {
    double F[12], P[12];
    mr_projections(a.ssd, a.gs, a.ge, V, g, F, P);
#pragma unroll
    for (int al = 0; al < 12; ++al) k += (double)a.ssd[(size_t)al * V + g] + a.rhom_c * sqrt(P[al] * F[al]);
  } else {
    k += (double)a.rho[g];
  }
  return k;
}

// One nucleation test on the state after an increment: a voxel with a face
// neighbour of another grain nucleates when its total dislocation density
// exceeds its strength. A nucleus becomes a single-voxel grain (id
// -(index + 1)), keeps s_soften of its GND densities (Eq. 16) and draws a new
// strength with s_nucl kc. Grain ids are read from one buffer and written to
// another.
template <typename T, bool MRLAW>
__global__ __launch_bounds__(256) void k_drx(DrxArgs<T> a) {
  const size_t V = a.V;
  double cnt[2] = {0.0, 0.0};
  const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    const int x = (int)(g % n0), y = (int)((g / n0) % n1), z = (int)(g / ((size_t)n0 * n1));
    const size_t sy = (size_t)n0, sz = (size_t)n0 * n1;
    const int me = a.grain[g];
    const size_t nb[6] = {x + 1 < n0 ? g + 1 : g + 1 - n0, x > 0 ? g - 1 : g - 1 + n0,
                          y + 1 < n1 ? g + sy : g + sy - (size_t)n1 * sy, y > 0 ? g - sy : g - sy + (size_t)n1 * sy,
                          z + 1 < n2 ? g + sz : g + sz - (size_t)n2 * sz, z > 0 ? g - sz : g - sz + (size_t)n2 * sz};
    bool site = false;
#pragma unroll
    for (int k = 0; k < 6; ++k) site |= a.grain[nb[k]] != me;
    int out = me;
    if (site) {
      const double k = drx_total_density<T, MRLAW>(a, g);
      if (k > (double)a.kappa[g]) {
        out = -(int)(g + 1);
        cnt[0] += 1.0;
#pragma unroll
        for (int al = 0; al < 12; ++al) {
          a.gs[(size_t)al * V + g] = (T)(a.s_soften * (double)a.gs[(size_t)al * V + g]);
          a.ge[(size_t)al * V + g] = (T)(a.s_soften * (double)a.ge[(size_t)al * V + g]);
        }
        a.kappa[g] = (T)(a.kc_new * pow(-log1p(-a.u[g]), a.iq));
      }
    }
    a.grain_out[g] = out;
  }
  block_reduce<2, 0>(cnt, a.partial + (size_t)blockIdx.x * 2);
}

// scale x total dislocation density of every voxel (the stored energy
// E_store = rho_tot zeta mu b^2 of Eq. 14, in the units the scale gives)
template <typename T, bool MRLAW>
__global__ __launch_bounds__(256) void k_rho_tot(DrxArgs<T> a, double scale, double* __restrict__ out) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < a.V; g += (size_t)gridDim.x * 256)
    out[g] = scale * drx_total_density<T, MRLAW>(a, g);
}

// After grain growth: voxels whose grain changed are counted; those now in a
// recrystallised grain (negative id) keep s_soften of their GND densities
// (Eq. 16, as material points of a new grain).
template <typename T>
__global__ __launch_bounds__(256) void k_sweep(DrxArgs<T> a) {
  const size_t V = a.V;
  double cnt[2] = {0.0, 0.0};
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    const int before = a.grain[g], after = a.grain_out[g];
    if (after != before) {
      cnt[0] += 1.0;
      if (after < 0) {
        cnt[1] += 1.0;
#pragma unroll
        for (int al = 0; al < 12; ++al) {
          a.gs[(size_t)al * V + g] = (T)(a.s_soften * (double)a.gs[(size_t)al * V + g]);
          a.ge[(size_t)al * V + g] = (T)(a.s_soften * (double)a.ge[(size_t)al * V + g]);
        }
      }
    }
  }
  block_reduce<2, 0>(cnt, a.partial + (size_t)blockIdx.x * 2);
}

template <typename T>
__global__ __launch_bounds__(256) void k_export_int(const int* __restrict__ src, double* __restrict__ dst, size_t V) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) dst[g] = src[g];
}

__global__ __launch_bounds__(256) void k_sum2(const double* __restrict__ p, int n, double* out) {
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += 256) {
    v[0] += p[2 * b];
    v[1] += p[2 * b + 1];
  }
  block_reduce<2, 0>(v, out);
}

// ---------------------------------------------------------------------------
// adjoint of one increment (reverse mode through the converged fixed point)
// ---------------------------------------------------------------------------
// Flow quantities at a stress, crystal frame, FP64: x_a, |x_a|^n, |x_a|^(n-1).
__device__ __forceinline__ void adj_flow(const AdjArgsBase& a, const double (&sc)[6], double itauc,
                                         double (&x)[12], double (&p)[12], double (&w)[12]) {
  static_for<0, 12>([&](auto ac) {
    constexpr int A = decltype(ac)::value;
    x[A] = resolved<A>(sc) * itauc;
  });
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const double ax = fabs(x[q]);
    double wq;
    if (a.n_int > 0) {
      wq = 1.0;
      double bq = ax;
      for (int e = a.n_int - 1; e != 0; e >>= 1) {
        if (e & 1) wq *= bq;
        bq *= bq;
      }
    } else {
      wq = ax > 0.0 ? exp((a.n - 1.0) * log(ax)) : (a.n == 1.0 ? 1.0 : 0.0);
    }
    w[q] = wq;
    p[q] = wq * ax;
  }
}

template <int A>
__device__ __forceinline__ void add_schmid(double (&v)[6], double c) {
  static_for<0, 6>([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    acc_sign<kSign[A][K]>(v[K], c * (K < 3 ? kUN : kUS));
  });
}

// eigenstrain of the adjoint linear problem:
//   eta = dt [ sum_a gdot'_a m_a (m_a : a_eps) + a_rho h sum_a sign(tau_a) gdot'_a m_a ]
template <typename T>
__global__ __launch_bounds__(256) void k_adj_setup(AdjArgs<T> a) {
  const size_t V = a.nvox;
  double part[1] = {0.0};
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    double R[9], s[6], sc[6], ae[6], aec[6];
    quat_rot<double>(a.quat[g], a.quat[V + g], a.quat[2 * V + g], a.quat[3 * V + g], R);
    for (int k = 0; k < 6; ++k) {
      s[k] = a.sig_t[k * V + g];
      ae[k] = a.a_eps[k * V + g];
    }
    to_crystal(R, s, sc);
    to_crystal(R, ae, aec);
    const double rho = a.rho0[g], sr = sqrt(rho);
    const double tauc = a.b.tau0 + a.b.taylor * sr;
    const double h = a.b.k1 * sr - a.b.k2 * rho;
    const double arho = a.a_rho[g];
    double x[12], p[12], w[12];
    adj_flow(a.b, sc, 1.0 / tauc, x, p, w);
    double ec[6] = {0, 0, 0, 0, 0, 0};
    const double gd1 = a.b.gdot0 * a.b.n / tauc;  // dgdot/dtau = gd1 |x|^(n-1)
    static_for<0, 12>([&](auto ac) {
      constexpr int A = decltype(ac)::value;
      const double ma = resolved<A>(aec);
      const double sg = x[A] < 0.0 ? -1.0 : (x[A] > 0.0 ? 1.0 : 0.0);
      add_schmid<A>(ec, a.b.dt * gd1 * w[A] * (ma + arho * h * sg));
    });
    double es[6];
    to_sample(R, ec, es);
    double n2 = 0.0;
    for (int k = 0; k < 6; ++k) {
      a.eta[k * V + g] = (T)(-es[k]);  // the tangent solve takes the offset q = -eta
      n2 += es[k] * es[k];
    }
    part[0] += n2;
  }
  block_reduce<1, 0>(part, a.partial + blockIdx.x);
}

// reverse update of the state adjoints and the parameter-gradient partials
template <typename T>
__global__ __launch_bounds__(256) void k_adj_update(AdjArgs<T> a) {
  const size_t V = a.nvox;
  double part[4] = {0.0, 0.0, 0.0, 0.0};  // d/d tau0, k1, k2, n
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    double R[9], s[6], sc[6], at[6], atc[6];
    quat_rot<double>(a.quat[g], a.quat[V + g], a.quat[2 * V + g], a.quat[3 * V + g], R);
    for (int k = 0; k < 6; ++k) {
      s[k] = a.sig_t[k * V + g];
      at[k] = (double)a.a_eps[k * V + g] + (double)a.z[k * V + g];
    }
    to_crystal(R, s, sc);
    to_crystal(R, at, atc);
    const double rho = a.rho0[g], sr = sqrt(rho);
    const double tauc = a.b.tau0 + a.b.taylor * sr;
    const double h = a.b.k1 * sr - a.b.k2 * rho;
    const double hp = a.b.k1 / (2.0 * sr) - a.b.k2;
    const double arho = a.a_rho[g];
    double x[12], p[12], w[12];
    adj_flow(a.b, sc, 1.0 / tauc, x, p, w);
    double A1 = 0.0, gam = 0.0, dn1 = 0.0, dn2 = 0.0;
    static_for<0, 12>([&](auto ac) {
      constexpr int A = decltype(ac)::value;
      const double gdot = a.b.gdot0 * (x[A] < 0.0 ? -p[A] : p[A]);
      const double ma = resolved<A>(atc);
      const double lx = p[A] > 0.0 ? log(fabs(x[A])) : 0.0;
      A1 += ma * gdot;
      gam += fabs(gdot);
      dn1 += ma * gdot * lx;
      dn2 += fabs(gdot) * lx;
    });
    const double dt = a.b.dt;
    const double atau = -dt * (a.b.n / tauc) * (A1 + arho * h * gam);
    part[0] += atau;
    part[1] += arho * dt * sr * gam;
    part[2] -= arho * dt * rho * gam;
    part[3] += dt * (dn1 + arho * h * dn2);
    a.a_rho[g] = (T)(arho * (1.0 + dt * hp * gam) + atau * a.b.taylor / (2.0 * sr));
    for (int k = 0; k < 6; ++k) a.a_eps[k * V + g] = (T)at[k];
  }
  block_reduce<4, 0>(part, a.partial + blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_sum_rows(const double* __restrict__ p, int n, int rows,
                                                  double* out) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += 256)
    for (int r = 0; r < rows; ++r) v[r] += p[(size_t)r * n + b];
  block_reduce<4, 0>(v, out);
}

template <typename T>
hipError_t launch_adj_setup(const AdjArgs<T>& a, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_setup<T>, dim3(nblocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, (const double*)a.partial, nblocks, 1, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_update(const AdjArgs<T>& a, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_update<T>, dim3(nblocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, (const double*)a.partial, nblocks, 4, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// set-up, validation and field export
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ingest(const double* __restrict__ q, const double* __restrict__ rho,
                                                T* __restrict__ qo, T* __restrict__ ro, size_t V,
                                                double* partial) {
  double bad[2] = {0.0, 0.0};
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    double c[4], n2 = 0.0;
    for (int k = 0; k < 4; ++k) {
      c[k] = q[k * V + g];
      n2 += c[k] * c[k];
    }
    const double nrm = sqrt(n2);
    if (!(fabs(nrm - 1.0) <= 1e-6)) bad[0] += 1.0;
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int k = 0; k < 4; ++k) qo[k * V + g] = (T)(c[k] * inv);
    const double r = rho[g];
    if (!(r > 0.0 && isfinite(r))) bad[1] += 1.0;
    ro[g] = (T)r;
  }
  block_reduce<2, 0>(bad, partial + (size_t)blockIdx.x * 2);
}

template <typename T>
__global__ __launch_bounds__(256) void k_export(const T* __restrict__ src, double* __restrict__ dst, size_t V,
                                                int ncomp, int mandel) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V * ncomp; g += (size_t)gridDim.x * 256) {
    const int c = (int)(g / V);
    const double f = (mandel && c >= 3) ? kIR2 : 1.0;
    dst[g] = f * (double)src[g];
  }
}

// add a uniform strain to the x-DC coefficient of every x-line
template <typename T>
__global__ __launch_bounds__(256) void k_shift_dc(cx<T>* main, size_t planes, int h, Shift6 d) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < 6 * planes; g += (size_t)gridDim.x * 256) {
    const size_t line = g / 6;
    const int c = (int)(g - line * 6);
    main[line * h * 6 + c].x += (T)d.v[c];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* p, size_t n, T v) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256) p[g] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b < 8192 ? (b ? b : 1) : 8192);
}

template <typename T, int MODE>
hipError_t launch_local(int n0, const LocalArgs<T>& a, hipStream_t s) {
  const int planes = a.n1 * a.n2;
#define FFTEVP_LOCAL(N)                                                                       \
  case N: {                                                                                   \
    const int lpb = LocalShape<T, N>::LPB;                                                    \
    if constexpr (MODE == MODE_NEWTON) {                                                      \
      if (a.sysp) {                                                                           \
        hipLaunchKernelGGL((k_local<T, N, MODE, FLOW_MR>), dim3(planes / lpb), dim3(LocalShape<T, N>::NT), 0, s, a); \
        break;                                                                                \
      }                                                                                       \
    }                                                                                         \
    if (MODE == MODE_EXPORT || a.m.n_int > 0)                                                 \
      hipLaunchKernelGGL((k_local<T, N, MODE, FLOW_POWER_INT>), dim3(planes / lpb), dim3(LocalShape<T, N>::NT), 0, s, a); \
    else                                                                                      \
      hipLaunchKernelGGL((k_local<T, N, MODE, FLOW_POWER>), dim3(planes / lpb), dim3(LocalShape<T, N>::NT), 0, s, a); \
    break;                                                                                    \
  }
  switch (n0) {
    FFTEVP_LOCAL(8)
    FFTEVP_LOCAL(16)
    FFTEVP_LOCAL(32)
    FFTEVP_LOCAL(64)
    FFTEVP_LOCAL(128)
    FFTEVP_LOCAL(256)
    FFTEVP_LOCAL(512)
    default:
      return hipErrorInvalidValue;
  }
#undef FFTEVP_LOCAL
  return hipGetLastError();
}

template <typename T>
int local_blocks(int n0, int n1, int n2) {
  return n1 * n2 / local_lines_per_block(n0);
}

// number of x-frequency tiles of a y pass (= blocks in its reduction row)
template <typename T>
int ypass_tiles(int n1, int h) {
  const int tx = y_tile<T, false>(n1);
  return h / (h < tx ? h : tx);
}

// Launch with the largest tile TX <= TXM that divides the h x-frequencies.
template <typename T, int N, int TX, bool INV>
hipError_t ypass_tx(int n2, const YArgs<T>& a, hipStream_t s) {
  if constexpr (TX > 1) {
    if (a.h < TX) return ypass_tx<T, N, TX / 2, INV>(n2, a, s);
  }
  hipLaunchKernelGGL((k_ypass<T, N, TX, INV>), dim3(a.h / TX, n2 + (INV || a.no_reduce ? 0 : 1)), dim3(256), 0,
                     s, a);
  return hipGetLastError();
}

template <typename T, bool INV>
hipError_t launch_ypass(int n1, int n2, const YArgs<T>& a, hipStream_t s) {
  switch (n1) {
    case 8: return ypass_tx<T, 8, y_tile<T, INV>(8), INV>(n2, a, s);
    case 16: return ypass_tx<T, 16, y_tile<T, INV>(16), INV>(n2, a, s);
    case 32: return ypass_tx<T, 32, y_tile<T, INV>(32), INV>(n2, a, s);
    case 64: return ypass_tx<T, 64, y_tile<T, INV>(64), INV>(n2, a, s);
    case 128: return ypass_tx<T, 128, y_tile<T, INV>(128), INV>(n2, a, s);
    case 256: return ypass_tx<T, 256, y_tile<T, INV>(256), INV>(n2, a, s);
    case 512: return ypass_tx<T, 512, y_tile<T, INV>(512), INV>(n2, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int N, int TX>
hipError_t zgamma_tx(const ZArgs<T>& a, hipStream_t s) {
  if constexpr (TX > 1) {
    if (a.h < TX) return zgamma_tx<T, N, TX / 2>(a, s);
  }
  hipLaunchKernelGGL((k_zgamma<T, N, TX>), dim3(a.h / TX, a.n1), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zgamma(int n2, const ZArgs<T>& a, hipStream_t s) {
  switch (n2) {
    case 8: return zgamma_tx<T, 8, spec_tile<T>(8)>(a, s);
    case 16: return zgamma_tx<T, 16, spec_tile<T>(16)>(a, s);
    case 32: return zgamma_tx<T, 32, spec_tile<T>(32)>(a, s);
    case 64: return zgamma_tx<T, 64, spec_tile<T>(64)>(a, s);
    case 128: return zgamma_tx<T, 128, spec_tile<T>(128)>(a, s);
    case 256: return zgamma_tx<T, 256, spec_tile<T>(256)>(a, s);
    case 512: return zgamma_tx<T, 512, spec_tile<T>(512)>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int N, int TX>
hipError_t zspin_tx(const ZArgs<T>& a, hipStream_t s) {
  if constexpr (TX > 1) {
    if (a.h < TX) return zspin_tx<T, N, TX / 2>(a, s);
  }
  hipLaunchKernelGGL((k_zspin<T, N, TX>), dim3(a.h / TX, a.n1), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zspin(int n2, const ZArgs<T>& a, hipStream_t s) {
  switch (n2) {
    case 8: return zspin_tx<T, 8, spec_tile<T>(8)>(a, s);
    case 16: return zspin_tx<T, 16, spec_tile<T>(16)>(a, s);
    case 32: return zspin_tx<T, 32, spec_tile<T>(32)>(a, s);
    case 64: return zspin_tx<T, 64, spec_tile<T>(64)>(a, s);
    case 128: return zspin_tx<T, 128, spec_tile<T>(128)>(a, s);
    case 256: return zspin_tx<T, 256, spec_tile<T>(256)>(a, s);
    case 512: return zspin_tx<T, 512, spec_tile<T>(512)>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_cadd(const cx<T>* a, const cx<T>* b, cx<T>* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_cadd<T>, dim3(grid_for(n)), dim3(256), 0, s, a, b, out, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_state(const StateArgs<T>& a, int nblocks, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_state<T>, dim3(nblocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, (const double*)a.partial, nblocks, out2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gdot(const T* sig, const T* quat, const T* rho, double* out, size_t V, const Mat& m,
                       double gdot0, hipStream_t s) {
  hipLaunchKernelGGL((k_gdot<T, double>), dim3(grid_for(V)), dim3(256), 0, s, sig, quat, rho, out, V, m, gdot0);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_split12(const T* __restrict__ rho, T* __restrict__ ssd, size_t V) {
  for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < V; g += (size_t)gridDim.x * 256) {
    const T r = (T)((double)rho[g] / 12.0);
    for (int a = 0; a < 12; ++a) ssd[(size_t)a * V + g] = r;
  }
}

template <typename T>
hipError_t launch_split12(const T* rho, T* ssd, size_t V, hipStream_t s) {
  hipLaunchKernelGGL(k_split12<T>, dim3(grid_for(V)), dim3(256), 0, s, rho, ssd, V);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_state_mr(const StateArgs<T>& a, int nblocks, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_state_mr<T>, dim3(nblocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, (const double*)a.partial, nblocks, out2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mr_params(const T* ssd, const T* gnds, const T* gndet, T* sysp, size_t V, const MrConst& c,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_mr_params<T>, dim3(grid_for(V)), dim3(256), 0, s, ssd, gnds, gndet, sysp, V, c);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gdot_mr(const T* sig, const T* quat, const T* sysp, double* out, size_t V, hipStream_t s) {
  hipLaunchKernelGGL(k_gdot_mr<T>, dim3(grid_for(V)), dim3(256), 0, s, sig, quat, sysp, out, V);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_kappa(const double* u, T* kappa, size_t V, double kc, double q, double* partial, int nblocks,
                        double* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_kappa<T>, dim3(nblocks), dim3(256), 0, s, u, kappa, V, kc, 1.0 / q, partial);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, (const double*)partial, nblocks, out2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_drx(const DrxArgs<T>& a, bool mr, int nblocks, double* out2, hipStream_t s) {
  if (mr) hipLaunchKernelGGL((k_drx<T, true>), dim3(nblocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_drx<T, false>), dim3(nblocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, (const double*)a.partial, nblocks, out2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rotate(T* quat, const T* gd, const double* spin, size_t V, double dt, hipStream_t s) {
  hipLaunchKernelGGL(k_rotate<T>, dim3(grid_for(V)), dim3(256), 0, s, quat, gd, spin, V, dt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rho_tot(const DrxArgs<T>& a, bool mr, double scale, double* out, hipStream_t s) {
  if (mr) hipLaunchKernelGGL((k_rho_tot<T, true>), dim3(grid_for(a.V)), dim3(256), 0, s, a, scale, out);
  else hipLaunchKernelGGL((k_rho_tot<T, false>), dim3(grid_for(a.V)), dim3(256), 0, s, a, scale, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const DrxArgs<T>& a, int nblocks, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_sweep<T>, dim3(nblocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, (const double*)a.partial, nblocks, out2);
  return hipGetLastError();
}

hipError_t launch_export_int(const int* src, double* dst, size_t V, hipStream_t s) {
  hipLaunchKernelGGL(k_export_int<double>, dim3(grid_for(V)), dim3(256), 0, s, src, dst, V);
  return hipGetLastError();
}

// GND update of one increment from the slip rates k_state left in gd.
// Grids whose xy-planes hold whole blocks march along z in the longest
// chunks (16, 8 or 4 planes) that still give a minimum number of blocks;
// others take one thread per voxel. Longer chunks fetch fewer halo planes
// (2 per chunk); FP32 (three waves per SIMD against two for FP64) measured
// best with more, shorter chunks at 128^3: 512 and 2048 blocks minimum.
#ifndef FFTEVP_GND_MIN_BLOCKS_F64
#define FFTEVP_GND_MIN_BLOCKS_F64 512
#endif
#ifndef FFTEVP_GND_MIN_BLOCKS_F32
#define FFTEVP_GND_MIN_BLOCKS_F32 2048
#endif
template <typename T>
hipError_t launch_gnd(const GndArgs<T>& a, hipStream_t s) {
  const size_t P = (size_t)a.n0 * a.n1;
  if (FFTEVP_GND_MARCH && P % 256 == 0 && a.n2 % 4 == 0) {
    const size_t tiles = P / 256;
    const size_t min_blocks = sizeof(T) == 8 ? FFTEVP_GND_MIN_BLOCKS_F64 : FFTEVP_GND_MIN_BLOCKS_F32;
    auto fits = [&](int zc) { return a.n2 % zc == 0 && tiles * (a.n2 / zc) >= min_blocks; };
    if (fits(16))
      hipLaunchKernelGGL((k_gnd_z<T, 16>), dim3((unsigned)(tiles * (a.n2 / 16))), dim3(256), 0, s, a);
    else if (fits(8))
      hipLaunchKernelGGL((k_gnd_z<T, 8>), dim3((unsigned)(tiles * (a.n2 / 8))), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_gnd_z<T, 4>), dim3((unsigned)(tiles * (a.n2 / 4))), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  const int nb = (int)((a.V + 255) / 256);
  hipLaunchKernelGGL(k_gnd<T>, dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ingest(const double* q, const double* rho, T* qo, T* ro, size_t V, double* partial,
                         int nblocks, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_ingest<T>, dim3(nblocks), dim3(256), 0, s, q, rho, qo, ro, V, partial);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, (const double*)partial, nblocks, out2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_export(const T* src, double* dst, size_t V, int ncomp, int mandel, hipStream_t s) {
  hipLaunchKernelGGL(k_export<T>, dim3(grid_for(V * ncomp)), dim3(256), 0, s, src, dst, V, ncomp, mandel);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_shift_dc(cx<T>* main, size_t planes, int h, const double dE[6], hipStream_t s) {
  Shift6 d;
  for (int k = 0; k < 6; ++k) d.v[k] = dE[k];
  hipLaunchKernelGGL(k_shift_dc<T>, dim3(grid_for(6 * planes)), dim3(256), 0, s, main, planes, h, d);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, size_t n, T v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

#define FFTEVP_INST(T)                                                                          \
  template hipError_t launch_local<T, MODE_NEWTON>(int, const LocalArgs<T>&, hipStream_t);     \
  template hipError_t launch_local<T, MODE_TANGENT>(int, const LocalArgs<T>&, hipStream_t);    \
  template hipError_t launch_local<T, MODE_EXPORT>(int, const LocalArgs<T>&, hipStream_t);     \
  template int local_blocks<T>(int, int, int);                                                  \
  template int ypass_tiles<T>(int, int);                                                        \
  template hipError_t launch_ypass<T, false>(int, int, const YArgs<T>&, hipStream_t);          \
  template hipError_t launch_ypass<T, true>(int, int, const YArgs<T>&, hipStream_t);           \
  template hipError_t launch_zgamma<T>(int, const ZArgs<T>&, hipStream_t);                     \
  template hipError_t launch_state<T>(const StateArgs<T>&, int, double*, hipStream_t);         \
  template hipError_t launch_gdot<T>(const T*, const T*, const T*, double*, size_t, const Mat&, double, \
                                     hipStream_t);                                            \
  template hipError_t launch_gnd<T>(const GndArgs<T>&, hipStream_t);                          \
  template hipError_t launch_state_mr<T>(const StateArgs<T>&, int, double*, hipStream_t);      \
  template hipError_t launch_split12<T>(const T*, T*, size_t, hipStream_t);                   \
  template hipError_t launch_kappa<T>(const double*, T*, size_t, double, double, double*, int, double*, \
                                      hipStream_t);                                           \
  template hipError_t launch_drx<T>(const DrxArgs<T>&, bool, int, double*, hipStream_t);      \
  template hipError_t launch_rho_tot<T>(const DrxArgs<T>&, bool, double, double*, hipStream_t); \
  template hipError_t launch_rotate<T>(T*, const T*, const double*, size_t, double, hipStream_t); \
  template hipError_t launch_zspin<T>(int, const ZArgs<T>&, hipStream_t);                      \
  template hipError_t launch_cadd<T>(const cx<T>*, const cx<T>*, cx<T>*, size_t, hipStream_t); \
  template hipError_t launch_sweep<T>(const DrxArgs<T>&, int, double*, hipStream_t);          \
  template hipError_t launch_mr_params<T>(const T*, const T*, const T*, T*, size_t, const MrConst&, \
                                          hipStream_t);                                       \
  template hipError_t launch_gdot_mr<T>(const T*, const T*, const T*, double*, size_t, hipStream_t); \
  template hipError_t launch_ingest<T>(const double*, const double*, T*, T*, size_t, double*, int, \
                                       double*, hipStream_t);                                  \
  template hipError_t launch_export<T>(const T*, double*, size_t, int, int, hipStream_t);      \
  template hipError_t launch_shift_dc<T>(cx<T>*, size_t, int, const double*, hipStream_t);     \
  template hipError_t launch_fill<T>(T*, size_t, T, hipStream_t);                              \
  template hipError_t launch_adj_setup<T>(const AdjArgs<T>&, int, double*, hipStream_t);        \
  template hipError_t launch_adj_update<T>(const AdjArgs<T>&, int, double*, hipStream_t);

FFTEVP_INST(double)
FFTEVP_INST(float)

}  // namespace fftevp
