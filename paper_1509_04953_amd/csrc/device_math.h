// Per-voxel crystal mechanics for the local solve (device side).
//
// Symmetric tensors are Mandel 6-vectors [11, 22, 33, r2*23, r2*13, r2*12]
// (r2 = sqrt 2), so double contraction is a dot product. The local problem
// is solved in the crystal frame of the voxel: there the cubic compliance has
// three distinct entries, the isotropic reference medium is unchanged, and
// the Schmid tensors of the 12 FCC {111}<110> systems are fixed sign
// patterns, so each resolved shear costs a few additions.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace fftevp {

// Crystal-frame Schmid vectors: m_a[k] = kSign[a][k] * (1/sqrt6 for the
// normal slots, 1/sqrt12 for the shear slots). Systems: plane normals
// (111), (-111), (1-11), (11-1); per plane the three <110> directions in the
// plane, i.e. m = sym(d x n) with |n| = |d| = 1 and n.d = 0. Shear is signed,
// so each system appears once.
constexpr int kSign[12][6] = {
    {0, 1, -1, 0, -1, 1},  {1, 0, -1, -1, 0, 1},  {1, -1, 0, -1, 1, 0},
    {0, 1, -1, 0, 1, -1},  {-1, 0, 1, 1, 0, 1},   {-1, 1, 0, 1, 1, 0},
    {0, -1, 1, 0, 1, 1},   {1, 0, -1, 1, 0, -1},  {1, -1, 0, 1, 1, 0},
    {0, 1, -1, 0, 1, 1},   {1, 0, -1, 1, 0, 1},   {1, -1, 0, 1, -1, 0},
};

constexpr double kR2 = 1.41421356237309504880;
constexpr double kIR2 = 0.70710678118654752440;
constexpr double kUN = 0.40824829046386301637;   // 1/sqrt(6)
constexpr double kUS = 0.28867513459481288225;   // 1/sqrt(12)

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

__host__ __device__ constexpr int tri(int i, int j) {  // packed lower triangle
  return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

// Material constants of one solve, all FP64 on the host side.
struct Mat {
  double a_d, a_o, a_s;   // A = C0^-1 + S in the crystal frame (cubic form)
  double s_d, s_o, s_s;   // S in the crystal frame (cubic form)
  double c0l, c0m;        // reference medium: lambda0, mu0
  double ci_d, ci_o, ci_s;  // C0^-1 (Mandel: normal diag, normal off, shear)
  double c1;              // dt * gdot0
  double n;               // rate exponent
  int n_int;              // n if n is a positive integer, else 0
  int newton_max;
  double ntol;            // Newton step tolerance (relative)
  double qtol;            // full Newton steps below this are final (quadratic regime)
  double tau0, taylor;    // tauc = tau0 + taylor * sqrt(rho), taylor = alpha mu b
  double inv_n0;          // 1 / n0
  double dt;              // time increment (s)
};

// Flow rules of the local solve: the power law with a general or an integral
// exponent, or the paper's dislocation-based law (Sec. 2.2, Eq. 3) with
// per-system parameters frozen over the increment.
enum { FLOW_POWER = 0, FLOW_POWER_INT = 1, FLOW_MR = 2 };

// Per-voxel parameters of the paper's law, stored [3][12][V]: tau_pass (MPa),
// 1 / tau_cut (1/MPa), A = gdot_0 exp(-Q_slip / kB T) (1/s); the flow needs
// no division (tau_cut for the potential comes from a refined reciprocal).
template <typename T>
struct SysParams {
  const T* p;
  size_t V, g;
  __device__ __forceinline__ T tp(int a) const { return p[(size_t)a * V + g]; }
  __device__ __forceinline__ T itc(int a) const { return p[(size_t)(12 + a) * V + g]; }
  __device__ __forceinline__ T amp(int a) const { return p[(size_t)(24 + a) * V + g]; }
};

// The same parameters with the first Q rows (tau_pass and 1/tau_cut: 24, or
// all 36) staged in LDS, one column per thread (rows of stride ls); the rest
// read from global memory.
template <typename T, int Q>
struct SysParamsStaged {
  const T* p;
  size_t V, g;
  const T* l;
  int ls, t;
  __device__ __forceinline__ T tp(int a) const { return l[a * ls + t]; }
  __device__ __forceinline__ T itc(int a) const { return l[(12 + a) * ls + t]; }
  __device__ __forceinline__ T amp(int a) const {
    if constexpr (Q == 36) return l[(24 + a) * ls + t];
    else return p[(size_t)(24 + a) * V + g];
  }
};

// tau_pass and A staged in LDS (rows 0-11 and 12-23 of stride ls), 1/tau_cut
// held in registers
template <typename T>
struct SysParamsHybrid {
  const T* l;
  int ls, t;
  const T (&ir)[12];
  __device__ __forceinline__ T tp(int a) const { return l[a * ls + t]; }
  __device__ __forceinline__ T itc(int a) const { return ir[a]; }
  __device__ __forceinline__ T amp(int a) const { return l[(12 + a) * ls + t]; }
};

// 1/x: the hardware reciprocal, refined once by Newton's method in FP64
__device__ __forceinline__ float fast_recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_recip(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return r * __builtin_fma(-x, r, 2.0);
}

template <typename T>
__device__ __forceinline__ void quat_rot(T w, T x, T y, T z, T (&R)[9]) {
  R[0] = T(1) - T(2) * (y * y + z * z);
  R[1] = T(2) * (x * y - w * z);
  R[2] = T(2) * (x * z + w * y);
  R[3] = T(2) * (x * y + w * z);
  R[4] = T(1) - T(2) * (x * x + z * z);
  R[5] = T(2) * (y * z - w * x);
  R[6] = T(2) * (x * z - w * y);
  R[7] = T(2) * (y * z + w * x);
  R[8] = T(1) - T(2) * (x * x + y * y);
}

template <typename T>
__device__ __forceinline__ void to_sym3(const T (&a)[6], T (&A)[9]) {
  const T h = T(kIR2);
  A[0] = a[0];
  A[4] = a[1];
  A[8] = a[2];
  A[5] = A[7] = h * a[3];
  A[2] = A[6] = h * a[4];
  A[1] = A[3] = h * a[5];
}

// crystal components of a sample-frame tensor: R^T A R
template <typename T>
__device__ __forceinline__ void to_crystal(const T (&R)[9], const T (&a)[6], T (&o)[6]) {
  T A[9], B[9];
  to_sym3(a, A);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      B[3 * i + j] = A[3 * i] * R[j] + A[3 * i + 1] * R[3 + j] + A[3 * i + 2] * R[6 + j];
  auto c = [&](int i, int j) { return R[i] * B[j] + R[3 + i] * B[3 + j] + R[6 + i] * B[6 + j]; };
  const T r2 = T(kR2);
  o[0] = c(0, 0);
  o[1] = c(1, 1);
  o[2] = c(2, 2);
  o[3] = r2 * c(1, 2);
  o[4] = r2 * c(0, 2);
  o[5] = r2 * c(0, 1);
}

// sample components of a crystal-frame tensor: R A R^T
template <typename T>
__device__ __forceinline__ void to_sample(const T (&R)[9], const T (&a)[6], T (&o)[6]) {
  T A[9], B[9];
  to_sym3(a, A);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      B[3 * i + j] = A[3 * i] * R[3 * j] + A[3 * i + 1] * R[3 * j + 1] + A[3 * i + 2] * R[3 * j + 2];
  auto c = [&](int i, int j) {
    return R[3 * i] * B[j] + R[3 * i + 1] * B[3 + j] + R[3 * i + 2] * B[6 + j];
  };
  const T r2 = T(kR2);
  o[0] = c(0, 0);
  o[1] = c(1, 1);
  o[2] = c(2, 2);
  o[3] = r2 * c(1, 2);
  o[4] = r2 * c(0, 2);
  o[5] = r2 * c(0, 1);
}

template <int C, typename T>
__device__ __forceinline__ void acc_sign(T& acc, T v) {
  if constexpr (C > 0) acc += v;
  else if constexpr (C < 0) acc -= v;
}

// resolved shear of system A (crystal-frame Mandel stress)
template <int A, typename T>
__device__ __forceinline__ T resolved(const T (&s)[6]) {
  T tn = T(0), ts = T(0);
  acc_sign<kSign[A][0]>(tn, s[0]);
  acc_sign<kSign[A][1]>(tn, s[1]);
  acc_sign<kSign[A][2]>(tn, s[2]);
  acc_sign<kSign[A][3]>(ts, s[3]);
  acc_sign<kSign[A][4]>(ts, s[4]);
  acc_sign<kSign[A][5]>(ts, s[5]);
  return T(kUN) * tn + T(kUS) * ts;
}

// Structure of the 12 systems in the crystal frame, read off kSign. The
// normal part of m_a is kUN * nsgn(a) * d_t with t = ntype(a) the normal slot
// that is zero and d_0 = e1 - e2, d_1 = e0 - e2, d_2 = e0 - e1. The shear
// part is kUS * ssgn(a) * (e_p + srho(a) e_q), where (p, q), p < q, are the
// two shear slots other than t (the zero shear slot of every system is the
// one of its normal type). Resolved shears, flow sums and the Jacobian are
// assembled from the per-type sums these groupings allow.
__host__ __device__ constexpr int ntype(int a) {
  return kSign[a][0] == 0 ? 0 : (kSign[a][1] == 0 ? 1 : 2);
}
__host__ __device__ constexpr int nsgn(int a) { return ntype(a) == 0 ? kSign[a][1] : kSign[a][0]; }
__host__ __device__ constexpr int slot_p(int t) { return t == 0 ? 1 : 0; }
__host__ __device__ constexpr int slot_q(int t) { return t == 2 ? 1 : 2; }
__host__ __device__ constexpr int ssgn(int a) { return kSign[a][3 + slot_p(ntype(a))]; }
__host__ __device__ constexpr int srho(int a) {
  return kSign[a][3 + slot_p(ntype(a))] * kSign[a][3 + slot_q(ntype(a))];
}
// d_t as a 3-vector: component i of d_t
__host__ __device__ constexpr int dcomp(int t, int i) {
  return i == t ? 0 : ((t == 0) ? (i == 1 ? 1 : -1) : (i == 0 ? 1 : -1));
}
// position of system a among the four systems of its type
__host__ __device__ constexpr int tpos(int a) {
  int k = 0;
  for (int b = 0; b < a; ++b) k += ntype(b) == ntype(a);
  return k;
}
__host__ __device__ constexpr bool structure_ok() {
  for (int a = 0; a < 12; ++a) {
    const int t = ntype(a);
    for (int i = 0; i < 3; ++i)
      if (kSign[a][i] != nsgn(a) * dcomp(t, i)) return false;
    if (kSign[a][3 + t] != 0) return false;
    if (kSign[a][3 + slot_p(t)] != ssgn(a)) return false;
    if (kSign[a][3 + slot_q(t)] != ssgn(a) * srho(a)) return false;
    if (ssgn(a) == 0 || srho(a) == 0) return false;
  }
  for (int t = 0; t < 3; ++t) {
    int c = 0;
    for (int a = 0; a < 12; ++a) c += ntype(a) == t;
    if (c != 4) return false;
  }
  return true;
}
static_assert(structure_ok(), "slip-system sign table does not have the assumed structure");

// Resolved shears x_a = m_a : s * (scale), a in type t: cn = kUN * scale,
// cs = kUS * scale. One subtraction, two products, a sum and a difference
// serve the four systems of the type.
template <int TT, typename T>
__device__ __forceinline__ void resolved_type(const T (&s)[6], T cn, T cs, T (&x)[4]) {
  constexpr int P = slot_p(TT), Q = slot_q(TT);
  const T dn = cn * (TT == 0 ? s[1] - s[2] : (TT == 1 ? s[0] - s[2] : s[0] - s[1]));
  const T hp = cs * s[3 + P], hq = cs * s[3 + Q];
  const T pp = hp + hq, pm = hp - hq;
  static_for<0, 12>([&](auto ac) {
    constexpr int A = decltype(ac)::value;
    if constexpr (ntype(A) == TT) {
      constexpr int j = tpos(A);
      const T sh = srho(A) > 0 ? pp : pm;
      if constexpr (nsgn(A) > 0 && ssgn(A) > 0) x[j] = dn + sh;
      else if constexpr (nsgn(A) > 0) x[j] = dn - sh;
      else if constexpr (ssgn(A) > 0) x[j] = sh - dn;
      else x[j] = -(dn + sh);
    }
  });
}

// Flow at a crystal-frame stress s:
//   w[a]  = |x_a|^(n-1),  x_a = tau_a / tauc
//   g[k]  = sum_a sign(x_a)|x_a|^n kSign[a][k]   (epsdot_p = gdot0 * u_k g[k])
//   visc  = sum_a |x_a|^(n+1)
//   asum  = sum_a |x_a|^n
// INTN: n is a positive integer (n_int); the powers then come from a
// binary-exponent loop with a uniform trip count. Otherwise
// |x|^(n-1) = exp((n-1) log|x|). The systems are processed one normal type
// (four systems) at a time to bound the number of live registers.
template <bool INTN, int TT, typename T, typename W>
__device__ __forceinline__ void flow_type(const T (&s)[6], T cn, T cs, T n, int n_int, W (&w)[12],
                                          T (&g)[6], T& visc, T& asum) {
  T x[4], wg[4], ax[4];
  resolved_type<TT>(s, cn, cs, x);
#pragma unroll
  for (int a = 0; a < 4; ++a) ax[a] = fabs(x[a]);
  if constexpr (INTN) {
    // |x|^(n-1) by binary powers: the lowest bit sets the start value
    T base[4];
    int e = n_int - 1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      base[a] = ax[a];
      wg[a] = (e & 1) ? ax[a] : T(1);
    }
#pragma unroll 1
    for (e >>= 1; e != 0; e >>= 1) {
#pragma unroll
      for (int a = 0; a < 4; ++a) base[a] *= base[a];
      if (e & 1) {
#pragma unroll
        for (int a = 0; a < 4; ++a) wg[a] *= base[a];
      }
    }
  } else {
#pragma unroll
    for (int a = 0; a < 4; ++a)
      wg[a] = ax[a] > T(0) ? exp((n - T(1)) * log(ax[a])) : (n == T(1) ? T(1) : T(0));
  }
  // signed |x|^n, grouped: gn = sum nsgn sp (normal part), gs[r] = sum ssgn sp
  // over the systems with srho = +1 (r = 0) or -1 (r = 1)
  T gn = T(-0.0), gs0 = T(-0.0), gs1 = T(-0.0);
  static_for<0, 12>([&](auto ac) {
    constexpr int A = decltype(ac)::value;
    if constexpr (ntype(A) == TT) {
      constexpr int j = tpos(A);
      const T p = wg[j] * ax[j];
      w[A] = W(wg[j]);
      visc += p * ax[j];
      asum += p;
      const T sp = x[j] < T(0) ? -p : p;
      if constexpr (nsgn(A) > 0) gn += sp;
      else gn -= sp;
      if constexpr (srho(A) > 0) {
        if constexpr (ssgn(A) > 0) gs0 += sp;
        else gs0 -= sp;
      } else {
        if constexpr (ssgn(A) > 0) gs1 += sp;
        else gs1 -= sp;
      }
    }
  });
  static_for<0, 3>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    if constexpr (dcomp(TT, I) > 0) g[I] += gn;
    else if constexpr (dcomp(TT, I) < 0) g[I] -= gn;
  });
  g[3 + slot_p(TT)] += gs0 + gs1;
  g[3 + slot_q(TT)] += gs0 - gs1;
}

// The paper's flow rule for the four systems of a type: with
// x = (|tau| - tau_pass) / tau_cut > 0, gdot = A sinh(x) sign(tau), Jacobian
// weight dgdot/dtau = A cosh(x) / tau_cut and potential A tau_cut (cosh x - 1)
// (zero below the passing stress). g, visc and asum as for the power law, in
// rate units (the residual then takes dt instead of dt gdot0).
template <int TT, typename T, typename W, typename SP>
__device__ __forceinline__ void flow_type_mr(const T (&s)[6], const SP& sp, W (&w)[12], T (&g)[6],
                                             T& visc, T& asum) {
  T x[4];
  resolved_type<TT>(s, T(kUN), T(kUS), x);
  T gn = T(-0.0), gs0 = T(-0.0), gs1 = T(-0.0);
  static_for<0, 12>([&](auto ac) {
    constexpr int A = decltype(ac)::value;
    if constexpr (ntype(A) == TT) {
      constexpr int j = tpos(A);
      const T itc = sp.itc(A), amp = sp.amp(A);
      const T xx = (fabs(x[j]) - sp.tp(A)) * itc;
      T rate = T(0), wa = T(0), psi = T(0);
      if (xx > T(0)) {
        const T ex = exp(xx), iex = fast_recip(ex);
        const T sh = T(0.5) * (ex - iex), ch = T(0.5) * (ex + iex);
        rate = amp * sh;
        wa = amp * ch * itc;
        psi = amp * fast_recip(itc) * (ch - T(1));
      }
      w[A] = W(wa);
      visc += psi;
      asum += rate;
      const T sp_ = x[j] < T(0) ? -rate : rate;
      if constexpr (nsgn(A) > 0) gn += sp_;
      else gn -= sp_;
      if constexpr (srho(A) > 0) {
        if constexpr (ssgn(A) > 0) gs0 += sp_;
        else gs0 -= sp_;
      } else {
        if constexpr (ssgn(A) > 0) gs1 += sp_;
        else gs1 -= sp_;
      }
    }
  });
  static_for<0, 3>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    if constexpr (dcomp(TT, I) > 0) g[I] += gn;
    else if constexpr (dcomp(TT, I) < 0) g[I] -= gn;
  });
  g[3 + slot_p(TT)] += gs0 + gs1;
  g[3 + slot_q(TT)] += gs0 - gs1;
}

template <typename T, typename W, typename SP>
__device__ __forceinline__ void flow_eval_mr(const T (&s)[6], const SP& sp, W (&w)[12], T (&g)[6],
                                             T& visc, T& asum) {
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = T(-0.0);
  visc = T(-0.0);
  asum = T(-0.0);
  flow_type_mr<0>(s, sp, w, g, visc, asum);
  flow_type_mr<1>(s, sp, w, g, visc, asum);
  flow_type_mr<2>(s, sp, w, g, visc, asum);
}

template <bool INTN, typename T, typename W>
__device__ __forceinline__ void flow_eval(const T (&s)[6], T itauc, T n, int n_int, W (&w)[12],
                                          T (&g)[6], T& visc, T& asum) {
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = T(-0.0);
  visc = T(-0.0);
  asum = T(-0.0);
  const T cn = T(kUN) * itauc, cs = T(kUS) * itauc;
  flow_type<INTN, 0>(s, cn, cs, n, n_int, w, g, visc, asum);
  flow_type<INTN, 1>(s, cn, cs, n, n_int, w, g, visc, asum);
  flow_type<INTN, 2>(s, cn, cs, n, n_int, w, g, visc, asum);
}

// cubic-form 6x6 (Mandel) times vector: normal block (d, o), shear diag s
template <typename T>
__device__ __forceinline__ void cubic_mul(T d, T o, T sh, const T (&v)[6], T (&out)[6]) {
  out[0] = d * v[0] + o * (v[1] + v[2]);
  out[1] = d * v[1] + o * (v[0] + v[2]);
  out[2] = d * v[2] + o * (v[0] + v[1]);
  out[3] = sh * v[3];
  out[4] = sh * v[4];
  out[5] = sh * v[5];
}

// residual and potential of the local problem in the crystal frame:
//   r   = A s - b + c1 * m(g)
//   phi = 1/2 s.A s - b.s + c1 tauc/(n+1) visc   (power law, c1 = dt gdot0)
//   phi = 1/2 s.A s - b.s + dt visc              (paper's law, c1 = dt)
// The residual is formed in T (it cancels large terms); once formed it is
// returned in FP32 with the Jacobian weights w: the Newton direction is an
// FP32 solve, and rounding a small residual keeps its relative precision.
template <int FLOW, typename T, typename SP>
__device__ __forceinline__ void local_residual(const Mat& M, const T (&s)[6], const T (&b)[6],
                                               T tauc, T itauc, float (&w)[12], float (&r)[6], T& phi,
                                               const SP& sp) {
  T g[6], visc, asum;
  if constexpr (FLOW == FLOW_MR) flow_eval_mr(s, sp, w, g, visc, asum);
  else flow_eval<FLOW == FLOW_POWER_INT>(s, itauc, T(M.n), M.n_int, w, g, visc, asum);
  T As[6];
  cubic_mul(T(M.a_d), T(M.a_o), T(M.a_s), s, As);
  const T c1 = FLOW == FLOW_MR ? T(M.dt) : T(M.c1);
  T q = T(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T u = k < 3 ? T(kUN) : T(kUS);
    r[k] = float(As[k] - b[k] + c1 * u * g[k]);
    q += s[k] * (T(0.5) * As[k] - b[k]);
  }
  if constexpr (FLOW == FLOW_MR) phi = q + c1 * visc;
  else phi = q + c1 * tauc / (T(M.n) + T(1)) * visc;
}

// J = A + cj * sum_a w_a m_a m_a^T  (packed lower triangle, 21 entries),
// assembled in precision JT from per-type sums of the weights:
//   wp[t][r] = sum of w_a over type t with srho = +1 (r = 0) / -1 (r = 1),
//   v[t][r]  = the same sums of nsgn ssgn w_a.
// Normal block: (d_t d_t^T) (wp0 + wp1) / 6; shear block: on the pair (p, q)
// of type t, diagonal wp0 + wp1 and off-diagonal wp0 - wp1, times 1/12;
// mixed block: d_t (x) (e_p (v0 + v1) + e_q (v0 - v1)) kUN kUS.
template <typename JT, typename T>
__device__ __forceinline__ void local_jacobian(const Mat& M, const T (&w)[12], T cj, JT (&J)[21]) {
  JT wd[3], wo[3], vp[3], vm[3];
  static_for<0, 3>([&](auto tc) {
    constexpr int TT = decltype(tc)::value;
    JT w0 = JT(-0.0), w1 = JT(-0.0), v0 = JT(-0.0), v1 = JT(-0.0);
    static_for<0, 12>([&](auto ac) {
      constexpr int A = decltype(ac)::value;
      if constexpr (ntype(A) == TT) {
        const JT x = JT(w[A]);
        if constexpr (srho(A) > 0) {
          w0 += x;
          if constexpr (nsgn(A) * ssgn(A) > 0) v0 += x;
          else v0 -= x;
        } else {
          w1 += x;
          if constexpr (nsgn(A) * ssgn(A) > 0) v1 += x;
          else v1 -= x;
        }
      }
    });
    wd[TT] = w0 + w1;
    wo[TT] = w0 - w1;
    vp[TT] = v0 + v1;
    vm[TT] = v0 - v1;
  });
  const JT fn = JT(cj) * JT(1.0 / 6.0), fs = JT(cj) * JT(1.0 / 12.0), fm = JT(cj) * JT(kUN * kUS);
  const JT ad = JT(M.a_d), ao = JT(M.a_o), as = JT(M.a_s);
  // normal block: (i, i) = sum of wd over the two types with d_t[i] != 0,
  // (i, k) = -wd of the third type
  J[tri(0, 0)] = ad + fn * (wd[1] + wd[2]);
  J[tri(1, 1)] = ad + fn * (wd[0] + wd[2]);
  J[tri(2, 2)] = ad + fn * (wd[0] + wd[1]);
  J[tri(1, 0)] = ao - fn * wd[2];
  J[tri(2, 0)] = ao - fn * wd[1];
  J[tri(2, 1)] = ao - fn * wd[0];
  // shear block: slot j lies in the pairs of the two types t != j
  J[tri(3, 3)] = as + fs * (wd[1] + wd[2]);
  J[tri(4, 4)] = as + fs * (wd[0] + wd[2]);
  J[tri(5, 5)] = as + fs * (wd[0] + wd[1]);
  static_for<0, 3>([&](auto tc) {
    constexpr int TT = decltype(tc)::value;
    J[tri(3 + slot_q(TT), 3 + slot_p(TT))] = fs * wo[TT];
  });
  // mixed block: entry (i, 3 + j) = sum over types t with d_t[i] != 0 and
  // j in {p, q} of d_t[i] * (j == p ? vp : vm)
  static_for<0, 3>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    static_for<0, 3>([&](auto jc) {
      constexpr int J3 = decltype(jc)::value;
      JT h = JT(-0.0);
      static_for<0, 3>([&](auto tc) {
        constexpr int TT = decltype(tc)::value;
        if constexpr (dcomp(TT, I) != 0 && J3 != TT) {
          const JT c = (J3 == slot_p(TT)) ? vp[TT] : vm[TT];
          if constexpr (dcomp(TT, I) > 0) h += c;
          else h -= c;
        }
      });
      J[tri(3 + J3, I)] = fm * h;
    });
  });
}

// 1/d: the hardware reciprocal (1 ulp) for the FP32 Newton direction, a
// correctly rounded division in FP64
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double recip(double d) { return 1.0 / d; }

// Solve J x = rhs for SPD J (packed lower triangle) by J = L D L^T with unit
// lower L. P holds L scaled by D column-wise (P_ij = L_ij d_j), id = 1/d;
// L_ij = P_ij id_j is formed once per entry, so every update of the
// factorisation and of the forward substitution is one fused multiply-add.
template <typename T>
__device__ __forceinline__ void ldl_solve(const T (&J)[21], const T (&rhs)[6], T (&x)[6]) {
  T P[21], L[21], id[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T d = J[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= P[tri(j, k)] * L[tri(j, k)];
    id[j] = recip(d);
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      T v = J[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= P[tri(i, k)] * L[tri(j, k)];
      P[tri(i, j)] = v;
      L[tri(i, j)] = v * id[j];
    }
  }
  T y[6];  // L y = rhs
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T v = rhs[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[tri(i, k)] * y[k];
    y[i] = v;
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {  // L^T x = D^-1 y
    T v = y[i] * id[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) v -= L[tri(k, i)] * x[k];
    x[i] = v;
  }
}

}  // namespace fftevp
