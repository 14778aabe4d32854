// Phase-field growth of recrystallised grains (Sec. 2.4, Eq. 12-15) on
// sparse order parameters: 2:1 refinement of the grain map and stored energy,
// explicit Allen-Cahn steps with per-point truncation to the K largest order
// parameters, and the grain map read back on the mechanical grid. The
// contract is include/fftevp_pf.h.
//
// Layout on the PF grid (Vf points, [z][y][x]): a count byte per point and
// K slots of (int32 key, value), slot-major, the used slots of a point first
// and in decreasing value. Slots past a point's count are never read, so a
// step writes only the used ones: the traffic of a point scales with the
// order parameters it holds (one in a grain interior).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <string>

#include "../../include/fftevp_pf.h"

namespace {

constexpr int kNoKey = INT_MIN;  // key of an unused slot on export
constexpr int kBlock = 256;
constexpr int kList = 16;  // LDS list entries per thread in the step (see there)

// Coefficients in the solver's units (dx = 1, one step dt = 1,
// l_gb^2 = 9.6, 6 omega_gb = l_gb, M_gb = 0.0375 l_gb):
constexpr double kGrad = 1.2;   // gradient coefficient 3 omega l / 4
constexpr double kKin = 0.05;   // kinetic coefficient 4 M / (3 l)
// the well height 6 omega / l is 1 and is left out of the products

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// First point of this block's tile. Consecutive tiles go to one XCD (blocks
// are dealt to the 8 XCDs in turn), so the y and z neighbours of a tile are
// mostly read from the L2 that already holds them.
__device__ __forceinline__ int tile_base() {
  unsigned id = blockIdx.x;
  const unsigned nb = gridDim.x;
  if (nb % 8 == 0) id = (id % 8) * (nb / 8) + id / 8;
  return (int)(id * kBlock);
}

// Tile order of the step: when a z-plane splits into 8 equal runs of whole
// tiles, XCD x (blocks id = x mod 8) owns run x of every plane and walks
// through the planes in z order, so the plane below a tile was read only a
// run earlier (tens of tiles) and is still in that XCD's L2 when the tile
// reads it as a neighbour; the plane above is being brought in by the tiles
// that follow.
__device__ __forceinline__ int step_tile_base(int n0, int n1, int n2) {
  const unsigned plane = (unsigned)n0 * (unsigned)n1;
  if (plane % (8u * kBlock) == 0) {
    const unsigned ntp = plane / kBlock, run = ntp / 8;
    if (gridDim.x == ntp * (unsigned)n2) {
      const unsigned id = blockIdx.x, x = id % 8, k = id / 8;
      return (int)(((k / run) * ntp + x * run + k % run) * kBlock);
    }
  }
  return tile_base();
}

// Insert (v, k) into a list sorted by decreasing value (equal values: smaller
// key first); the smallest entry falls off the end.
template <typename T, int K>
__device__ __forceinline__ void keep_largest(T (&tv)[K], int (&tk)[K], T v, int k) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const bool take = v > tv[i] || (v == tv[i] && k < tk[i]);
    const T sv = tv[i];
    const int sk = tk[i];
    tv[i] = take ? v : sv;
    tk[i] = take ? k : sk;
    v = take ? sv : v;
    k = take ? sk : k;
  }
}

// Order (tv, tk) by decreasing value, equal values by increasing key, with
// the 12-comparator sorting network for six inputs (cheaper than inserting
// the six one by one).
template <typename T>
__device__ __forceinline__ void sort6(T (&tv)[6], int (&tk)[6]) {
  auto cx = [&](int i, int j) {
    const bool sw = tv[j] > tv[i] || (tv[j] == tv[i] && tk[j] < tk[i]);
    const T vi = tv[i], vj = tv[j];
    const int ki = tk[i], kj = tk[j];
    tv[i] = sw ? vj : vi;
    tv[j] = sw ? vi : vj;
    tk[i] = sw ? kj : ki;
    tk[j] = sw ? ki : kj;
  };
  cx(0, 5); cx(1, 3); cx(2, 4);
  cx(1, 2); cx(3, 4);
  cx(0, 3); cx(2, 5);
  cx(0, 1); cx(2, 3); cx(4, 5);
  cx(1, 2); cx(3, 4);
}

template <typename T>
struct StepArgs {
  const unsigned char* cnt;
  const int* key;
  const T* val;
  const T* E;  // stored energy [Vf]
  unsigned char* cnt_out;
  int* key_out;
  T* val_out;
  int n0, n1, n2, V;
  T thr;
};

// One explicit step of Eq. 15 for every order parameter that is non-zero at
// the point or at one of its six neighbours (the others stay zero), then
// truncation. The candidate keys are the point's own and, once each, those
// its neighbours hold that it does not.
// Occupancy: three waves per SIMD for FP64 (a few registers spill, which
// costs less than the latency the extra wave hides), four for FP32.
template <typename T, int K>
__global__ __launch_bounds__(kBlock, sizeof(T) == 8 ? 3 : 4) void k_pf_step(StepArgs<T> a) {
  const int V = a.V;
  const int p0 = step_tile_base(a.n0, a.n1, a.n2) + (int)threadIdx.x;
  const bool live = p0 < V;
  const int p = live ? p0 : V - 1;
  const int n0 = a.n0, n1 = a.n1, n2 = a.n2, pl = n0 * n1;
  const int x = p % n0, r = p / n0, y = r % n1, z = r / n1;
  // neighbours in the order z-1, z+1, y-1, y+1, x-1, x+1 (periodic)
  int nb[6];
  nb[0] = z > 0 ? p - pl : p + (n2 - 1) * pl;
  nb[1] = z < n2 - 1 ? p + pl : p - (n2 - 1) * pl;
  nb[2] = y > 0 ? p - n0 : p + (n1 - 1) * n0;
  nb[3] = y < n1 - 1 ? p + n0 : p - (n1 - 1) * n0;
  nb[4] = x > 0 ? p - 1 : p + n0 - 1;
  nb[5] = x < n0 - 1 ? p + 1 : p - (n0 - 1);

  const int c0 = a.cnt[p];
  int cn[6];
  int cm = c0;
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    cn[n] = a.cnt[nb[n]];
    cm = max(cm, cn[n]);
  }
  // slots in use anywhere in the wave's stencils; loops stop there
  int kmax = 0;
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (wave_any(cm > j)) kmax = j + 1;
  kmax = __builtin_amdgcn_readfirstlane(kmax);

  int ok[K];
  T ov[K];
  int nk[6][K];
  T nv[6][K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    ok[j] = kNoKey;
    ov[j] = T(0);
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      nk[n][j] = kNoKey;
      nv[n][j] = T(0);
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < kmax) {
      const size_t o = (size_t)j * V;
      if (j < c0) {
        ok[j] = a.key[o + p];
        ov[j] = a.val[o + p];
      }
#pragma unroll
      for (int n = 0; n < 6; ++n)
        if (j < cn[n]) {
          nk[n][j] = a.key[o + nb[n]];
          nv[n][j] = a.val[o + nb[n]];
        }
    }
  }

  // sum of squares, over the recrystallised and the deformed order parameters
  T s2 = T(0), R = T(0), D = T(0);
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j < kmax) {
      const T e2 = ov[j] * ov[j];
      s2 += e2;
      if (ok[j] & 1) R += e2;
      else D += e2;
    }
  // stored-energy derivatives (Eq. 14) per unit order parameter; they vanish
  // unless both kinds are present, so E is read only there
  T dfr = T(0), dfd = T(0);
  if (R > T(0) && D > T(0)) {
    const T e = a.E[p];
    const T S = R + D;
    const T S2 = S * S;
    dfr = T(-2) * e * D / S2;
    dfd = T(2) * e * R / S2;
  }

  T tv[K];
  int tk[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    tv[i] = T(0);
    tk[i] = INT_MAX;
  }
  int used = 0;

  // the point's own order parameters
#pragma unroll
  for (int i = 0; i < K; ++i) {
    if (i < kmax) {
      const T e = ov[i];
      const int q = ok[i];
      T lap = T(-6) * e;
#pragma unroll
      for (int n = 0; n < 6; ++n) {
        T w = T(0);  // value of q at neighbour n (at most one slot matches)
#pragma unroll
        for (int j = K - 1; j >= 0; --j)
          if (j < kmax) w = nk[n][j] == q ? nv[n][j] : w;
        lap += w;
      }
      const T e2 = e * e;
      const T well = e2 * e - e + T(3) * e * (s2 - e2);
      const T dF = well - T(kGrad) * lap + ((q & 1) ? dfr : dfd) * e;
      const T v = e - T(kKin) * dF;
      const bool keep = i < c0 && v > a.thr;
      if constexpr (K == 6) {
        // placed in slot order here, sorted by the network below
        tv[i] = keep ? v : T(0);
        tk[i] = keep ? q : INT_MAX;
      } else if (keep) {
        keep_largest(tv, tk, v, q);
      }
      used += keep ? 1 : 0;
    }
  }
  if constexpr (K == 6) sort6(tv, tk);
  // a candidate enters the list unless the list is full and it ranks below
  // the last entry
  auto enters = [&](T v, int q) {
    return used < K || v > tv[K - 1] || (v == tv[K - 1] && q < tk[K - 1]);
  };
  // Order parameters that diffuse in: zero here, so only the Laplacian acts.
  // The neighbour slots whose key the point lacks are appended, in neighbour
  // order, to a list of the thread's own in LDS; the first entry with a key
  // sums that key's values over the later entries (the same neighbour order
  // as a full scan), so the work scales with the few such slots of the point
  // rather than with all 6 K. A wave in which some point has more than
  // kList such slots scans all slots instead.
  __shared__ int lk[kList * kBlock];
  __shared__ T lv[kList * kBlock];
  const int tid = threadIdx.x;
  int nf = 0;
#pragma unroll
  for (int n = 0; n < 6; ++n)
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (j < kmax) {
        const int q = nk[n][j];
        bool f = j < cn[n];
#pragma unroll
        for (int i = 0; i < K; ++i)
          if (i < kmax) f = f && q != ok[i];
        if (f) {
          if (nf < kList) {
            lk[nf * kBlock + tid] = q;
            lv[nf * kBlock + tid] = nv[n][j];
          }
          ++nf;
        }
      }
  if (!wave_any(nf > kList)) {
    for (int e = 0; e < nf; ++e) {
      const int q = lk[e * kBlock + tid];
      bool first = true;
      for (int f = 0; f < e; ++f) first = first && lk[f * kBlock + tid] != q;
      if (!first) continue;
      T s = lv[e * kBlock + tid];
      for (int f = e + 1; f < nf; ++f)
        if (lk[f * kBlock + tid] == q) s += lv[f * kBlock + tid];
      const T v = T(kKin) * (T(kGrad) * s);
      if (v > a.thr) {
        if (enters(v, q)) keep_largest(tv, tk, v, q);
        ++used;
      }
    }
  } else {
#pragma unroll
    for (int n = 0; n < 6; ++n) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j < kmax) {
          const int q = nk[n][j];
          bool fresh = j < cn[n];
#pragma unroll
          for (int i = 0; i < K; ++i)
            if (i < kmax) fresh = fresh && q != ok[i];
          if (!wave_any(fresh)) continue;
#pragma unroll
          for (int m = 0; m < n; ++m)
#pragma unroll
            for (int jj = 0; jj < K; ++jj)
              if (jj < kmax) fresh = fresh && q != nk[m][jj];
          if (!wave_any(fresh)) continue;
          // value of q at the later neighbours: at most one slot each matches
          T s = nv[n][j];
#pragma unroll
          for (int m = n + 1; m < 6; ++m) {
            T w = T(0);
#pragma unroll
            for (int jj = K - 1; jj >= 0; --jj)
              if (jj < kmax) w = nk[m][jj] == q ? nv[m][jj] : w;
            s += w;
          }
          const T v = T(kKin) * (T(kGrad) * s);
          const bool cand = fresh && v > a.thr;
          if (wave_any(cand && enters(v, q))) {
            if (cand) keep_largest(tv, tk, v, q);
          }
          used += cand ? 1 : 0;
        }
      }
    }
  }

  if (live) {
    const int cnew = min(used, K);
    a.cnt_out[p] = (unsigned char)cnew;
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (i < cnew) {
        a.key_out[(size_t)i * V + p] = tk[i];
        a.val_out[(size_t)i * V + p] = tv[i];
      }
  }
}

// Range checks of refine's inputs: grain ids in [-2^30, 2^30), finite energy.
__global__ __launch_bounds__(kBlock) void k_pf_check_coarse(const int* grain, const double* E, int V,
                                                            int* flag) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= V) return;
  const int g = grain[p];
  if (g < -(1 << 30) || g >= (1 << 30) || !isfinite(E[p])) atomicOr(flag, 1);
}

// 2:1 refinement (Sec. 2.4): the grain of the mechanical point, and the
// stored energy interpolated linearly along z, then y, then x (periodic).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pf_refine(const int* grain, const double* Ec, int n0,
                                                      int n1, int n2, unsigned char* cnt, int* key,
                                                      T* val, T* E) {
  const int N0 = 2 * n0, N1 = 2 * n1, N2 = 2 * n2;
  const int Vf = N0 * N1 * N2;
  const int p = tile_base() + (int)threadIdx.x;
  if (p >= Vf) return;
  const int X = p % N0, Y = (p / N0) % N1, Z = p / (N0 * N1);
  const int xc = X >> 1, yc = Y >> 1, zc = Z >> 1;
  const int g = grain[(zc * n1 + yc) * n0 + xc];
  cnt[p] = 1;
  key[p] = 2 * g + (g < 0 ? 1 : 0);
  val[p] = T(1);
  const int xs[2] = {xc, xc + 1 < n0 ? xc + 1 : 0};
  const int ys[2] = {yc, yc + 1 < n1 ? yc + 1 : 0};
  const int zs[2] = {zc, zc + 1 < n2 ? zc + 1 : 0};
  const bool ox = X & 1, oy = Y & 1, oz = Z & 1;
  double b[2];
#pragma unroll
  for (int dx = 0; dx < 2; ++dx) {
    double a2[2];
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const double f0 = Ec[((size_t)zs[0] * n1 + ys[dy]) * n0 + xs[dx]];
      const double f1 = Ec[((size_t)zs[1] * n1 + ys[dy]) * n0 + xs[dx]];
      a2[dy] = oz ? 0.5 * (f0 + f1) : f0;
    }
    b[dx] = oy ? 0.5 * (a2[0] + a2[1]) : a2[0];
  }
  E[p] = (T)(ox ? 0.5 * (b[0] + b[1]) : b[0]);
}

// Checks of import's inputs (the same "used" test as the import itself).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pf_check_import(const int* keys, const double* vals, int kin,
                                                            const double* E, int Vf, T thr, int* flag) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= Vf) return;
  bool bad = !isfinite(E[p]);
  for (int j = 0; j < kin; ++j) {
    const double v = vals[(size_t)j * Vf + p];
    if (!isfinite(v)) bad = true;
    if (!((T)v > thr)) continue;
    const int k = keys[(size_t)j * Vf + p];
    if (k == kNoKey) bad = true;
    for (int i = 0; i < j; ++i)
      if ((T)vals[(size_t)i * Vf + p] > thr && keys[(size_t)i * Vf + p] == k) bad = true;
  }
  if (bad) atomicOr(flag, 1);
}

template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_pf_import(const int* keys, const double* vals, int kin,
                                                      const double* Ein, int Vf, T thr,
                                                      unsigned char* cnt, int* key, T* val, T* E) {
  const int p = tile_base() + (int)threadIdx.x;
  if (p >= Vf) return;
  T tv[K];
  int tk[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    tv[i] = T(0);
    tk[i] = INT_MAX;
  }
  int used = 0;
  for (int j = 0; j < kin; ++j) {
    const T v = (T)vals[(size_t)j * Vf + p];
    if (v > thr) {
      keep_largest(tv, tk, v, keys[(size_t)j * Vf + p]);
      ++used;
    }
  }
  const int c = min(used, K);
  cnt[p] = (unsigned char)c;
#pragma unroll
  for (int i = 0; i < K; ++i)
    if (i < c) {
      key[(size_t)i * Vf + p] = tk[i];
      val[(size_t)i * Vf + p] = tv[i];
    }
  E[p] = (T)Ein[p];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pf_export(const unsigned char* cnt, const int* key,
                                                      const T* val, int K, int Vf, int* kout,
                                                      double* vout) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= Vf) return;
  const int c = cnt[p];
  for (int j = 0; j < K; ++j) {
    const size_t o = (size_t)j * Vf + p;
    kout[o] = j < c ? key[o] : kNoKey;
    vout[o] = j < c ? (double)val[o] : 0.0;
  }
}

// Mechanical point i takes the grain of slot 0 (the largest) at PF point 2i.
__global__ __launch_bounds__(kBlock) void k_pf_grains(const unsigned char* cnt, const int* key, int n0,
                                                      int n1, int n2, const int* before, int* out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n0 * n1 * n2) return;
  const int x = i % n0, y = (i / n0) % n1, z = i / (n0 * n1);
  const int p = ((2 * z) * (2 * n1) + 2 * y) * (2 * n0) + 2 * x;
  const int g0 = before[i];
  out[i] = cnt[p] > 0 ? (key[p] >> 1) : g0;
}

}  // namespace

struct fftevp_pf {
  int n0 = 0, n1 = 0, n2 = 0;  // mechanical grid
  int V = 0, Vf = 0;
  int K = 0;
  double thr = 0.0;
  fftevp_precision prec = FFTEVP_FP64;
  size_t ts = 8;
  hipStream_t stream = nullptr;
  unsigned char* cnt[2] = {};
  int* key[2] = {};
  void* val[2] = {};
  void* E = nullptr;
  int* flag = nullptr;
  int cur = 0;
  bool have = false;
  std::string err;
};

namespace {

fftevp_status pf_fail(fftevp_pf* pf, fftevp_status s, const std::string& m) {
  if (pf) pf->err = m;
  return s;
}

fftevp_status pf_hip(fftevp_pf* pf, hipError_t e, const char* what) {
  return pf_fail(pf, FFTEVP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define PFCHK(call)                                   \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return pf_hip(pf, e_, #call); \
  } while (0)

int nblocks(int n) { return (n + kBlock - 1) / kBlock; }

// Clear the flag, run a check launch, read the flag back.
template <typename F>
fftevp_status checked(fftevp_pf* pf, F&& launch, int* bad) {
  PFCHK(hipMemsetAsync(pf->flag, 0, sizeof(int), pf->stream));
  launch();
  PFCHK(hipGetLastError());
  PFCHK(hipMemcpyAsync(bad, pf->flag, sizeof(int), hipMemcpyDeviceToHost, pf->stream));
  PFCHK(hipStreamSynchronize(pf->stream));
  return FFTEVP_OK;
}

template <typename T, int K>
void launch_step(fftevp_pf* pf) {
  StepArgs<T> a;
  const int c = pf->cur, o = 1 - c;
  a.cnt = pf->cnt[c];
  a.key = pf->key[c];
  a.val = (const T*)pf->val[c];
  a.E = (const T*)pf->E;
  a.cnt_out = pf->cnt[o];
  a.key_out = pf->key[o];
  a.val_out = (T*)pf->val[o];
  a.n0 = 2 * pf->n0;
  a.n1 = 2 * pf->n1;
  a.n2 = 2 * pf->n2;
  a.V = pf->Vf;
  a.thr = (T)pf->thr;
  hipLaunchKernelGGL((k_pf_step<T, K>), dim3(nblocks(pf->Vf)), dim3(kBlock), 0, pf->stream, a);
}

template <typename T, int K>
void launch_import(fftevp_pf* pf, const int* keys, const double* vals, int kin, const double* E) {
  hipLaunchKernelGGL((k_pf_import<T, K>), dim3(nblocks(pf->Vf)), dim3(kBlock), 0, pf->stream, keys, vals,
                     kin, E, pf->Vf, (T)pf->thr, pf->cnt[pf->cur], pf->key[pf->cur], (T*)pf->val[pf->cur],
                     (T*)pf->E);
}

// K as a template argument: the register lists of the step are sized by it.
template <typename T, template <typename, int> class Fn, typename... A>
void by_k(int K, A&&... args) {
  switch (K) {
    case 1: Fn<T, 1>::run(args...); break;
    case 2: Fn<T, 2>::run(args...); break;
    case 3: Fn<T, 3>::run(args...); break;
    case 4: Fn<T, 4>::run(args...); break;
    case 5: Fn<T, 5>::run(args...); break;
    default: Fn<T, 6>::run(args...); break;
  }
}

template <typename T, int K>
struct StepFn {
  static void run(fftevp_pf* pf) { launch_step<T, K>(pf); }
};
template <typename T, int K>
struct ImportFn {
  static void run(fftevp_pf* pf, const int* k, const double* v, int kin, const double* E) {
    launch_import<T, K>(pf, k, v, kin, E);
  }
};

void release(fftevp_pf* pf) {
  for (int i = 0; i < 2; ++i) {
    if (pf->cnt[i]) (void)hipFree(pf->cnt[i]);
    if (pf->key[i]) (void)hipFree(pf->key[i]);
    if (pf->val[i]) (void)hipFree(pf->val[i]);
  }
  if (pf->E) (void)hipFree(pf->E);
  if (pf->flag) (void)hipFree(pf->flag);
}

}  // namespace

extern "C" {

fftevp_status fftevp_pf_create(int n0, int n1, int n2, int K, double threshold, int precision, void* stream,
                               fftevp_pf** out) {
  if (!out) return FFTEVP_EINVAL;
  *out = nullptr;
  if (n0 < 1 || n1 < 1 || n2 < 1) return FFTEVP_EINVAL;
  const long long vf = 8LL * n0 * n1 * n2;
  if (vf >= (1LL << 31)) return FFTEVP_EINVAL;
  if (K < 1 || K > FFTEVP_PF_KMAX) return FFTEVP_EINVAL;
  if (!(threshold >= 0.0 && threshold < 1.0)) return FFTEVP_EINVAL;
  if (precision != FFTEVP_FP64 && precision != FFTEVP_MIXED) return FFTEVP_EINVAL;
  fftevp_pf* pf = new fftevp_pf;
  pf->n0 = n0;
  pf->n1 = n1;
  pf->n2 = n2;
  pf->V = n0 * n1 * n2;
  pf->Vf = (int)vf;
  pf->K = K;
  pf->thr = threshold;
  pf->prec = (fftevp_precision)precision;
  pf->ts = precision == FFTEVP_FP64 ? 8 : 4;
  pf->stream = (hipStream_t)stream;
  const size_t Vf = (size_t)vf;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipMalloc((void**)&pf->cnt[i], Vf);
    if (e == hipSuccess) e = hipMalloc((void**)&pf->key[i], (size_t)K * Vf * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&pf->val[i], (size_t)K * Vf * pf->ts);
  }
  if (e == hipSuccess) e = hipMalloc(&pf->E, Vf * pf->ts);
  if (e == hipSuccess) e = hipMalloc((void**)&pf->flag, sizeof(int));
  if (e != hipSuccess) {
    release(pf);
    delete pf;
    (void)hipGetLastError();
    return FFTEVP_ENOMEM;
  }
  *out = pf;
  return FFTEVP_OK;
}

fftevp_status fftevp_pf_destroy(fftevp_pf* pf) {
  if (!pf) return FFTEVP_EINVAL;
  if (pf->stream) (void)hipStreamSynchronize(pf->stream);
  else (void)hipDeviceSynchronize();
  release(pf);
  delete pf;
  return FFTEVP_OK;
}

fftevp_status fftevp_pf_refine(fftevp_pf* pf, const int* grain_dev, const double* estore_dev) {
  if (!pf) return FFTEVP_EINVAL;
  if (!grain_dev || !estore_dev) return pf_fail(pf, FFTEVP_EINVAL, "null argument");
  int bad = 0;
  fftevp_status s = checked(
      pf,
      [&] {
        hipLaunchKernelGGL(k_pf_check_coarse, dim3(nblocks(pf->V)), dim3(kBlock), 0, pf->stream, grain_dev,
                           estore_dev, pf->V, pf->flag);
      },
      &bad);
  if (s != FFTEVP_OK) return s;
  if (bad) return pf_fail(pf, FFTEVP_EINVAL, "grain id outside [-2^30, 2^30) or stored energy not finite");
  const int c = pf->cur;
  if (pf->prec == FFTEVP_FP64)
    hipLaunchKernelGGL(k_pf_refine<double>, dim3(nblocks(pf->Vf)), dim3(kBlock), 0, pf->stream, grain_dev,
                       estore_dev, pf->n0, pf->n1, pf->n2, pf->cnt[c], pf->key[c], (double*)pf->val[c],
                       (double*)pf->E);
  else
    hipLaunchKernelGGL(k_pf_refine<float>, dim3(nblocks(pf->Vf)), dim3(kBlock), 0, pf->stream, grain_dev,
                       estore_dev, pf->n0, pf->n1, pf->n2, pf->cnt[c], pf->key[c], (float*)pf->val[c],
                       (float*)pf->E);
  PFCHK(hipGetLastError());
  pf->have = true;
  return FFTEVP_OK;
}

fftevp_status fftevp_pf_import(fftevp_pf* pf, const int* keys_dev, const double* vals_dev, int kin,
                               const double* estore_dev) {
  if (!pf) return FFTEVP_EINVAL;
  if (!keys_dev || !vals_dev || !estore_dev) return pf_fail(pf, FFTEVP_EINVAL, "null argument");
  if (kin < 1 || kin > 64) return pf_fail(pf, FFTEVP_EINVAL, "kin must be in 1..64");
  int bad = 0;
  const bool d = pf->prec == FFTEVP_FP64;
  fftevp_status s = checked(
      pf,
      [&] {
        if (d)
          hipLaunchKernelGGL(k_pf_check_import<double>, dim3(nblocks(pf->Vf)), dim3(kBlock), 0, pf->stream,
                             keys_dev, vals_dev, kin, estore_dev, pf->Vf, pf->thr, pf->flag);
        else
          hipLaunchKernelGGL(k_pf_check_import<float>, dim3(nblocks(pf->Vf)), dim3(kBlock), 0, pf->stream,
                             keys_dev, vals_dev, kin, estore_dev, pf->Vf, (float)pf->thr, pf->flag);
      },
      &bad);
  if (s != FFTEVP_OK) return s;
  if (bad) return pf_fail(pf, FFTEVP_EINVAL, "duplicate or reserved key, or a value that is not finite");
  if (d) by_k<double, ImportFn>(pf->K, pf, keys_dev, vals_dev, kin, estore_dev);
  else by_k<float, ImportFn>(pf->K, pf, keys_dev, vals_dev, kin, estore_dev);
  PFCHK(hipGetLastError());
  pf->have = true;
  return FFTEVP_OK;
}

fftevp_status fftevp_pf_steps(fftevp_pf* pf, int nsteps) {
  if (!pf) return FFTEVP_EINVAL;
  if (nsteps < 0) return pf_fail(pf, FFTEVP_EINVAL, "nsteps < 0");
  if (!pf->have) return pf_fail(pf, FFTEVP_ESTATE, "no state: call fftevp_pf_refine or fftevp_pf_import");
  for (int i = 0; i < nsteps; ++i) {
    if (pf->prec == FFTEVP_FP64) by_k<double, StepFn>(pf->K, pf);
    else by_k<float, StepFn>(pf->K, pf);
    PFCHK(hipGetLastError());
    pf->cur = 1 - pf->cur;
  }
  return FFTEVP_OK;
}

fftevp_status fftevp_pf_export(fftevp_pf* pf, int* keys_dev, double* vals_dev) {
  if (!pf) return FFTEVP_EINVAL;
  if (!keys_dev || !vals_dev) return pf_fail(pf, FFTEVP_EINVAL, "null argument");
  if (!pf->have) return pf_fail(pf, FFTEVP_ESTATE, "no state");
  const int c = pf->cur;
  if (pf->prec == FFTEVP_FP64)
    hipLaunchKernelGGL(k_pf_export<double>, dim3(nblocks(pf->Vf)), dim3(kBlock), 0, pf->stream, pf->cnt[c],
                       pf->key[c], (const double*)pf->val[c], pf->K, pf->Vf, keys_dev, vals_dev);
  else
    hipLaunchKernelGGL(k_pf_export<float>, dim3(nblocks(pf->Vf)), dim3(kBlock), 0, pf->stream, pf->cnt[c],
                       pf->key[c], (const float*)pf->val[c], pf->K, pf->Vf, keys_dev, vals_dev);
  PFCHK(hipGetLastError());
  return FFTEVP_OK;
}

fftevp_status fftevp_pf_grains(fftevp_pf* pf, const int* grain_before_dev, int* grain_out_dev) {
  if (!pf) return FFTEVP_EINVAL;
  if (!grain_before_dev || !grain_out_dev) return pf_fail(pf, FFTEVP_EINVAL, "null argument");
  if (!pf->have) return pf_fail(pf, FFTEVP_ESTATE, "no state");
  const int c = pf->cur;
  hipLaunchKernelGGL(k_pf_grains, dim3(nblocks(pf->V)), dim3(kBlock), 0, pf->stream, pf->cnt[c], pf->key[c],
                     pf->n0, pf->n1, pf->n2, grain_before_dev, grain_out_dev);
  PFCHK(hipGetLastError());
  return FFTEVP_OK;
}

fftevp_status fftevp_pf_dims(const fftevp_pf* pf, int* n0, int* n1, int* n2) {
  if (!pf || !n0 || !n1 || !n2) return FFTEVP_EINVAL;
  *n0 = pf->n0;
  *n1 = pf->n1;
  *n2 = pf->n2;
  return FFTEVP_OK;
}

int fftevp_pf_step_count(double dt, double omega_gb, double mobility) {
  if (!(std::isfinite(dt) && dt > 0.0 && std::isfinite(omega_gb) && omega_gb > 0.0 &&
        std::isfinite(mobility) && mobility > 0.0))
    return -1;
  const double n = std::floor(dt / (0.225 * omega_gb / mobility));
  return n < 2147483647.0 ? (int)n : -1;
}

const char* fftevp_pf_last_error(const fftevp_pf* pf) { return pf ? pf->err.c_str() : "null context"; }

}  // extern "C"
