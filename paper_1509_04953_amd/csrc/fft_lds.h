// Batched power-of-two complex FFTs on lines held in LDS (gfx950).
//
// Each stage is a Stockham autosort radix-R pass (natural order in and out):
// every thread loads its butterflies' inputs into registers, the block
// synchronises, then the thread applies twiddles, the in-register radix-R
// DFT and writes the outputs back to the same LDS buffer. Reading everything
// before any write lets one buffer serve as both source and destination.
// Twiddles come from a table w[m] = exp(-2 pi i m / N), m in [0, N), built on
// the host in extended precision. Forward transforms are unnormalised; the
// inverse uses conjugate twiddles and is unnormalised too.
#pragma once
#include <hip/hip_runtime.h>

namespace fftevp {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  if constexpr (INV) return {-a.y, a.x};
  else return {a.y, -a.x};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
  cx<T> t2 = v[1] + v[3], t3 = rot90<T, INV>(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
  const T h = T(0.70710678118654752440);
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  // o[k] *= exp(-+ i pi k / 4)
  cx<T> o1, o3;
  if constexpr (INV) {
    o1 = {h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)};
    o3 = {-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)};
  } else {
    o1 = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
    o3 = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
  }
  cx<T> o2 = rot90<T, INV>(o[2]);
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

// o * exp(-+ 2 pi i k / 16) for a compile-time k in [1, 8)
template <typename T, bool INV, int K>
__device__ __forceinline__ cx<T> w16(cx<T> o) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
  constexpr double h = 0.70710678118654752440;
  if constexpr (K == 4) {
    return rot90<T, INV>(o);
  } else if constexpr (K == 2 || K == 6) {
    // (1 -+ i) h or (-1 -+ i) h
    const T a = T(h) * (o.x + (INV ? -o.y : o.y)), b = T(h) * (o.y - (INV ? -o.x : o.x));
    if constexpr (K == 2) return {a, b};
    else return INV ? cx<T>{-b, a} : cx<T>{b, -a};  // times -+ i
  } else {
    constexpr double cr = K == 1 ? c1 : (K == 3 ? s1 : (K == 5 ? -s1 : -c1));
    constexpr double ci = K == 1 ? -s1 : (K == 3 ? -c1 : (K == 5 ? -c1 : -s1));
    const cx<T> w = {T(cr), T(INV ? -ci : ci)};
    return cmul(o, w);
  }
}

// 16-point DFT: two 8-point DFTs of the even and odd elements and one
// radix-2 combination with the 16th roots of unity.
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cx<T>* v) {
  cx<T> e[8], o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e[k] = v[2 * k];
    o[k] = v[2 * k + 1];
  }
  dft8<T, INV>(e);
  dft8<T, INV>(o);
  const cx<T> t[8] = {o[0], w16<T, INV, 1>(o[1]), w16<T, INV, 2>(o[2]), w16<T, INV, 3>(o[3]),
                      w16<T, INV, 4>(o[4]), w16<T, INV, 5>(o[5]), w16<T, INV, 6>(o[6]), w16<T, INV, 7>(o[7])};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = e[k] + t[k];
    v[k + 8] = e[k] - t[k];
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else dft16<T, INV>(v);
}

// One Stockham stage over LINES lines of length N (line stride LS, unit
// element stride) with NT cooperating threads. Thread order: line-major
// (consecutive threads take the same butterfly of consecutive lines, so with
// an odd line stride their LDS accesses spread over the banks in every
// stage) for FP64 and for many lines; butterfly-major (unit-stride reads,
// R-strided writes) for a few FP32 lines, where it measured faster.
template <typename T, int N, int R, int NS, bool INV, int LINES, int LS, int NT>
__device__ __forceinline__ void stockham_stage(cx<T>* __restrict__ buf,
                                               const cx<T>* __restrict__ tw) {
  constexpr int BF = N / R;
  constexpr int TOTAL = LINES * BF;
  constexpr int PER = (TOTAL + NT - 1) / NT;
  constexpr bool LM = sizeof(T) == 8 || LINES >= 32;
  cx<T> v[PER][R];
  cx<T> wt[PER][R > 1 && NS > 1 ? R - 1 : 1];
  const int tid = threadIdx.x;
  // inputs and twiddles are requested before the barrier, so the twiddle
  // loads (cached table) overlap the wait for the other waves
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = tid + b * NT;
    if ((TOTAL % NT) == 0 || idx < TOTAL) {
      const int line = LM ? idx % LINES : idx / BF, j = LM ? idx / LINES : idx % BF;
      const cx<T>* src = buf + line * LS + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = src[r * BF];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) wt[b][r - 1] = tw[k * r * (N / (NS * R))];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = tid + b * NT;
    if ((TOTAL % NT) == 0 || idx < TOTAL) {
      const int line = LM ? idx % LINES : idx / BF, j = LM ? idx / LINES : idx % BF;
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r)
          v[b][r] = INV ? cmulc(v[b][r], wt[b][r - 1]) : cmul(v[b][r], wt[b][r - 1]);
      }
      dftR<T, R, INV>(v[b]);
      cx<T>* dst = buf + line * LS + (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * NS] = v[b][r];
    }
  }
  __syncthreads();
}

// radix plan: 16 where it leaves a factor of at least 8 (or is the whole
// transform), else 8s, then a final 4 or 2:
// 16 -> 16, 32 -> 8x4, 64 -> 8x8, 128 -> 16x8, 256 -> 16x16, 512 -> 8x8x8
__host__ __device__ constexpr int radix_at(int n, int ns) {
  const int rem = n / ns;
  return (rem == 16 || rem == 128 || rem == 256) ? 16 : (rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : 2));
}
// NS of the plan's last stage (1 for a one-stage plan)
__host__ __device__ constexpr int last_stage_ns(int n) {
  int ns = 1;
  while (ns * radix_at(n, ns) < n) ns *= radix_at(n, ns);
  return ns;
}

// the stages of the plan from NS up to (not including) the one at STOP
template <typename T, int N, int NS, int STOP, bool INV, int LINES, int LS, int NT>
__device__ __forceinline__ void fft_stages(cx<T>* buf, const cx<T>* tw) {
  if constexpr (NS < STOP) {
    constexpr int R = radix_at(N, NS);
    stockham_stage<T, N, R, NS, INV, LINES, LS, NT>(buf, tw);
    fft_stages<T, N, NS * R, STOP, INV, LINES, LS, NT>(buf, tw);
  }
}

// P complex values of row `row` at column w (P = 2: one 16-byte FP32 access)
template <typename T, int P>
__device__ __forceinline__ void load_row(const cx<T>* __restrict__ p, cx<T> (&o)[P]) {
  if constexpr (P == 2) {
    static_assert(sizeof(T) == 4, "pairs are FP32");
    const float4 f = *reinterpret_cast<const float4*>(p);
    o[0] = {f.x, f.y};
    o[1] = {f.z, f.w};
  } else {
    o[0] = p[0];
  }
}
template <typename T, int P>
__device__ __forceinline__ void store_row(cx<T>* __restrict__ p, const cx<T> (&o)[P]) {
  if constexpr (P == 2) {
    *reinterpret_cast<float4*>(p) = make_float4(o[0].x, o[0].y, o[1].x, o[1].y);
  } else {
    p[0] = o[0];
  }
}

// First stage of the plan (NS = 1, no twiddles) read straight from global
// rows: row i of a tile holds element i of its W lines (row stride rs, W
// contiguous complex values, P lines per thread). Thread (column w, butterfly
// j) loads rows j + r N/R, applies the radix-R DFT and writes the outputs to
// LDS line w at j R + r (line stride LS). Consecutive threads take
// neighbouring columns, so each load covers whole rows. Ends with a barrier.
template <typename T, int N, int W, bool INV, int LS, int NT, int P>
__device__ __forceinline__ void first_stage_from_rows(const cx<T>* __restrict__ src, size_t rs,
                                                      cx<T>* sh) {
  constexpr int R = radix_at(N, 1);
  constexpr int BF = N / R;
  constexpr int WP = W / P;
  constexpr int TOTAL = WP * BF;
  constexpr int PER = (TOTAL + NT - 1) / NT;
  static_assert(W % P == 0, "whole pairs");
  cx<T> v[PER][P][R];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + b * NT;
    if ((TOTAL % NT) == 0 || idx < TOTAL) {
      const int w = (idx % WP) * P, j = idx / WP;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cx<T> o[P];
        load_row<T, P>(src + (size_t)(j + r * BF) * rs + w, o);
#pragma unroll
        for (int p = 0; p < P; ++p) v[b][p][r] = o[p];
      }
    }
  }
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + b * NT;
    if ((TOTAL % NT) == 0 || idx < TOTAL) {
      const int w = (idx % WP) * P, j = idx / WP;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        dftR<T, R, INV>(v[b][p]);
        cx<T>* dst = sh + (w + p) * LS + j * R;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r] = v[b][p][r];
      }
    }
  }
  __syncthreads();
}

// Last stage of the plan (NS = N / R) written straight to global rows:
// thread (column w, butterfly j) reads inputs j + r NS of LDS line w,
// applies the twiddles and the radix-R DFT and stores output r (element
// j + r NS) to that row. The stage before must have ended with a barrier. A
// one-stage plan (NS = 1) makes this the whole transform.
template <typename T, int N, int W, bool INV, int LS, int NT, int P>
__device__ __forceinline__ void last_stage_to_rows(const cx<T>* sh, const cx<T>* __restrict__ tw,
                                                   cx<T>* __restrict__ dst, size_t rs) {
  constexpr int NSL = last_stage_ns(N);
  constexpr int R = N / NSL;
  constexpr int WP = W / P;
  constexpr int TOTAL = WP * NSL;
  constexpr int PER = (TOTAL + NT - 1) / NT;
  static_assert(W % P == 0, "whole pairs");
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int idx = threadIdx.x + b * NT;
    if ((TOTAL % NT) == 0 || idx < TOTAL) {
      const int w = (idx % WP) * P, j = idx / WP;
      cx<T> v[P][R];
      cx<T> wt[R > 1 && NSL > 1 ? R - 1 : 1];
      if constexpr (NSL > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) wt[r - 1] = tw[j * r];
      }
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = sh[(w + p) * LS + j + r * NSL];
      }
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if constexpr (NSL > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r)
            v[p][r] = INV ? cmulc(v[p][r], wt[r - 1]) : cmul(v[p][r], wt[r - 1]);
        }
        dftR<T, R, INV>(v[p]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cx<T> o[P];
#pragma unroll
        for (int p = 0; p < P; ++p) o[p] = v[p][r];
        store_row<T, P>(dst + (size_t)(j + r * NSL) * rs + w, o);
      }
    }
  }
}

// In-place FFT of LINES lines of length N held in LDS (line stride LS).
// Must be called by all NT threads of the block; ends with a barrier.
template <typename T, int N, bool INV, int LINES, int LS, int NT>
__device__ __forceinline__ void fft_lines(cx<T>* buf, const cx<T>* __restrict__ tw) {
  fft_stages<T, N, 1, N, INV, LINES, LS, NT>(buf, tw);
}

}  // namespace fftevp
