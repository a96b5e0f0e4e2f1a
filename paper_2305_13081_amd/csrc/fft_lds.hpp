// LDS-staged Stockham autosort FFT for gfx950 (64-lane wavefronts).
//
// A workgroup transforms NSIG contiguous signals of length N held in LDS.
// Each stage of radix R reads R strided values per butterfly, applies the
// twiddles exp(-2 pi i k r / (Ns R)) (k = position inside the current
// sub-transform of length Ns), runs an R-point DFT in registers and writes
// the results to their self-sorted positions (j / Ns) * Ns * R + k + r * Ns.
// The transform is in place: every thread loads all of its butterflies into
// registers, the workgroup synchronises, then stores.  The twiddle of r = 1
// comes from a per-length table tw[t] = exp(-2 pi i t / N) built once on the
// host in FP64; its powers r = 2 .. R-1 are formed by complex products in
// registers (one table load per butterfly instead of R - 1: the loads compete
// with the streaming traffic of the passes, the products are cheap; the
// error of w^r grows by about one rounding per product).
//
// Radix plans for N = 3^a 2^b, the 3s first.  Plan 0: radix 8, with 8*2 ->
// 4*4 and a single trailing 4 so that no radix-2 pass is needed for b >= 2.
// Plan 1: radix 16 where it fits (16*2 -> 8*4, then a trailing 8 or 4), one
// LDS round trip and barrier pair fewer per four factors of 2 at the cost of
// fewer, larger butterflies per stage.  Which is faster depends on the pass
// and its signals per block, so the row and column passes take the plan as a
// template parameter and the mechanics passes time both (autotuner).
#pragma once
#include <hip/hip_runtime.h>

namespace fgcg {

template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C cmul_mi(C a) {
  return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

// LDS index of complex element i: one 16-byte pad per 8 elements.  With it the
// R-strided Stockham writes of the first stages (lane l writes 8 l + r, or
// 64 (l / 8) + l % 8 + 8 r) land on 8 distinct 16-byte bank groups for every
// 8 consecutive lanes, and contiguous accesses stay conflict-free.
__device__ __forceinline__ int lds(int i) { return i + (i >> 3); }
constexpr int lds_size(int n) { return n + n / 8 + 1; }

// LDS position of element x of signal sig.  FlatIdx: the signals back to back
// in one padded array (lds(sig N + x)).  PitchIdx: signals P apart with P odd,
// so that the 16 (FP64) or 32 (FP32) lanes that write element x of
// consecutive signals (a transposing load) hit distinct banks.
template <int N> struct FlatIdx {
  static __device__ __forceinline__ int at(int sig, int x) { return lds(sig * N + x); }
};
constexpr int pitch_for(int n) { return (n + n / 8) | 1; }
template <int N> struct PitchIdx {
  static __device__ __forceinline__ int at(int sig, int x) { return sig * pitch_for(N) + lds(x); }
};

// ---------------------------------------------------------------- radix plan
constexpr int count3(int n) { return n % 3 == 0 ? 1 + count3(n / 3) : 0; }
constexpr int pow3(int a) { return a == 0 ? 1 : 3 * pow3(a - 1); }
constexpr int log2i(int n) { return n <= 1 ? 0 : 1 + log2i(n / 2); }

struct Plan {
  int n;
  int nst;
  int r[16];
};

constexpr Plan make_plan(int N, int P = 0) {
  Plan p{N, 0, {0}};
  int a = count3(N);
  int b = log2i(N / pow3(a));
  for (int i = 0; i < a; ++i) p.r[p.nst++] = 3;
  if (P == 1 && b >= 4) {
    int n16 = b / 4, rem = b % 4;
    int tail[2] = {0, 0}, nt = 0;
    if (rem == 1) {
      n16 -= 1;
      tail[nt++] = 8;
      tail[nt++] = 4;
    } else if (rem == 2) {
      tail[nt++] = 4;
    } else if (rem == 3) {
      tail[nt++] = 8;
    }
    for (int i = 0; i < n16; ++i) p.r[p.nst++] = 16;
    for (int i = 0; i < nt; ++i) p.r[p.nst++] = tail[i];
    return p;
  }
  int n8 = b / 3, rem = b % 3;
  int n4 = 0, n2 = 0;
  if (rem == 2) n4 = 1;
  if (rem == 1) {
    if (n8 > 0) { n8 -= 1; n4 = 2; } else { n2 = 1; }
  }
  for (int i = 0; i < n8; ++i) p.r[p.nst++] = 8;
  for (int i = 0; i < n4; ++i) p.r[p.nst++] = 4;
  for (int i = 0; i < n2; ++i) p.r[p.nst++] = 2;
  return p;
}

constexpr bool fft_size_ok(int N) {
  return N >= 2 && (N / pow3(count3(N))) * pow3(count3(N)) == N &&
         ((N / pow3(count3(N))) & ((N / pow3(count3(N))) - 1)) == 0;
}

// ----------------------------------------------------------- small DFTs
template <int R, bool INV, typename T> struct Dft;

template <bool INV, typename T> struct Dft<2, INV, T> {
  using C = typename cvec<T>::type;
  static __device__ __forceinline__ void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV, typename T> struct Dft<3, INV, T> {
  using C = typename cvec<T>::type;
  static __device__ __forceinline__ void run(C* v) {
    const T s = (T)0.86602540378443864676372317075294;  // sin(2 pi / 3)
    C a0 = v[0], a1 = v[1], a2 = v[2];
    C sum = cadd(a1, a2);
    C dif = csub(a1, a2);
    C t = C{a0.x - (T)0.5 * sum.x, a0.y - (T)0.5 * sum.y};
    // forward: -i s (a1 - a2); inverse: +i s (a1 - a2)
    C u = cmul_mi<INV>(C{s * dif.x, s * dif.y});
    v[0] = cadd(a0, sum);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
  }
};

template <bool INV, typename T> struct Dft<4, INV, T> {
  using C = typename cvec<T>::type;
  static __device__ __forceinline__ void run(C* v) {
    C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    C s13 = cadd(v[1], v[3]), d13 = cmul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  }
};

template <bool INV, typename T> struct Dft<8, INV, T> {
  using C = typename cvec<T>::type;
  static __device__ __forceinline__ void run(C* v) {
    const T r2 = (T)0.70710678118654752440084436210485;
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV, T>::run(e);
    Dft<4, INV, T>::run(o);
    // o[k] *= exp(-+ 2 pi i k / 8)
    C o1 = o[1], o3 = o[3];
    if (!INV) {
      o[1] = C{r2 * (o1.x + o1.y), r2 * (o1.y - o1.x)};
      o[3] = C{r2 * (o3.y - o3.x), -r2 * (o3.x + o3.y)};
    } else {
      o[1] = C{r2 * (o1.x - o1.y), r2 * (o1.x + o1.y)};
      o[3] = C{-r2 * (o3.x + o3.y), r2 * (o3.x - o3.y)};
    }
    o[2] = cmul_mi<INV>(o[2]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

// 16 points as 4 x 4: DFT-4 over n1 for each n2, twiddle W16^(n2 k1), DFT-4
// over n2; output k1 + 4 k2.  W16^m = (cos, -+sin)(2 pi m / 16).
template <bool INV, typename T> struct Dft<16, INV, T> {
  using C = typename cvec<T>::type;
  static __device__ __forceinline__ C tw16(C a, int m) {
    const T c1 = (T)0.92387953251128675612818318939679;  // cos(pi / 8)
    const T s1 = (T)0.38268343236508977172845998403040;  // sin(pi / 8)
    const T r2 = (T)0.70710678118654752440084436210485;
    // forward multiplies by (c, -s); inverse by (c, +s)
    auto rot = [&](T c, T sn) {
      const T ss = INV ? sn : -sn;
      return C{a.x * c - a.y * ss, a.x * ss + a.y * c};
    };
    switch (m) {
      case 1: return rot(c1, s1);
      case 2: return INV ? C{r2 * (a.x - a.y), r2 * (a.x + a.y)} : C{r2 * (a.x + a.y), r2 * (a.y - a.x)};
      case 3: return rot(s1, c1);
      case 4: return cmul_mi<INV>(a);
      case 6: return INV ? C{-r2 * (a.x + a.y), r2 * (a.x - a.y)} : C{r2 * (a.y - a.x), -r2 * (a.x + a.y)};
      case 9: return rot(-c1, -s1);
      default: return a;
    }
  }
  static __device__ __forceinline__ void run(C* v) {
    C y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      C t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<4, INV, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = tw16(t[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<4, INV, T>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// ------------------------------------------------------------ one stage
template <typename T, int N, int R, int NS, int NSIG, int NT, bool INV, class Idx>
__device__ __forceinline__ void stockham_stage(typename cvec<T>::type* buf,
                                               const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  constexpr int M = N / R;
  constexpr int TOT = NSIG * M;
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr int TSTEP = N / (NS * R);
  C v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if (TOT % NT == 0 || b < TOT) {
      const int sig = b / M, j = b - sig * M;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[Idx::at(sig, j + r * M)];
      if (NS > 1) {
        const int k = j % NS;
        C w1 = tw[k * TSTEP];
        if (INV) w1.y = -w1.y;
        C w = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[q][r] = cmul(v[q][r], w);
          if (r + 1 < R) w = cmul(w, w1);
        }
      }
      Dft<R, INV, T>::run(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if (TOT % NT == 0 || b < TOT) {
      const int sig = b / M, j = b - sig * M;
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[Idx::at(sig, base + r * NS)] = v[q][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int NSIG, int NT, bool INV, int ST, int NS, class Idx, int P>
struct StageRunner {
  static __device__ __forceinline__ void run(typename cvec<T>::type* buf,
                                             const typename cvec<T>::type* __restrict__ tw) {
    constexpr Plan p = make_plan(N, P);
    if constexpr (ST < p.nst) {
      constexpr int R = p.r[ST];
      stockham_stage<T, N, R, NS, NSIG, NT, INV, Idx>(buf, tw);
      StageRunner<T, N, NSIG, NT, INV, ST + 1, NS * R, Idx, P>::run(buf, tw);
    }
  }
};

// Transform NSIG signals of length N in LDS (element i of signal g at
// Idx::at(g, i), by default lds(g N + i)) with radix plan P; callers
// synchronise before.  Forward uses exp(-2 pi i k x / N); inverse uses
// exp(+...) without 1/N.
template <typename T, int N, int NSIG, int NT, bool INV, class Idx = FlatIdx<N>, int P = 0>
__device__ __forceinline__ void fft_lds(typename cvec<T>::type* buf,
                                        const typename cvec<T>::type* __restrict__ tw) {
  static_assert(fft_size_ok(N), "FFT length must be 2^a 3^b");
  StageRunner<T, N, NSIG, NT, INV, 0, 1, Idx, P>::run(buf, tw);
}

// Whether plan 1 is a different schedule from plan 0 for length N.
constexpr bool plan1_differs(int N) {
  const Plan a = make_plan(N, 0), b = make_plan(N, 1);
  if (a.nst != b.nst) return true;
  for (int i = 0; i < a.nst; ++i)
    if (a.r[i] != b.r[i]) return true;
  return false;
}

}  // namespace fgcg
