// Fused 2D FFT passes: the building blocks of every operator application.
//
// Real fields are stored component-major, [sample][comp][ny][nx] with x
// fastest.  Half spectra are stored TRANSPOSED, [sample][comp][nx/2+1][ny], so
// that the y-direction (column) transforms read and write contiguous memory.
//
//   row_fwd : per block ROWS rows.  A pointwise prologue functor produces NOUT
//             real values per voxel (e.g. the stress of a CG direction), the
//             rows are packed two by two into complex signals z = a + i b,
//             transformed along x in LDS, unpacked into the half spectra of a
//             and b, and stored transposed.
//   col     : per block one kx column.  NIN spectra are transformed along y,
//             a per-mode symbol functor maps them to NOUT spectra (projection,
//             Laplacian, gradient, divergence; the 1/N of the inverse is folded
//             in here), and NOUT inverse transforms along y follow.
//   row_inv : per block ROWS rows.  NIN half spectra are rebuilt into full
//             Hermitian spectra two rows at a time, inverse-transformed along x,
//             and an epilogue functor consumes the NIN real values per voxel
//             (e.g. the CG update x += alpha p, r -= alpha q).
//   row_mid : inverse x transform, pointwise map, forward x transform in one
//             block (the D(x) multiplication of the diffusion operator).
//
// Functors are immutable and expose begin(s, red, sc) (uniform: false = the
// whole block exits; may set the block scalar sc, e.g. the CG beta or alpha),
// point(..., acc, sc) and partial(s, value) (block-reduced FP64 sum, thread 0
// stores).  Optional members: Ld / load / apply (row_fwd: loads issued a voxel
// ahead), NPRE / prefetch (row_inv: inputs of the epilogue loaded before the
// transforms), EARLY (those loads go before begin()), Pre / pre / mode_pre
// (col: per-mode symbol data loaded before the forward transform).  The grid's
// y index s names a sample, or a (sample, component) pair for one-component
// functors.
#pragma once
#include "fft_lds.hpp"

namespace fgcg {

constexpr int NT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum (fixed order) of one value per thread.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Deterministic block sum of an array of partial sums.  A thread's loads
// are issued B at a time and added in index order (the result of adding
// them one at a time, without a memory round trip per element).
template <int B = 4>
__device__ __forceinline__ double block_sum_array(const double* a, int n, double* red) {
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += B * NT) {
    double v[B];
#pragma unroll
    for (int k = 0; k < B; ++k) v[k] = i + k * NT < n ? a[i + k * NT] : 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (i + k * NT < n) t += v[k];
  }
  return block_sum(t, red);
}

// Default rows per block of the row passes: about 2048 voxels per block, so a
// 1024^2 grid gives 512 blocks (two per CU) instead of one block per CU.  The
// mechanics passes of 2D contexts take ROWS as a template argument chosen at
// run time among rows_for / 2, rows_for and 2 rows_for by timing them.
constexpr int rows_for(int nx) {
  return nx >= 768 ? 2 : nx >= 384 ? 4 : nx >= 256 ? 8 : 16;
}

// The hardware hands block b to XCD b % 8.  Give every XCD a contiguous
// range of logical row blocks, so the blocks that share the 128-byte lines of
// a transposed spectrum column (ROWS * 16 bytes each) meet in the same L2.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int x = b & 7, q = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + q;
}

template <typename T>
__device__ __forceinline__ T* as_real(typename cvec<T>::type* p) { return reinterpret_cast<T*>(p); }

// -------------------------------------------------------------- row forward
// Prologues may split point() into load(s, y, x, Ld&) and apply(s, y, x,
// const Ld&, out, acc, sc): the kernel then issues the loads of the next voxel
// before the stores of the current one (the compiler cannot reorder them
// itself, since the fields might alias).
template <class P, class = void> struct ProLoads {
  static constexpr bool value = false;
};
template <class P> struct ProLoads<P, decltype((void)sizeof(typename P::Ld))> {
  static constexpr bool value = true;
};
// P::EARLY: issue the first loads (or the prefetch) before begin()
template <class P, class = void> struct ProEarly {
  static constexpr bool value = false;
};
template <class P> struct ProEarly<P, decltype((void)P::EARLY)> {
  static constexpr bool value = P::EARLY;
};
template <class P, bool = ProLoads<P>::value> struct ProLd {
  struct type {};
};
template <class P> struct ProLd<P, true> {
  using type = typename P::Ld;
};

template <typename T, int NX, int NOUT, class Pro, int ROWS = rows_for(NX), int PL = 0>
__global__ void __launch_bounds__(NT) k_row_fwd(Pro pro, typename cvec<T>::type* spec, int ny,
                                                long long spec_ss,
                                                const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  static_assert(ROWS >= 2 && ROWS % 2 == 0, "rows per block: even, at least 2");
  constexpr int NP = ROWS / 2;
  constexpr int NXH = NX / 2 + 1;
  constexpr int VOX = ROWS * NX;
  constexpr int VPT = (VOX + NT - 1) / NT;
  __shared__ C buf[lds_size(NP * NX)];
  __shared__ double red[NT / 64];
  const int s = blockIdx.y;
  const int tid = threadIdx.x;
  const int y0 = xcd_block() * ROWS;
  auto valid = [&](int i) {
    const int v = tid + i * NT;
    return (VOX % NT == 0 || v < VOX) && y0 + v / NX < ny;
  };
  // The loads of the first voxel do not depend on the CG scalars.  Where
  // begin() reduces many partial sums (Pro::EARLY), they are issued first so
  // that the two latencies overlap (the empty asm keeps them from being sunk
  // below the early exit; it emits no instruction).  Otherwise they follow
  // begin(): its state check would wait for them.
  typename ProLd<Pro>::type cur;
  constexpr bool EARLY = ProEarly<Pro>::value;
  if constexpr (EARLY) {
    if (valid(0)) pro.load(s, y0 + tid / NX, tid % NX, cur);
    asm volatile("" ::: "memory");
  }
  double sc = 0.0;
  if (!pro.begin(s, red, sc)) return;
  if constexpr (ProLoads<Pro>::value && !EARLY) {
    if (valid(0)) pro.load(s, y0 + tid / NX, tid % NX, cur);
  }
  T vals[VPT][NOUT];
  double acc = 0.0;
  if constexpr (ProLoads<Pro>::value) {
    // loads of voxel i + 1 are issued before the stores of voxel i
    typename Pro::Ld nxt;
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * NT;
      const int row = v / NX, x = v - (v / NX) * NX;
      if (i + 1 < VPT && valid(i + 1)) {
        const int v1 = v + NT;
        pro.load(s, y0 + v1 / NX, v1 % NX, nxt);
      }
      if (valid(i)) {
        pro.apply(s, y0 + row, x, cur, vals[i], acc, sc);
      } else {
#pragma unroll
        for (int c = 0; c < NOUT; ++c) vals[i][c] = (T)0;
      }
      cur = nxt;
    }
  } else {
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * NT;
      const int row = v / NX, x = v - (v / NX) * NX;
      if (valid(i)) {
        pro.point(s, y0 + row, x, vals[i], acc, sc);
      } else {
#pragma unroll
        for (int c = 0; c < NOUT; ++c) vals[i][c] = (T)0;
      }
    }
  }
  pro.partial(s, block_sum(acc, red));
  C* out = spec + s * spec_ss;
  T* rb = as_real<T>(buf);
#pragma unroll
  for (int c = 0; c < NOUT; ++c) {
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * NT;
      if (VOX % NT == 0 || v < VOX) {
        const int row = v / NX, x = v - (v / NX) * NX;
        rb[2 * lds((row >> 1) * NX + x) + (row & 1)] = vals[i][c];
      }
    }
    __syncthreads();
    fft_lds<T, NX, NP, NT, false, FlatIdx<NX>, PL>(buf, tw);
    for (int idx = tid; idx < NXH * NP; idx += NT) {
      const int pair = idx % NP, kx = idx / NP;
      const C z = buf[lds(pair * NX + kx)];
      const C zm = buf[lds(pair * NX + (NX - kx) % NX)];
      const C a = C{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)};
      const C b = C{(T)0.5 * (z.y + zm.y), (T)0.5 * (zm.x - z.x)};
      const int y = y0 + 2 * pair;
      C* o = out + ((long long)c * NXH + kx) * ny;
      if (y < ny) o[y] = a;
      if (y + 1 < ny) o[y + 1] = b;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ column
// Sym::Pre: per-mode data the symbol can take from registers (sym.pre(s, kx, ky)
// loaded before the forward transform, used by sym.mode_pre).
template <class S, class = void> struct SymPre {
  static constexpr bool value = false;
  struct type {};
};
template <class S> struct SymPre<S, decltype((void)sizeof(typename S::Pre))> {
  static constexpr bool value = true;
  using type = typename S::Pre;
};

template <typename T, int NY, int NIN, int NOUT, class Sym, int PL = 0>
__global__ void __launch_bounds__(NT) k_col(Sym sym, const typename cvec<T>::type* spec_in,
                                            typename cvec<T>::type* spec_out, int nxh,
                                            long long ss_in, long long ss_out,
                                            const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  constexpr int NB = NIN > NOUT ? NIN : NOUT;
  __shared__ C buf[lds_size(NB * NY)];
  __shared__ double red[NT / 64];
  const int s = blockIdx.y;
  const int kx = blockIdx.x;
  const int tid = threadIdx.x;
  // The state check comes first: blocks of samples whose solve has ended (in
  // a batch) exit before loading anything.
  const C* in = spec_in + s * ss_in;
  double sc = 0.0;
  if (!sym.begin(s, red, sc)) return;
  for (int idx = tid; idx < NIN * NY; idx += NT) {
    const int c = idx / NY, y = idx - (idx / NY) * NY;
    buf[lds(c * NY + y)] = in[((long long)c * nxh + kx) * NY + y];
  }
  // per-mode symbol data loaded before the transform (Sym::Pre), so the
  // loads are not on the path between the two transforms
  constexpr int KPT = (NY + NT - 1) / NT;
  typename SymPre<Sym>::type spre[KPT];
  if constexpr (SymPre<Sym>::value) {
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
      const int ky = tid + k * NT;
      if (NY % NT == 0 || ky < NY) spre[k] = sym.pre(s, kx, ky);
    }
  }
  __syncthreads();
  fft_lds<T, NY, NIN, NT, false, FlatIdx<NY>, PL>(buf, tw);
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < KPT; ++k) {
    const int ky = tid + k * NT;
    if (NY % NT == 0 || ky < NY) {
      C a[NIN], b[NOUT];
#pragma unroll
      for (int c = 0; c < NIN; ++c) a[c] = buf[lds(c * NY + ky)];
      if constexpr (SymPre<Sym>::value)
        sym.mode_pre(s, kx, ky, spre[k], a, b, acc, sc);
      else
        sym.mode(s, kx, ky, a, b, acc, sc);
#pragma unroll
      for (int c = 0; c < NOUT; ++c) buf[lds(c * NY + ky)] = b[c];
    }
  }
  __syncthreads();
  sym.partial(s, block_sum(acc, red));
  fft_lds<T, NY, NOUT, NT, true, FlatIdx<NY>, PL>(buf, tw);
  C* out = spec_out + s * ss_out;
  for (int idx = tid; idx < NOUT * NY; idx += NT) {
    const int c = idx / NY, y = idx - (idx / NY) * NY;
    out[((long long)c * nxh + kx) * NY + y] = buf[lds(c * NY + y)];
  }
}

// ------------------------------------------------- column, one wave per column
// One 64-lane wavefront (a block of 64 threads) transforms a whole column of
// length N in registers: lane l holds the elements l + 64 m, m < E = N / 64.
// A Stockham stage of radix R (E a multiple of R) gives lane l the butterflies
// j = l + 64 q, whose inputs j + r N / R = l + 64 (q + r E / R) are again the
// lane's own elements, so a stage needs no exchange to read; its outputs go
// to LDS (positions (j / Ns) Ns R + j % Ns + r Ns) and come back as the next
// stage's elements l + 64 m, except after the last stage, whose outputs
// j + r Ns already are the lane's own elements.  The column is loaded and
// stored in that layout (64 consecutive complex values per access), and the
// symbol is applied to the lane's modes between the forward and the inverse
// transform: two LDS round trips per direction for N = 1024 (radix 16, 16,
// 4), no barrier across wavefronts.
struct WPlan {
  int nst;
  int r[6];
};
constexpr WPlan wave_plan(int N) {
  return N == 256 ? WPlan{4, {4, 4, 4, 4, 0, 0}}
         : N == 512 ? WPlan{3, {8, 8, 8, 0, 0, 0}}
         : N == 1024 ? WPlan{3, {16, 16, 4, 0, 0, 0}}
         : N == 2048 ? WPlan{3, {16, 16, 8, 0, 0, 0}}
                     : WPlan{0, {0, 0, 0, 0, 0, 0}};
}
constexpr bool wave_col_ok(int N) { return wave_plan(N).nst > 0; }

// Twiddles of the stages before stage ST: a lane holds B = E / R of them for
// every stage after the first (one per butterfly), loaded once per kernel;
// the inverse transform uses their conjugates.
constexpr int wave_tw_before(int N, int ST) {
  int t = 0;
  for (int i = 1; i < ST; ++i) t += N / 64 / wave_plan(N).r[i];
  return t;
}
constexpr int wave_tw_count(int N) { return wave_tw_before(N, wave_plan(N).nst); }

// Load the lane's twiddles: stage ST (sub-transform length NS, radix R),
// butterfly q takes w = exp(-2 pi i k / (NS R)), k = (l + 64 q) mod NS.
template <typename T, int N, int ST, int NS>
__device__ __forceinline__ void wave_tw_load(typename cvec<T>::type* W, const typename cvec<T>::type* __restrict__ tw) {
  constexpr WPlan p = wave_plan(N);
  if constexpr (ST < p.nst) {
    constexpr int R = p.r[ST];
    if constexpr (ST > 0) {
      constexpr int B = N / 64 / R, TSTEP = N / (NS * R), OFF = wave_tw_before(N, ST);
#pragma unroll
      for (int q = 0; q < B; ++q) W[OFF + q] = tw[((threadIdx.x + 64 * q) % NS) * TSTEP];
    }
    wave_tw_load<T, N, ST + 1, NS * R>(W, tw);
  }
}

// One stage (radix R, sub-transform length NS) on the lane's elements V, with
// the lane's twiddles of this stage in W[0 .. B).
template <typename T, int N, int R, int NS, bool INV, bool LAST>
__device__ __forceinline__ void wave_stage(typename cvec<T>::type* V, typename cvec<T>::type* buf,
                                           const typename cvec<T>::type* W) {
  using C = typename cvec<T>::type;
  constexpr int E = N / 64, B = E / R;  // butterflies per lane
  const int l = threadIdx.x;
#pragma unroll
  for (int q = 0; q < B; ++q) {
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = V[q + r * B];
    if (NS > 1) {
      C w1 = W[q];
      if (INV) w1.y = -w1.y;
      C w = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        v[r] = cmul(v[r], w);
        if (r + 1 < R) w = cmul(w, w1);
      }
    }
    Dft<R, INV, T>::run(v);
    if constexpr (LAST) {
      // outputs j + r NS with j = l + 64 q and NS = 64 B: the lane's own
      // elements q + r B, the ones this butterfly read
#pragma unroll
      for (int r = 0; r < R; ++r) V[q + r * B] = v[r];
    } else {
      const int j = l + 64 * q;
      const int base = (j / NS) * NS * R + j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lds(base + r * NS)] = v[r];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) V[m] = buf[lds(l + 64 * m)];
    __syncthreads();
  }
}

template <typename T, int N, bool INV, int ST, int NS>
__device__ __forceinline__ void wave_fft(typename cvec<T>::type* V, typename cvec<T>::type* buf,
                                         const typename cvec<T>::type* W) {
  constexpr WPlan p = wave_plan(N);
  if constexpr (ST < p.nst) {
    constexpr int R = p.r[ST];
    wave_stage<T, N, R, NS, INV, ST + 1 == p.nst>(V, buf, W + (ST > 0 ? wave_tw_before(N, ST) : 0));
    wave_fft<T, N, INV, ST + 1, NS * R>(V, buf, W);
  }
}

__device__ __forceinline__ double wave_sum64(double v) { return wave_sum(v); }

// One-component column pass (NIN = NOUT = 1) for the Green symbols: block
// (kx, s) of 64 threads.  Same contract as k_col<T, NY, 1, 1, Sym>.  The
// lane's column elements, twiddles and symbol data are loaded together at the
// start; with EARLY (single-sample contexts, where no block can find its
// sample's solve ended while others run) before the state check, so its
// latency overlaps theirs.
template <typename T, int NY, class Sym, bool EARLY>
__global__ void __launch_bounds__(64) k_colw(Sym sym, const typename cvec<T>::type* spec_in,
                                             typename cvec<T>::type* spec_out, int nxh, long long ss_in,
                                             long long ss_out, const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  constexpr int E = NY / 64;
  constexpr int NW = wave_tw_count(NY) > 0 ? wave_tw_count(NY) : 1;
  __shared__ C buf[lds_size(NY)];
  __shared__ double red[1];
  const int s = blockIdx.y;
  const int kx = blockIdx.x;
  const int l = threadIdx.x;
  const C* in = spec_in + s * ss_in + (long long)kx * NY;
  C V[E], W[NW];
  typename SymPre<Sym>::type spre[E];
  auto load = [&]() {
#pragma unroll
    for (int m = 0; m < E; ++m) V[m] = in[l + 64 * m];
    wave_tw_load<T, NY, 0, 1>(W, tw);
    if constexpr (SymPre<Sym>::value) {
#pragma unroll
      for (int m = 0; m < E; ++m) spre[m] = sym.pre(s, kx, l + 64 * m);
    }
  };
  double sc = 0.0;
  if constexpr (EARLY) load();
  if (!sym.begin(s, red, sc)) return;
  if constexpr (!EARLY) load();
  wave_fft<T, NY, false, 0, 1>(V, buf, W);
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    C b[1];
    if constexpr (SymPre<Sym>::value)
      sym.mode_pre(s, kx, l + 64 * m, spre[m], &V[m], b, acc, sc);
    else
      sym.mode(s, kx, l + 64 * m, &V[m], b, acc, sc);
    V[m] = b[0];
  }
  acc = wave_sum64(acc);
  sym.partial(s, acc);
  wave_fft<T, NY, true, 0, 1>(V, buf, W);
  C* out = spec_out + s * ss_out + (long long)kx * NY;
#pragma unroll
  for (int m = 0; m < E; ++m) out[l + 64 * m] = V[m];
}

// Load NIN half spectra of ROWS rows, inverse transform, into registers.
// The half spectrum of component c + 1 is loaded into registers before the
// transform of component c (the barriers wait for LDS traffic only), so its
// transposed reads overlap the LDS work.
template <typename T, int NX, int NIN, int ROWS = rows_for(NX), int PL = 0>
__device__ __forceinline__ void rows_inverse(
    const typename cvec<T>::type* in, int ny, int y0, typename cvec<T>::type* buf,
    T (*vals)[NIN], const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  static_assert(ROWS >= 2 && ROWS % 2 == 0, "rows per block: even, at least 2");
  constexpr int NP = ROWS / 2;
  constexpr int NXH = NX / 2 + 1;
  constexpr int VOX = ROWS * NX;
  constexpr int VPT = (VOX + NT - 1) / NT;
  constexpr int NL = (NXH * NP + NT - 1) / NT;  // (pair, kx) entries per thread
  const int tid = threadIdx.x;
  T* rb = as_real<T>(buf);
  C ra[NL], rbv[NL];
  auto load = [&](int c) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int idx = tid + l * NT;
      ra[l] = C{(T)0, (T)0};
      rbv[l] = C{(T)0, (T)0};
      if (idx < NXH * NP) {
        const int pair = idx % NP, kx = idx / NP;
        const int y = y0 + 2 * pair;
        const C* o = in + ((long long)c * NXH + kx) * ny;
        if (y < ny) ra[l] = o[y];
        if (y + 1 < ny) rbv[l] = o[y + 1];
      }
    }
  };
  load(0);
#pragma unroll
  for (int c = 0; c < NIN; ++c) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int idx = tid + l * NT;
      if (idx < NXH * NP) {
        const int pair = idx % NP, kx = idx / NP;
        C a = ra[l], b = rbv[l];
        if (kx == 0 || 2 * kx == NX) {
          a.y = (T)0;
          b.y = (T)0;
        }
        buf[lds(pair * NX + kx)] = C{a.x - b.y, a.y + b.x};
        if (kx > 0 && 2 * kx < NX) buf[lds(pair * NX + NX - kx)] = C{a.x + b.y, b.x - a.y};
      }
    }
    if (c + 1 < NIN) load(c + 1);
    __syncthreads();
    fft_lds<T, NX, NP, NT, true, FlatIdx<NX>, PL>(buf, tw);
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * NT;
      if (VOX % NT == 0 || v < VOX) {
        const int row = v / NX, x = v - (v / NX) * NX;
        vals[i][c] = rb[2 * lds((row >> 1) * NX + x) + (row & 1)];
      }
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------- row inverse
// Epilogues that read fields of their own voxels may declare NPRE > 0 and a
// prefetch(s, y, x, pre) member: those values are loaded into registers
// before the transforms and handed to point(..., pre), so their reads overlap
// the LDS work instead of following it.
template <class E, class = void> struct EpiPre {
  static constexpr int N = 0;
};
template <class E> struct EpiPre<E, decltype((void)E::NPRE)> {
  static constexpr int N = E::NPRE;
};

template <typename T, int NX, int NIN, class Epi, int ROWS = rows_for(NX), int PL = 0>
__global__ void __launch_bounds__(NT) k_row_inv(Epi epi, const typename cvec<T>::type* spec, int ny,
                                                long long spec_ss,
                                                const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  static_assert(ROWS >= 2 && ROWS % 2 == 0, "rows per block: even, at least 2");
  constexpr int NP = ROWS / 2;
  constexpr int VOX = ROWS * NX;
  constexpr int VPT = (VOX + NT - 1) / NT;
  constexpr int NPRE = EpiPre<Epi>::N;
  __shared__ C buf[lds_size(NP * NX)];
  __shared__ double red[NT / 64];
  const int s = blockIdx.y;
  const int tid = threadIdx.x;
  const int y0 = xcd_block() * ROWS;
  // The prefetch of the epilogue's inputs does not depend on the CG scalars:
  // issued before begin() where that reduces many partial sums (Epi::EARLY),
  // after it otherwise (as in the forward pass).
  T pre[VPT][NPRE > 0 ? NPRE : 1];
  auto prefetch = [&](auto& e) {
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * NT;
      const int row = v / NX, x = v - (v / NX) * NX;
      if ((VOX % NT == 0 || v < VOX) && y0 + row < ny) e.prefetch(s, y0 + row, x, pre[i]);
    }
  };
  constexpr bool EARLY = NPRE > 0 && ProEarly<Epi>::value;
  if constexpr (EARLY) {
    prefetch(epi);
    asm volatile("" ::: "memory");
  }
  double sc = 0.0;
  if (!epi.begin(s, red, sc)) return;
  if constexpr (NPRE > 0 && !EARLY) prefetch(epi);
  T vals[VPT][NIN];
  rows_inverse<T, NX, NIN, ROWS, PL>(spec + s * spec_ss, ny, y0, buf, vals, tw);
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int v = tid + i * NT;
    const int row = v / NX, x = v - (v / NX) * NX;
    if ((VOX % NT == 0 || v < VOX) && y0 + row < ny) {
      if constexpr (NPRE > 0)
        epi.point(s, y0 + row, x, vals[i], acc, sc, pre[i]);
      else
        epi.point(s, y0 + row, x, vals[i], acc, sc);
    }
  }
  epi.partial(s, block_sum(acc, red));
}

// -------------------------------------------------- row inverse + forward
template <typename T, int NX, int NIN, int NOUT, class Mid>
__global__ void __launch_bounds__(NT) k_row_mid(Mid mid, typename cvec<T>::type* spec, int ny,
                                                long long spec_ss,
                                                const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  constexpr int ROWS = rows_for(NX);
  constexpr int NP = ROWS / 2;
  constexpr int NXH = NX / 2 + 1;
  constexpr int VOX = ROWS * NX;
  constexpr int VPT = (VOX + NT - 1) / NT;
  __shared__ C buf[lds_size(NP * NX)];
  __shared__ double red[NT / 64];
  const int s = blockIdx.y;
  const int tid = threadIdx.x;
  double sc = 0.0;
  if (!mid.begin(s, red, sc)) return;
  const int y0 = xcd_block() * ROWS;
  T vin[VPT][NIN];
  T vout[VPT][NOUT];
  C* sp = spec + s * spec_ss;
  rows_inverse<T, NX, NIN>(sp, ny, y0, buf, vin, tw);
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int v = tid + i * NT;
    const int row = v / NX, x = v - (v / NX) * NX;
    if ((VOX % NT == 0 || v < VOX) && y0 + row < ny) {
      mid.point(s, y0 + row, x, vin[i], vout[i], acc, sc);
    } else {
#pragma unroll
      for (int c = 0; c < NOUT; ++c) vout[i][c] = (T)0;
    }
  }
  mid.partial(s, block_sum(acc, red));
  T* rb = as_real<T>(buf);
#pragma unroll
  for (int c = 0; c < NOUT; ++c) {
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int v = tid + i * NT;
      if (VOX % NT == 0 || v < VOX) {
        const int row = v / NX, x = v - (v / NX) * NX;
        rb[2 * lds((row >> 1) * NX + x) + (row & 1)] = vout[i][c];
      }
    }
    __syncthreads();
    fft_lds<T, NX, NP, NT, false>(buf, tw);
    for (int idx = tid; idx < NXH * NP; idx += NT) {
      const int pair = idx % NP, kx = idx / NP;
      const C z = buf[lds(pair * NX + kx)];
      const C zm = buf[lds(pair * NX + (NX - kx) % NX)];
      const C a = C{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)};
      const C b = C{(T)0.5 * (z.y + zm.y), (T)0.5 * (zm.x - z.x)};
      const int y = y0 + 2 * pair;
      C* o = sp + ((long long)c * NXH + kx) * ny;
      if (y < ny) o[y] = a;
      if (y + 1 < ny) o[y + 1] = b;
    }
    __syncthreads();
  }
}

}  // namespace fgcg
