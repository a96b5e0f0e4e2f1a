// Mechanics PCG of 2D FP64 contexts with the residual kept in Fourier space.
//
// The displacement-form PCG of mech_u.hpp (K u = f, M = (grad^H grad)^-1,
// Sec. 2.3 / App. A) needs r only through r_hat: the Green operator is applied
// to r_hat, r.z is a Parseval sum over r_hat, and r -= alpha q is linear, so
// it can be carried out on the spectra, r_hat -= alpha FFT(q).  The solution
// update x += alpha p can wait until the pass that forms the next direction,
// which reads p anyway.  One iteration is then three passes instead of four:
//   k_kp_fwd2          q = K p as a real-space stencil for the rows of the
//                      block (both displacement components; k_kp_fwd: one
//                      per block), the forward x transforms of q, partial
//                      sums of p.Kp in the energy form
//                      sum sym(grad p) : g C : sym(grad p)
//   col (MechGreenSR)  alpha = r.z / p.Kp; y transforms; r_hat -= alpha q_hat
//                      (stored); z_hat = r_hat / |D|^2 / N; partial sums of
//                      r.z; inverse y transforms of z_hat
//   row_inv (MechUEpiSRC) inverse x transforms; stop test on r.z; beta;
//                      x += alpha p; p = z + beta p
// with the alpha, beta and stop test of the four-pass form, iterate by
// iterate.  When the stop test ends the solve inside the inverse pass, the
// last x update is still due; k_sr_finish applies it after the solve.
// Algorithmic bytes per voxel (FP64, 2 components, half spectra
// (nx/2+1)/nx * 16 B per component): 41 + 64.1 + 80.0 = 185 against 233 for
// the four-pass form.  The two-pass form (k_sr_row, below) does the inverse
// pass of one iteration and the stiffness pass of the next in one kernel:
// 105.1 + 64.1 = 169.2 bytes per voxel and one launch fewer.
#pragma once
#include "mech_u.hpp"

namespace fgcg {

// Sum of an array of partial sums by a block of 64 or NT threads (fixed order
// for a given block size).
__device__ __forceinline__ double group_sum_array(const double* a, int n, double* red) {
  if (blockDim.x == 64) {
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) t += a[i];
    return wave_sum(t);
  }
  return block_sum_array(a, n, red);
}

// q = K p for the ROWS rows y0 .. y0 + ROWS - 1 of displacement component
// c = blockIdx.y % 2 (sample blockIdx.y / 2), transformed along x and stored
// transposed as k_row_fwd does; partial sums of this component's share of the
// energy form of p.Kp (c = 0: e11 s11 + e12 s12, c = 1: e22 s22 + e12 s12),
// one per grid row at part[blockIdx.y * ny + y], so that the sum does not
// depend on the rows per block.
//
// EF: the material is a per-voxel E field (else phase tables).  KT threads
// per block (kp_threads: four columns per thread on rows of 1024 and more);
// thread t owns the XPT = NX / KT consecutive columns x = t XPT + j.  Every
// global load of the block is issued first: p (both components) on the rows
// y0 - 1 .. y0 + ROWS, the right neighbour p(y, (t + 1) XPT) on the rows
// y0 - 1 .. y0 + ROWS - 1 and the material there.  The rows are then walked
// with registers only: the stress at (y, x) takes p at (y, x), (y, x + 1) and
// (y + 1, x); the divergence at (y, x) takes the stress at (y, x - 1) (the
// thread's own column j - 1, or for j = 0 the left thread's last column
// through LDS, double-buffered: one barrier per row) and at (y - 1, x) (the
// previous row).  The two component blocks of a row strip share an XCD, so the
// second reads p and the material from L2.
constexpr int kp_threads(int nx) { return nx >= 2048 ? nx / 4 : NT; }

template <typename T, int NX, int ROWS, int PL, bool EF, int KT = kp_threads(NX)>
__global__ void __launch_bounds__(KT) k_kp_fwd(MechMat m, const T* __restrict__ p, CgState* st, double* part,
                                               typename cvec<T>::type* spec, int ny, long long spec_ss, T ih,
                                               const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  static_assert(NX % KT == 0 && KT % 64 == 0, "k_kp_fwd: NX must be a multiple of the block size");
  static_assert(ROWS >= 2 && ROWS % 2 == 0, "rows per block: even, at least 2");
  constexpr int XPT = NX / KT;
  constexpr int NP = ROWS / 2;
  constexpr int NXH = NX / 2 + 1;
  __shared__ C buf[lds_size(NP * NX)];
  __shared__ T edge[2][KT];             // x flux of each thread's last column, per row parity
  __shared__ double rsum[ROWS][KT / 64];  // per-row energy sums of each wavefront
  const int s2 = blockIdx.y, s = s2 >> 1, c = s2 & 1;
  const int tid = threadIdx.x;
  const int y0 = xcd_block() * ROWS;
  const long long n = m.ss;
  const T* ps = p + 2 * n * s;
  // periodic row index (a block's rows may pass the last row more than once on
  // grids of fewer rows than a block holds)
  auto wrap = [&](int y) { return ((y % ny) + ny) % ny; };
  const int x0 = tid * XPT, xr = (x0 + XPT) % NX;
  long long rowi[ROWS + 2];
#pragma unroll
  for (int k = 0; k < ROWS + 2; ++k) rowi[k] = (long long)wrap(y0 - 1 + k) * NX;
  // Loads in straight-line groups (the material's kind is uniform: branches
  // around whole groups, not per voxel), so that they are all in flight
  // before the first use.  A single sample (two component blocks) issues them
  // before the state check: no block can find its solve ended while others
  // run; in batches the blocks of converged samples exit first.
  T p0[ROWS + 2][XPT], p1[ROWS + 2][XPT], r0[ROWS + 1], r1[ROWS + 1];
  uint8_t ph[EF ? 1 : ROWS + 1][XPT];
  double ev[EF ? ROWS + 1 : 1][XPT], dd[ROWS + 1][XPT];
  const bool dmg = m.d != nullptr;
  auto load = [&]() {
#pragma unroll
    for (int k = 0; k < ROWS + 2; ++k)
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        p0[k][j] = ps[rowi[k] + x0 + j];
        p1[k][j] = ps[n + rowi[k] + x0 + j];
      }
#pragma unroll
    for (int k = 0; k < ROWS + 1; ++k) {
      r0[k] = ps[rowi[k] + xr];
      r1[k] = ps[n + rowi[k] + xr];
    }
    const long long so = s * n;
#pragma unroll
    for (int k = 0; k < ROWS + 1; ++k)
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        if constexpr (EF)
          ev[k][j] = m.Efield[so + rowi[k] + x0 + j];
        else
          ph[k][j] = m.phase[so + rowi[k] + x0 + j];
      }
    if (dmg) {
#pragma unroll
      for (int k = 0; k < ROWS + 1; ++k)
#pragma unroll
        for (int j = 0; j < XPT; ++j) dd[k][j] = m.d[so + rowi[k] + x0 + j];
    }
  };
  const bool early = gridDim.y == 2;
  if (early) load();
  if (!cg_running(st, s)) return;
  if (lead() && c == 0) st[s].k = st[s].k_next;
  if (!early) load();
  // Lame constants of voxel (row k, column j), degraded (the per-sample
  // tables of a batch are read per voxel)
  auto lame = [&](int k, int j, double& lam, double& mu) {
    if constexpr (EF) {
      lam = ev[k][j] * m.lam_per_E;
      mu = ev[k][j] * m.mu_per_E;
    } else if (m.lm_dev) {
      lam = m.lm_dev[16 * s + ph[k][j]];
      mu = m.lm_dev[16 * s + 8 + ph[k][j]];
    } else if (m.nphase <= 2) {  // (uniform) one selection instead of the eight-way one
      lam = ph[k][j] ? m.lm.a[1] : m.lm.a[0];
      mu = ph[k][j] ? m.lm.b[1] : m.lm.b[0];
    } else {
      pick(m.lm, ph[k][j], lam, mu);
    }
    if (dmg) {
      const double g = (1.0 - dd[k][j]) * (1.0 - dd[k][j]) + m.kappa;
      lam *= g;
      mu *= g;
    }
  };
  T* rb = as_real<T>(buf);
  T fy_prev[XPT];
#pragma unroll
  for (int k = 0; k < ROWS + 1; ++k) {  // row y0 - 1 + k
    const int rr = k - 1;
    const bool own = rr >= 0 && y0 + rr < ny;  // a row of this block (not the halo row, not past the grid)
    T fx[XPT], fy[XPT];
    double e_row = 0.0;
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const T px0 = j + 1 < XPT ? p0[k][j + 1] : r0[k];
      const T px1 = j + 1 < XPT ? p1[k][j + 1] : r1[k];
      const T g11 = (px0 - p0[k][j]) * ih;
      const T g12 = (p0[k + 1][j] - p0[k][j]) * ih;
      const T g21 = (px1 - p1[k][j]) * ih;
      const T g22 = (p1[k + 1][j] - p1[k][j]) * ih;
      const T e0 = g11, e1 = g22, e2 = (T)0.5 * (g12 + g21);
      double lam, mu;
      lame(k, j, lam, mu);
      T sg[3];
      stress2<T>(lam, mu, e0, e1, e2, sg);
      fx[j] = c == 0 ? sg[0] : sg[2];
      fy[j] = c == 0 ? sg[2] : sg[1];
      e_row += c == 0 ? (double)e0 * sg[0] + (double)e2 * sg[2] : (double)e1 * sg[1] + (double)e2 * sg[2];
    }
    edge[k & 1][tid] = fx[XPT - 1];
    __syncthreads();
    if (rr >= 0) {
      const T left = edge[k & 1][tid == 0 ? KT - 1 : tid - 1];
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        const T fxm = j > 0 ? fx[j - 1] : left;
        const T q = ((fxm - fx[j]) + (fy_prev[j] - fy[j])) * ih;
        rb[2 * lds((rr >> 1) * NX + x0 + j) + (rr & 1)] = own ? q : (T)0;
      }
      const double w = wave_sum(own ? e_row : 0.0);
      if ((tid & 63) == 0) rsum[rr][tid >> 6] = w;
    }
#pragma unroll
    for (int j = 0; j < XPT; ++j) fy_prev[j] = fy[j];
  }
  __syncthreads();
  if (tid < ROWS && y0 + tid < ny) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < KT / 64; ++w) t += rsum[tid][w];
    part[(long long)s2 * ny + y0 + tid] = t;
  }
  fft_lds<T, NX, NP, KT, false, FlatIdx<NX>, PL>(buf, tw);
  C* out = spec + s2 * spec_ss;
  for (int idx = tid; idx < NXH * NP; idx += KT) {
    const int pair = idx % NP, kx = idx / NP;
    const C z = buf[lds(pair * NX + kx)];
    const C zm = buf[lds(pair * NX + (NX - kx) % NX)];
    const C a = C{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)};
    const C b = C{(T)0.5 * (z.y + zm.y), (T)0.5 * (zm.x - z.x)};
    const int yy = y0 + 2 * pair;
    C* o = out + (long long)kx * ny;
    if (yy < ny) o[yy] = a;
    if (yy + 1 < ny) o[yy + 1] = b;
  }
}

// The same pass with both displacement components in one block (grid (row
// blocks, samples)): the stress of a voxel is evaluated once for both
// components' divergences, p and the material are read once, and the 2 ROWS
// real rows of q (ROWS of each component) are transformed as ROWS complex
// signals.  The p.Kp partial sums are the full energy sum e11 s11 + e22 s22
// + 2 e12 s12 of each grid row, at part[sample * ny + y].
template <typename T, int NX, int ROWS, int PL, bool EF, int KT = kp_threads(NX)>
__global__ void __launch_bounds__(KT) k_kp_fwd2(MechMat m, const T* __restrict__ p, CgState* st, double* part,
                                                typename cvec<T>::type* spec, int ny, long long spec_ss, T ih,
                                                const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  static_assert(NX % KT == 0 && KT % 64 == 0, "k_kp_fwd2: NX must be a multiple of the block size");
  static_assert(ROWS >= 2 && ROWS % 2 == 0, "rows per block: even, at least 2");
  constexpr int XPT = NX / KT;
  constexpr int NP = ROWS / 2;  // complex signals per component
  constexpr int NXH = NX / 2 + 1;
  __shared__ C buf[lds_size(2 * NP * NX)];
  __shared__ T edge[2][2][KT];
  __shared__ double rsum[ROWS][KT / 64];
  const int s = blockIdx.y;
  const int tid = threadIdx.x;
  const int y0 = xcd_block() * ROWS;
  const long long n = m.ss;
  const T* ps = p + 2 * n * s;
  auto wrap = [&](int y) { return ((y % ny) + ny) % ny; };
  const int x0 = tid * XPT, xr = (x0 + XPT) % NX;
  long long rowi[ROWS + 2];
#pragma unroll
  for (int k = 0; k < ROWS + 2; ++k) rowi[k] = (long long)wrap(y0 - 1 + k) * NX;
  T p0[ROWS + 2][XPT], p1[ROWS + 2][XPT], r0[ROWS + 1], r1[ROWS + 1];
  uint8_t ph[EF ? 1 : ROWS + 1][XPT];
  double ev[EF ? ROWS + 1 : 1][XPT], dd[ROWS + 1][XPT];
  const bool dmg = m.d != nullptr;
  auto load = [&]() {
#pragma unroll
    for (int k = 0; k < ROWS + 2; ++k)
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        p0[k][j] = ps[rowi[k] + x0 + j];
        p1[k][j] = ps[n + rowi[k] + x0 + j];
      }
#pragma unroll
    for (int k = 0; k < ROWS + 1; ++k) {
      r0[k] = ps[rowi[k] + xr];
      r1[k] = ps[n + rowi[k] + xr];
    }
    const long long so = s * n;
#pragma unroll
    for (int k = 0; k < ROWS + 1; ++k)
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        if constexpr (EF)
          ev[k][j] = m.Efield[so + rowi[k] + x0 + j];
        else
          ph[k][j] = m.phase[so + rowi[k] + x0 + j];
      }
    if (dmg) {
#pragma unroll
      for (int k = 0; k < ROWS + 1; ++k)
#pragma unroll
        for (int j = 0; j < XPT; ++j) dd[k][j] = m.d[so + rowi[k] + x0 + j];
    }
  };
  const bool early = gridDim.y == 1;
  if (early) load();
  if (!cg_running(st, s)) return;
  if (lead()) st[s].k = st[s].k_next;
  if (!early) load();
  auto lame = [&](int k, int j, double& lam, double& mu) {
    if constexpr (EF) {
      lam = ev[k][j] * m.lam_per_E;
      mu = ev[k][j] * m.mu_per_E;
    } else if (m.lm_dev) {
      lam = m.lm_dev[16 * s + ph[k][j]];
      mu = m.lm_dev[16 * s + 8 + ph[k][j]];
    } else if (m.nphase <= 2) {  // (uniform) one selection instead of the eight-way one
      lam = ph[k][j] ? m.lm.a[1] : m.lm.a[0];
      mu = ph[k][j] ? m.lm.b[1] : m.lm.b[0];
    } else {
      pick(m.lm, ph[k][j], lam, mu);
    }
    if (dmg) {
      const double g = (1.0 - dd[k][j]) * (1.0 - dd[k][j]) + m.kappa;
      lam *= g;
      mu *= g;
    }
  };
  T* rb = as_real<T>(buf);
  T s12_prev[XPT], s22_prev[XPT];
#pragma unroll
  for (int k = 0; k < ROWS + 1; ++k) {  // row y0 - 1 + k
    const int rr = k - 1;
    const bool own = rr >= 0 && y0 + rr < ny;
    T s11[XPT], s22[XPT], s12[XPT];
    double e_row = 0.0;
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const T px0 = j + 1 < XPT ? p0[k][j + 1] : r0[k];
      const T px1 = j + 1 < XPT ? p1[k][j + 1] : r1[k];
      const T g11 = (px0 - p0[k][j]) * ih;
      const T g12 = (p0[k + 1][j] - p0[k][j]) * ih;
      const T g21 = (px1 - p1[k][j]) * ih;
      const T g22 = (p1[k + 1][j] - p1[k][j]) * ih;
      const T e0 = g11, e1 = g22, e2 = (T)0.5 * (g12 + g21);
      double lam, mu;
      lame(k, j, lam, mu);
      T sg[3];
      stress2<T>(lam, mu, e0, e1, e2, sg);
      s11[j] = sg[0];
      s22[j] = sg[1];
      s12[j] = sg[2];
      e_row += (double)e0 * sg[0] + (double)e1 * sg[1] + 2.0 * (double)e2 * sg[2];
    }
    edge[k & 1][0][tid] = s11[XPT - 1];
    edge[k & 1][1][tid] = s12[XPT - 1];
    __syncthreads();
    if (rr >= 0) {
      const int tl = tid == 0 ? KT - 1 : tid - 1;
      const T l11 = edge[k & 1][0][tl], l12 = edge[k & 1][1][tl];
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        const T m11 = j > 0 ? s11[j - 1] : l11, m12 = j > 0 ? s12[j - 1] : l12;
        const T q0 = ((m11 - s11[j]) + (s12_prev[j] - s12[j])) * ih;
        const T q1 = ((m12 - s12[j]) + (s22_prev[j] - s22[j])) * ih;
        rb[2 * lds((rr >> 1) * NX + x0 + j) + (rr & 1)] = own ? q0 : (T)0;
        rb[2 * lds((NP + (rr >> 1)) * NX + x0 + j) + (rr & 1)] = own ? q1 : (T)0;
      }
      const double w = wave_sum(own ? e_row : 0.0);
      if ((tid & 63) == 0) rsum[rr][tid >> 6] = w;
    }
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      s12_prev[j] = s12[j];
      s22_prev[j] = s22[j];
    }
  }
  __syncthreads();
  if (tid < ROWS && y0 + tid < ny) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < KT / 64; ++w) t += rsum[tid][w];
    part[(long long)s * ny + y0 + tid] = t;
  }
  fft_lds<T, NX, 2 * NP, KT, false, FlatIdx<NX>, PL>(buf, tw);
  for (int idx = tid; idx < NXH * 2 * NP; idx += KT) {
    const int sig = idx % (2 * NP), kx = idx / (2 * NP);
    const int comp = sig / NP, pair = sig % NP;
    const C z = buf[lds(sig * NX + kx)];
    const C zm = buf[lds(sig * NX + (NX - kx) % NX)];
    const C a = C{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)};
    const C b = C{(T)0.5 * (z.y + zm.y), (T)0.5 * (zm.x - z.x)};
    const int yy = y0 + 2 * pair;
    C* o = spec + (2LL * s + comp) * spec_ss + (long long)kx * ny;
    if (yy < ny) o[yy] = a;
    if (yy + 1 < ny) o[yy + 1] = b;
  }
}

// Green operator of the unit reference medium on the residual spectrum, one
// displacement component per block (s2 = 2 s + c; spectra of (s, c) at
// s2 * rs).  init: r_hat = q_hat (the transform of f) is stored and no alpha
// is formed; otherwise alpha = rz_k / p.Kp (the partial sums of k_kp_fwd) and
// r_hat -= alpha q_hat.  Then z_hat = r_hat / (N |D|^2) (zero at k = 0) and
// the partial sums of r.z by Parseval over the half spectrum.
template <typename T> struct MechGreenSR {
  const double2* Dx;
  const double2* Dy;
  double inv_n;
  int nx;
  CgState* st;
  double* part;          // r.z partial sums
  const double* part_a;  // p.Kp partial sums of k_kp_fwd (two per grid row), np_a per sample
  int np_a;
  typename cvec<T>::type* rhat;
  long long rs;  // per (sample, component) stride of rhat
  int ny;
  int init;
  __device__ bool begin(int s2, double* red, double& sc) const {
    const int s = s2 >> 1;
    if (init) {
      sc = 0.0;
      return true;
    }
    if (!cg_running(st, s)) return false;
    CgState* S = st + s;
    // the iteration starts here: k = k_next (the row passes set k_next; no
    // block of this pass reads k)
    const int k = S->k_next;
    const bool w = blockIdx.x == 0 && threadIdx.x == 0 && (s2 & 1) == 0;
    if (w) S->k = k;
    const double pap = group_sum_array(part_a + (long long)s * np_a, np_a, red);
    const double rz = S->rz[k & 1];
    if (!(pap > 0.0) || !isfinite(pap)) {
      if (w) {
        S->done = 3;
        S->iter = k;
        S->rr_final = rz;
      }
      return false;
    }
    sc = rz / pap;
    if (w) S->alpha = sc;
    return true;
  }
  // |D_y|^2 and the stored r_hat of the mode, loaded before the forward transform
  struct Pre {
    double dy2;
    typename cvec<T>::type rh;
  };
  __device__ Pre pre(int s2, int kx, int ky) const {
    const double2 d = Dy[ky];
    Pre v;
    v.dy2 = d.x * d.x + d.y * d.y;
    v.rh = init ? typename cvec<T>::type{(T)0, (T)0} : rhat[s2 * rs + (long long)kx * ny + ky];
    return v;
  }
  template <typename CC>
  __device__ void mode(int s2, int kx, int ky, const CC* a, CC* b, double& acc, double sc) const {
    mode_pre(s2, kx, ky, pre(s2, kx, ky), a, b, acc, sc);
  }
  template <typename CC>
  __device__ void mode_pre(int s2, int kx, int ky, const Pre& v, const CC* a, CC* b, double& acc, double sc) const {
    const CC rh = init ? a[0] : CC{v.rh.x - (T)sc * a[0].x, v.rh.y - (T)sc * a[0].y};
    rhat[s2 * rs + (long long)kx * ny + ky] = rh;
    const double2 d1 = Dx[kx];
    const double n2 = (d1.x * d1.x + d1.y * d1.y) + v.dy2;
    if (n2 == 0.0) {
      b[0] = CC{(T)0, (T)0};
      return;
    }
    const double f = inv_n / n2;
    const T ft = (T)f;
    b[0] = CC{rh.x * ft, rh.y * ft};
    const double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
    acc += w * f * ((double)rh.x * rh.x + (double)rh.y * rh.y);
  }
  __device__ void partial(int s2, double v) const {
    if (part && threadIdx.x == 0) part[(long long)s2 * gridDim.x + blockIdx.x] = v;
  }
};

// Inverse pass of the iteration, one component per block: p = z + beta p and
// x += alpha p (p of the previous direction, prefetched with x); init: p = z.
// m.sr must be 1 (the stop test then marks the last x update as due).
// E: prefetch before begin() (single-sample contexts, as MechUEpiC).
template <typename T, bool E> struct MechUEpiSRC {
  MechUEpi<T, 2> m;
  Field<T> x;
  static constexpr int NPRE = 2;
  static constexpr bool EARLY = E;
  __device__ bool begin(int s2, double* red, double& sc) const { return m.begin(s2 / 2, red, sc); }
  __device__ void prefetch(int s2, int y, int xx, T* pre) const {
    const long long i = (long long)y * m.nx + xx;
    pre[0] = m.init ? (T)0 : m.p.at(s2 / 2, s2 % 2, i);
    pre[1] = m.init ? (T)0 : x.at(s2 / 2, s2 % 2, i);
  }
  __device__ void point(int s2, int y, int xx, const T* z, double&, double sc, const T* pre) const {
    const int s = s2 / 2, c = s2 % 2;
    const long long i = (long long)y * m.nx + xx;
    if (m.init) {
      m.p.at(s, c, i) = z[0];
    } else {
      m.p.at(s, c, i) = z[0] + (T)sc * pre[0];
      x.at(s, c, i) = pre[1] + (T)m.st[s].alpha * pre[0];
    }
  }
  __device__ void partial(int, double) const {}
};

// ------------------------------------------------------- two-pass form
// The row stage of the residual-spectrum PCG in one pass: the inverse x
// transforms of z_hat and the direction update that end iteration k, then
// the stiffness stencil, its forward x transforms and the p.Kp partial sums
// that start iteration k + 1 (with the Green column pass, two passes per
// iteration).  A block owns SR_ROWS grid rows and transforms one more row
// above and below them, so that the stencil finds the new direction of its
// neighbour rows without waiting for the blocks that own them; every row is
// one complex signal z_x + i z_y (the two displacement components of the
// row), so a halo row is computed exactly as its owner computes it.  Hence p
// is double-buffered (blocks read halo rows of p_k while owners write
// p_{k+1}) and q_hat goes to a spectrum buffer of its own (blocks read halo
// rows of z_hat while owners write q_hat).  init: p_0 = z_0 and the state of
// the solve, as MechUEpi's init; otherwise the stop test, beta, x += alpha p_k
// (own rows) and p_{k+1} = z + beta p_k.  When the stop test ends the solve
// the pass does nothing but mark the last x update as due (k_sr_finish).
// The iteration counter k is advanced by the Green pass (k = k_next), since
// the lead block here sets k_next while other blocks still read k.
constexpr int SR_ROWS = 2;
// Threads per block: two columns per thread on rows of 1024 and more (the
// registers of NR rows of p per column bound occupancy); shorter rows: NT
// threads where they divide the row, else 128 or one wavefront (rows that
// are a multiple of 64).
constexpr int sr_threads(int nx) {
  return nx >= 1024 ? nx / 2 : nx % NT == 0 ? NT : nx % 128 == 0 ? 128 : 64;
}

template <typename T> struct SrRowArgs {
  const typename cvec<T>::type* zs;  // z_hat, [(2 s + c) spec_ss + kx ny + y]
  typename cvec<T>::type* qs;        // q_hat, same layout, another buffer
  const T* pin;                      // p_k, [s][c][y][x] (2 n per sample)
  T* pout;                           // p_{k+1}
  T* x;
  CgState* st;
  const double* part_rz;  // r.z partial sums of the Green pass, np_rz per sample
  int np_rz;
  double* part_a;  // p.Kp of every grid row, ny per sample
  int ny;
  long long spec_ss;
  T ih;
  int init;
  double tol;
  int maxit;
};

// Fixed-order sum of n partial sums by a block of KT threads (every block
// gets the same value).
template <int KT> __device__ __forceinline__ double kt_sum_array(const double* a, int n, double* red) {
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += KT) t += a[i];
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < KT / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

template <typename T, int NX, int PL, bool EF, int KT = sr_threads(NX)>
__global__ void __launch_bounds__(KT) k_sr_row(SrRowArgs<T> a, MechMat m,
                                               const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  static_assert(NX % KT == 0 && KT % 64 == 0, "k_sr_row: NX must be a multiple of the block size");
  constexpr int R = SR_ROWS;
  constexpr int NR = R + 2;  // transformed rows: y0 - 1 .. y0 + R
  constexpr int XPT = NX / KT;
  constexpr int NXH = NX / 2 + 1;
  constexpr int ITEMS = (NR * NXH + KT - 1) / KT;
  __shared__ C buf[lds_size(NR * NX)];
  __shared__ double red[KT / 64];
  __shared__ double rsum[R][KT / 64];
  const int s = blockIdx.y;
  const int tid = threadIdx.x;
  const int ny = a.ny;
  const int y0 = xcd_block() * R;
  const long long n = m.ss;
  int rowy[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) rowy[r] = (((y0 - 1 + r) % ny) + ny) % ny;
  // z_hat of the NR rows (both components), issued before the CG scalars
  const C* z0 = a.zs + 2LL * s * a.spec_ss;
  const C* z1 = z0 + a.spec_ss;
  C za[ITEMS], zb[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int idx = tid + i * KT;
    if ((NR * NXH) % KT == 0 || idx < NR * NXH) {
      const int r = idx % NR, kx = idx / NR;
      const long long o = (long long)kx * ny + rowy[r];
      za[i] = z0[o];
      zb[i] = z1[o];
    }
  }
  CgState* S = a.st + s;
  if (!a.init && !cg_running(a.st, s)) return;
  const double rz = kt_sum_array<KT>(a.part_rz + (long long)s * a.np_rz, a.np_rz, red);
  double beta = 0.0;
  if (a.init) {
    const double thr = a.tol * a.tol * rz;
    const int done = !isfinite(rz) ? 4 : (rz <= thr ? 1 : (a.maxit <= 0 ? 2 : 0));
    if (lead()) {
      CgState t;
      t.rr_cur = t.rr_prev = 0.0;
      t.bnorm2 = rz;
      t.thr = thr;
      t.rr_final = rz;
      t.rz[0] = rz;
      t.rz[1] = 0.0;
      t.maxit = a.maxit;
      t.k = 0;
      t.k_next = 0;
      t.iter = 0;
      t.done = done;
      t.zero_rhs = rz == 0.0;
      t.alpha = 0.0;
      t.x_pending = 0;
      t.kk[0] = t.kk[1] = 0;
      t.gam[0] = t.gam[1] = t.stp[0] = t.stp[1] = 0.0;
      *S = t;
    }
    if (done) return;
  } else {
    const int k = S->k;
    int code = 0;
    if (!isfinite(rz)) code = 3;
    else if (rz <= S->thr) code = 1;
    else if (k + 1 >= S->maxit) code = 2;
    if (code) {
      if (lead()) {
        S->done = code;
        S->iter = k + 1;
        S->rr_final = rz;
        S->x_pending = 1;
      }
      return;
    }
    beta = rz / S->rz[k & 1];
    if (lead()) {
      S->rz[(k + 1) & 1] = rz;
      S->k_next = k + 1;
    }
  }
  // the rows as complex signals z_x + i z_y over the full spectrum (Hermitian
  // extension of the half spectra; the imaginary parts at kx = 0 and NX / 2
  // are not part of a real field's spectrum and are dropped)
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int idx = tid + i * KT;
    if ((NR * NXH) % KT == 0 || idx < NR * NXH) {
      const int r = idx % NR, kx = idx / NR;
      const C A = za[i], B = zb[i];
      if (kx == 0 || 2 * kx == NX) {
        buf[lds(r * NX + kx)] = C{A.x, B.x};
      } else {
        buf[lds(r * NX + kx)] = C{A.x - B.y, A.y + B.x};
        buf[lds(r * NX + NX - kx)] = C{A.x + B.y, B.x - A.y};
      }
    }
  }
  const T alpha = a.init ? (T)0 : (T)S->alpha;
  // p_k of the NR rows at the thread's columns, issued before the transforms
  const int x0 = tid * XPT;
  const T* pin = a.pin + 2 * n * s;
  T* pout = a.pout + 2 * n * s;
  T* xs = a.x + 2 * n * s;
  T po0[NR][XPT], po1[NR][XPT], xo0[R][XPT], xo1[R][XPT];
  if (!a.init) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        const long long i = (long long)rowy[r] * NX + x0 + j;
        po0[r][j] = pin[i];
        po1[r][j] = pin[n + i];
      }
  }
  __syncthreads();
  fft_lds<T, NX, NR, KT, true, FlatIdx<NX>, PL>(buf, tw);
  // x of the own rows and the material of the stress points (rows
  // y0 - 1 .. y0 + R - 1, columns x0 - 1 .. x0 + XPT - 1), issued after the
  // transforms (fewer registers held across them)
  if (!a.init) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        const long long i = (long long)rowy[r + 1] * NX + x0 + j;
        xo0[r][j] = xs[i];
        xo1[r][j] = xs[n + i];
      }
  }
  const long long so = s * n;
  const bool dmg = m.d != nullptr;
  uint8_t ph[EF ? 1 : R + 1][XPT + 1];
  double ev[EF ? R + 1 : 1][XPT + 1], dd[R + 1][XPT + 1];
#pragma unroll
  for (int r = 0; r < R + 1; ++r)
#pragma unroll
    for (int j = 0; j < XPT + 1; ++j) {
      const long long i = so + (long long)rowy[r] * NX + (x0 - 1 + j + NX) % NX;
      if constexpr (EF)
        ev[r][j] = m.Efield[i];
      else
        ph[r][j] = m.phase[i];
      if (dmg) dd[r][j] = m.d[i];
    }
  // p_{k+1} = z + beta p_k on the NR rows (into LDS for the stencil), x and p
  // of the own rows to memory
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const bool own = r >= 1 && r <= R && y0 + r - 1 < ny;
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const int li = lds(r * NX + x0 + j);
      const C z = buf[li];
      const T p0 = a.init ? z.x : (T)(z.x + (T)beta * po0[r][j]);
      const T p1 = a.init ? z.y : (T)(z.y + (T)beta * po1[r][j]);
      buf[li] = C{p0, p1};
      if (own) {
        const long long i = (long long)rowy[r] * NX + x0 + j;
        pout[i] = p0;
        pout[n + i] = p1;
        if (!a.init) {
          xs[i] = xo0[r - 1][j] + alpha * po0[r][j];
          xs[n + i] = xo1[r - 1][j] + alpha * po1[r][j];
        }
      }
    }
  }
  __syncthreads();
  auto lame = [&](int r, int j, double& lam, double& mu) {
    if constexpr (EF) {
      lam = ev[r][j] * m.lam_per_E;
      mu = ev[r][j] * m.mu_per_E;
    } else if (m.lm_dev) {
      lam = m.lm_dev[16 * s + ph[r][j]];
      mu = m.lm_dev[16 * s + 8 + ph[r][j]];
    } else if (m.nphase <= 2) {
      lam = ph[r][j] ? m.lm.a[1] : m.lm.a[0];
      mu = ph[r][j] ? m.lm.b[1] : m.lm.b[0];
    } else {
      pick(m.lm, ph[r][j], lam, mu);
    }
    if (dmg) {
      const double g = (1.0 - dd[r][j]) * (1.0 - dd[r][j]) + m.kappa;
      lam *= g;
      mu *= g;
    }
  };
  // stress row by row (rows y0 - 1 .. y0 + R - 1, columns x0 - 1 ..
  // x0 + XPT - 1, p from LDS), q = K p_{k+1} and the energy form of p.Kp on
  // the own rows
  const T ih = a.ih;
  T q0[R][XPT], q1[R][XPT];
  T s12p[XPT + 1], s22p[XPT + 1];
#pragma unroll
  for (int r = 0; r < R + 1; ++r) {
    C pc[XPT + 2], pd[XPT + 1];
#pragma unroll
    for (int j = 0; j < XPT + 2; ++j) pc[j] = buf[lds(r * NX + (x0 - 1 + j + NX) % NX)];
#pragma unroll
    for (int j = 0; j < XPT + 1; ++j) pd[j] = buf[lds((r + 1) * NX + (x0 - 1 + j + NX) % NX)];
    T s11[XPT + 1], s22[XPT + 1], s12[XPT + 1];
    double e_row = 0.0;
#pragma unroll
    for (int j = 0; j < XPT + 1; ++j) {
      const T g11 = (pc[j + 1].x - pc[j].x) * ih;
      const T g12 = (pd[j].x - pc[j].x) * ih;
      const T g21 = (pc[j + 1].y - pc[j].y) * ih;
      const T g22 = (pd[j].y - pc[j].y) * ih;
      const T e0 = g11, e1 = g22, e2 = (T)0.5 * (g12 + g21);
      double lam, mu;
      lame(r, j, lam, mu);
      T sg[3];
      stress2<T>(lam, mu, e0, e1, e2, sg);
      s11[j] = sg[0];
      s22[j] = sg[1];
      s12[j] = sg[2];
      if (j >= 1) e_row += (double)e0 * sg[0] + (double)e1 * sg[1] + 2.0 * (double)e2 * sg[2];
    }
    if (r >= 1) {
      const int rr = r - 1;
      const bool own = y0 + rr < ny;
#pragma unroll
      for (int j = 0; j < XPT; ++j) {
        q0[rr][j] = own ? ((s11[j] - s11[j + 1]) + (s12p[j + 1] - s12[j + 1])) * ih : (T)0;
        q1[rr][j] = own ? ((s12[j] - s12[j + 1]) + (s22p[j + 1] - s22[j + 1])) * ih : (T)0;
      }
      const double w = wave_sum(own ? e_row : 0.0);
      if ((tid & 63) == 0) rsum[rr][tid >> 6] = w;
    }
#pragma unroll
    for (int j = 0; j < XPT + 1; ++j) {
      s12p[j] = s12[j];
      s22p[j] = s22[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < R; ++rr)
#pragma unroll
    for (int j = 0; j < XPT; ++j) buf[lds(rr * NX + x0 + j)] = C{q0[rr][j], q1[rr][j]};
  if (tid < R && y0 + tid < ny) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < KT / 64; ++w) t += rsum[tid][w];
    a.part_a[(long long)s * ny + y0 + tid] = t;
  }
  __syncthreads();
  fft_lds<T, NX, R, KT, false, FlatIdx<NX>, PL>(buf, tw);
  // the two components' half spectra from each row's signal, stored
  // transposed (R consecutive y of a (component, kx) together)
  C* q0s = a.qs + 2LL * s * a.spec_ss;
  for (int idx = tid; idx < NXH * 2 * R; idx += KT) {
    const int rr = idx % R, comp = (idx / R) & 1, kx = idx / (2 * R);
    const int y = y0 + rr;
    if (y < ny) {
      const C z = buf[lds(rr * NX + kx)];
      const C zm = buf[lds(rr * NX + (NX - kx) % NX)];
      const C v = comp == 0 ? C{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)}
                            : C{(T)0.5 * (z.y + zm.y), (T)0.5 * (zm.x - z.x)};
      q0s[comp * a.spec_ss + (long long)kx * ny + y] = v;
    }
  }
}

// The x update still due when the stop test ended the solve in the inverse
// pass: x += alpha p for every sample whose state says so (one launch after
// the solve; p is the last direction, alpha its step).
// p_odd: the direction buffer of odd iterations (the two-pass form keeps p
// double-buffered; the same buffer as p otherwise).
template <typename T>
__global__ void __launch_bounds__(PT) k_sr_finish(T* __restrict__ x, const T* p, const T* p_odd, const CgState* st,
                                                  long long n2) {
  const int s = blockIdx.y;
  if (!st[s].x_pending) return;
  const T a = (T)st[s].alpha;
  if (st[s].k & 1) p = p_odd;
  x += n2 * s;
  p += n2 * s;
  for (long long i = blockIdx.x * (long long)PT + threadIdx.x; i < n2; i += (long long)gridDim.x * PT)
    x[i] += a * p[i];
}

// Identity symbol with the 1/N of the inverse transform (the kernel-level
// hook that brings q back to real space), one component per block.
template <typename T> struct ScaleSym {
  double inv_n;
  __device__ bool begin(int, double*, double&) const { return true; }
  template <typename CC>
  __device__ void mode(int, int, int, const CC* a, CC* b, double&, double) const {
    b[0] = CC{a[0].x * (T)inv_n, a[0].y * (T)inv_n};
  }
  __device__ void partial(int, double) const {}
};

// out = z, one component per block (the same hook's inverse row pass).
template <typename T> struct StoreCompEpi {
  Field<T> out;
  int nx;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s2, int y, int xx, const T* z, double&, double) const {
    out.at(s2 / 2, s2 % 2, (long long)y * nx + xx) = z[0];
  }
  __device__ void partial(int, double) const {}
};

}  // namespace fgcg
