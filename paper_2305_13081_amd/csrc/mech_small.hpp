// Mechanics PCG for small square 2D grids in one workgroup, one launch.
//
// The same method and iteration as mech_u.hpp (displacement form of the
// projected CG of Sec. 2.3 / App. A: K u = f with K = grad^H g C grad, Green
// preconditioner 1/|D|^2 with the forward-difference symbol of Sec. 2.6), for
// an N x N grid with N <= 64, FP64, one sample.  A grid this small leaves the
// GPU idle between the four passes of an iteration, so here 1024 threads run
// the whole solve: every thread keeps p of its own voxels in registers and
// x, r, q of its own voxels in memory (no other thread touches them); the
// transform buffer in LDS holds r (then z) for the Green operator (full
// complex 2D transforms, rows then columns) and p for the stiffness stencil,
// which reads the neighbours' p from there.  The stop test, alpha,
// beta and the breakdown and iteration-limit outcomes are those of the
// multi-pass solver; results agree with it up to rounding.
#pragma once
#include "mech_u.hpp"

namespace fgcg {

constexpr int NTS = 1024;                 // threads of the single workgroup
constexpr int SMALL_MAX = 64;             // largest side handled here

__device__ __forceinline__ double block_sum_small(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NTS / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Column signals of the [comp][y][x] buffer: signal sig = c N + x, element y.
template <int N> struct ColIdx {
  static __device__ __forceinline__ int at(int sig, int y) {
    const int c = sig / N, x = sig - c * N;
    return lds((c * N + y) * N + x);
  }
};

// r holds f on entry and x = 0; x holds the solution on exit; q is scratch;
// *st the outcome.  Components are N^2 apart.
template <int N>
__global__ void __launch_bounds__(NTS) k_mech_small(MechMat m, double* __restrict__ x, double* __restrict__ r,
                                                    double* __restrict__ q, double ih,
                                                    const double2* __restrict__ Dx,
                                                    const double2* __restrict__ Dy,
                                                    const double2* __restrict__ tw, double tol, int maxit,
                                                    CgState* st) {
  using C = double2;
  constexpr int NN = N * N;
  constexpr int J = (NN + NTS - 1) / NTS;  // own voxels per thread
  __shared__ C buf[lds_size(2 * NN)];
  __shared__ double red[NTS / 64];
  const int tid = threadIdx.x;
  const double inv_n = 1.0 / (double)NN;
  double pr[J][2];
  double lamv[J], muv[J];  // g C of the own voxels, looked up once
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int i = tid + j * NTS;
    pr[j][0] = pr[j][1] = 0.0;
    lamv[j] = muv[j] = 0.0;
    if (i < NN) m.get(0, i, lamv[j], muv[j]);
  }
  // z = M r into buf (real parts), returns r.z (Parseval over the full spectrum)
  auto green = [&]() -> double {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = tid + j * NTS;
      if (i < NN) {
        buf[lds(i)] = C{r[i], 0.0};
        buf[lds(NN + i)] = C{r[NN + i], 0.0};
      }
    }
    __syncthreads();
    fft_lds<double, N, 2 * N, NTS, false, FlatIdx<N>, true>(buf, tw);
    fft_lds<double, N, 2 * N, NTS, false, ColIdx<N>, true>(buf, tw);
    double acc = 0.0;
    int t0 = tid;
    asm volatile("" : "+v"(t0));  // symbol loads stay inside the iteration loop
    for (int i = t0; i < 2 * NN; i += NTS) {
      const int rem = i % NN, ky = rem / N, kx = rem - ky * N;
      const double2 d1 = Dx[kx <= N / 2 ? kx : N - kx], d2 = Dy[ky];
      const double n2 = d1.x * d1.x + d1.y * d1.y + d2.x * d2.x + d2.y * d2.y;
      C a = buf[lds(i)];
      if (n2 == 0.0) {
        a = C{0.0, 0.0};
      } else {
        const double fct = inv_n / n2;
        acc += fct * (a.x * a.x + a.y * a.y);
        a = C{a.x * fct, a.y * fct};
      }
      buf[lds(i)] = a;
    }
    const double rz = block_sum_small(acc, red);
    fft_lds<double, N, 2 * N, NTS, true, ColIdx<N>, true>(buf, tw);
    fft_lds<double, N, 2 * N, NTS, true, FlatIdx<N>, true>(buf, tw);
    return rz;
  };
  // p = z + beta p (own voxels), and p into buf for the stencil
  auto direction = [&](double beta, bool first) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = tid + j * NTS;
      if (i < NN) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const double z = buf[lds(c * NN + i)].x;
          pr[j][c] = first ? z : z + beta * pr[j][c];
          buf[lds(c * NN + i)] = C{pr[j][c], 0.0};
        }
      }
    }
    __syncthreads();
  };
  auto pv = [&](int c, int y, int xx) -> double { return buf[lds(c * NN + y * N + xx)].x; };
  double* sgb = reinterpret_cast<double*>(buf);  // stresses [3][NN] over the p buffer
  double rz = green();
  const double thr = tol * tol * rz;
  int done = !isfinite(rz) ? 4 : (rz <= thr ? 1 : (maxit <= 0 ? 2 : 0));
  int iter = 0;
  const double bnorm2 = rz;
  double rr_final = rz;
  direction(0.0, true);
  for (int k = 0; done == 0; ++k) {
    // q = K p, p.Kp: the stress of the own voxels from p in buf, then (with p
    // in registers) the stresses replace p in buf and the divergence takes the
    // x - 1 and y - 1 neighbours from there
    double acc = 0.0;
    double sg[J][3];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = tid + j * NTS;
      sg[j][0] = sg[j][1] = sg[j][2] = 0.0;
      if (i < NN) {
        const int y = i / N, xx = i - y * N;
        const int xp = xx + 1 == N ? 0 : xx + 1, yp = y + 1 == N ? 0 : y + 1;
        const double u1 = pv(0, y, xx), u2 = pv(1, y, xx);
        const double g11 = (pv(0, y, xp) - u1) * ih, g12 = (pv(0, yp, xx) - u1) * ih;
        const double g21 = (pv(1, y, xp) - u2) * ih, g22 = (pv(1, yp, xx) - u2) * ih;
        const double e12 = 0.5 * (g12 + g21);
        stress2<double>(lamv[j], muv[j], g11, g22, e12, sg[j]);
        acc += g11 * sg[j][0] + g22 * sg[j][1] + 2.0 * e12 * sg[j][2];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = tid + j * NTS;
      if (i < NN)
#pragma unroll
        for (int c = 0; c < 3; ++c) sgb[c * NN + i] = sg[j][c];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = tid + j * NTS;
      if (i < NN) {
        const int y = i / N, xx = i - y * N;
        const int ixm = y * N + (xx == 0 ? N - 1 : xx - 1), iym = (y == 0 ? N - 1 : y - 1) * N + xx;
        const double sx[3] = {sgb[ixm], sgb[NN + ixm], sgb[2 * NN + ixm]};
        const double sy[3] = {sgb[iym], sgb[NN + iym], sgb[2 * NN + iym]};
        double qq[2];
        div_adj<double>(sg[j], sx, sy, ih, qq);
        q[i] = qq[0];
        q[NN + i] = qq[1];
      }
    }
    const double pap = block_sum_small(acc, red);
    if (!(pap > 0.0) || !isfinite(pap)) {
      done = 3;
      iter = k;
      rr_final = rz;
      break;
    }
    const double alpha = rz / pap;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = tid + j * NTS;
      if (i < NN) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          x[c * NN + i] += alpha * pr[j][c];
          r[c * NN + i] -= alpha * q[c * NN + i];
        }
      }
    }
    const double rzn = green();
    if (!isfinite(rzn)) {
      done = 3;
      iter = k + 1;
      rr_final = rzn;
    } else if (rzn <= thr) {
      done = 1;
      iter = k + 1;
      rr_final = rzn;
    } else if (k + 1 >= maxit) {
      done = 2;
      iter = k + 1;
      rr_final = rzn;
    } else {
      direction(rzn / rz, false);
      rz = rzn;
    }
  }
  if (tid == 0) {
    CgState s;
    s.rr_cur = s.rr_prev = 0.0;
    s.thr = thr;
    s.bnorm2 = bnorm2;
    s.rr_final = rr_final;
    s.rz[0] = s.rz[1] = 0.0;
    s.maxit = maxit;
    s.k = s.k_next = iter;
    s.iter = iter;
    s.done = done;
    s.zero_rhs = bnorm2 == 0.0;
    *st = s;
  }
}

}  // namespace fgcg
