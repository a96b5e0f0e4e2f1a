// Pointwise kernels of the path (no transforms): CG set-up, post-processing,
// precipitation/eigenstrain, history update, observables.  The non-template
// kernels have internal linkage: every translation unit that includes this
// header launches its own copy.
#pragma once
#include "ops2d.hpp"

namespace fgcg {

constexpr int PT = 256;

// Sum the partial array of ||b||^2, set the CG state of sample s (one block
// per sample).  done = 1 with zero_rhs = 1 when b = 0; done = 4 when ||b|| is
// not finite.
static __global__ void __launch_bounds__(NT) k_cg_init(CgState* st, const double* part_b, int np,
                                                int pstride, double tol, int maxit) {
  __shared__ double red[NT / 64];
  const int s = blockIdx.x;
  const double b2 = block_sum_array(part_b + (long long)s * pstride, np, red);
  if (threadIdx.x == 0) {
    CgState t;
    t.rr_cur = t.rr_prev = 0.0;
    t.bnorm2 = b2;
    t.thr = tol * tol * b2;
    t.rr_final = b2;
    t.maxit = maxit;
    t.k = 0;
    t.iter = 0;
    t.zero_rhs = b2 == 0.0;
    t.done = !isfinite(b2) ? 4 : (b2 == 0.0 ? 1 : 0);
    t.rz[0] = t.rz[1] = 0.0;
    t.k_next = 0;
    t.alpha = 0.0;
    t.x_pending = 0;
    t.kk[0] = t.kk[1] = 0;
    t.gam[0] = t.gam[1] = t.stp[0] = t.stp[1] = 0.0;
    st[s] = t;
  }
}

// Block partial sums of |v|^2 for a double field of n voxels.
static __global__ void __launch_bounds__(PT) k_norm2(const double* v, long long n, double* part) {
  __shared__ double red[NT / 64];
  double a = 0.0;
  for (long long i = blockIdx.x * (long long)PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT)
    a += v[i] * v[i];
  const double t = block_sum(a, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename TO, typename TI>
__global__ void __launch_bounds__(PT) k_convert(TO* out, const TI* in, long long n) {
  for (long long i = blockIdx.x * (long long)PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT)
    out[i] = (TO)in[i];
}

// c = c_dir on the band, x elsewhere (spectral diffusion step)
template <typename T>
__global__ void __launch_bounds__(PT) k_diff_finish(double* c, const T* x, long long n, int nx,
                                                    int band, double c_dir) {
  for (long long i = blockIdx.x * (long long)PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT)
    c[i] = (int)(i % nx) < band ? c_dir : (double)x[i];
}

// Empty kernel (the event-gap calibration of the profiling hooks).
static __global__ void __launch_bounds__(NT) k_noop(int) {}

// Precipitation (first-order, the same rate as the sink of the diffusion
// step): f = min(1, f + dt k(phase) c) wherever the phase's rate k is
// positive (f unchanged elsewhere); e = e_per_f f (eq. eigen-simplify with a
// linear precipitate-to-strain map).  With diffuse = 0 the eigenstrain of the
// pores (phase 0) follows the prescribed ramp value e_pres instead.
static __global__ void __launch_bounds__(PT) k_precip(const uint8_t* phase, const double* c, double* f,
                                               double* e, long long n, PhaseTab dtk, double e_per_f,
                                               int diffuse, double e_pres) {
  for (long long i = blockIdx.x * (long long)PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT) {
    const int ph = phase[i];
    if (diffuse) {
      double rate, unused;
      pick(dtk, ph, rate, unused);
      const double fv = rate > 0.0 ? fmin(1.0, f[i] + rate * c[i]) : f[i];
      f[i] = fv;
      e[i] = e_per_f * fv;
    } else {
      e[i] = ph == 0 ? e_pres : 0.0;
    }
  }
}

// H = max(H, psi+(eps - e I)) with the undegraded Lame constants (Sec. 2.4,
// eq. energy, 2D): psi+ = (lambda + mu)/2 <tr>_+^2 + mu dev:dev.
static __global__ void __launch_bounds__(PT) k_history(MechMat m, const double* strain, const double* e,
                                                double* H, long long n) {
  for (long long i = blockIdx.x * (long long)PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT) {
    double lam, mu;
    m.get(0, i, lam, mu);  // m.d is null here: undegraded
    const double ev = e[i];
    const double l11 = strain[i] - ev, l22 = strain[n + i] - ev, l12 = strain[2 * n + i];
    const double tr = l11 + l22;
    const double trp = 0.5 * (tr + fabs(tr));
    const double d11 = l11 - 0.5 * tr, d22 = l22 - 0.5 * tr;
    const double devdev = d11 * d11 + d22 * d22 + 2.0 * l12 * l12;
    const double psi = 0.5 * (lam + mu) * trp * trp + mu * devdev;
    H[i] = fmax(H[i], psi);
  }
}

// Observables: partial [max d, count(solid & d > 0.9), sum_solid d, sum f, count solid]
static __global__ void __launch_bounds__(PT) k_observe(const uint8_t* phase, const double* d,
                                                const double* f, long long n, double* part) {
  __shared__ double red[NT / 64];
  __shared__ double redm[NT];
  double mx = 0.0, cnt = 0.0, sd = 0.0, sf = 0.0, ns = 0.0;
  for (long long i = blockIdx.x * (long long)PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT) {
    const double dv = d[i];
    mx = fmax(mx, dv);
    sf += f[i];
    if (phase[i] != 0) {
      ns += 1.0;
      sd += dv;
      cnt += dv > 0.9 ? 1.0 : 0.0;
    }
  }
  redm[threadIdx.x] = mx;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) redm[threadIdx.x] = fmax(redm[threadIdx.x], redm[threadIdx.x + w]);
    __syncthreads();
  }
  const double t1 = block_sum(cnt, red), t2 = block_sum(sd, red), t3 = block_sum(sf, red),
               t4 = block_sum(ns, red);
  if (threadIdx.x == 0) {
    part[5 * blockIdx.x + 0] = redm[0];
    part[5 * blockIdx.x + 1] = t1;
    part[5 * blockIdx.x + 2] = t2;
    part[5 * blockIdx.x + 3] = t3;
    part[5 * blockIdx.x + 4] = t4;
  }
}

}  // namespace fgcg
