// Physics functors plugged into the fused 2D passes, CG control state, and
// the materials.
//
// Materials of the mechanics (Sec. 2.3): isotropic per phase or per voxel,
// degraded by g = (1-d)^2 + kappa (Sec. 2.4); the solvers themselves are in
// mech_u.hpp (2D) and mech3.hpp (3D).
//
// Phase field (Sec. 2.4, eq. crack-fft): A d = (Gc/(2 l0) + H) d
// + (Gc l0 / 2) F^-1[|D|^2 F d].
//
// Diffusion step: A c = (1/dt + k_r) c + sum_a F^-1[conj(D_a) F[D(x) F^-1[D_a F c]]],
// on the free voxels of a Dirichlet band x < band_width.
//
// The CG solves of these scalar operators through the FFT passes (the
// spectral option) take three (phase field) or five (diffusion) launches per
// iteration: the first pass reduces the partial sums of r.r left by the
// previous iteration, checks convergence, forms beta and p = r + beta p in its
// prologue and accumulates p.Ap from pointwise quantities (the diagonal part
// plus the Parseval sum of the Laplacian part, or plus sum D |grad p|^2); the
// last pass then knows alpha = r.r / p.Ap and applies x += alpha p,
// r -= alpha q without storing q.  All sums are FP64, block-reduced in a fixed
// order, so repeated runs are bitwise identical.
#pragma once
#include <stdint.h>

#include "passes2d.hpp"

namespace fgcg {

struct CgState {
  double rr_cur;   // r.r of the current iteration (written by the forward pass)
  double rr_prev;  // r.r of the previous iteration (written by the inverse pass)
  double thr;      // tol^2 ||b||^2
  double bnorm2;
  double rr_final;
  double rz[2];    // preconditioned CG: r.z of iterations with parity 0 / 1
  int maxit;
  int k;           // iteration counter
  int k_next;      // preconditioned CG: next counter value, published by the first pass
  int iter;        // iterations taken when the solve ended
  int done;        // 0 running, 1 converged, 2 iteration limit, 3 breakdown, 4 non-finite rhs
  int zero_rhs;
  double alpha;    // residual-spectrum PCG: step of the current direction
  int x_pending;   // residual-spectrum PCG: the last x update is still due
  // one-reduction scalar CG: iteration counter, r.r and step of the previous
  // iteration, by the parity of the launch that reads them (the launch of
  // parity P reads slot P and its lead writes slot P ^ 1)
  int kk[2];
  double gam[2], stp[2];
};

// The iteration number lives in device memory so that a chunk of iterations
// can be captured once in a graph and replayed.  Within one launch only the
// lead thread of block 0 writes the state, and it writes fields that no other
// block of that launch reads.
struct CgCtl {
  CgState* st;
  double* part_a;   // p.Ap partial sums
  double* part_rr;  // r.r partial sums
  int np_a, np_rr;
  int pa_stride, prr_stride;
};

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

// Voxel range of this block for the kernels that walk a grid of `rows` rows of
// nx voxels (row = z ny + y): the rows are cut into 8 contiguous slabs, one per
// XCD (the hardware hands block b to XCD b % 8), and the blocks of a slab walk
// it together, so the neighbour rows a block reads were brought into the same
// L2 by the blocks beside it.  gridDim.x must be a multiple of 8.  Grids hold
// fewer than 2^31 voxels, so the row of voxel v is (unsigned)v / nx.
struct SlabIter {
  long long v0, v1, step;
  __device__ SlabIter(int nx, long long rows) {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b & 7, q = b >> 3, nq = nb >> 3;
    const long long r0 = rows * x / 8, r1 = rows * (x + 1) / 8;
    v0 = r0 * nx + (long long)q * NT + threadIdx.x;
    v1 = r1 * nx;
    step = (long long)nq * NT;
  }
};

__device__ __forceinline__ bool cg_running(const CgState* st, int s) {
  return !__syncthreads_or(st[s].done != 0);
}

// Forward pass of an iteration: beta (0 on the first iteration, which the
// prologues use to take p = r), convergence and iteration-limit tests.
__device__ __forceinline__ bool cg_begin_dir(const CgCtl& c, int s, double* red, double& beta) {
  CgState* st = c.st + s;
  if (!cg_running(c.st, s)) return false;
  const int k = st->k;
  const double rr = block_sum_array(c.part_rr + (long long)s * c.prr_stride, c.np_rr, red);
  int code = 0;
  if (!isfinite(rr)) code = 3;
  else if (rr <= st->thr) code = 1;
  else if (k >= st->maxit) code = 2;
  if (code) {
    if (lead()) {
      st->done = code;
      st->iter = k;
      st->rr_final = rr;
    }
    return false;
  }
  beta = k == 0 ? 0.0 : rr / st->rr_prev;
  if (lead()) st->rr_cur = rr;
  return true;
}

// Inverse pass of an iteration: alpha = r.r / p.Ap, breakdown test, and the
// lead thread advances the iteration counter.
__device__ __forceinline__ bool cg_begin_step(const CgCtl& c, int s, double* red, double& alpha) {
  CgState* st = c.st + s;
  if (!cg_running(c.st, s)) return false;
  const double pap = block_sum_array(c.part_a + (long long)s * c.pa_stride, c.np_a, red);
  const double rr = st->rr_cur;
  if (!(pap > 0.0) || !isfinite(pap)) {
    if (lead()) {
      st->done = 3;
      st->iter = st->k;
      st->rr_final = rr;
    }
    return false;
  }
  alpha = rr / pap;
  if (lead()) {
    st->rr_prev = rr;
    st->k = st->k + 1;
  }
  return true;
}

__device__ __forceinline__ void store_partial(double* a, int stride, int s, int off, double v) {
  if (threadIdx.x == 0) a[(long long)s * stride + off + blockIdx.x] = v;
}

template <typename T> struct Field {
  T* p;
  long long n;   // voxels per component
  long long ss;  // per-sample stride
  __device__ __forceinline__ T& at(int s, int c, long long i) const { return p[s * ss + c * n + i]; }
};

// ------------------------------------------------------------- materials
constexpr int MAXPH = 8;
struct PhaseTab {
  double a[MAXPH];
  double b[MAXPH];
};

// Select the entries of phase ph with static indices only, so the table stays
// in kernel-argument registers instead of being copied to scratch memory.
__device__ __forceinline__ void pick(const PhaseTab& t, int ph, double& a, double& b) {
  a = t.a[0];
  b = t.b[0];
#pragma unroll
  for (int q = 1; q < MAXPH; ++q) {
    if (ph == q) {
      a = t.a[q];
      b = t.b[q];
    }
  }
}

struct MechMat {
  const uint8_t* phase;
  const double* d;       // nullable
  const double* Efield;  // nullable: per-voxel Young's modulus
  const double* lm_dev;  // nullable: per-sample tables [s][lambda[8], mu[8]] (batches)
  long long ss;          // per-sample stride of the scalar fields
  int nphase;            // entries of lm in use (0 with Efield)
  double kappa;
  double lam_per_E, mu_per_E;  // used with Efield
  PhaseTab lm;                 // a = lambda, b = mu per phase
  __device__ __forceinline__ void get(int s, long long i, double& lam, double& mu) const {
    if (Efield) {
      const double E = Efield[s * ss + i];
      lam = E * lam_per_E;
      mu = E * mu_per_E;
    } else if (lm_dev) {
      const int ph = phase[s * ss + i];
      lam = lm_dev[16 * s + ph];
      mu = lm_dev[16 * s + 8 + ph];
    } else {
      pick(lm, phase[s * ss + i], lam, mu);
    }
    if (d) {
      const double dd = d[s * ss + i];
      const double g = (1.0 - dd) * (1.0 - dd) + kappa;
      lam *= g;
      mu *= g;
    }
  }
};

template <typename T>
__device__ __forceinline__ void stress2(double lam, double mu, T e11, T e22, T e12, T* sg) {
  const T tr = e11 + e22;
  const T l = (T)lam, m2 = (T)(2.0 * mu);
  sg[0] = l * tr + m2 * e11;
  sg[1] = l * tr + m2 * e22;
  sg[2] = m2 * e12;
}

// out = sign * q ; optionally x = 0 ; partial |out|^2 into part
template <typename T, int NC> struct StoreEpi {
  Field<T> out;
  Field<T> zero;  // nullable
  T sign;
  int nx;
  double* part;
  int pstride;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int xx, const T* q, double& acc, double sc) const {
    const long long i = (long long)y * nx + xx;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T v = sign * q[k];
      out.at(s, k, i) = v;
      if (zero.p) zero.at(s, k, i) = (T)0;
      acc += (double)v * (double)v;
    }
  }
  __device__ void partial(int s, double v) const {
    if (part) store_partial(part, pstride, s, 0, v);
  }
};

// ------------------------------------------------------------ phase field
template <typename T> struct PfCgPro {
  Field<T> p, r;
  const double* H;
  long long ss;
  double a;  // Gc / (2 l0)
  int nx;
  CgCtl c;
  __device__ bool begin(int s, double* red, double& sc) const { return cg_begin_dir(c, s, red, sc); }
  __device__ void point(int s, int y, int x, T* out, double& acc, double sc) const {
    const long long i = (long long)y * nx + x;
    const T rv = r.at(s, 0, i);
    const T pp = sc == 0.0 ? rv : rv + (T)sc * p.at(s, 0, i);
    p.at(s, 0, i) = pp;
    out[0] = pp;
    acc += (a + H[s * ss + i]) * (double)pp * (double)pp;
  }
  __device__ void partial(int s, double v) const { store_partial(c.part_a, c.pa_stride, s, 0, v); }
};

template <typename T> struct CopyPro {
  Field<T> v;
  int nx;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int x, T* out, double&, double) const { out[0] = v.at(s, 0, (long long)y * nx + x); }
  __device__ void partial(int, double) const {}
};

template <typename T> struct PfLap {
  const double2* Dx;
  const double2* Dy;
  double cl;  // (Gc l0 / 2) / N
  int nx;
  const CgState* st;  // nullable
  double* part;       // nullable: Parseval partial of p.Lp
  int pstride, poff;
  __device__ bool begin(int s, double*, double&) const { return st == nullptr || cg_running(st, s); }
  template <typename C>
  __device__ void mode(int, int kx, int ky, const C* a, C* b, double& acc, double) const {
    const double2 d1 = Dx[kx], d2 = Dy[ky];
    const double n2 = d1.x * d1.x + d1.y * d1.y + d2.x * d2.x + d2.y * d2.y;
    const T f = (T)(cl * n2);
    b[0] = C{a[0].x * f, a[0].y * f};
    const double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
    acc += w * (double)f * ((double)a[0].x * a[0].x + (double)a[0].y * a[0].y);
  }
  __device__ void partial(int s, double v) const {
    if (part) store_partial(part, pstride, s, poff, v);
  }
};

template <typename T> struct PfCgEpi {
  Field<T> x, r, p;
  const double* H;
  long long ss;
  double a;
  int nx;
  CgCtl c;
  __device__ bool begin(int s, double* red, double& sc) const { return cg_begin_step(c, s, red, sc); }
  __device__ void point(int s, int y, int xx, const T* q, double& acc, double sc) const {
    const long long i = (long long)y * nx + xx;
    const T pv = p.at(s, 0, i);
    const T qv = (T)(a + H[s * ss + i]) * pv + q[0];
    const T al = (T)sc;
    x.at(s, 0, i) += al * pv;
    const T rv = r.at(s, 0, i) - al * qv;
    r.at(s, 0, i) = rv;
    acc += (double)rv * (double)rv;
  }
  __device__ void partial(int s, double v) const { store_partial(c.part_rr, c.prr_stride, s, 0, v); }
};

// r = H - A x (initial residual of a warm start), partial |r|^2
template <typename T> struct PfResEpi {
  Field<T> x, r;
  const double* H;
  long long ss;
  double a;
  int nx;
  double* part;
  int pstride;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int xx, const T* q, double& acc, double sc) const {
    const long long i = (long long)y * nx + xx;
    const double h = H[s * ss + i];
    const T rv = (T)(h - ((a + h) * (double)x.at(s, 0, i) + (double)q[0]));
    r.at(s, 0, i) = rv;
    acc += (double)rv * (double)rv;
  }
  __device__ void partial(int s, double v) const { store_partial(part, pstride, s, 0, v); }
};

// -------------------------------------------------------------- diffusion
struct DiffCoef {
  const uint8_t* phase;
  long long ss;
  PhaseTab dk;  // a = D, b = reaction rate, per phase
  double inv_dt;
  int band;  // voxels with x < band are Dirichlet
};

template <typename T> struct DiffCgPro {
  Field<T> p, r;
  DiffCoef co;
  int nx;
  CgCtl c;
  __device__ bool begin(int s, double* red, double& sc) const { return cg_begin_dir(c, s, red, sc); }
  __device__ void point(int s, int y, int x, T* out, double& acc, double sc) const {
    const long long i = (long long)y * nx + x;
    const T rv = r.at(s, 0, i);
    const T pp = sc == 0.0 ? rv : rv + (T)sc * p.at(s, 0, i);
    p.at(s, 0, i) = pp;
    out[0] = pp;
    double D, kr;
    pick(co.dk, co.phase[s * co.ss + i], D, kr);
    acc += (co.inv_dt + kr) * (double)pp * (double)pp;
  }
  __device__ void partial(int s, double v) const { store_partial(c.part_a, c.pa_stride, s, 0, v); }
};

// v = c_dir on the band, else (src ? src : 0)
template <typename T> struct BandSrcPro {
  const double* src;  // nullable
  long long ss;
  int band;
  double c_dir;
  int nx;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int x, T* out, double&, double) const {
    const long long i = (long long)y * nx + x;
    out[0] = (T)(x < band ? c_dir : (src ? src[s * ss + i] : 0.0));
  }
  __device__ void partial(int, double) const {}
};

template <typename T> struct DiffGrad {
  const double2* Dx;
  const double2* Dy;
  double inv_n;
  const CgState* st;
  __device__ bool begin(int s, double*, double&) const { return st == nullptr || cg_running(st, s); }
  template <typename C>
  __device__ void mode(int, int kx, int ky, const C* a, C* b, double&, double) const {
    const double2 d1 = Dx[kx], d2 = Dy[ky];
    const C D1 = C{(T)(d1.x * inv_n), (T)(d1.y * inv_n)};
    const C D2 = C{(T)(d2.x * inv_n), (T)(d2.y * inv_n)};
    b[0] = cmul(D1, a[0]);
    b[1] = cmul(D2, a[0]);
  }
  __device__ void partial(int, double) const {}
};

template <typename T> struct DiffMid {
  DiffCoef co;
  int nx;
  const CgState* st;  // nullable
  double* part;       // nullable: sum D |grad p|^2
  int pstride, poff;
  __device__ bool begin(int s, double*, double&) const { return st == nullptr || cg_running(st, s); }
  __device__ void point(int s, int y, int x, const T* g, T* j, double& acc, double) const {
    const long long i = (long long)y * nx + x;
    double D, kr;
    pick(co.dk, co.phase[s * co.ss + i], D, kr);
    j[0] = (T)D * g[0];
    j[1] = (T)D * g[1];
    acc += D * ((double)g[0] * g[0] + (double)g[1] * g[1]);
  }
  __device__ void partial(int s, double v) const {
    if (part) store_partial(part, pstride, s, poff, v);
  }
};

template <typename T> struct DiffDiv {
  const double2* Dx;
  const double2* Dy;
  double inv_n;
  const CgState* st;
  __device__ bool begin(int s, double*, double&) const { return st == nullptr || cg_running(st, s); }
  template <typename C>
  __device__ void mode(int, int kx, int ky, const C* a, C* b, double&, double) const {
    const double2 d1 = Dx[kx], d2 = Dy[ky];
    const C D1 = C{(T)(d1.x * inv_n), (T)(-d1.y * inv_n)};
    const C D2 = C{(T)(d2.x * inv_n), (T)(-d2.y * inv_n)};
    b[0] = cadd(cmul(D1, a[0]), cmul(D2, a[1]));
  }
  __device__ void partial(int, double) const {}
};

template <typename T> struct DiffCgEpi {
  Field<T> x, r, p;
  DiffCoef co;
  int nx;
  CgCtl c;
  __device__ bool begin(int s, double* red, double& sc) const { return cg_begin_step(c, s, red, sc); }
  __device__ void point(int s, int y, int xx, const T* q, double& acc, double sc) const {
    const long long i = (long long)y * nx + xx;
    if (xx < co.band) return;  // p, r, x stay zero on the Dirichlet band
    double D, kr;
    pick(co.dk, co.phase[s * co.ss + i], D, kr);
    const T pv = p.at(s, 0, i);
    const T qv = (T)(co.inv_dt + kr) * pv + q[0];
    const T al = (T)sc;
    x.at(s, 0, i) += al * pv;
    const T rv = r.at(s, 0, i) - al * qv;
    r.at(s, 0, i) = rv;
    acc += (double)rv * (double)rv;
  }
  __device__ void partial(int s, double v) const { store_partial(c.part_rr, c.prr_stride, s, 0, v); }
};

// out = M (c^n/dt - A v) where the pass computed the divergence part of A v;
// v is rebuilt pointwise (band value or the source field); optionally also
// x = M c^n.  Partial |out|^2 into part.
template <typename T> struct DiffResEpi {
  Field<T> out;
  Field<T> xinit;     // nullable: receives M c^n
  const double* cn;   // c^n
  const double* vsrc; // nullable: v off the band (else 0)
  long long ss;
  DiffCoef co;
  double c_dir;
  int nx;
  double* part;
  int pstride;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int xx, const T* q, double& acc, double sc) const {
    const long long i = (long long)y * nx + xx;
    const bool fixed = xx < co.band;
    const double cnv = cn[s * ss + i];
    if (xinit.p) xinit.at(s, 0, i) = fixed ? (T)0 : (T)cnv;
    if (fixed) {
      out.at(s, 0, i) = (T)0;
      return;
    }
    double D, kr;
    pick(co.dk, co.phase[s * co.ss + i], D, kr);
    const double v = vsrc ? vsrc[s * ss + i] : 0.0;
    const double res = cnv * co.inv_dt - ((co.inv_dt + kr) * v + (double)q[0]);
    out.at(s, 0, i) = (T)res;
    acc += res * res;
  }
  __device__ void partial(int s, double v) const { store_partial(part, pstride, s, 0, v); }
};

}  // namespace fgcg
