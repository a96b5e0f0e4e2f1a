// Projected CG in the paper's own variables, through the 2D transform passes:
// the symmetric strain for the mechanics (Sec. 2.3, eq. solid-final with the
// projection of App. A) and the concentration gradient for the static
// diffusion homogenisation (Sec. 2.1, eq. diffusion-final).  Only the gradient
// symbol tables enter, so these solvers serve every gradient operator of
// Sec. 2.6 (forward, central, eighth-order central, Fourier), where the
// displacement-form solvers need the forward difference's local stencil.
//
// Unknown x: the compatible fluctuation, NC components (strain: Voigt 11,
// 22, 12 with tensor shear, inner product weights 1, 1, 2; gradient: 2
// components, weights 1).  A x = G[L x] with L pointwise (g C, or D(x)).  Since
// p is compatible, p.A p = sum_x p : L p needs no transform, so an iteration
// is three passes, as for the spectral scalar solves:
//   row_fwd (VecCgPro)  beta, the stop test, p = r + beta p, L p, partial sums
//                       of p : L p
//   col (SymProj/VecProj) the projection of the spectra (1/N folded in)
//   row_inv (VecCgEpi)  alpha = r.r / p.Ap, x += alpha p, r -= alpha q,
//                       partial sums of r.r
#pragma once
#include "ops2d.hpp"

namespace fgcg {

template <int NC> __device__ __forceinline__ double vweight(int c) { return NC == 3 && c == 2 ? 2.0 : 1.0; }

// Pointwise L of the two problems.
struct StrainLaw {
  MechMat m;
  template <typename T> __device__ void apply(int s, long long i, const T* e, T* out) const {
    double lam, mu;
    m.get(s, i, lam, mu);
    stress2<T>(lam, mu, e[0], e[1], e[2], out);
  }
};
struct FluxLaw {
  const double* Df;
  template <typename T> __device__ void apply(int, long long i, const T* g, T* out) const {
    const T d = (T)Df[i];
    out[0] = d * g[0];
    out[1] = d * g[1];
  }
};

template <typename T, int NC, class Law> struct VecCgPro {
  Field<T> p, r;
  Law law;
  int nx;
  CgCtl c;
  __device__ bool begin(int s, double* red, double& sc) const { return cg_begin_dir(c, s, red, sc); }
  __device__ void point(int s, int y, int x, T* out, double& acc, double sc) const {
    const long long i = (long long)y * nx + x;
    T pp[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T rv = r.at(s, k, i);
      pp[k] = sc == 0.0 ? rv : rv + (T)sc * p.at(s, k, i);
      p.at(s, k, i) = pp[k];
    }
    law.apply(s, i, pp, out);
#pragma unroll
    for (int k = 0; k < NC; ++k) acc += vweight<NC>(k) * (double)pp[k] * (double)out[k];
  }
  __device__ void partial(int s, double v) const { store_partial(c.part_a, c.pa_stride, s, 0, v); }
};

// Right-hand side: L applied to the macroscopic field minus the eigenstrain
// (strain: eps_mac - e I; gradient: grad c_mac).
template <typename T, int NC, class Law> struct VecSrcPro {
  Law law;
  const double* eig;  // nullable (strain only)
  double g0[3];
  int nx;
  long long ss;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int x, T* out, double&, double) const {
    const long long i = (long long)y * nx + x;
    const double e = eig ? eig[ss * s + i] : 0.0;
    T v[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) v[k] = (T)(g0[k] - (NC == 3 && k < 2 ? e : 0.0));
    law.apply(s, i, v, out);
  }
  __device__ void partial(int, double) const {}
};

// r = -q (q = G[L E0]), x = 0; partial sums of r.r into part_a and part_b (the
// first iteration's r.r and ||b||^2).
template <typename T, int NC> struct VecRhsEpi {
  Field<T> x, r;
  int nx;
  double* part_rr;
  double* part_b;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int xx, const T* q, double& acc, double) const {
    const long long i = (long long)y * nx + xx;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T v = -q[k];
      r.at(s, k, i) = v;
      x.at(s, k, i) = (T)0;
      acc += vweight<NC>(k) * (double)v * (double)v;
    }
  }
  __device__ void partial(int s, double v) const {
    store_partial(part_rr, 0, s, 0, v);
    store_partial(part_b, 0, s, 0, v);
  }
};

template <typename T, int NC> struct VecCgEpi {
  Field<T> x, r, p;
  int nx;
  CgCtl c;
  __device__ bool begin(int s, double* red, double& sc) const { return cg_begin_step(c, s, red, sc); }
  __device__ void point(int s, int y, int xx, const T* q, double& acc, double sc) const {
    const long long i = (long long)y * nx + xx;
    const T al = (T)sc;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const T pv = p.at(s, k, i);
      x.at(s, k, i) += al * pv;
      const T rv = r.at(s, k, i) - al * q[k];
      r.at(s, k, i) = rv;
      acc += vweight<NC>(k) * (double)rv * (double)rv;
    }
  }
  __device__ void partial(int s, double v) const { store_partial(c.part_rr, c.prr_stride, s, 0, v); }
};

// Projection of a symmetric 2 x 2 tensor field (Voigt 11, 22, 12) onto the
// symmetric gradients sym(u (x) D), orthogonal in the Frobenius product: with
// t_c = t conj(D), u = (2/|D|^2) [t_c - D (D^H t_c) / (2 |D|^2)], out =
// sym(u (x) D); zero at |D| = 0 (App. A's projection in symmetric storage).
template <typename T> struct SymProj {
  const double2* Dx;
  const double2* Dy;
  double inv_n;
  const CgState* st;  // nullable
  __device__ bool begin(int s, double*, double&) const { return st == nullptr || cg_running(st, s); }
  template <typename C>
  __device__ void mode(int, int kx, int ky, const C* a, C* b, double&, double) const {
    const double2 d1 = Dx[kx], d2 = Dy[ky];
    const double n2 = d1.x * d1.x + d1.y * d1.y + d2.x * d2.x + d2.y * d2.y;
    if (n2 == 0.0) {
      b[0] = b[1] = b[2] = C{(T)0, (T)0};
      return;
    }
    const double2 s11{(double)a[0].x, (double)a[0].y}, s22{(double)a[1].x, (double)a[1].y},
        s12{(double)a[2].x, (double)a[2].y};
    // t_c = t conj(D): tc1 = s11 conj(D1) + s12 conj(D2), tc2 = s12 conj(D1) + s22 conj(D2)
    auto mulc = [](double2 v, double2 d) { return double2{v.x * d.x + v.y * d.y, v.y * d.x - v.x * d.y}; };
    auto add = [](double2 a, double2 b) { return double2{a.x + b.x, a.y + b.y}; };
    auto mul = [](double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; };
    const double2 tc1 = add(mulc(s11, d1), mulc(s12, d2)), tc2 = add(mulc(s12, d1), mulc(s22, d2));
    const double2 dh = add(mulc(tc1, d1), mulc(tc2, d2));  // D^H t_c
    const double f = 2.0 / n2, g = 1.0 / (2.0 * n2);
    const double2 u1{f * (tc1.x - g * (d1.x * dh.x - d1.y * dh.y)), f * (tc1.y - g * (d1.x * dh.y + d1.y * dh.x))};
    const double2 u2{f * (tc2.x - g * (d2.x * dh.x - d2.y * dh.y)), f * (tc2.y - g * (d2.x * dh.y + d2.y * dh.x))};
    const double2 o11 = mul(u1, d1), o22 = mul(u2, d2);
    const double2 o12 = add(mul(u1, d2), mul(u2, d1));
    b[0] = C{(T)(o11.x * inv_n), (T)(o11.y * inv_n)};
    b[1] = C{(T)(o22.x * inv_n), (T)(o22.y * inv_n)};
    b[2] = C{(T)(0.5 * o12.x * inv_n), (T)(0.5 * o12.y * inv_n)};
  }
  __device__ void partial(int, double) const {}
};

// Vector projection onto gradients, out = D (conj(D) . a) / |D|^2 (App. A,
// eq. g-42); zero at |D| = 0.
template <typename T> struct VecProj {
  const double2* Dx;
  const double2* Dy;
  double inv_n;
  const CgState* st;  // nullable
  __device__ bool begin(int s, double*, double&) const { return st == nullptr || cg_running(st, s); }
  template <typename C>
  __device__ void mode(int, int kx, int ky, const C* a, C* b, double&, double) const {
    const double2 d1 = Dx[kx], d2 = Dy[ky];
    const double n2 = d1.x * d1.x + d1.y * d1.y + d2.x * d2.x + d2.y * d2.y;
    if (n2 == 0.0) {
      b[0] = b[1] = C{(T)0, (T)0};
      return;
    }
    // s = conj(D) . a / |D|^2
    const double sx = (d1.x * a[0].x + d1.y * a[0].y + d2.x * a[1].x + d2.y * a[1].y) / n2 * inv_n;
    const double sy = (d1.x * a[0].y - d1.y * a[0].x + d2.x * a[1].y - d2.y * a[1].x) / n2 * inv_n;
    b[0] = C{(T)(d1.x * sx - d1.y * sy), (T)(d1.x * sy + d1.y * sx)};
    b[1] = C{(T)(d2.x * sx - d2.y * sy), (T)(d2.x * sy + d2.y * sx)};
  }
  __device__ void partial(int, double) const {}
};

// Post-processing of the strain form: eps = eps_mac + x, sigma = g C : (eps -
// e I); partial sums of sigma (3) and (eps - e I) : sigma (4 per block).
static __global__ void __launch_bounds__(NT) k_sf_post(MechMat m, const double* __restrict__ xs, long long n,
                                                       const double* eig, double em0, double em1, double em2,
                                                       double* strain, double* stress, double* part) {
  __shared__ double red[NT / 64];
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const double e11 = em0 + xs[i], e22 = em1 + xs[n + i], e12 = em2 + xs[2 * n + i];
    strain[i] = e11;
    strain[n + i] = e22;
    strain[2 * n + i] = e12;
    const double e = eig ? eig[i] : 0.0;
    double lam, mu;
    m.get(0, i, lam, mu);
    const double l11 = e11 - e, l22 = e22 - e, tr = l11 + l22;
    const double s11 = lam * tr + 2.0 * mu * l11, s22 = lam * tr + 2.0 * mu * l22, s12 = 2.0 * mu * e12;
    if (stress) {
      stress[i] = s11;
      stress[n + i] = s22;
      stress[2 * n + i] = s12;
    }
    a0 += s11;
    a1 += s22;
    a2 += s12;
    a3 += l11 * s11 + l22 * s22 + 2.0 * e12 * s12;
  }
  const double t0 = block_sum(a0, red), t1 = block_sum(a1, red), t2 = block_sum(a2, red), t3 = block_sum(a3, red);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = t0;
    part[4 * blockIdx.x + 1] = t1;
    part[4 * blockIdx.x + 2] = t2;
    part[4 * blockIdx.x + 3] = t3;
  }
}

// Post-processing of the gradient form: grad c = grad c_mac + x, optional
// output, partial sums of the flux (2) and of grad c . D grad c (4 per block).
static __global__ void __launch_bounds__(NT) k_hg_post(const double* __restrict__ Df, const double* __restrict__ xs,
                                                       long long n, double g0, double g1, double* grad_c,
                                                       double* part) {
  __shared__ double red[NT / 64];
  double a[4] = {0, 0, 0, 0};
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const double c0 = g0 + xs[i], c1 = g1 + xs[n + i];
    if (grad_c) {
      grad_c[i] = c0;
      grad_c[n + i] = c1;
    }
    const double d = Df[i];
    a[0] -= d * c0;
    a[1] -= d * c1;
    a[3] += d * (c0 * c0 + c1 * c1);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double t = block_sum(a[c], red);
    if (threadIdx.x == 0) part[4 * blockIdx.x + c] = t;
  }
}

}  // namespace fgcg
