// Mechanics CG in displacement form.
//
// The compatible fluctuation of Sec. 2.3 is a forward-difference gradient,
// x = grad u, and the projection of App. A factors as
// G = grad (grad^H grad)^-1 grad^H.  CG on x with the Frobenius inner product
// (the projected CG of eq. solid-final) is therefore the same iteration, in
// exact arithmetic, as CG on the displacement u (2 components) for
//     K u = f,   K = grad^H g C grad,   f = -grad^H g C : (eps_mac - e I),
// preconditioned by the Green operator M = (grad^H grad)^-1 of a unit
// reference medium, which is diagonal in Fourier space (1 / |D(k)|^2, zero at
// k = 0).  Its iterates are x_k = grad u_k; its alpha, beta and stop test
// coincide because ||G[g C x]||^2 = r.z and p_x . A p_x = p . K p.
//
// One iteration, four passes:
//   k_mech_kp          q = K p as a real-space stencil (grad and grad^H are
//                      the periodic forward/backward differences), partial
//                      sums of p.Kp = sum_x sym(grad p) : g C : sym(grad p)
//   row_fwd (MechUProC) alpha = r.z / p.Kp; x += alpha p; r -= alpha q; r
//                      transformed along x (one component per block)
//   col (MechGreen)    z_hat = r_hat / |D|^2 / N, partial sums of r.z by
//                      Parseval over the half spectrum (one component per
//                      block)
//   row_inv (MechUEpiC) z back in real space; stop test on r.z; beta;
//                      p = z + beta p (one component per block)
// so q and z are never stored except q between the first two passes.  The
// all-component functors MechUPro / MechUEpi serve the 3D passes where those
// measured faster and the one-component wrappers MechUProC / MechUEpiC the
// rest.
#pragma once
#include "ops2d.hpp"

namespace fgcg {

// sigma = g C : sym(grad u) at voxel (y, x): forward differences to (y, x+1)
// and (y+1, x), periodic.  Returns the symmetric gradient in e[3] too.
template <typename T>
__device__ __forceinline__ void sigma_u(const MechMat& m, int s, const T* u, long long n, int nx, int ny, int y,
                                        int x, T ih, T* sg, T* e) {
  const int xp = x + 1 == nx ? 0 : x + 1;
  const int yp = y + 1 == ny ? 0 : y + 1;
  const long long i = (long long)y * nx + x;
  const long long ix = (long long)y * nx + xp;
  const long long iy = (long long)yp * nx + x;
  const T u1 = u[i], u2 = u[n + i];
  const T g11 = (u[ix] - u1) * ih;
  const T g12 = (u[iy] - u1) * ih;
  const T g21 = (u[n + ix] - u2) * ih;
  const T g22 = (u[n + iy] - u2) * ih;
  e[0] = g11;
  e[1] = g22;
  e[2] = (T)0.5 * (g12 + g21);
  double lam, mu;
  m.get(s, i, lam, mu);
  stress2<T>(lam, mu, e[0], e[1], e[2], sg);
}

// sigma = g C : (eps_mac - e I) at voxel i
template <typename T>
__device__ __forceinline__ void sigma_src(const MechMat& m, int s, const double* eig, const double* em, long long i,
                                          T* sg) {
  double lam, mu;
  m.get(s, i, lam, mu);
  const double e = eig ? eig[m.ss * s + i] : 0.0;
  stress2<T>(lam, mu, (T)(em[0] - e), (T)(em[1] - e), (T)em[2], sg);
}

// q_i(x) = sum_j (sigma_ij(x - e_j) - sigma_ij(x)) / h  (the adjoint of the
// forward difference), sigma in Voigt order (11, 22, 12).
template <typename T>
__device__ __forceinline__ void div_adj(const T* s0, const T* sxm, const T* sym_, T ih, T* q) {
  q[0] = ((sxm[0] - s0[0]) + (sym_[2] - s0[2])) * ih;
  q[1] = ((sxm[2] - s0[2]) + (sym_[1] - s0[1])) * ih;
}

// q = K p with partial sums of p.Kp; the lead thread publishes the iteration
// counter (k = k_next) for the later passes of this iteration.
//
// Tiled: a tile of KP_TX x KP_TY voxels computes the stress once per voxel of
// the tile and of its halo column x0 - 1 and halo row y0 - 1 (1.08 stress
// evaluations per voxel instead of 3), keeps it in LDS, and takes the
// divergence from there.  Each block walks a contiguous range of tiles
// (row-major, x fastest), the ranges laid out XCD by XCD (xcd_block), so the
// rows a tile shares with the tiles beside it meet in one L2.
constexpr int KP_TX = 64, KP_TY = 16;

inline int kp_tiles(int nx, int ny) { return ((nx + KP_TX - 1) / KP_TX) * ((ny + KP_TY - 1) / KP_TY); }

template <typename T>
__global__ void __launch_bounds__(NT) k_mech_kp(MechMat m, const T* __restrict__ p, T* __restrict__ q,
                                                long long n, int nx, int ny, T ih, CgState* st,
                                                double* part) {
  constexpr int HX = KP_TX + 1, HY = KP_TY + 1, HP = HX * HY;
  __shared__ T sg[3][HP];
  __shared__ double red[NT / 64];
  const int s = blockIdx.y;  // sample of a batch
  st += s;
  p += 2 * n * s;
  q += 2 * n * s;
  // (the state check stays first: blocks of samples whose solve has ended,
  // in a batch, exit before loading anything)
  if (!cg_running(st, 0)) return;
  if (lead()) st->k = st->k_next;
  const int ntx = (nx + KP_TX - 1) / KP_TX;
  const int ntiles = ntx * ((ny + KP_TY - 1) / KP_TY);
  const int lb = xcd_block(), nb = gridDim.x;
  const int t0 = (int)((long long)ntiles * lb / nb), t1 = (int)((long long)ntiles * (lb + 1) / nb);
  const int tx = threadIdx.x & (KP_TX - 1), ty = threadIdx.x / KP_TX;
  double acc = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int x0 = (t % ntx) * KP_TX, y0 = (t / ntx) * KP_TY;
    // a fixed trip count, unrolled: the loads of all of a thread's halo
    // points are issued together instead of one round trip per point
#pragma unroll
    for (int k = 0; k < (HP + NT - 1) / NT; ++k) {
      const int hp = threadIdx.x + k * NT;
      const int hy = hp / HX, hx = hp - hy * HX;
      int x = x0 - 1 + hx, y = y0 - 1 + hy;
      // past the halo, or past the edge of a partial tile (never read)
      if (hp >= HP || x >= nx || y >= ny) continue;
      if (x < 0) x += nx;
      if (y < 0) y += ny;
      T sv[3], e[3];
      sigma_u<T>(m, s, p, n, nx, ny, y, x, ih, sv, e);
      sg[0][hp] = sv[0];
      sg[1][hp] = sv[1];
      sg[2][hp] = sv[2];
      if (hx >= 1 && hy >= 1) acc += (double)e[0] * sv[0] + (double)e[1] * sv[1] + 2.0 * (double)e[2] * sv[2];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KP_TY / (NT / KP_TX); ++k) {
      const int yy = ty + k * (NT / KP_TX);
      const int x = x0 + tx, y = y0 + yy;
      if (x < nx && y < ny) {
        const int hp = (yy + 1) * HX + tx + 1;
        const T s0[3] = {sg[0][hp], sg[1][hp], sg[2][hp]};
        const T sx[3] = {sg[0][hp - 1], sg[1][hp - 1], sg[2][hp - 1]};
        const T sy[3] = {sg[0][hp - HX], sg[1][hp - HX], sg[2][hp - HX]};
        T qq[2];
        div_adj<T>(s0, sx, sy, ih, qq);
        const long long i = (long long)y * nx + x;
        q[i] = qq[0];
        q[n + i] = qq[1];
      }
    }
    __syncthreads();
  }
  const double tsum = block_sum(acc, red);
  if (threadIdx.x == 0) part[(long long)s * gridDim.x + blockIdx.x] = tsum;
}

// r = f = -grad^H g C : (eps_mac - e I); x = 0.  Sample s = blockIdx.y uses
// em[3 s .. 3 s + 2].
template <typename T>
__global__ void __launch_bounds__(NT) k_mech_rhs(MechMat m, const double* eig, const double* __restrict__ ems,
                                                 T* __restrict__ r, T* __restrict__ x, long long n, int nx, int ny,
                                                 T ih) {
  const int s = blockIdx.y;
  const double em[3] = {ems[3 * s], ems[3 * s + 1], ems[3 * s + 2]};
  r += 2 * n * s;
  x += 2 * n * s;
  const SlabIter it(nx, ny);
  for (long long i = it.v0; i < it.v1; i += it.step) {
    const int y = (int)((unsigned)i / (unsigned)nx), xx = (int)(i - (long long)y * nx);
    const int xm = xx == 0 ? nx - 1 : xx - 1;
    const int ym = y == 0 ? ny - 1 : y - 1;
    T s0[3], sx[3], sy[3], qq[2];
    sigma_src<T>(m, s, eig, em, i, s0);
    sigma_src<T>(m, s, eig, em, (long long)y * nx + xm, sx);
    sigma_src<T>(m, s, eig, em, (long long)ym * nx + xx, sy);
    div_adj<T>(s0, sx, sy, ih, qq);
    r[i] = -qq[0];
    r[n + i] = -qq[1];
    x[i] = (T)0;
    x[n + i] = (T)0;
  }
}

// Post-processing: eps = eps_mac + sym(grad u), sigma = g C : (eps - e I);
// partial sums of sigma (3) and (eps - e I) : sigma.
template <typename T>
__global__ void __launch_bounds__(NT) k_mech_post_u(MechMat m, const T* __restrict__ u, long long n, int nx,
                                                    int ny, T ih, const double* eig, const double* __restrict__ ems,
                                                    double* strain, double* stress, double* part) {
  __shared__ double red[NT / 64];
  const int s = blockIdx.y;
  const double em0 = ems[3 * s], em1 = ems[3 * s + 1], em2 = ems[3 * s + 2];
  u += 2 * n * s;
  strain += 3 * n * s;
  if (stress) stress += 3 * n * s;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const int y = (int)(i / nx), x = (int)(i - (long long)y * nx);
    const int xp = x + 1 == nx ? 0 : x + 1;
    const int yp = y + 1 == ny ? 0 : y + 1;
    const long long ix = (long long)y * nx + xp, iy = (long long)yp * nx + x;
    const double u1 = (double)u[i], u2 = (double)u[n + i];
    const double g11 = ((double)u[ix] - u1) * (double)ih;
    const double g12 = ((double)u[iy] - u1) * (double)ih;
    const double g21 = ((double)u[n + ix] - u2) * (double)ih;
    const double g22 = ((double)u[n + iy] - u2) * (double)ih;
    const double e11 = em0 + g11, e22 = em1 + g22, e12 = em2 + 0.5 * (g12 + g21);
    strain[i] = e11;
    strain[n + i] = e22;
    strain[2 * n + i] = e12;
    const double e = eig ? eig[m.ss * s + i] : 0.0;
    double lam, mu;
    m.get(s, i, lam, mu);
    const double l11 = e11 - e, l22 = e22 - e;
    const double tr = l11 + l22;
    const double s11 = lam * tr + 2.0 * mu * l11;
    const double s22 = lam * tr + 2.0 * mu * l22;
    const double s12 = 2.0 * mu * e12;
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
  const double t0 = block_sum(a0, red), t1 = block_sum(a1, red), t2 = block_sum(a2, red),
               t3 = block_sum(a3, red);
  if (threadIdx.x == 0) {
    double* pp = part + 4 * ((long long)s * gridDim.x + blockIdx.x);
    pp[0] = t0;
    pp[1] = t1;
    pp[2] = t2;
    pp[3] = t3;
  }
}

// alpha = r.z / p.Kp of iteration k with the breakdown test (uniform per block).
__device__ __forceinline__ bool mech_alpha(CgState* st, const double* part_a, int np_a, double* red,
                                           double& alpha) {
  if (!cg_running(st, 0)) return false;
  const int k = st->k;
  const double pap = block_sum_array(part_a, np_a, red);
  const double rz = st->rz[k & 1];
  if (!(pap > 0.0) || !isfinite(pap)) {
    if (lead()) {
      st->done = 3;
      st->iter = k;
      st->rr_final = rz;
    }
    return false;
  }
  alpha = rz / pap;
  return true;
}

// Mixed precision, reliable update (every tenth iteration): fold the FP32
// increments into the FP64 solution, x_hi += x_lo + alpha p, x_lo = 0.
template <typename T>
__global__ void __launch_bounds__(NT) k_mech_fold(T* __restrict__ xlo, double* __restrict__ xhi,
                                                  const T* __restrict__ p, long long n2, CgState* st,
                                                  const double* part_a, int np_a) {
  __shared__ double red[NT / 64];
  const int s = blockIdx.y;
  xlo += n2 * s;
  xhi += n2 * s;
  p += n2 * s;
  double alpha;
  if (!mech_alpha(st + s, part_a + (long long)s * np_a, np_a, red, alpha)) return;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n2; i += (long long)gridDim.x * NT) {
    xhi[i] += (double)xlo[i] + alpha * (double)p[i];
    xlo[i] = (T)0;
  }
}

// Mixed precision: the true residual r = f - K x_hi with the FP64 operator.
template <typename T>
__global__ void __launch_bounds__(NT) k_mech_true_res(MechMat m, const double* __restrict__ xhi,
                                                      const double* __restrict__ f, T* __restrict__ r, long long n,
                                                      int nx, int ny, double ih, const CgState* st) {
  const int s = blockIdx.y;
  xhi += 2 * n * s;
  f += 2 * n * s;
  r += 2 * n * s;
  if (!cg_running(st, s)) return;
  const SlabIter it(nx, ny);
  for (long long i = it.v0; i < it.v1; i += it.step) {
    const int y = (int)((unsigned)i / (unsigned)nx), x = (int)(i - (long long)y * nx);
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int ym = y == 0 ? ny - 1 : y - 1;
    double s0[3], sx[3], sy[3], e[3], qq[2];
    sigma_u<double>(m, s, xhi, n, nx, ny, y, x, ih, s0, e);
    sigma_u<double>(m, s, xhi, n, nx, ny, y, xm, ih, sx, e);
    sigma_u<double>(m, s, xhi, n, nx, ny, ym, x, ih, sy, e);
    div_adj<double>(s0, sx, sy, ih, qq);
    r[i] = (T)(f[i] - qq[0]);
    r[n + i] = (T)(f[n + i] - qq[1]);
  }
}

// x_hi += x_lo (end of a mixed-precision solve)
template <typename T>
__global__ void __launch_bounds__(NT) k_fold_final(const T* __restrict__ xlo, double* __restrict__ xhi, long long n2) {
  xlo += n2 * blockIdx.y;
  xhi += n2 * blockIdx.y;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n2; i += (long long)gridDim.x * NT)
    xhi[i] += (double)xlo[i];
}

// Forward row pass of iteration k (NC displacement components).
template <typename T, int NC = 2> struct MechUPro {
  Field<T> x, r, p, q;
  int nx;
  CgState* st;
  const double* part_a;
  int np_a;
  __device__ bool begin(int s, double* red, double& sc) const {
    return mech_alpha(st + s, part_a + (long long)s * np_a, np_a, red, sc);
  }
  // 2D (two components): begin() sums the stiffness pass's partials itself,
  // so the first loads are issued before it; the 3D passes get one
  // pre-reduced value and keep loads after it (EARLY)
  static constexpr bool EARLY = NC == 2;
  struct Ld {
    T x[NC], r[NC], p[NC], q[NC];
  };
  __device__ void load(int s, int y, int xx, Ld& l) const {
    const long long i = (long long)y * nx + xx;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      l.x[c] = x.at(s, c, i);
      l.r[c] = r.at(s, c, i);
      l.p[c] = p.at(s, c, i);
      l.q[c] = q.at(s, c, i);
    }
  }
  __device__ void apply(int s, int y, int xx, const Ld& l, T* out, double&, double sc) const {
    const long long i = (long long)y * nx + xx;
    const T a = (T)sc;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      x.at(s, c, i) = l.x[c] + a * l.p[c];
      const T rv = l.r[c] - a * l.q[c];
      r.at(s, c, i) = rv;
      out[c] = rv;
    }
  }
  __device__ void partial(int, double) const {}
};

// out = v (NC components)
template <typename T, int NC> struct CopyProN {
  Field<T> v;
  int nx;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int x, T* out, double&, double) const {
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = v.at(s, c, (long long)y * nx + x);
  }
  __device__ void partial(int, double) const {}
};

// Green operator of the unit reference medium with partial sums of r.z, one
// component per block: the column pass runs over (sample, component) pairs
// s2 = NC s + c (component stride nxh ny), and the partial sums of sample s
// fill part[NC s gridDim.x .. NC (s + 1) gridDim.x).  NC = 2: the mechanics
// displacement; NC = 1: the scalar fluctuation of the diffusion homogenisation.
template <typename T, int NC = 2> struct MechGreen {
  const double2* Dx;
  const double2* Dy;
  double inv_n;
  int nx;
  const CgState* st;  // nullable
  double* part;       // nullable
  __device__ bool begin(int s2, double*, double&) const { return st == nullptr || cg_running(st, s2 / NC); }
  // the column pass loads |D_y|^2 of its modes before the forward transform
  using Pre = double;
  __device__ Pre pre(int, int, int ky) const {
    const double2 d = Dy[ky];
    return d.x * d.x + d.y * d.y;
  }
  template <typename C>
  __device__ void mode(int s2, int kx, int ky, const C* a, C* b, double& acc, double sc) const {
    mode_pre(s2, kx, ky, pre(s2, kx, ky), a, b, acc, sc);
  }
  template <typename C>
  __device__ void mode_pre(int, int kx, int, const double dy2, const C* a, C* b, double& acc, double) const {
    const double2 d1 = Dx[kx];
    const double n2 = (d1.x * d1.x + d1.y * d1.y) + dy2;
    if (n2 == 0.0) {
      b[0] = C{(T)0, (T)0};
      return;
    }
    const double f = inv_n / n2;
    const T ft = (T)f;
    b[0] = C{a[0].x * ft, a[0].y * ft};
    const double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
    acc += w * f * ((double)a[0].x * a[0].x + (double)a[0].y * a[0].y);
  }
  __device__ void partial(int s2, double v) const {
    if (part && threadIdx.x == 0) part[(long long)s2 * gridDim.x + blockIdx.x] = v;
  }
};

// Green operator of an isotropic reference medium (lam0, mu0), both
// displacement components of a column in one block: per mode the 2 x 2
// Hermitian system K0 z_hat = r_hat with
//     K0(k) = mu0 |D|^2 I + lam0 conj(D) D^T + mu0 D D^H
// (the stiffness of the homogeneous reference medium in Fourier space; zero at
// k = 0), solved in closed form in FP64, and the Parseval partial sums of
// r.z = (1/N) sum_k Re(r_hat^H z_hat) (one per block, blocks of sample s at
// part[s gridDim.x ..]).  Only lam0 / mu0 matters to the CG; mu0 is taken
// as 1.
template <typename T> struct MechRefGreen {
  const double2* Dx;
  const double2* Dy;
  double inv_n;
  double lam0, mu0;
  int nx;
  const CgState* st;  // nullable
  double* part;       // nullable
  __device__ bool begin(int s, double*, double&) const { return st == nullptr || cg_running(st, s); }
  using Pre = double2;
  __device__ Pre pre(int, int, int ky) const { return Dy[ky]; }
  template <typename C>
  __device__ void mode(int s, int kx, int ky, const C* a, C* b, double& acc, double sc) const {
    mode_pre(s, kx, ky, Dy[ky], a, b, acc, sc);
  }
  template <typename C>
  __device__ void mode_pre(int, int kx, int, const double2 d2, const C* a, C* b, double& acc, double) const {
    const double2 d1 = Dx[kx];
    const double m1 = d1.x * d1.x + d1.y * d1.y, m2 = d2.x * d2.x + d2.y * d2.y;
    const double n2 = m1 + m2;
    if (n2 == 0.0) {
      b[0] = C{(T)0, (T)0};
      b[1] = C{(T)0, (T)0};
      return;
    }
    const double lm = lam0 + mu0;
    const double a11 = mu0 * n2 + lm * m1, a22 = mu0 * n2 + lm * m2;
    // a12 = lam0 conj(D1) D2 + mu0 D1 conj(D2)
    const double c1r = d1.x * d2.x + d1.y * d2.y, c1i = d1.x * d2.y - d1.y * d2.x;  // conj(D1) D2
    const double a12r = (lam0 + mu0) * c1r, a12i = (lam0 - mu0) * c1i;
    const double det = a11 * a22 - (a12r * a12r + a12i * a12i);
    const double f = inv_n / det;
    const double r1x = a[0].x, r1y = a[0].y, r2x = a[1].x, r2y = a[1].y;
    // z1 = (a22 r1 - a12 r2) / det, z2 = (a11 r2 - conj(a12) r1) / det
    const double z1x = f * (a22 * r1x - (a12r * r2x - a12i * r2y));
    const double z1y = f * (a22 * r1y - (a12r * r2y + a12i * r2x));
    const double z2x = f * (a11 * r2x - (a12r * r1x + a12i * r1y));
    const double z2y = f * (a11 * r2y - (a12r * r1y - a12i * r1x));
    b[0] = C{(T)z1x, (T)z1y};
    b[1] = C{(T)z2x, (T)z2y};
    const double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
    acc += w * (r1x * z1x + r1y * z1y + r2x * z2x + r2y * z2y);
  }
  __device__ void partial(int s, double v) const {
    if (part && threadIdx.x == 0) part[(long long)s * gridDim.x + blockIdx.x] = v;
  }
};

// Inverse row pass: stop test, beta, p = z + beta p.  With init set it starts
// the solve instead: r.z of the right-hand side gives ||b||^2 and the
// threshold, and p = z.
template <typename T, int NC = 2> struct MechUEpi {
  Field<T> p;
  int nx;
  CgState* st;
  const double* part_rz;
  int np_rz;
  int init;
  double tol;
  int maxit;
  int sr = 0;  // the solution update of the iteration happens in this pass (sr2d.hpp)
  __device__ bool begin(int s, double* red, double& sc) const {
    CgState* S = st + s;
    if (!init && !cg_running(st, s)) return false;
    const double rz = block_sum_array(part_rz + (long long)s * np_rz, np_rz, red);
    if (init) {
      const double thr = tol * tol * rz;
      const int done = !isfinite(rz) ? 4 : (rz <= thr ? 1 : (maxit <= 0 ? 2 : 0));
      if (lead()) {
        CgState t;
        t.rr_cur = t.rr_prev = 0.0;
        t.bnorm2 = rz;
        t.thr = thr;
        t.rr_final = rz;
        t.rz[0] = rz;
        t.rz[1] = 0.0;
        t.maxit = maxit;
        t.k = 0;
        t.k_next = 0;
        t.iter = 0;
        t.done = done;
        t.zero_rhs = rz == 0.0;
        t.alpha = 0.0;
        t.x_pending = 0;
        *S = t;
      }
      sc = 0.0;
      return done == 0;
    }
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
        if (sr) S->x_pending = 1;
      }
      return false;
    }
    sc = rz / S->rz[k & 1];
    if (lead()) {
      S->rz[(k + 1) & 1] = rz;
      S->k_next = k + 1;
    }
    return true;
  }
  static constexpr int NPRE = NC;  // p of the voxel, loaded before the transforms
  // 2D: begin() sums the column pass's partials itself: prefetch before it
  // (3D: one pre-reduced value, prefetch after it)
  static constexpr bool EARLY = NC == 2;
  __device__ void prefetch(int s, int y, int xx, T* pre) const {
    const long long i = (long long)y * nx + xx;
#pragma unroll
    for (int c = 0; c < NC; ++c) pre[c] = init ? (T)0 : p.at(s, c, i);
  }
  __device__ void point(int s, int y, int xx, const T* z, double&, double sc, const T* pre) const {
    const long long i = (long long)y * nx + xx;
#pragma unroll
    for (int c = 0; c < NC; ++c) p.at(s, c, i) = init ? z[c] : z[c] + (T)sc * pre[c];
  }
  __device__ void partial(int, double) const {}
};

// One displacement component per block (row passes): the pass runs over
// (sample, component) pairs s2 = NC s + c with the spectrum stride of one
// component, as the column pass does.  NC times the blocks of the
// all-component passes, each with 1/NC of the registers for its values; the CG
// scalars and the stop test are those of sample s (every component block
// computes and stores the same values).  EARLY as for MechUPro.
template <typename T, int NC = 2> struct MechUProC {
  MechUPro<T, NC> m;
  static constexpr bool EARLY = MechUPro<T, NC>::EARLY;
  __device__ bool begin(int s2, double* red, double& sc) const { return m.begin(s2 / NC, red, sc); }
  struct Ld {
    T x, r, p, q;
  };
  __device__ void load(int s2, int y, int xx, Ld& l) const {
    const int s = s2 / NC, c = s2 - s * NC;
    const long long i = (long long)y * m.nx + xx;
    l.x = m.x.at(s, c, i);
    l.r = m.r.at(s, c, i);
    l.p = m.p.at(s, c, i);
    l.q = m.q.at(s, c, i);
  }
  __device__ void apply(int s2, int y, int xx, const Ld& l, T* out, double&, double sc) const {
    const int s = s2 / NC, c = s2 - s * NC;
    const long long i = (long long)y * m.nx + xx;
    const T a = (T)sc;
    m.x.at(s, c, i) = l.x + a * l.p;
    const T rv = l.r - a * l.q;
    m.r.at(s, c, i) = rv;
    out[0] = rv;
  }
  __device__ void partial(int, double) const {}
};

// E: prefetch before begin() (as MechUEpi::EARLY); batches of several
// samples take E = false, so that the blocks of samples whose solve has ended
// exit before reading p.
template <typename T, int NC = 2, bool E = MechUEpi<T, NC>::EARLY> struct MechUEpiC {
  MechUEpi<T, NC> m;
  static constexpr int NPRE = 1;
  static constexpr bool EARLY = E;
  __device__ bool begin(int s2, double* red, double& sc) const { return m.begin(s2 / NC, red, sc); }
  __device__ void prefetch(int s2, int y, int xx, T* pre) const {
    const long long i = (long long)y * m.nx + xx;
    pre[0] = m.init ? (T)0 : m.p.at(s2 / NC, s2 % NC, i);
  }
  __device__ void point(int s2, int y, int xx, const T* z, double&, double sc, const T* pre) const {
    const long long i = (long long)y * m.nx + xx;
    m.p.at(s2 / NC, s2 % NC, i) = m.init ? z[0] : z[0] + (T)sc * pre[0];
  }
  __device__ void partial(int, double) const {}
};

}  // namespace fgcg
