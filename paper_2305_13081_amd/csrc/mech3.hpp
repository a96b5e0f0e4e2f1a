// Mechanics on 3D grids: the real-space parts of the displacement-form PCG.
//
// Same method as the 2D engine (Sec. 2.3 with the forward difference of
// Sec. 2.6; the projection of App. A factored through the displacement):
// unknown u (3 components), K = grad^H g C grad, Green preconditioner
// (grad^H grad)^-1 applied by the 3D transforms.  Strain and stress use Voigt
// order (11, 22, 33, 23, 13, 12) with tensor shear; index 1 is x, the fastest
// axis, then y, then z.
//
// The stencil kernels walk the grid row by row (row = z ny + y).  Rows are cut
// into 8 contiguous slabs, one per XCD (the hardware hands block b to XCD
// b % 8), so that the y and z neighbours a block reads were mostly brought into
// the same L2 by the blocks next to it.
#pragma once
#include "ops2d.hpp"

namespace fgcg {

struct Grid3 {
  int nx, ny, nz;
  long long n;
};

struct Em6 {
  double v[6];
};

// Voxel range of this block: slab of XCD (blockIdx.x % 8), block q of nq in it.
// gridDim.x is a multiple of 8.
struct SlabIter {
  long long v0, v1;  // voxels [v0, v1) of the slab
  long long step;
  __device__ SlabIter(const Grid3& g) {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b & 7, q = b >> 3, nq = nb >> 3;
    const long long rows = (long long)g.ny * g.nz;
    const long long r0 = rows * x / 8, r1 = rows * (x + 1) / 8;
    v0 = r0 * g.nx + (long long)q * NT + threadIdx.x;
    v1 = r1 * g.nx;
    step = (long long)nq * NT;
  }
};

// Periodic neighbour offsets of voxel i = (z ny + y) nx + x.
struct Off3 {
  long long xp, xm, yp, ym, zp, zm;
  __device__ Off3(const Grid3& g, long long i, int& x, int& y, int& z) {
    const unsigned iu = (unsigned)i;  // 3D grids hold fewer than 2^31 voxels
    const unsigned row = iu / (unsigned)g.nx;
    x = (int)(iu - row * (unsigned)g.nx);
    y = (int)(row % (unsigned)g.ny);
    z = (int)(row / (unsigned)g.ny);
    const long long px = g.nx, pl = (long long)g.nx * g.ny;
    xp = x + 1 == g.nx ? -(long long)(g.nx - 1) : 1;
    xm = x == 0 ? (long long)(g.nx - 1) : -1;
    yp = y + 1 == g.ny ? -(long long)(g.ny - 1) * px : px;
    ym = y == 0 ? (long long)(g.ny - 1) * px : -px;
    zp = z + 1 == g.nz ? -(long long)(g.nz - 1) * pl : pl;
    zm = z == 0 ? (long long)(g.nz - 1) * pl : -pl;
  }
};

template <typename T>
__device__ __forceinline__ void stress3(double lam, double mu, const T* e, T* s) {
  const T l = (T)lam, m2 = (T)(2.0 * mu);
  const T tr = e[0] + e[1] + e[2];
  s[0] = l * tr + m2 * e[0];
  s[1] = l * tr + m2 * e[1];
  s[2] = l * tr + m2 * e[2];
  s[3] = m2 * e[3];
  s[4] = m2 * e[4];
  s[5] = m2 * e[5];
}

// sym(grad u) at voxel i from its forward neighbours ix, iy, iz.
template <typename T>
__device__ __forceinline__ void symgrad3(const T* u, long long n, long long i, long long ix, long long iy,
                                         long long iz, T ih, T* e) {
  T g[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T* ua = u + a * n;
    const T u0 = ua[i];
    g[a][0] = (ua[ix] - u0) * ih;
    g[a][1] = (ua[iy] - u0) * ih;
    g[a][2] = (ua[iz] - u0) * ih;
  }
  e[0] = g[0][0];
  e[1] = g[1][1];
  e[2] = g[2][2];
  e[3] = (T)0.5 * (g[1][2] + g[2][1]);
  e[4] = (T)0.5 * (g[0][2] + g[2][0]);
  e[5] = (T)0.5 * (g[0][1] + g[1][0]);
}

// sym(grad u) and the stress g C : sym(grad u) at voxel i.
template <typename T>
__device__ __forceinline__ void sigma3(const MechMat& m, const T* u, long long n, long long i, long long ix,
                                       long long iy, long long iz, T ih, T* sg, T* e) {
  symgrad3<T>(u, n, i, ix, iy, iz, ih, e);
  double lam, mu;
  m.get(0, i, lam, mu);
  stress3<T>(lam, mu, e, sg);
}

// sigma = g C : (eps_mac - e I) at voxel i
template <typename T>
__device__ __forceinline__ void sigma3_src(const MechMat& m, const double* eig, const Em6& em, long long i, T* sg) {
  double lam, mu;
  m.get(0, i, lam, mu);
  const double e = eig ? eig[i] : 0.0;
  const T el[6] = {(T)(em.v[0] - e), (T)(em.v[1] - e), (T)(em.v[2] - e), (T)em.v[3], (T)em.v[4], (T)em.v[5]};
  stress3<T>(lam, mu, el, sg);
}

// q_a(x) = sum_b (sigma_ab(x - e_b) - sigma_ab(x)) / h
template <typename T>
__device__ __forceinline__ void div_adj3(const T* s0, const T* sx, const T* sy, const T* sz, T ih, T* q) {
  q[0] = ((sx[0] - s0[0]) + (sy[5] - s0[5]) + (sz[4] - s0[4])) * ih;
  q[1] = ((sx[5] - s0[5]) + (sy[1] - s0[1]) + (sz[3] - s0[3])) * ih;
  q[2] = ((sx[4] - s0[4]) + (sy[3] - s0[3]) + (sz[2] - s0[2])) * ih;
}

template <typename T> __device__ __forceinline__ double edots(const T* e, const T* s) {
  return (double)e[0] * s[0] + (double)e[1] * s[1] + (double)e[2] * s[2] +
         2.0 * ((double)e[3] * s[3] + (double)e[4] * s[4] + (double)e[5] * s[5]);
}

// q = K u at voxel i (stress at the voxel and at its three backward neighbours).
template <typename T>
__device__ __forceinline__ void kapply3(const MechMat& m, const T* u, long long n, long long i, const Off3& o, T ih,
                                        T* q, double* ed) {
  T s0[6], e0[6], sx[6], sy[6], sz[6], t[6];
  sigma3<T>(m, u, n, i, i + o.xp, i + o.yp, i + o.zp, ih, s0, e0);
  const long long jx = i + o.xm, jy = i + o.ym, jz = i + o.zm;
  sigma3<T>(m, u, n, jx, i, jx + o.yp, jx + o.zp, ih, sx, t);
  sigma3<T>(m, u, n, jy, jy + o.xp, i, jy + o.zp, ih, sy, t);
  sigma3<T>(m, u, n, jz, jz + o.xp, jz + o.yp, i, ih, sz, t);
  div_adj3<T>(s0, sx, sy, sz, ih, q);
  if (ed) *ed = edots<T>(e0, s0);
}

// q = K p with partial sums of p.Kp; publishes k = k_next (see the 2D kernel).
template <typename T>
__global__ void __launch_bounds__(NT) k_mech3_kp(MechMat m, const T* __restrict__ p, T* __restrict__ q, Grid3 g,
                                                 T ih, CgState* st, double* part) {
  __shared__ double red[NT / 64];
  if (!cg_running(st, 0)) return;
  if (lead()) st->k = st->k_next;
  const long long n = g.n;
  double acc = 0.0;
  const SlabIter it(g);
  for (long long i = it.v0; i < it.v1; i += it.step) {
    int x, y, z;
    const Off3 o(g, i, x, y, z);
    T qq[3];
    double ed;
    kapply3<T>(m, p, n, i, o, ih, qq, &ed);
    q[i] = qq[0];
    q[n + i] = qq[1];
    q[2 * n + i] = qq[2];
    acc += ed;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// r = f = -grad^H g C : (eps_mac - e I); x = 0.
template <typename T>
__global__ void __launch_bounds__(NT) k_mech3_rhs(MechMat m, const double* eig, Em6 em, T* __restrict__ r,
                                                  T* __restrict__ x, Grid3 g, T ih) {
  const long long n = g.n;
  const SlabIter it(g);
  for (long long i = it.v0; i < it.v1; i += it.step) {
    int xx, y, z;
    const Off3 o(g, i, xx, y, z);
    T s0[6], sx[6], sy[6], sz[6], qq[3];
    sigma3_src<T>(m, eig, em, i, s0);
    sigma3_src<T>(m, eig, em, i + o.xm, sx);
    sigma3_src<T>(m, eig, em, i + o.ym, sy);
    sigma3_src<T>(m, eig, em, i + o.zm, sz);
    div_adj3<T>(s0, sx, sy, sz, ih, qq);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r[a * n + i] = -qq[a];
      x[a * n + i] = (T)0;
    }
  }
}

// Mixed precision: r = f - K x_hi with the FP64 operator.
template <typename T>
__global__ void __launch_bounds__(NT) k_mech3_true_res(MechMat m, const double* __restrict__ xhi,
                                                       const double* __restrict__ f, T* __restrict__ r, Grid3 g,
                                                       double ih, const CgState* st) {
  if (!cg_running(st, 0)) return;
  const long long n = g.n;
  const SlabIter it(g);
  for (long long i = it.v0; i < it.v1; i += it.step) {
    int x, y, z;
    const Off3 o(g, i, x, y, z);
    double qq[3];
    kapply3<double>(m, xhi, n, i, o, ih, qq, nullptr);
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a * n + i] = (T)(f[a * n + i] - qq[a]);
  }
}

// eps = eps_mac + sym(grad u), sigma = g C : (eps - e I); partial sums of
// sigma (6) and (eps - e I) : sigma, 7 per block.
__global__ void __launch_bounds__(NT) k_mech3_post(MechMat m, const double* __restrict__ u, Grid3 g, double ih,
                                                   const double* eig, Em6 em, double* strain, double* stress,
                                                   double* part) {
  __shared__ double red[NT / 64];
  const long long n = g.n;
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  const SlabIter it(g);
  for (long long i = it.v0; i < it.v1; i += it.step) {
    int x, y, z;
    const Off3 o(g, i, x, y, z);
    double sg[6], e[6];
    symgrad3<double>(u, n, i, i + o.xp, i + o.yp, i + o.zp, ih, e);
    const double ev = eig ? eig[i] : 0.0;
    double eps[6], el[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      eps[c] = em.v[c] + e[c];
      el[c] = eps[c] - (c < 3 ? ev : 0.0);
      strain[c * n + i] = eps[c];
    }
    double lam, mu;
    m.get(0, i, lam, mu);
    stress3<double>(lam, mu, el, sg);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (stress) stress[c * n + i] = sg[c];
      a[c] += sg[c];
    }
    a[6] += edots<double>(el, sg);
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    const double t = block_sum(a[c], red);
    if (threadIdx.x == 0) part[7 * blockIdx.x + c] = t;
  }
}

// H = max(H, psi+(eps - e I)) on 3D grids with the undegraded Lame constants:
// psi+ = K/2 <tr>_+^2 + mu dev:dev, K = lambda + 2 mu / 3.
__global__ void __launch_bounds__(NT) k_history3(MechMat m, const double* strain, const double* e, double* H,
                                                 long long n) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    double lam, mu;
    m.get(0, i, lam, mu);  // m.d is null here: undegraded
    const double ev = e[i];
    const double l0 = strain[i] - ev, l1 = strain[n + i] - ev, l2 = strain[2 * n + i] - ev;
    const double s3 = strain[3 * n + i], s4 = strain[4 * n + i], s5 = strain[5 * n + i];
    const double tr = l0 + l1 + l2;
    const double trp = 0.5 * (tr + fabs(tr));
    const double d0 = l0 - tr / 3.0, d1 = l1 - tr / 3.0, d2 = l2 - tr / 3.0;
    const double devdev = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * (s3 * s3 + s4 * s4 + s5 * s5);
    const double psi = 0.5 * (lam + 2.0 * mu / 3.0) * trp * trp + mu * devdev;
    H[i] = fmax(H[i], psi);
  }
}

// Debug transforms: internal half spectrum [kx][z][y] <-> the usual
// [z][y][kx] layout of a real-input transform.
__global__ void __launch_bounds__(NT) k_spec_out(const double2* __restrict__ in, double2* __restrict__ out, int nxh,
                                                 int ny, int nz) {
  const long long tot = (long long)nxh * ny * nz;
  for (long long o = blockIdx.x * (long long)NT + threadIdx.x; o < tot; o += (long long)gridDim.x * NT) {
    const int kx = (int)(o % nxh);
    const long long zy = o / nxh;  // z ny + y
    out[o] = in[(long long)kx * ny * nz + zy];
  }
}

__global__ void __launch_bounds__(NT) k_spec_in(const double2* __restrict__ in, double2* __restrict__ out, int nxh,
                                                int ny, int nz) {
  const long long tot = (long long)nxh * ny * nz;
  for (long long o = blockIdx.x * (long long)NT + threadIdx.x; o < tot; o += (long long)gridDim.x * NT) {
    const int kx = (int)(o % nxh);
    const long long zy = o / nxh;
    out[(long long)kx * ny * nz + zy] = in[o];
  }
}

}  // namespace fgcg
