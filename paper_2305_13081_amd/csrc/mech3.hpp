// Mechanics on 3D grids: the real-space parts of the displacement-form PCG.
//
// Same method as the 2D engine (Sec. 2.3 with the forward difference of
// Sec. 2.6; the projection of App. A factored through the displacement):
// unknown u (3 components), K = grad^H g C grad, Green preconditioner
// (grad^H grad)^-1 applied by the 3D transforms.  Strain and stress use Voigt
// order (11, 22, 33, 23, 13, 12) with tensor shear; index 1 is x, the fastest
// axis, then y, then z.
//
// The stencil kernels walk the grid row by row (row = z ny + y) in XCD slabs
// (SlabIter), so the y and z neighbours a block reads were mostly brought into
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

// q = K p, tiled: a block takes an x-y tile of K3_TX x K3_TY voxels and marches it
// through K3_ZC planes.  On each plane the stress is computed once per voxel
// of the tile and of its halo column x0 - 1 and halo row y0 - 1 and kept in
// LDS; the stress of the plane below stays in registers, so the divergence
// needs no other evaluation (about 1.4 stress evaluations per voxel instead
// of 4).  Tile-chunks are ordered x, y, then z, and each block walks a
// contiguous range of them laid out XCD by XCD (xcd_block).
constexpr int K3_TX = 64, K3_TY = 8, K3_ZC = 8;

inline int kp3_chunks(int nx, int ny, int nz) {
  return ((nx + K3_TX - 1) / K3_TX) * ((ny + K3_TY - 1) / K3_TY) * ((nz + K3_ZC - 1) / K3_ZC);
}

template <typename T>
__device__ __forceinline__ void sigma3_at(const MechMat& m, const T* u, const Grid3& g, int x, int y, int z, T ih,
                                          T* sv, T* e) {
  const long long pl = (long long)g.nx * g.ny;
  const long long i = (long long)z * pl + (long long)y * g.nx + x;
  const long long ix = i + (x + 1 == g.nx ? -(long long)(g.nx - 1) : 1);
  const long long iy = i + (y + 1 == g.ny ? -(long long)(g.ny - 1) * g.nx : (long long)g.nx);
  const long long iz = i + (z + 1 == g.nz ? -(long long)(g.nz - 1) * pl : pl);
  sigma3<T>(m, u, g.n, i, ix, iy, iz, ih, sv, e);
}

// T: type of q; TU: type of p and of the arithmetic.  RES = false: the CG
// pass, q = K p with p.Kp partial sums, publishing k = k_next.  RES = true:
// the FP64 true residual of the mixed-precision solve, q = (T)(f - K p)
// (p = x_hi), nothing else.
template <typename T, typename TU, bool RES>
__global__ void __launch_bounds__(NT) k_mech3_kpx(MechMat m, const TU* __restrict__ p, T* __restrict__ q,
                                                  const double* __restrict__ f, Grid3 g, TU ih, CgState* st,
                                                  double* part) {
  constexpr int HX = K3_TX + 1, HY = K3_TY + 1, HP = HX * HY;
  constexpr int RPT = K3_TY / (NT / K3_TX);  // own rows per thread
  __shared__ TU sg[6][HP];
  __shared__ double red[NT / 64];
  if (!cg_running(st, 0)) return;
  if (!RES && lead()) st->k = st->k_next;
  const long long n = g.n;
  const int ntx = (g.nx + K3_TX - 1) / K3_TX, nty = (g.ny + K3_TY - 1) / K3_TY;
  const int nch = ntx * nty * ((g.nz + K3_ZC - 1) / K3_ZC);
  const int lb = xcd_block(), nb = gridDim.x;
  const int c0 = (int)((long long)nch * lb / nb), c1 = (int)((long long)nch * (lb + 1) / nb);
  const int tx = threadIdx.x & (K3_TX - 1), ty = threadIdx.x / K3_TX;
  double acc = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int x0 = (c % ntx) * K3_TX, y0 = ((c / ntx) % nty) * K3_TY;
    const int z0 = (c / (ntx * nty)) * K3_ZC, z1 = min(z0 + K3_ZC, g.nz);
    const int xo = x0 + tx;
    // stress of the own points on the plane below the chunk
    TU below[RPT][6];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int yo = y0 + ty + k * (NT / K3_TX);
      if (xo < g.nx && yo < g.ny) {
        TU e[6];
        sigma3_at<TU>(m, p, g, xo, yo, z0 == 0 ? g.nz - 1 : z0 - 1, ih, below[k], e);
      }
    }
    for (int z = z0; z < z1; ++z) {
      for (int hp = threadIdx.x; hp < HP; hp += NT) {
        const int hy = hp / HX, hx = hp - hy * HX;
        int x = x0 - 1 + hx, y = y0 - 1 + hy;
        if (x >= g.nx || y >= g.ny) continue;  // past the edge of a partial tile: never read
        if (x < 0) x += g.nx;
        if (y < 0) y += g.ny;
        TU sv[6], e[6];
        sigma3_at<TU>(m, p, g, x, y, z, ih, sv, e);
#pragma unroll
        for (int j = 0; j < 6; ++j) sg[j][hp] = sv[j];
        if (!RES && hx >= 1 && hy >= 1) acc += edots<TU>(e, sv);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int yy = ty + k * (NT / K3_TX);
        const int yo = y0 + yy;
        if (xo < g.nx && yo < g.ny) {
          const int hp = (yy + 1) * HX + tx + 1;
          TU s0[6], sx[6], sy[6], qq[3];
#pragma unroll
          for (int j = 0; j < 6; ++j) {
            s0[j] = sg[j][hp];
            sx[j] = sg[j][hp - 1];
            sy[j] = sg[j][hp - HX];
          }
          div_adj3<TU>(s0, sx, sy, below[k], ih, qq);
          const long long i = ((long long)z * g.ny + yo) * g.nx + xo;
          if (RES) {
            q[i] = (T)(f[i] - qq[0]);
            q[n + i] = (T)(f[n + i] - qq[1]);
            q[2 * n + i] = (T)(f[2 * n + i] - qq[2]);
          } else {
            q[i] = (T)qq[0];
            q[n + i] = (T)qq[1];
            q[2 * n + i] = (T)qq[2];
          }
#pragma unroll
          for (int j = 0; j < 6; ++j) below[k][j] = s0[j];
        }
      }
      __syncthreads();
    }
  }
  if (!RES) {
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

// r = f = -grad^H g C : (eps_mac - e I); x = 0.
template <typename T>
__global__ void __launch_bounds__(NT) k_mech3_rhs(MechMat m, const double* eig, Em6 em, T* __restrict__ r,
                                                  T* __restrict__ x, Grid3 g, T ih) {
  const long long n = g.n;
  const SlabIter it(g.nx, (long long)g.ny * g.nz);
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

// eps = eps_mac + sym(grad u), sigma = g C : (eps - e I); partial sums of
// sigma (6) and (eps - e I) : sigma, 7 per block.
static __global__ void __launch_bounds__(NT) k_mech3_post(MechMat m, const double* __restrict__ u, Grid3 g, double ih,
                                                   const double* eig, Em6 em, double* strain, double* stress,
                                                   double* part) {
  __shared__ double red[NT / 64];
  const long long n = g.n;
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  const SlabIter it(g.nx, (long long)g.ny * g.nz);
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
static __global__ void __launch_bounds__(NT) k_history3(MechMat m, const double* strain, const double* e, double* H,
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
static __global__ void __launch_bounds__(NT) k_spec_out(const double2* __restrict__ in, double2* __restrict__ out, int nxh,
                                                 int ny, int nz) {
  const long long tot = (long long)nxh * ny * nz;
  for (long long o = blockIdx.x * (long long)NT + threadIdx.x; o < tot; o += (long long)gridDim.x * NT) {
    const int kx = (int)(o % nxh);
    const long long zy = o / nxh;  // z ny + y
    out[o] = in[(long long)kx * ny * nz + zy];
  }
}

static __global__ void __launch_bounds__(NT) k_spec_in(const double2* __restrict__ in, double2* __restrict__ out, int nxh,
                                                int ny, int nz) {
  const long long tot = (long long)nxh * ny * nz;
  for (long long o = blockIdx.x * (long long)NT + threadIdx.x; o < tot; o += (long long)gridDim.x * NT) {
    const int kx = (int)(o % nxh);
    const long long zy = o / nxh;
    out[(long long)kx * ny * nz + zy] = in[o];
  }
}

}  // namespace fgcg
