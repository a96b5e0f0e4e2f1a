// Static diffusion homogenisation on the representative volume (Sec. 2.1)
// and the concentration reconstruction (eqs. micro-gradient to
// concentration-correct): the real-space kernels.
//
// The paper solves for the compatible fluctuation x of the concentration
// gradient with G[D (grad c_mac + x)] = 0 (eq. diffusion-final, the vector
// projection G of App. A).  With the forward difference of Sec. 2.6 every
// compatible periodic field is a gradient, x = grad phi, and G factors as
// grad (grad^H grad)^-1 grad^H, so the projected CG on x is, iterate by
// iterate, CG on the scalar fluctuation phi for
//     K phi = f,   K = grad^H D grad,   f = -grad^H D grad c_mac,
// preconditioned by the Green operator (grad^H grad)^-1 -- the mechanics
// engine with one component.  K is the 5-point (7-point in 3D) flux stencil:
//     (K p)(x) = sum_a [j_a(x - e_a) - j_a(x)] / h,   j_a = D (p(x + e_a) - p(x)) / h.
#pragma once
#include "mech3.hpp"
#include "scalar_cg.hpp"

namespace fgcg {

// q = K p with partial sums of p.Kp = sum_x grad p . D grad p (2D).  Tiled
// as the mechanics stiffness pass: the flux is formed once per voxel of a
// 64 x 16 tile and of its halo column x0 - 1 and halo row y0 - 1 and kept in
// LDS; the lead thread publishes the iteration counter.
constexpr int FK_TX = 64, FK_TY = 16;

inline int fk_tiles(int nx, int ny) { return ((nx + FK_TX - 1) / FK_TX) * ((ny + FK_TY - 1) / FK_TY); }

template <typename T>
__global__ void __launch_bounds__(NT) k_flux_kp(const double* __restrict__ Df, const T* __restrict__ p,
                                                T* __restrict__ q, int nx, int ny, T ih, CgState* st,
                                                double* part) {
  constexpr int HX = FK_TX + 1, HY = FK_TY + 1, HP = HX * HY;
  __shared__ T jx[HP], jy[HP];
  __shared__ double red[NT / 64];
  if (!cg_running(st, 0)) return;
  if (lead()) st->k = st->k_next;
  const int ntx = (nx + FK_TX - 1) / FK_TX;
  const int ntiles = ntx * ((ny + FK_TY - 1) / FK_TY);
  const int lb = xcd_block(), nb = gridDim.x;
  const int t0 = (int)((long long)ntiles * lb / nb), t1 = (int)((long long)ntiles * (lb + 1) / nb);
  const int tx = threadIdx.x & (FK_TX - 1), ty = threadIdx.x / FK_TX;
  double acc = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int x0 = (t % ntx) * FK_TX, y0 = (t / ntx) * FK_TY;
#pragma unroll
    for (int k = 0; k < (HP + NT - 1) / NT; ++k) {
      const int hp = threadIdx.x + k * NT;
      const int hy = hp / HX, hx = hp - hy * HX;
      int x = x0 - 1 + hx, y = y0 - 1 + hy;
      // past the halo, or past the edge of a partial tile (never read)
      if (hp >= HP || x >= nx || y >= ny) continue;
      if (x < 0) x += nx;
      if (y < 0) y += ny;
      const int xp = x + 1 == nx ? 0 : x + 1, yp = y + 1 == ny ? 0 : y + 1;
      const long long i = (long long)y * nx + x;
      const T p0 = p[i];
      const T g1 = (p[(long long)y * nx + xp] - p0) * ih;
      const T g2 = (p[(long long)yp * nx + x] - p0) * ih;
      const T d = (T)Df[i];
      const T f1 = d * g1, f2 = d * g2;
      jx[hp] = f1;
      jy[hp] = f2;
      if (hx >= 1 && hy >= 1) acc += (double)g1 * f1 + (double)g2 * f2;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < FK_TY / (NT / FK_TX); ++k) {
      const int yy = ty + k * (NT / FK_TX);
      const int x = x0 + tx, y = y0 + yy;
      if (x < nx && y < ny) {
        const int hp = (yy + 1) * HX + tx + 1;
        q[(long long)y * nx + x] = ((jx[hp - 1] - jx[hp]) + (jy[hp - HX] - jy[hp])) * ih;
      }
    }
    __syncthreads();
  }
  const double tsum = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tsum;
}

// The same operator on 3D grids: 64 x 8 tiles marching through 8 planes; the
// z flux of the plane below stays in registers.
constexpr int F3_TX = 64, F3_TY = 8, F3_ZC = 8;

inline int f3_chunks(int nx, int ny, int nz) {
  return ((nx + F3_TX - 1) / F3_TX) * ((ny + F3_TY - 1) / F3_TY) * ((nz + F3_ZC - 1) / F3_ZC);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_flux3_kp(const double* __restrict__ Df, const T* __restrict__ p,
                                                 T* __restrict__ q, Grid3 g, T ih, CgState* st, double* part) {
  constexpr int HX = F3_TX + 1, HY = F3_TY + 1, HP = HX * HY;
  constexpr int RPT = F3_TY / (NT / F3_TX);
  __shared__ T jx[HP], jy[HP];
  __shared__ double red[NT / 64];
  if (!cg_running(st, 0)) return;
  if (lead()) st->k = st->k_next;
  const long long pl = (long long)g.nx * g.ny;
  const int ntx = (g.nx + F3_TX - 1) / F3_TX, nty = (g.ny + F3_TY - 1) / F3_TY;
  const int nch = ntx * nty * ((g.nz + F3_ZC - 1) / F3_ZC);
  const int lb = xcd_block(), nb = gridDim.x;
  const int c0 = (int)((long long)nch * lb / nb), c1 = (int)((long long)nch * (lb + 1) / nb);
  const int tx = threadIdx.x & (F3_TX - 1), ty = threadIdx.x / F3_TX;
  // z flux D (p(z + 1) - p(z)) / h at (x, y, z) and its gradient
  auto jz_at = [&](int x, int y, int z, T& gz) -> T {
    const long long i = (long long)z * pl + (long long)y * g.nx + x;
    const long long iz = (long long)(z + 1 == g.nz ? 0 : z + 1) * pl + (long long)y * g.nx + x;
    gz = (p[iz] - p[i]) * ih;
    return (T)Df[i] * gz;
  };
  double acc = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int x0 = (c % ntx) * F3_TX, y0 = ((c / ntx) % nty) * F3_TY;
    const int z0 = (c / (ntx * nty)) * F3_ZC, z1 = min(z0 + F3_ZC, g.nz);
    const int xo = x0 + tx;
    T below[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int yo = y0 + ty + k * (NT / F3_TX);
      T gz;
      below[k] = (xo < g.nx && yo < g.ny) ? jz_at(xo, yo, z0 == 0 ? g.nz - 1 : z0 - 1, gz) : (T)0;
    }
    for (int z = z0; z < z1; ++z) {
      for (int hp = threadIdx.x; hp < HP; hp += NT) {
        const int hy = hp / HX, hx = hp - hy * HX;
        int x = x0 - 1 + hx, y = y0 - 1 + hy;
        if (x >= g.nx || y >= g.ny) continue;  // past the edge of a partial tile: never read
        if (x < 0) x += g.nx;
        if (y < 0) y += g.ny;
        const int xp = x + 1 == g.nx ? 0 : x + 1, yp = y + 1 == g.ny ? 0 : y + 1;
        const long long i = (long long)z * pl + (long long)y * g.nx + x;
        const T p0 = p[i];
        const T g1 = (p[(long long)z * pl + (long long)y * g.nx + xp] - p0) * ih;
        const T g2 = (p[(long long)z * pl + (long long)yp * g.nx + x] - p0) * ih;
        const T d = (T)Df[i];
        jx[hp] = d * g1;
        jy[hp] = d * g2;
        if (hx >= 1 && hy >= 1) acc += (double)g1 * (d * g1) + (double)g2 * (d * g2);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int yy = ty + k * (NT / F3_TX);
        const int yo = y0 + yy;
        if (xo < g.nx && yo < g.ny) {
          const int hp = (yy + 1) * HX + tx + 1;
          T gz;
          const T jz = jz_at(xo, yo, z, gz);
          acc += (double)gz * jz;
          q[(long long)z * pl + (long long)yo * g.nx + xo] =
              ((jx[hp - 1] - jx[hp]) + (jy[hp - HX] - jy[hp]) + (below[k] - jz)) * ih;
          below[k] = jz;
        }
      }
      __syncthreads();
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

struct Vec3 {
  double v[3];
};

// r = f = -grad^H D grad c_mac, x = 0 (2D: nz = 1, gm.v[2] unused).
static __global__ void __launch_bounds__(NT) k_flux_rhs(const double* __restrict__ Df, Vec3 gm, double* __restrict__ r,
                                                 double* __restrict__ x, int nx, int ny, int nz, double ih) {
  const SlabIter it(nx, (long long)ny * nz);
  for (long long v = it.v0; v < it.v1; v += it.step) {
    const int row = (int)((unsigned)v / (unsigned)nx), xx = (int)(v - (long long)row * nx);
    const Nbr b = nbrs(row, xx, nx, ny, nz);
    const double d0 = Df[b.i];
    double f = (Df[b.ixm] - d0) * gm.v[0] + (Df[b.iym] - d0) * gm.v[1];
    if (b.three) f += (Df[b.izm] - d0) * gm.v[2];
    r[b.i] = -f * ih;
    x[b.i] = 0.0;
  }
}

// grad c = grad c_mac + grad phi, flux j = -D grad c; optional outputs grad c
// (component-major) and phi; partial sums per block: the dim mean-flux sums and
// sum grad c . D grad c (4 per block).
static __global__ void __launch_bounds__(NT) k_flux_post(const double* __restrict__ Df, const double* __restrict__ u,
                                                  Vec3 gm, int nx, int ny, int nz, double ih, double* grad_c,
                                                  double* phi, double* part) {
  __shared__ double red[NT / 64];
  const long long n = (long long)nx * ny * nz;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  const SlabIter it(nx, (long long)ny * nz);
  for (long long v = it.v0; v < it.v1; v += it.step) {
    const int row = (int)((unsigned)v / (unsigned)nx), xx = (int)(v - (long long)row * nx);
    const Nbr b = nbrs(row, xx, nx, ny, nz);
    const double u0 = u[b.i];
    const double gc[3] = {gm.v[0] + (u[b.ixp] - u0) * ih, gm.v[1] + (u[b.iyp] - u0) * ih,
                          b.three ? gm.v[2] + (u[b.izp] - u0) * ih : 0.0};
    const double d = Df[b.i];
    const int dim = b.three ? 3 : 2;
    for (int c = 0; c < dim; ++c) {
      if (grad_c) grad_c[c * n + b.i] = gc[c];
      a[c] -= d * gc[c];
      a[3] += d * gc[c] * gc[c];
    }
    if (phi) phi[b.i] = u0;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double t = block_sum(a[c], red);
    if (threadIdx.x == 0) part[4 * blockIdx.x + c] = t;
  }
}

// Concentration reconstruction, eq. phi-fft through the inverse gradient of
// eq. g-42 on the 3D half spectrum [comp][kx][z][y] of grad c:
// out = sum_a conj(D_a) g_a / |D|^2 / N into component 0 (zero at k = 0).
static __global__ void __launch_bounds__(NT) k_invgrad3(double2* spec, const double2* __restrict__ Dx,
                                                 const double2* __restrict__ Dy, const double2* __restrict__ Dz,
                                                 int nxh, int ny, int nz, double inv_n) {
  const long long per = (long long)nxh * nz * ny;
  for (long long o = blockIdx.x * (long long)NT + threadIdx.x; o < per; o += (long long)gridDim.x * NT) {
    const int y = (int)(o % ny);
    const long long r = o / ny;
    const int z = (int)(r % nz), kx = (int)(r / nz);
    const double2 d[3] = {Dx[kx], Dy[y], Dz[z]};
    const double n2 = d[0].x * d[0].x + d[0].y * d[0].y + d[1].x * d[1].x + d[1].y * d[1].y + d[2].x * d[2].x +
                      d[2].y * d[2].y;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double2 g = spec[a * per + o];
      re += d[a].x * g.x + d[a].y * g.y;  // conj(D) g
      im += d[a].x * g.y - d[a].y * g.x;
    }
    const double f = n2 > 0.0 ? inv_n / n2 : 0.0;
    spec[o] = double2{re * f, im * f};
  }
}

// Column symbol of the 2D reconstruction: NIN = 2 spectra of grad c -> phi_hat.
template <typename T> struct InvGradSym {
  const double2* Dx;
  const double2* Dy;
  double inv_n;
  __device__ bool begin(int, double*, double&) const { return true; }
  template <typename C>
  __device__ void mode(int, int kx, int ky, const C* a, C* b, double&, double) const {
    const double2 d1 = Dx[kx], d2 = Dy[ky];
    const double n2 = d1.x * d1.x + d1.y * d1.y + d2.x * d2.x + d2.y * d2.y;
    const double f = n2 > 0.0 ? inv_n / n2 : 0.0;
    const double re = d1.x * a[0].x + d1.y * a[0].y + d2.x * a[1].x + d2.y * a[1].y;
    const double im = d1.x * a[0].y - d1.y * a[0].x + d2.x * a[1].y - d2.y * a[1].x;
    b[0] = C{(T)(re * f), (T)(im * f)};
  }
  __device__ void partial(int, double) const {}
};

// Per-block sums for the two constants of eq. psi-two-values: [sum phi,
// sum grad c_mac . x, count] over the pores, then the same over the solid
// (6 per block); x of voxel (ix, iy, iz) is (ix, iy, iz) h.
static __global__ void __launch_bounds__(NT) k_conc_sums(const uint8_t* __restrict__ phase, const double* __restrict__ phi,
                                                  Vec3 gm, double h, int nx, int ny, int nz, double* part) {
  __shared__ double red[NT / 64];
  double a[6] = {0, 0, 0, 0, 0, 0};
  const SlabIter it(nx, (long long)ny * nz);
  for (long long v = it.v0; v < it.v1; v += it.step) {
    const int row = (int)((unsigned)v / (unsigned)nx), xx = (int)(v - (long long)row * nx);
    const int y = row % ny, z = row / ny;
    const double lin = h * (gm.v[0] * xx + gm.v[1] * y + gm.v[2] * z);
    const int o = phase[v] == 0 ? 0 : 3;
    a[o] += phi[v];
    a[o + 1] += lin;
    a[o + 2] += 1.0;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double t = block_sum(a[c], red);
    if (threadIdx.x == 0) part[6 * blockIdx.x + c] = t;
  }
}

// c = grad c_mac . x + phi + beta_phase (eq. concentration with the constants
// of eq. psi-two-values; eq. concentration-correct in the pores).
static __global__ void __launch_bounds__(NT) k_conc_write(const uint8_t* __restrict__ phase, const double* __restrict__ phi,
                                                   Vec3 gm, double h, int nx, int ny, int nz, double beta_pore,
                                                   double beta_solid, double* __restrict__ c) {
  const SlabIter it(nx, (long long)ny * nz);
  for (long long v = it.v0; v < it.v1; v += it.step) {
    const int row = (int)((unsigned)v / (unsigned)nx), xx = (int)(v - (long long)row * nx);
    const int y = row % ny, z = row / ny;
    const double lin = h * (gm.v[0] * xx + gm.v[1] * y + gm.v[2] * z);
    c[v] = lin + phi[v] + (phase[v] == 0 ? beta_pore : beta_solid);
  }
}

}  // namespace fgcg
