// CG for the scalar operators of the path with the operators applied as
// real-space stencils (2D and 3D grids).
//
// Both scalar operators are local: with the forward difference of Sec. 2.6
// (D_a <-> (f(x + e_a) - f(x))/h) the Laplacian symbol -|D|^2 of the phase
// field (Sec. 2.4, eq. crack-fft) is the periodic 5-point stencil, and the
// diffusion operator grad^H D(x) grad is the 5-point flux stencil
//     sum_a [D(x - e_a)(c(x) - c(x - e_a)) - D(x)(c(x + e_a) - c(x))] / h^2
// (7-point stencils on 3D grids).
// Applying them in real space gives the same operator as the Fourier-space
// product (up to rounding) with one pass over the data.  CG is textbook CG;
// one iteration is two passes:
//   k_scg_dir : beta = rr_k / rr_{k-1} and the stop tests; p = r + beta p is
//               formed at the voxel and at its four neighbours from r and the
//               previous p (double-buffered by iteration parity), q = A p;
//               writes p, q; sum p.q
//   k_scg_upd : alpha = rr_k / p.q; x += alpha p; r -= alpha q; sum r.r
// CG control is that of the other solves (cg_begin_dir / cg_begin_step):
// each pass stores one FP64 partial sum per block and the next pass adds them
// in block order, so the result is deterministic and cross-block visibility
// comes from kernel boundaries only (a grid-wide fence inside a launch would
// write back the L2 of every XCD).
#pragma once
#include "ops2d.hpp"

namespace fgcg {

__device__ __forceinline__ int block_linear() { return blockIdx.y * gridDim.x + blockIdx.x; }

// Neighbours of voxel (z, y, x) on the periodic grid, as linear indices
// (row = z ny + y; nz = 1 for 2D grids).  x, xm, xp are the x coordinates of
// the voxel and its x neighbours (the other neighbours share x).
struct Nbr {
  long long i, ixm, ixp, iym, iyp, izm, izp;
  int x, xm, xp;
  bool three;
};

__device__ __forceinline__ Nbr nbrs(int row, int x, int nx, int ny, int nz) {
  Nbr b;
  const int y = nz == 1 ? row : row % ny;
  const int z = nz == 1 ? 0 : row / ny;
  const long long rb = (long long)row * nx;
  b.i = rb + x;
  b.x = x;
  b.xm = x == 0 ? nx - 1 : x - 1;
  b.xp = x + 1 == nx ? 0 : x + 1;
  b.ixm = rb + b.xm;
  b.ixp = rb + b.xp;
  const long long zb = (long long)z * ny;
  b.iym = (zb + (y == 0 ? ny - 1 : y - 1)) * nx + x;
  b.iyp = (zb + (y + 1 == ny ? 0 : y + 1)) * nx + x;
  b.three = nz > 1;
  b.izm = ((long long)(z == 0 ? nz - 1 : z - 1) * ny + y) * nx + x;
  b.izp = ((long long)(z + 1 == nz ? 0 : z + 1) * ny + y) * nx + x;
  return b;
}

// Stencil operators.  v(j, x) is the value at linear index j (x coordinate x)
// from a functor, so the CG direction p = r + beta p can be formed at the
// neighbours on the fly.
struct PfStencil {
  const double* H;
  double a;     // Gc / (2 l0)
  double cih2;  // (Gc l0 / 2) / h^2
  template <typename V>
  __device__ __forceinline__ double apply(double v0, const V& v, const Nbr& b) const {
    double lap = (b.three ? 6.0 : 4.0) * v0 - v(b.ixm, b.xm) - v(b.ixp, b.xp) - v(b.iym, b.x) - v(b.iyp, b.x);
    if (b.three) lap = lap - v(b.izm, b.x) - v(b.izp, b.x);
    return (a + H[b.i]) * v0 + cih2 * lap;
  }
};

struct DiffStencil {
  DiffCoef co;
  const uint8_t* phase;
  double ih2;
  __device__ __forceinline__ double D(long long j) const {
    double d, kr;
    pick(co.dk, phase[j], d, kr);
    return d;
  }
  template <typename V>
  __device__ __forceinline__ double apply(double v0, const V& v, const Nbr& b) const {
    double d0, kr;
    pick(co.dk, phase[b.i], d0, kr);
    double flux = D(b.ixm) * (v0 - v(b.ixm, b.xm)) - d0 * (v(b.ixp, b.xp) - v0) + D(b.iym) * (v0 - v(b.iym, b.x)) -
                  d0 * (v(b.iyp, b.x) - v0);
    if (b.three) flux = flux + D(b.izm) * (v0 - v(b.izm, b.x)) - d0 * (v(b.izp, b.x) - v0);
    return (co.inv_dt + kr) * v0 + ih2 * flux;
  }
};

// The kernels walk the rows (z ny + y) in XCD slabs (SlabIter); the grid is
// one-dimensional with a multiple of 8 blocks.

// First pass of iteration k.  band > 0: voxels with x < band are fixed
// (p = q = 0 there).
// p is double-buffered (pin -> pout): the direction at the neighbours is formed
// from the previous p, which other threads of this launch must not overwrite.
template <typename T, class Op>
__global__ void __launch_bounds__(NT) k_scg_dir(Op op, const T* __restrict__ r, const T* __restrict__ pin,
                                                T* __restrict__ pout, T* __restrict__ q, int nx, int ny, int nz,
                                                int band, CgCtl cc) {
  __shared__ double red[NT / 64];
  double beta;
  if (!cg_begin_dir(cc, 0, red, beta)) return;
  const bool first = beta == 0.0;  // beta is 0 exactly on the first iteration
  const T b = (T)beta;
  auto pn = [&](long long j, int) -> double { return first ? (double)r[j] : (double)(r[j] + b * pin[j]); };
  double acc = 0.0;
  const SlabIter it(nx, (long long)ny * nz);
  for (long long v = it.v0; v < it.v1; v += it.step) {
    const int row = (int)((unsigned)v / (unsigned)nx), x = (int)(v - (long long)row * nx);
    const Nbr nb = nbrs(row, x, nx, ny, nz);
    const double p0 = pn(nb.i, x);
    const double qv = x < band ? 0.0 : op.apply(p0, pn, nb);
    pout[nb.i] = (T)p0;
    q[nb.i] = (T)qv;
    acc += p0 * qv;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) cc.part_a[block_linear()] = t;
}

template <typename T>
__global__ void __launch_bounds__(NT) k_scg_upd(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                                const T* __restrict__ q, int nx, int rows, CgCtl cc) {
  __shared__ double red[NT / 64];
  double alpha;
  if (!cg_begin_step(cc, 0, red, alpha)) return;
  const T a = (T)alpha;
  double acc = 0.0;
  const SlabIter it(nx, rows);
  for (long long i = it.v0; i < it.v1; i += it.step) {
    x[i] += a * p[i];
    const T rv = r[i] - a * q[i];
    r[i] = rv;
    acc += (double)rv * (double)rv;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) cc.part_rr[block_linear()] = t;
}

// Initial residual r = b - A x0 with x0 = xin (mask band), partial sums of
// ||b||^2 and r.r (k_cg_init then sets the state).  b = bsrc: the phase field passes H; the diffusion step
// passes c^n / dt on the free voxels, with A applied to c~ (c^n, band = c_dir)
// and b_F = M(c^n/dt - A c_B).
template <typename T, class Op>
__global__ void __launch_bounds__(NT) k_scg_init(Op op, const double* __restrict__ xin, double bscale,
                                                 const double* __restrict__ bsrc, int band, double c_dir,
                                                 T* __restrict__ x, T* __restrict__ r, int nx, int ny, int nz,
                                                 double* part_b, double* part_rr) {
  __shared__ double red[NT / 64];
  auto vt = [&](long long j, int xx) -> double { return xx < band ? c_dir : xin[j]; };
  auto vb = [&](long long, int xx) -> double { return xx < band ? c_dir : 0.0; };
  double acc[2] = {0.0, 0.0};
  const SlabIter it(nx, (long long)ny * nz);
  for (long long v = it.v0; v < it.v1; v += it.step) {
    const int row = (int)((unsigned)v / (unsigned)nx), xx = (int)(v - (long long)row * nx);
    const Nbr nb = nbrs(row, xx, nx, ny, nz);
    const long long i = nb.i;
    if (xx < band) {
      x[i] = (T)0;
      r[i] = (T)0;
      continue;
    }
    const double b = bscale * bsrc[i];
    const double ax = op.apply(vt(i, xx), vt, nb);
    double bf = b;
    if (band > 0) bf = b - op.apply(0.0, vb, nb);
    const double res = b - ax;
    x[i] = (T)xin[i];
    r[i] = (T)res;
    acc[0] += bf * bf;
    acc[1] += res * res;
  }
  const double t0 = block_sum(acc[0], red), t1 = block_sum(acc[1], red);
  if (threadIdx.x == 0) {
    part_b[block_linear()] = t0;
    part_rr[block_linear()] = t1;
  }
}

}  // namespace fgcg
