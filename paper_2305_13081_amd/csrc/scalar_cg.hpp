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
//               formed from r and the previous p (double-buffered by iteration
//               parity) once per voxel of an LDS tile, q = A p from the tile;
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

// Stencil operators.  apply_vals takes the value at the voxel and at its
// neighbours vn = {x-1, x+1, y-1, y+1, z-1, z+1} (the z entries only on 3D
// grids); apply gathers them from a functor v(j, x) (value at linear index j,
// x coordinate x).  coef(b) loads the voxel's coefficients and apply_coef
// applies the operator with them (apply_vals is the two in a row), so the
// stencil pass can issue the coefficient loads early.
struct PfStencil {
  const double* H;
  double a;     // Gc / (2 l0)
  double cih2;  // (Gc l0 / 2) / h^2
  __device__ __forceinline__ bool fixed(long long, int) const { return false; }
  __device__ __forceinline__ bool has_fixed() const { return false; }
  struct Coef {
    double h;
  };
  __device__ __forceinline__ Coef coef(const Nbr& b) const { return Coef{H[b.i]}; }
  __device__ __forceinline__ double apply_coef(const Coef& c, const Nbr& b, double v0, const double* vn) const {
    double lap = (b.three ? 6.0 : 4.0) * v0 - vn[0] - vn[1] - vn[2] - vn[3];
    if (b.three) lap = lap - vn[4] - vn[5];
    return (a + c.h) * v0 + cih2 * lap;
  }
  __device__ __forceinline__ double apply_vals(const Nbr& b, double v0, const double* vn) const {
    return apply_coef(coef(b), b, v0, vn);
  }
  template <typename V>
  __device__ __forceinline__ double apply(double v0, const V& v, const Nbr& b) const {
    const double vn[6] = {v(b.ixm, b.xm), v(b.ixp, b.xp), v(b.iym, b.x), v(b.iyp, b.x),
                          b.three ? v(b.izm, b.x) : 0.0, b.three ? v(b.izp, b.x) : 0.0};
    return apply_vals(b, v0, vn);
  }
};

struct DiffStencil {
  DiffCoef co;
  const uint8_t* phase;
  double ih2;
  // Dirichlet voxels: the band x < co.band
  __device__ __forceinline__ bool fixed(long long, int x) const { return x < co.band; }
  __device__ __forceinline__ bool has_fixed() const { return co.band > 0; }
  __device__ __forceinline__ double D(long long j) const {
    double d, kr;
    pick(co.dk, phase[j], d, kr);
    return d;
  }
  struct Coef {
    uint8_t p0, pxm, pym, pzm;  // phases of the voxel and of its -x, -y, -z neighbours
  };
  __device__ __forceinline__ Coef coef(const Nbr& b) const {
    return Coef{phase[b.i], phase[b.ixm], phase[b.iym], b.three ? phase[b.izm] : (uint8_t)0};
  }
  __device__ __forceinline__ double apply_coef(const Coef& c, const Nbr& b, double v0, const double* vn) const {
    double d0, kr, dxm, dym, dzm, t;
    pick(co.dk, c.p0, d0, kr);
    pick(co.dk, c.pxm, dxm, t);
    pick(co.dk, c.pym, dym, t);
    double flux = dxm * (v0 - vn[0]) - d0 * (vn[1] - v0) + dym * (v0 - vn[2]) - d0 * (vn[3] - v0);
    if (b.three) {
      pick(co.dk, c.pzm, dzm, t);
      flux = flux + dzm * (v0 - vn[4]) - d0 * (vn[5] - v0);
    }
    return (co.inv_dt + kr) * v0 + ih2 * flux;
  }
  __device__ __forceinline__ double apply_vals(const Nbr& b, double v0, const double* vn) const {
    return apply_coef(coef(b), b, v0, vn);
  }
  template <typename V>
  __device__ __forceinline__ double apply(double v0, const V& v, const Nbr& b) const {
    const double vn[6] = {v(b.ixm, b.xm), v(b.ixp, b.xp), v(b.iym, b.x), v(b.iyp, b.x),
                          b.three ? v(b.izm, b.x) : 0.0, b.three ? v(b.izp, b.x) : 0.0};
    return apply_vals(b, v0, vn);
  }
};

// Diffusion step with per-voxel fields (Sec. 2.1 defines D point by point):
// D and the first-order rate k_r are device arrays, the Dirichlet voxels are
// those with mask != 0 (no mask: none).
struct DiffFieldStencil {
  const double* D;
  const double* kr;       // nullable: no sink
  const uint8_t* mask;    // nullable: no Dirichlet voxels
  double inv_dt;
  double ih2;
  __device__ __forceinline__ bool fixed(long long i, int) const { return mask != nullptr && mask[i] != 0; }
  __device__ __forceinline__ bool has_fixed() const { return mask != nullptr; }
  struct Coef {
    double d0, dxm, dym, dzm, k;
  };
  __device__ __forceinline__ Coef coef(const Nbr& b) const {
    return Coef{D[b.i], D[b.ixm], D[b.iym], b.three ? D[b.izm] : 0.0, kr ? kr[b.i] : 0.0};
  }
  __device__ __forceinline__ double apply_coef(const Coef& c, const Nbr& b, double v0, const double* vn) const {
    double flux = c.dxm * (v0 - vn[0]) - c.d0 * (vn[1] - v0) + c.dym * (v0 - vn[2]) - c.d0 * (vn[3] - v0);
    if (b.three) flux = flux + c.dzm * (v0 - vn[4]) - c.d0 * (vn[5] - v0);
    return (inv_dt + c.k) * v0 + ih2 * flux;
  }
  __device__ __forceinline__ double apply_vals(const Nbr& b, double v0, const double* vn) const {
    return apply_coef(coef(b), b, v0, vn);
  }
  template <typename V>
  __device__ __forceinline__ double apply(double v0, const V& v, const Nbr& b) const {
    const double vn[6] = {v(b.ixm, b.xm), v(b.ixp, b.xp), v(b.iym, b.x), v(b.iyp, b.x),
                          b.three ? v(b.izm, b.x) : 0.0, b.three ? v(b.izp, b.x) : 0.0};
    return apply_vals(b, v0, vn);
  }
};

// k_scg_upd and k_scg_init walk the rows (z ny + y) in XCD slabs (SlabIter);
// their grid is one-dimensional with a multiple of 8 blocks.

// First pass of iteration k.  Dirichlet voxels (op.fixed) keep p = q = 0.
// p is double-buffered (pin -> pout): the direction at the neighbours is formed
// from the previous p, which other threads of this launch must not overwrite.
//
// Tiled: a block forms p = r + beta p once per voxel of an SC_TX x SC_TY tile
// and its one-voxel halo ring into LDS and applies the stencil from there; on
// 3D grids it marches the tile through SC_ZC planes with two LDS planes (z and
// z + 1) and p of the plane below in registers.  Tile-chunks are ordered x, y,
// z and each block walks a contiguous range of them, XCD by XCD.
constexpr int SC_TX = 64, SC_TY = 16, SC_ZC = 8;

inline int scg_chunks(int nx, int ny, int nz) {
  return ((nx + SC_TX - 1) / SC_TX) * ((ny + SC_TY - 1) / SC_TY) * (nz > 1 ? (nz + SC_ZC - 1) / SC_ZC : 1);
}

template <typename T, class Op>
__global__ void __launch_bounds__(NT) k_scg_dir(Op op, const T* __restrict__ r, const T* __restrict__ pin,
                                                T* __restrict__ pout, T* __restrict__ q, int nx, int ny, int nz,
                                                CgCtl cc) {
  constexpr int HX = SC_TX + 2, HY = SC_TY + 2, HP = HX * HY;
  constexpr int RPT = SC_TY / (NT / SC_TX);  // own rows per thread
  __shared__ double pl[2][HP];
  __shared__ double red[NT / 64];
  double beta;
  if (!cg_begin_dir(cc, 0, red, beta)) return;
  const bool first = beta == 0.0;  // beta is 0 exactly on the first iteration
  const T b = (T)beta;
  const bool three = nz > 1;
  const long long plane = (long long)nx * ny;
  auto pval = [&](long long j) -> double { return first ? (double)r[j] : (double)(r[j] + b * pin[j]); };
  const int ntx = (nx + SC_TX - 1) / SC_TX, nty = (ny + SC_TY - 1) / SC_TY;
  const int nch = ntx * nty * (three ? (nz + SC_ZC - 1) / SC_ZC : 1);
  const int lb = xcd_block(), nb = gridDim.x;
  const int c0 = (int)((long long)nch * lb / nb), c1 = (int)((long long)nch * (lb + 1) / nb);
  const int tx = threadIdx.x & (SC_TX - 1), ty = threadIdx.x / SC_TX;
  // halo tile of plane z: the tile, the columns x0 - 1 and x0 + SC_TX and the
  // rows y0 - 1 and y0 + SC_TY (periodic); entries past the edge of a partial
  // tile are never read and are skipped
  auto fill = [&](double* buf, int x0, int y0, int z) {
    for (int hp = threadIdx.x; hp < HP; hp += NT) {
      const int hy = hp / HX, hx = hp - hy * HX;
      int x = x0 - 1 + hx, y = y0 - 1 + hy;
      if (x > nx || y > ny) continue;
      x = x < 0 ? nx - 1 : (x == nx ? 0 : x);
      y = y < 0 ? ny - 1 : (y == ny ? 0 : y);
      buf[hp] = pval((long long)z * plane + (long long)y * nx + x);
    }
  };
  double acc = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int x0 = (c % ntx) * SC_TX, y0 = ((c / ntx) % nty) * SC_TY;
    const int z0 = three ? (c / (ntx * nty)) * SC_ZC : 0;
    const int z1 = three ? min(z0 + SC_ZC, nz) : 1;
    const int xo = x0 + tx;
    double pm[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int yo = y0 + ty + k * (NT / SC_TX);
      pm[k] = 0.0;
      if (three && xo < nx && yo < ny)
        pm[k] = pval((long long)(z0 == 0 ? nz - 1 : z0 - 1) * plane + (long long)yo * nx + xo);
    }
    int cur = 0;
    fill(pl[0], x0, y0, z0);
    for (int z = z0; z < z1; ++z) {
      if (three) fill(pl[cur ^ 1], x0, y0, z + 1 == nz ? 0 : z + 1);
      // the voxels' coefficients (phases, history) are loaded before the
      // barrier, so their latency overlaps the halo fill's
      Nbr nbr[RPT];
      typename Op::Coef cf[RPT];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int yo = y0 + ty + k * (NT / SC_TX);
        nbr[k].i = ((long long)z * ny + yo) * nx + xo;
        nbr[k].ixm = nbr[k].i + (xo == 0 ? nx - 1 : -1);
        nbr[k].iym = nbr[k].i + (yo == 0 ? (long long)(ny - 1) * nx : -(long long)nx);
        nbr[k].izm = nbr[k].i + (z == 0 ? (long long)(nz - 1) * plane : -plane);
        nbr[k].three = three;
        if (xo < nx && yo < ny) cf[k] = op.coef(nbr[k]);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int yy = ty + k * (NT / SC_TX);
        const int yo = y0 + yy;
        if (xo < nx && yo < ny) {
          const int hp = (yy + 1) * HX + tx + 1;
          const double* P = pl[cur];
          const double v0 = P[hp];
          const double vn[6] = {P[hp - 1], P[hp + 1], P[hp - HX], P[hp + HX], three ? pm[k] : 0.0,
                                three ? pl[cur ^ 1][hp] : 0.0};
          const Nbr& nb = nbr[k];
          const double qv = op.fixed(nb.i, xo) ? 0.0 : op.apply_coef(cf[k], nb, v0, vn);
          pout[nb.i] = (T)v0;
          q[nb.i] = (T)qv;
          acc += v0 * qv;
          pm[k] = v0;
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) cc.part_a[blockIdx.x] = t;
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

// Initial residual r = b - A x0 with x0 = xin (zero on the Dirichlet voxels),
// partial sums of ||b||^2 and r.r (k_cg_init then sets the state).
// b = bsrc: the phase field passes H; the diffusion step passes c^n / dt on
// the free voxels, with A applied to c~ (c^n, c_dir on the Dirichlet voxels)
// and b_F = M(c^n/dt - A c_B).
template <typename T, class Op>
__global__ void __launch_bounds__(NT) k_scg_init(Op op, const double* __restrict__ xin, double bscale,
                                                 const double* __restrict__ bsrc, double c_dir,
                                                 T* __restrict__ x, T* __restrict__ r, int nx, int ny, int nz,
                                                 double* part_b, double* part_rr) {
  __shared__ double red[NT / 64];
  auto vt = [&](long long j, int xx) -> double { return op.fixed(j, xx) ? c_dir : xin[j]; };
  auto vb = [&](long long j, int xx) -> double { return op.fixed(j, xx) ? c_dir : 0.0; };
  double acc[2] = {0.0, 0.0};
  const SlabIter it(nx, (long long)ny * nz);
  for (long long v = it.v0; v < it.v1; v += it.step) {
    const int row = (int)((unsigned)v / (unsigned)nx), xx = (int)(v - (long long)row * nx);
    const Nbr nb = nbrs(row, xx, nx, ny, nz);
    const long long i = nb.i;
    if (op.fixed(i, xx)) {
      x[i] = (T)0;
      r[i] = (T)0;
      continue;
    }
    const double b = bscale * bsrc[i];
    const double ax = op.apply(vt(i, xx), vt, nb);
    double bf = b;
    if (op.has_fixed()) bf = b - op.apply(0.0, vb, nb);
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

// ------------------------------------------- one-reduction form (2D grids)
// CG in the one-reduction form of Chronopoulos and Gear: with w = A r and
// s = A p carried along, gamma_k = r_k.r_k and delta_k = w_k.r_k give
//     beta_k = gamma_k / gamma_{k-1},
//     alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
// (beta_0 = 0, alpha_0 = gamma_0 / delta_0), the alpha and beta of textbook
// CG in exact arithmetic, and one pass per iteration:
//     p = r + beta p, s = w + beta s, x += alpha p, r -= alpha s, w = A r,
// with gamma_{k+1} and delta_{k+1} summed on the way.  The stencil of the new
// r takes its values on the tile's halo, formed there from the old r, w and s
// (double-buffered by iteration parity, as are the partial sums and the
// scalars of CgState that every block reads: see CgState::kk).  The stop test
// (||r_k||^2 <= tol^2 ||b||^2, k < maxit) is textbook CG's, before the
// update of iteration k.  Dirichlet voxels (op.fixed) keep r = w = s = p = 0.
// init: only w_0 = A r_0 and the partial sums of gamma_0, delta_0.
// Partial sums: part[parity][0][block] = gamma, part[parity][1][block] = delta
// (np blocks).  2D grids (nz = 1).
template <typename T, class Op>
__global__ void __launch_bounds__(NT) k_scg_cg(Op op, T* __restrict__ x, T* __restrict__ p,
                                               const T* __restrict__ rin, T* __restrict__ rout,
                                               const T* __restrict__ win, T* __restrict__ wout,
                                               const T* __restrict__ sin, T* __restrict__ sout, int nx, int ny,
                                               CgState* st, double* part, int np, int parity, int init) {
  constexpr int HX = SC_TX + 2, HY = SC_TY + 2, HP = HX * HY;
  constexpr int RPT = SC_TY / (NT / SC_TX);  // own rows per thread
  __shared__ double rl[HP];  // new r on the tile and its halo
  __shared__ double r0l[HP], s1l[HP];  // old r and new s there (the own voxels' updates read them)
  __shared__ double red[NT / 64];
  double alpha = 0.0, beta = 0.0;
  int k = 0;
  if (!init) {
    // scalars of this iteration (every block computes them alike)
    if (!cg_running(st, 0)) return;
    CgState* S = st;
    k = S->kk[parity];
    const double* pin = part + (long long)parity * 2 * np;
    const double g = block_sum_array(pin, np, red), dl = block_sum_array(pin + np, np, red);
    int code = 0;
    if (!isfinite(g)) code = 3;
    else if (g <= S->thr) code = 1;
    else if (k >= S->maxit) code = 2;
    double den = dl;
    if (!code) {
      if (k > 0) {
        beta = g / S->gam[parity];
        den = dl - beta * g / S->stp[parity];
      }
      if (!(den > 0.0) || !isfinite(den)) code = 3;
    }
    if (code) {
      if (lead()) {
        S->done = code;
        S->iter = k;
        S->rr_final = g;
      }
      return;
    }
    alpha = g / den;
    if (lead()) {
      S->kk[parity ^ 1] = k + 1;
      S->gam[parity ^ 1] = g;
      S->stp[parity ^ 1] = alpha;
      S->k = k + 1;
    }
  }
  const bool first = k == 0;  // (p and s of the previous iteration are not read)
  const T a = (T)alpha, b = (T)beta;
  // at linear index j: old r, new s = w + beta s and new r = r - alpha s
  auto fillpt = [&](int hp, long long j) {
    const T r0 = rin[j];
    if (init) {
      rl[hp] = (double)r0;
      return;
    }
    const T sv = first ? win[j] : (T)(win[j] + b * sin[j]);
    r0l[hp] = (double)r0;
    s1l[hp] = (double)sv;
    rl[hp] = (double)(r0 - a * sv);
  };
  const int ntx = (nx + SC_TX - 1) / SC_TX, nty = (ny + SC_TY - 1) / SC_TY;
  const int nch = ntx * nty;
  const int lb = xcd_block(), nb = gridDim.x;
  const int c0 = (int)((long long)nch * lb / nb), c1 = (int)((long long)nch * (lb + 1) / nb);
  const int tx = threadIdx.x & (SC_TX - 1), ty = threadIdx.x / SC_TX;
  double accg = 0.0, accd = 0.0;
  for (int c = c0; c < c1; ++c) {
    const int x0 = (c % ntx) * SC_TX, y0 = (c / ntx) * SC_TY;
    const int xo = x0 + tx;
    for (int hp = threadIdx.x; hp < HP; hp += NT) {
      const int hy = hp / HX, hx = hp - hy * HX;
      int xx = x0 - 1 + hx, yy = y0 - 1 + hy;
      if (xx > nx || yy > ny) continue;  // past the edge of a partial tile (never read)
      xx = xx < 0 ? nx - 1 : (xx == nx ? 0 : xx);
      yy = yy < 0 ? ny - 1 : (yy == ny ? 0 : yy);
      fillpt(hp, (long long)yy * nx + xx);
    }
    // the voxels' coefficients, previous direction and solution are loaded
    // before the barrier
    Nbr nbr[RPT];
    typename Op::Coef cf[RPT];
    T pold[RPT], xold[RPT];
#pragma unroll
    for (int kk = 0; kk < RPT; ++kk) {
      const int yo = y0 + ty + kk * (NT / SC_TX);
      nbr[kk].i = (long long)yo * nx + xo;
      nbr[kk].ixm = nbr[kk].i + (xo == 0 ? nx - 1 : -1);
      nbr[kk].iym = nbr[kk].i + (yo == 0 ? (long long)(ny - 1) * nx : -(long long)nx);
      nbr[kk].izm = nbr[kk].i;
      nbr[kk].three = false;
      pold[kk] = xold[kk] = (T)0;
      if (xo < nx && yo < ny) {
        cf[kk] = op.coef(nbr[kk]);
        if (!init) {
          if (!first) pold[kk] = p[nbr[kk].i];
          xold[kk] = x[nbr[kk].i];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < RPT; ++kk) {
      const int yy = ty + kk * (NT / SC_TX);
      const int yo = y0 + yy;
      if (xo < nx && yo < ny) {
        const int hp = (yy + 1) * HX + tx + 1;
        const Nbr& nb = nbr[kk];
        const long long i = nb.i;
        const double r1 = rl[hp];
        const double vn[6] = {rl[hp - 1], rl[hp + 1], rl[hp - HX], rl[hp + HX], 0.0, 0.0};
        const double w1 = op.fixed(i, xo) ? 0.0 : op.apply_coef(cf[kk], nb, r1, vn);
        if (init) {
          wout[i] = (T)w1;
        } else {
          const T r0 = (T)r0l[hp];
          const T pv = first ? r0 : (T)(r0 + b * pold[kk]);
          p[i] = pv;
          sout[i] = (T)s1l[hp];
          x[i] = xold[kk] + a * pv;
          rout[i] = (T)r1;
          wout[i] = (T)w1;
        }
        accg += r1 * r1;
        accd += w1 * r1;
      }
    }
    __syncthreads();
  }
  const double tg = block_sum(accg, red), td = block_sum(accd, red);
  if (threadIdx.x == 0) {
    double* po = part + (long long)(init ? 0 : parity ^ 1) * 2 * np;
    po[blockIdx.x] = tg;
    po[np + blockIdx.x] = td;
  }
}

// c = c_dir on the Dirichlet voxels, x elsewhere
template <typename T, class Op>
__global__ void __launch_bounds__(NT) k_scg_finish(Op op, double* c, const T* x, long long n, int nx, double c_dir) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    c[i] = op.fixed(i, (int)(i % nx)) ? c_dir : (double)x[i];
}

}  // namespace fgcg
