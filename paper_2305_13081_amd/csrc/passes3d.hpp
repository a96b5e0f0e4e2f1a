// Transforms along y and z of the half spectra of 3D grids.
//
// The x-direction passes of the 2D engine (k_row_fwd / k_row_inv) run
// unchanged on a 3D grid taken as ny nz rows of length nx, and leave the half
// spectra as [comp][kx][z][y] with y contiguous.  Two more passes complete the
// transform:
//   k_ypass : in-place transforms of the y lines (contiguous), several lines
//             per block for short lines;
//   k_zpass : a block loads a tile of YT consecutive ky values over all z
//             (YT contiguous complex values per z, so the loads stay
//             coalesced), transforms along z in LDS with a bank-conflict-free
//             signal pitch, applies a per-mode symbol (the Green operator),
//             transforms back and stores the tile in place.
// A CG iteration of the 3D mechanics is then x-fwd, y-fwd, z (fwd + symbol +
// inv), y-inv, x-inv around the real-space stencil pass.
#pragma once
#include "ops2d.hpp"

namespace fgcg {

// y lines per block: at least about 1024 complex values per block.
constexpr int ylines_for(int ny, int nc) { return nc * ny >= 1024 ? 1 : 1024 / (nc * ny); }
// ky values per z tile: 128 contiguous bytes per z (8 in FP64, 16 in FP32),
// half that for z lines longer than 256.
template <typename T> constexpr int ztile_for(int nz) {
  return (sizeof(T) == 8 ? 8 : 16) / (nz > 256 ? 2 : 1);
}

// Deterministic single-block sum of np partial sums into out[0].
static __global__ void __launch_bounds__(NT) k_reduce(const double* __restrict__ part, int np, double* out) {
  __shared__ double red[NT / 64];
  const double t = block_sum_array<16>(part, np, red);  // up to 4096 partials: one round of loads
  if (threadIdx.x == 0) out[0] = t;
}

// NC spectra, lines [c][line][y] with nlines lines per component.
// st (nullable): the whole pass is skipped once the CG solve has ended.
template <typename T, int NY, int NC, bool INV>
__global__ void __launch_bounds__(NT) k_ypass(const CgState* st, typename cvec<T>::type* spec, int nlines,
                                              const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  constexpr int LPB = ylines_for(NY, NC);
  constexpr int NS = LPB * NC;
  __shared__ C buf[lds_size(NS * NY)];
  if (st && !cg_running(st, 0)) return;
  const int l0 = blockIdx.x * LPB;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NS * NY; idx += NT) {
    const int sig = idx / NY, y = idx - sig * NY;
    const int c = sig / LPB, l = sig - c * LPB;
    buf[lds(idx)] = l0 + l < nlines ? spec[((long long)c * nlines + l0 + l) * NY + y] : C{(T)0, (T)0};
  }
  __syncthreads();
  fft_lds<T, NY, NS, NT, INV>(buf, tw);
  for (int idx = tid; idx < NS * NY; idx += NT) {
    const int sig = idx / NY, y = idx - sig * NY;
    const int c = sig / LPB, l = sig - c * LPB;
    if (l0 + l < nlines) spec[((long long)c * nlines + l0 + l) * NY + y] = buf[lds(idx)];
  }
}

// Blocks: ZPT consecutive (component, kx, ky tile) entries each, tile
// fastest.  With ZPT = 2 the values of the next entry are loaded into
// registers while the current one is transformed, so the loads overlap the LDS
// work; ZPT = 1 loads its one tile straight into LDS.  zpt_for<T>() is the
// default where the context does not tune it (two in FP64, one in FP32, as
// measured on 256^3 grids).  FWD / INV select the transforms (the debug hook
// uses one of them alone); the symbol is applied between them and may reduce
// one FP64 partial sum per block.
template <typename T> constexpr int zpt_for() { return sizeof(T) == 8 ? 2 : 1; }

template <typename T, int NZ, bool FWD, bool INV, class Sym, int ZPT = zpt_for<T>()>
__global__ void __launch_bounds__(NT) k_zpass(Sym sym, typename cvec<T>::type* spec, int nxh, int ny, int ntiles,
                                              const typename cvec<T>::type* __restrict__ tw) {
  using C = typename cvec<T>::type;
  using Idx = PitchIdx<NZ>;
  constexpr int YT = ztile_for<T>(NZ);
  constexpr int PT = (YT * NZ + NT - 1) / NT;  // values per thread and tile
  __shared__ C buf[YT * pitch_for(NZ)];
  __shared__ double red[NT / 64];
  if (!sym.begin()) return;
  const int nty = (ny + YT - 1) / YT;
  const int tid = threadIdx.x;
  static_assert(ZPT == 1 || ZPT == 2, "one or two z tiles per block");
  if constexpr (ZPT == 1) {
    // one tile per block, loaded straight into LDS
    const int t = blockIdx.x % nty, ckx = blockIdx.x / nty;
    const int kx = ckx % nxh, ky0 = t * YT;
    C* base = spec + (long long)ckx * NZ * ny;
    for (int idx = tid; idx < YT * NZ; idx += NT) {
      const int z = idx / YT, l = idx - z * YT;
      buf[Idx::at(l, z)] = ky0 + l < ny ? base[(long long)z * ny + ky0 + l] : C{(T)0, (T)0};
    }
    __syncthreads();
    if (FWD) fft_lds<T, NZ, YT, NT, false, Idx>(buf, tw);
    double acc1 = 0.0;
    for (int idx = tid; idx < YT * NZ; idx += NT) {
      const int l = idx / NZ, kz = idx - l * NZ;
      if (ky0 + l < ny) {
        C& a = buf[Idx::at(l, kz)];
        a = sym.mode(kx, ky0 + l, kz, a, acc1);
      }
    }
    __syncthreads();
    sym.partial(block_sum(acc1, red));
    if (INV) fft_lds<T, NZ, YT, NT, true, Idx>(buf, tw);
    for (int idx = tid; idx < YT * NZ; idx += NT) {
      const int z = idx / YT, l = idx - z * YT;
      if (ky0 + l < ny) base[(long long)z * ny + ky0 + l] = buf[Idx::at(l, z)];
    }
    return;
  }
  const int e0 = blockIdx.x * ZPT, e1 = min(e0 + ZPT, ntiles);
  C pre[PT];
  auto load = [&](int e) {
    const int t = e % nty, ckx = e / nty, ky0 = t * YT;
    const C* base = spec + (long long)ckx * NZ * ny;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int idx = tid + u * NT;
      const int z = idx / YT, l = idx - z * YT;
      pre[u] = (idx < YT * NZ && ky0 + l < ny) ? base[(long long)z * ny + ky0 + l] : C{(T)0, (T)0};
    }
  };
  double acc = 0.0;
  load(e0);
  for (int e = e0; e < e1; ++e) {
    const int t = e % nty, ckx = e / nty;
    const int kx = ckx % nxh, ky0 = t * YT;
    C* base = spec + (long long)ckx * NZ * ny;  // the [z][y] plane of (component, kx)
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int idx = tid + u * NT;
      if (idx < YT * NZ) {
        const int z = idx / YT, l = idx - z * YT;
        buf[Idx::at(l, z)] = pre[u];
      }
    }
    if (e + 1 < e1) load(e + 1);
    __syncthreads();
    if (FWD) fft_lds<T, NZ, YT, NT, false, Idx>(buf, tw);
    for (int idx = tid; idx < YT * NZ; idx += NT) {
      const int l = idx / NZ, kz = idx - l * NZ;
      if (ky0 + l < ny) {
        C& a = buf[Idx::at(l, kz)];
        a = sym.mode(kx, ky0 + l, kz, a, acc);
      }
    }
    __syncthreads();
    if (INV) fft_lds<T, NZ, YT, NT, true, Idx>(buf, tw);
    for (int idx = tid; idx < YT * NZ; idx += NT) {
      const int z = idx / YT, l = idx - z * YT;
      if (ky0 + l < ny) base[(long long)z * ny + ky0 + l] = buf[Idx::at(l, z)];
    }
    __syncthreads();
  }
  sym.partial(block_sum(acc, red));
}

// Green operator of the unit reference medium on a 3D grid,
// z_hat = r_hat / (N |D(k)|^2) (0 at k = 0), with the Parseval partial sum of
// r.z over the half spectrum (weight 2 except on the kx = 0 and Nyquist planes).
template <typename T> struct Green3 {
  const double2* Dx;
  const double2* Dy;
  const double2* Dz;
  double inv_n;
  int nx;
  const CgState* st;  // nullable
  double* part;       // nullable; one partial per block
  __device__ bool begin() const { return st == nullptr || cg_running(st, 0); }
  template <typename C> __device__ C mode(int kx, int ky, int kz, C a, double& acc) const {
    const double2 d1 = Dx[kx], d2 = Dy[ky], d3 = Dz[kz];
    const double n2 = d1.x * d1.x + d1.y * d1.y + d2.x * d2.x + d2.y * d2.y + d3.x * d3.x + d3.y * d3.y;
    if (n2 == 0.0) return C{(T)0, (T)0};
    const double f = inv_n / n2;
    const double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
    acc += w * f * ((double)a.x * a.x + (double)a.y * a.y);
    const T ft = (T)f;
    return C{a.x * ft, a.y * ft};
  }
  __device__ void partial(double v) const {
    if (part && threadIdx.x == 0) part[blockIdx.x] = v;
  }
};

// Identity symbol that skips the pass once the CG solve has ended (st
// nullable: never skip).
struct StateSym {
  const CgState* st;
  __device__ bool begin() const { return st == nullptr || cg_running(st, 0); }
  template <typename C> __device__ C mode(int, int, int, C a, double&) const { return a; }
  __device__ void partial(double) const {}
};

// Green operator of an isotropic reference medium (lam0, mu0) on the 3D half
// spectrum [comp][kx][z][y] of the three displacement components: per mode
// the Hermitian positive definite system
//     K0(k) z_hat = r_hat,  K0 = mu0 |D|^2 I + lam0 conj(D) D^T + mu0 D D^H
// (zero at k = 0), solved by a 3 x 3 Cholesky factorisation in FP64, with
// the 1/N of the inverse transform folded in and the Parseval partial sum of
// r.z (weight 2 except on the kx = 0 and Nyquist planes), one per block.
struct Cd {
  double x, y;
};
__device__ __forceinline__ Cd cd_mul(Cd a, Cd b) { return Cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ Cd cd_conj_mul(Cd a, Cd b) { return Cd{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }

template <typename T>
__global__ void __launch_bounds__(NT) k_ref3(const CgState* st, typename cvec<T>::type* spec,
                                             const double2* __restrict__ Dx, const double2* __restrict__ Dy,
                                             const double2* __restrict__ Dz, double lam0, double mu0, double inv_n,
                                             int nxh, int ny, int nz, int nx, double* part) {
  using C = typename cvec<T>::type;
  __shared__ double red[NT / 64];
  if (st && !cg_running(st, 0)) return;
  const long long per = (long long)nxh * nz * ny;
  double acc = 0.0;
  for (long long o = blockIdx.x * (long long)NT + threadIdx.x; o < per; o += (long long)gridDim.x * NT) {
    const int y = (int)(o % ny);
    const long long rz = o / ny;
    const int z = (int)(rz % nz), kx = (int)(rz / nz);
    const double2 d1 = Dx[kx], d2 = Dy[y], d3 = Dz[z];
    const Cd D[3] = {{d1.x, d1.y}, {d2.x, d2.y}, {d3.x, d3.y}};
    const double n2 = D[0].x * D[0].x + D[0].y * D[0].y + D[1].x * D[1].x + D[1].y * D[1].y + D[2].x * D[2].x +
                      D[2].y * D[2].y;
    C* v[3] = {spec + o, spec + per + o, spec + 2 * per + o};
    if (n2 == 0.0) {
      for (int a = 0; a < 3; ++a) *v[a] = C{(T)0, (T)0};
      continue;
    }
    // A_ij = mu0 n2 d_ij + lam0 conj(D_i) D_j + mu0 D_i conj(D_j), lower triangle
    Cd A[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j <= i; ++j) {
        const Cd a = cd_conj_mul(D[i], D[j]);  // conj(D_i) D_j
        // D_i conj(D_j) = conj(conj(D_i) D_j)
        A[i][j] = Cd{(lam0 + mu0) * a.x + (i == j ? mu0 * n2 : 0.0), (lam0 - mu0) * a.y};
      }
    // Cholesky A = L L^H (real positive diagonal)
    const double l11 = sqrt(A[0][0].x);
    const Cd l21{A[1][0].x / l11, A[1][0].y / l11}, l31{A[2][0].x / l11, A[2][0].y / l11};
    const double l22 = sqrt(A[1][1].x - (l21.x * l21.x + l21.y * l21.y));
    const Cd t32 = cd_mul(l31, Cd{l21.x, -l21.y});  // l31 conj(l21)
    const Cd l32{(A[2][1].x - t32.x) / l22, (A[2][1].y - t32.y) / l22};
    const double l33 = sqrt(A[2][2].x - (l31.x * l31.x + l31.y * l31.y) - (l32.x * l32.x + l32.y * l32.y));
    const Cd r[3] = {{(double)v[0]->x, (double)v[0]->y}, {(double)v[1]->x, (double)v[1]->y},
                     {(double)v[2]->x, (double)v[2]->y}};
    // L w = r
    const Cd w1{r[0].x / l11, r[0].y / l11};
    const Cd u2 = cd_mul(l21, w1);
    const Cd w2{(r[1].x - u2.x) / l22, (r[1].y - u2.y) / l22};
    const Cd u31 = cd_mul(l31, w1), u32 = cd_mul(l32, w2);
    const Cd w3{(r[2].x - u31.x - u32.x) / l33, (r[2].y - u31.y - u32.y) / l33};
    // L^H z = w
    const Cd z3{w3.x / l33, w3.y / l33};
    const Cd e32 = cd_conj_mul(l32, z3);  // conj(l32) z3
    const Cd z2{(w2.x - e32.x) / l22, (w2.y - e32.y) / l22};
    const Cd e21 = cd_conj_mul(l21, z2), e31 = cd_conj_mul(l31, z3);
    const Cd z1{(w1.x - e21.x - e31.x) / l11, (w1.y - e21.y - e31.y) / l11};
    const Cd zz[3] = {z1, z2, z3};
    const double wgt = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
    for (int a = 0; a < 3; ++a) {
      const double zx = zz[a].x * inv_n, zy = zz[a].y * inv_n;
      acc += wgt * (r[a].x * zx + r[a].y * zy);
      *v[a] = C{(T)zx, (T)zy};
    }
  }
  const double t = block_sum(acc, red);
  if (part && threadIdx.x == 0) part[blockIdx.x] = t;
}

// Identity symbol (the debug transforms).
struct NoSym {
  __device__ bool begin() const { return true; }
  template <typename C> __device__ C mode(int, int, int, C a, double&) const { return a; }
  __device__ void partial(double) const {}
};

}  // namespace fgcg
