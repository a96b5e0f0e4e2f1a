// Launch helpers of the 3D transform passes, shared by the translation units
// that run CG on 3D grids (mechanics, diffusion homogenisation).
#pragma once
#include "engine.hpp"
#include "mech3.hpp"
#include "passes3d.hpp"

namespace fgcg {

// Axis lengths of 3D grids.
#define FGCG_SIZES3(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

template <class F> bool with_n3(int n, F&& f) {
  switch (n) {
#define FGCG_CASE3(N)                      \
  case N:                                  \
    f(std::integral_constant<int, N>{});   \
    return true;
    FGCG_SIZES3(FGCG_CASE3)
#undef FGCG_CASE3
    default:
      return false;
  }
}

inline constexpr int RELIABLE_EVERY3 = 10;  // FP32-mixed: true residual every tenth iteration
inline constexpr int KP3_MAX_BLOCKS = 4096;  // blocks of the tiled stiffness pass (partial sums in part_a)

template <typename T> inline const CT<T>* tw_z(const fgcg_ctx* c) {
  return (const CT<T>*)(std::is_same<T, double>::value ? c->twz : c->twz32);
}

inline Grid3 grid3(const fgcg_ctx* c) { return Grid3{c->nx, c->ny, c->nz, c->n}; }

// Blocks of the slab-walking stencil kernels: a multiple of 8, at most 1024.
inline int nslab(const fgcg_ctx* c) {
  const int rows = c->ny * c->nz;
  return std::max(8, std::min(1024, rows) & ~7);
}

template <typename T> inline int ztiles(const fgcg_ctx* c) {
  int nty = 0;
  with_n3(c->nz, [&](auto NZc) {
    constexpr int YT = ztile_for<T>(decltype(NZc)::value);
    nty = (c->ny + YT - 1) / YT;
  });
  return nty;
}

template <typename T, int NC>
int launch_ypass(fgcg_ctx* c, int kind, bool inv, const CgState* st, CT<T>* spec) {
  int rc = 0;
  const int nlines = c->nxh * c->nz;
  with_n3(c->ny, [&](auto NYc) {
    constexpr int NY = decltype(NYc)::value;
    constexpr int LPB = ylines_for(NY, NC);
    dim3 g((nlines + LPB - 1) / LPB);
    if (kind >= 0) set_kname(c, kind, inv ? "k_ypass<%s, %d, 3, true" : "k_ypass<%s, %d, 3, false", tname<T>(), NY);
    if (inv)
      rc = launch(c, kind, (const void*)&k_ypass<T, NY, NC, true>, g, st, spec, nlines, tw_y<T>(c));
    else
      rc = launch(c, kind, (const void*)&k_ypass<T, NY, NC, false>, g, st, spec, nlines, tw_y<T>(c));
  });
  return rc;
}

// z tiles per block of the context's z passes: the tuned or fixed choice,
// else zpt_for<T>().
template <typename T> inline int zpt_of(const fgcg_ctx* c) { return c->zpt_pick ? c->zpt_pick : zpt_for<T>(); }

// Blocks of the z pass over ncomp components (zpt tiles per block; by
// default the context's).
template <typename T> inline int zblocks(const fgcg_ctx* c, int ncomp, int zpt = 0) {
  const int z = zpt ? zpt : zpt_of<T>(c);
  return (ncomp * c->nxh * ztiles<T>(c) + z - 1) / z;
}

template <typename T, bool FWD, bool INV, class Sym>
int launch_zpass(fgcg_ctx* c, int kind, const Sym& sym, CT<T>* spec, int ncomp) {
  int rc = 0;
  const int ntiles = ncomp * c->nxh * ztiles<T>(c);
  const int zpt = zpt_of<T>(c);
  with_n3(c->nz, [&](auto NZc) {
    constexpr int NZ = decltype(NZc)::value;
    dim3 g(zblocks<T>(c, ncomp));
    if (kind >= 0) set_kname(c, kind, "k_zpass<%s, %d", tname<T>(), NZ);
    const void* fn = zpt == 1 ? (const void*)&k_zpass<T, NZ, FWD, INV, Sym, 1>
                              : (const void*)&k_zpass<T, NZ, FWD, INV, Sym, 2>;
    rc = launch(c, kind, fn, g, sym, spec, c->nxh, c->ny, ntiles, tw_z<T>(c));
  });
  return rc;
}

inline int launch_reduce(fgcg_ctx* c, const double* part, int np, double* out) {
  return launch(c, -1, (const void*)&k_reduce, dim3(1), part, np, out);
}

}  // namespace fgcg
