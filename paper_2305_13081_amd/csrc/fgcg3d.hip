// 3D grids: workspace, the y/z transform passes, the mechanics PCG in
// displacement form (FP64 and FP32-mixed with reliable updates), the 3D
// history update and the transform test hook.  The phase-field and diffusion
// solves use the stencil CG of the 2D engine, which handles both.
#include "engine.hpp"
#include "mech3.hpp"
#include "launch3d.hpp"

#include <array>
#include <map>
#include <mutex>
#include <tuple>

namespace fgcg {

namespace {

template <typename T> Field<T> fld3(void* p, const fgcg_ctx* c) { return Field<T>{(T*)p, c->n, 3 * c->n}; }

// z = M r (the Green operator by x, y, z transforms), r.z reduced into red[1].
// spectrum stride of one displacement component
inline long long comp_stride3(const fgcg_ctx* c) { return (long long)c->nxh * c->rows; }

// NOUT = 3: pro covers the three components in one block; NOUT = 1: pro is
// a one-component functor, launched over the three components.
template <typename T, int NOUT, class Pro>
int green3(fgcg_ctx* c, const Pro& pro, const CgState* st, bool timed) {
  CT<T>* spec = (CT<T>*)c->spec;
  int r = NOUT == 3 ? launch_row_fwd<T, NOUT>(c, timed ? FGCG_K_MECH_ROW_FWD : -1, pro, spec)
                    : launch_row_fwd<T, NOUT>(c, timed ? FGCG_K_MECH_ROW_FWD : -1, pro, spec, 3, comp_stride3(c));
  r |= launch_ypass<T, 3>(c, timed ? FGCG_K_MECH_Y_FWD : -1, false, st, spec);
  if (c->precond == 1) {
    // forward z transforms, the reference-medium solve mode by mode, inverse z
    const StateSym ss{st};
    r |= launch_zpass<T, true, false>(c, timed ? FGCG_K_MECH_COL : -1, ss, spec, 3);
    const long long per = comp_stride3(c);
    const int nref = (int)std::min<long long>((per + NT - 1) / NT, c->nzb);
    r |= launch(c, -1, (const void*)&k_ref3<T>, dim3(nref), st, spec, (const double2*)c->Dx, (const double2*)c->Dy,
                (const double2*)c->Dz, c->use_lam, c->use_mu, 1.0 / (double)c->n, c->nxh, c->ny, c->nz, c->nx,
                c->part_z);
    r |= launch_reduce(c, c->part_z, nref, c->red + 1);
    r |= launch_zpass<T, false, true>(c, -1, ss, spec, 3);
  } else {
    const Green3<T> g{c->Dx, c->Dy, c->Dz, 1.0 / (double)c->n, c->nx, st, c->part_z};
    r |= launch_zpass<T, true, true>(c, timed ? FGCG_K_MECH_COL : -1, g, spec, 3);
    r |= launch_reduce(c, c->part_z, zblocks<T>(c, 3), c->red + 1);
  }
  r |= launch_ypass<T, 3>(c, timed ? FGCG_K_MECH_Y_INV : -1, true, st, spec);
  return r;
}

template <typename T> int mech3_init(fgcg_ctx* c, double tol, int maxit) {
  const CopyProN<T, 3> cp{fld3<T>(c->r, c), c->nx};
  int r = green3<T, 3>(c, cp, nullptr, false);
  const MechUEpi<T, 3> e0{fld3<T>(c->p, c), c->nx, c->st, c->red + 1, 1, 1, tol, maxit};
  r |= launch_row_inv<T, 3>(c, -1, e0, (const CT<T>*)c->spec);
  HIPCHK(hipGetLastError());
  return r;
}

// Row passes with one displacement component per block (launched over the
// three components) or all three in one block, as the context's split3 says
// (tuned on large grids; the default per precision as measured at 256^3:
// FP64 inverse pass 277 -> 253 us split, forward pass 556 -> 611 us split;
// FP32 forward pass 304 -> 284 us split, inverse pass 129 -> 133 us split).
inline int split_bits(const fgcg_ctx* c) { return c->split3 ? c->split3 - 1 : (c->prec == FGCG_FP64 ? 2 : 1); }

template <typename T> int mech3_iter(fgcg_ctx* c, const MechMat& m, double tol, int maxit, bool reliable) {
  const int sp = split_bits(c);
  const bool split_fwd = (sp & 1) != 0, split_inv = (sp & 2) != 0;
  const Field<T> X = fld3<T>(c->x, c), R = fld3<T>(c->r, c), P = fld3<T>(c->p, c), Q = fld3<T>(c->tmp, c);
  const Grid3 g = grid3(c);
  const int nb = nslab(c);
  const int nkp = std::min(kp3_chunks(c->nx, c->ny, c->nz), KP3_MAX_BLOCKS);
  set_kname(c, FGCG_K_MECH_KP, "k_mech3_kpx<%s%.0d", tname<T>(), 0);
  int r = launch(c, FGCG_K_MECH_KP, (const void*)&k_mech3_kpx<T, T, false>, dim3(nkp), m, (const T*)P.p, Q.p,
                 (const double*)nullptr, g, (T)(1.0 / c->h), c->st, c->part_a);
  r |= launch_reduce(c, c->part_a, nkp, c->red);
  if (!reliable) {
    if (split_fwd) {
      const MechUProC<T, 3> pro{{X, R, P, Q, c->nx, c->st, c->red, 1}};
      r |= green3<T, 1>(c, pro, c->st, true);
    } else {
      const MechUPro<T, 3> pro{X, R, P, Q, c->nx, c->st, c->red, 1};
      r |= green3<T, 3>(c, pro, c->st, true);
    }
  } else {
    r |= launch(c, -1, (const void*)&k_mech_fold<T>, dim3(c->npost), X.p, c->xh, (const T*)P.p, 3 * c->n, c->st,
                (const double*)c->red, 1);
    r |= launch(c, -1, (const void*)&k_mech3_kpx<T, double, true>, dim3(nkp), m, (const double*)c->xh, R.p,
                (const double*)c->fh, g, 1.0 / c->h, c->st, (double*)nullptr);
    const CopyProN<T, 3> cp{R, c->nx};
    r |= green3<T, 3>(c, cp, c->st, false);
  }
  if (split_inv) {
    const MechUEpiC<T, 3> epi{{P, c->nx, c->st, c->red + 1, 1, 0, tol, maxit}};
    r |= launch_row_inv<T, 1>(c, FGCG_K_MECH_ROW_INV, epi, (const CT<T>*)c->spec, 3, comp_stride3(c));
  } else {
    const MechUEpi<T, 3> epi{P, c->nx, c->st, c->red + 1, 1, 0, tol, maxit};
    r |= launch_row_inv<T, 3>(c, FGCG_K_MECH_ROW_INV, epi, (const CT<T>*)c->spec);
  }
  return r;
}

struct Mech3IterFn {
  fgcg_ctx* c;
  MechMat m;
  double tol;
  int maxit;
  int j = 0;
  int operator()() {
    if (c->prec == FGCG_FP64) return mech3_iter<double>(c, m, tol, maxit, false);
    const bool rel = j == RELIABLE_EVERY3 - 1;
    j = rel ? 0 : j + 1;
    return mech3_iter<float>(c, m, tol, maxit, rel);
  }
};

// Autotuning of the 3D mechanics passes, before the first solve of a grid of
// at least 2^18 voxels: the forward and the inverse row pass each with one
// displacement component per block or all three (timed separately; the
// choice never changes results), and one or two z tiles per block in the
// Green z pass (a different block count orders the r.z partial sums
// differently, so the other choice must win by more than 3 %).  Each
// candidate is timed over 3 + 10 back-to-back launches between HIP events on
// the context's own workspace: zero fields and spectra, a running CG state
// and unit scalars (so every launch does its full work).  Smaller grids take
// the defaults.  Picks are kept per process, keyed by the device, the grid,
// the precision, the preconditioner and the values fixed through the options.
template <typename T> int timing3(fgcg_ctx* c) {
  int rc = running_state(c);
  if (rc) return rc;
  const size_t nv = sizeof(T) * 3 * (size_t)c->n;
  for (void* b : {c->x, c->r, c->p, c->tmp}) HIPCHK(hipMemsetAsync(b, 0, nv, c->stream));
  HIPCHK(hipMemsetAsync(c->spec, 0, sizeof(CT<T>) * 3 * (size_t)c->nxh * c->rows, c->stream));
  const double ones[8] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
  HIPCHK(hipMemcpyAsync(c->red, ones, sizeof ones, hipMemcpyHostToDevice, c->stream));
  // the host array is read by the copy: wait before it goes out of scope
  HIPCHK(hipStreamSynchronize(c->stream));
  return 0;
}

template <typename T> int tune3_t(fgcg_ctx* c) {
  int rc = timing3<T>(c);
  if (rc) return rc;
  const Field<T> X = fld3<T>(c->x, c), R = fld3<T>(c->r, c), P = fld3<T>(c->p, c), Q = fld3<T>(c->tmp, c);
  CT<T>* spec = (CT<T>*)c->spec;
  const long long cs = comp_stride3(c);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(FGCG_EHIP, "hipEventCreate");
  auto time_it = [&](auto&& f) -> float {
    for (int rep = 0; rep < 13 && !rc; ++rep) {
      if (rep == 3 && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(FGCG_EHIP, "hipEventRecord");
      rc |= f();
    }
    float ms = 0.f;
    if (!rc && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = fail(FGCG_EHIP, "timing a 3D pass candidate failed");
    return ms;
  };
  int split = c->split3 ? c->split3 - 1 : -1;
  if (split < 0 && !rc) {
    const MechUPro<T, 3> pw{X, R, P, Q, c->nx, c->st, c->red, 1};
    const MechUProC<T, 3> pc{{X, R, P, Q, c->nx, c->st, c->red, 1}};
    const MechUEpi<T, 3> ew{P, c->nx, c->st, c->red + 1, 1, 0, 0.0, 1 << 30};
    const MechUEpiC<T, 3> ec{{P, c->nx, c->st, c->red + 1, 1, 0, 0.0, 1 << 30}};
    const float fw = time_it([&] { return launch_row_fwd<T, 3>(c, -1, pw, spec); });
    const float fs = time_it([&] { return launch_row_fwd<T, 1>(c, -1, pc, spec, 3, cs); });
    const float iw = time_it([&] { return launch_row_inv<T, 3>(c, -1, ew, (const CT<T>*)spec); });
    const float is = time_it([&] { return launch_row_inv<T, 1>(c, -1, ec, (const CT<T>*)spec, 3, cs); });
    split = (fs < fw ? 1 : 0) | (is < iw ? 2 : 0);
  }
  int zpt = c->zpt_pick;
  if (!zpt && !rc) {
    const Green3<T> g{c->Dx, c->Dy, c->Dz, 1.0 / (double)c->n, c->nx, c->st, c->part_z};
    float tz[3] = {0.f, 0.f, 0.f};
    for (int z = 1; z <= 2 && !rc; ++z) {
      c->zpt_pick = z;
      tz[z] = time_it([&] { return launch_zpass<T, true, true>(c, -1, g, spec, 3); });
    }
    constexpr float MARGIN = 0.97f;
    const int def = zpt_for<T>(), alt = 3 - def;
    zpt = tz[alt] < MARGIN * tz[def] ? alt : def;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  HIPCHK(hipGetLastError());
  if (rc) return rc;
  c->split3 = 1 + split;
  c->zpt_pick = zpt;
  return 0;
}

struct Tune3Key {
  int dev, nx, ny, nz, prec, precond, split, zpt;
  bool operator<(const Tune3Key& o) const {
    return std::tie(dev, nx, ny, nz, prec, precond, split, zpt) <
           std::tie(o.dev, o.nx, o.ny, o.nz, o.prec, o.precond, o.split, o.zpt);
  }
};
std::mutex tune3_mu;
std::map<Tune3Key, std::array<int, 2>> tune3_cache;

// Overwrites the workspace and the CG state: runs before a solve forms its
// right-hand side.
int tune3(fgcg_ctx* c) {
  if (c->split3 && c->zpt_pick) return 0;
  const bool f64 = c->prec == FGCG_FP64;
  if (c->n < (1LL << 18)) {
    if (!c->split3) c->split3 = 1 + split_bits(c);
    if (!c->zpt_pick) c->zpt_pick = f64 ? zpt_for<double>() : zpt_for<float>();
    return 0;
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const Tune3Key key{dev, c->nx, c->ny, c->nz, c->prec, c->precond, c->split3, c->zpt_pick};
  {
    std::lock_guard<std::mutex> g(tune3_mu);
    auto it = tune3_cache.find(key);
    if (it != tune3_cache.end()) {
      c->split3 = it->second[0];
      c->zpt_pick = it->second[1];
      return 0;
    }
  }
  const int rc = f64 ? tune3_t<double>(c) : tune3_t<float>(c);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(tune3_mu);
  tune3_cache[key] = {c->split3, c->zpt_pick};
  return 0;
}

}  // namespace

bool size3_supported(int n) {
  return with_n3(n, [](auto) {});
}

int alloc3d(fgcg_ctx* c) {
  auto tw = [&](int n, bool f32, void** out) -> int {
    if (f32) {
      std::vector<float2> t(n);
      for (int k = 0; k < n; ++k) {
        const double th = 2.0 * M_PI * (double)k / (double)n;
        t[k] = float2{(float)std::cos(th), (float)-std::sin(th)};
      }
      HIPCHK(hipMalloc(out, sizeof(float2) * n));
      HIPCHK(hipMemcpy(*out, t.data(), sizeof(float2) * n, hipMemcpyHostToDevice));
    } else {
      std::vector<double2> t(n);
      for (int k = 0; k < n; ++k) {
        const double th = 2.0 * M_PI * (double)k / (double)n;
        t[k] = double2{std::cos(th), -std::sin(th)};
      }
      HIPCHK(hipMalloc(out, sizeof(double2) * n));
      HIPCHK(hipMemcpy(*out, t.data(), sizeof(double2) * n, hipMemcpyHostToDevice));
    }
    return 0;
  };
  int rc;
  if ((rc = tw(c->nz, false, &c->twz))) return rc;
  if (c->prec == FGCG_FP32_MIXED && (rc = tw(c->nz, true, &c->twz32))) return rc;
  std::vector<double2> dz(c->nz);
  for (int k = 0; k < c->nz; ++k) {
    const double th = 2.0 * M_PI * k / c->nz, sh = std::sin(0.5 * th);
    dz[k] = double2{-2.0 * sh * sh / c->h, std::sin(th) / c->h};
  }
  HIPCHK(hipMalloc(&c->Dz, sizeof(double2) * c->nz));
  HIPCHK(hipMemcpy(c->Dz, dz.data(), sizeof(double2) * c->nz, hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&c->red, sizeof(double) * 8));
  HIPCHK(hipMemset(c->red, 0, sizeof(double) * 8));
  // partial sums of the z passes: the most blocks any of them launches (one
  // tile per block, three components, either precision's tile width)
  c->nzb = std::max(zblocks<double>(c, 3, 1), zblocks<float>(c, 3, 1));
  HIPCHK(hipMalloc(&c->part_z, sizeof(double) * c->nzb));
  c->nslab = nslab(c);
  return 0;
}

int mech3_solve(fgcg_ctx* c, const MechMat& m, const double* eig, const double* em, double tol, int maxit,
                double* strain, double* stress, double* mean_stress, double* energy, fgcg_info* info) {
  const double t0 = now();
  resolve_reference(c, m);
  int rc = tune3(c);
  if (rc) return rc;
  const Grid3 g = grid3(c);
  const int nb = nslab(c);
  Em6 e6;
  for (int j = 0; j < 6; ++j) e6.v[j] = em[j];
  // right-hand side f = -grad^H g C : (eps_mac - e I), x = 0
  if (c->prec == FGCG_FP64) {
    hipLaunchKernelGGL((k_mech3_rhs<double>), dim3(nb), dim3(NT), 0, c->stream, m, eig, e6, (double*)c->r,
                       (double*)c->x, g, 1.0 / c->h);
  } else {
    hipLaunchKernelGGL((k_mech3_rhs<double>), dim3(nb), dim3(NT), 0, c->stream, m, eig, e6, c->fh, c->xh, g,
                       1.0 / c->h);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(c->npost), dim3(PT), 0, c->stream, (float*)c->r,
                       (const double*)c->fh, 3 * c->n);
    HIPCHK(hipMemsetAsync(c->x, 0, sizeof(float) * 3 * c->n, c->stream));
  }
  HIPCHK(hipGetLastError());
  rc = c->prec == FGCG_FP64 ? mech3_init<double>(c, tol, maxit) : mech3_init<float>(c, tol, maxit);
  if (rc) return rc;
  Mech3IterFn it{c, m, tol, maxit};
  const int K = c->prec == FGCG_FP64 ? c->chunk : 2 * RELIABLE_EVERY3;
  Key key;
  key.add(m.phase).add(m.d).add(m.Efield).add(m.lm_dev).add(m.kappa).add(m.lam_per_E).add(m.mu_per_E).add(m.lm).add(c->prec);
  key.add(c->precond).add(c->use_lam).add(c->use_mu);
  key.add(tol).add(maxit);
  if ((rc = run_cg(c, c->prec == FGCG_FP64 ? 0 : 5, key, c->st, c->h_st, it, maxit, K))) return rc;
  const CgState s = *c->h_st;
  const double* u = (const double*)c->x;
  if (c->prec != FGCG_FP64) {
    hipLaunchKernelGGL((k_fold_final<float>), dim3(c->npost), dim3(PT), 0, c->stream, (const float*)c->x, c->xh,
                       3 * c->n);
    u = c->xh;
  }
  hipLaunchKernelGGL(k_mech3_post, dim3(nb), dim3(NT), 0, c->stream, m, u, g, 1.0 / c->h, eig, e6, strain, stress,
                     c->part_post);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_part, c->part_post, sizeof(double) * 7 * nb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < nb; ++b)
    for (int j = 0; j < 7; ++j) acc[j] += c->h_part[7 * b + j];
  if (mean_stress)
    for (int j = 0; j < 6; ++j) mean_stress[j] = acc[j] / (double)c->n;
  if (energy) *energy = 0.5 * c->h * c->h * c->h * acc[6];
  fill_info(info, s, now() - t0);
  return status_of(s);
}

// Kernel-level hook on 3D grids: q = K p through the tiled stiffness pass of
// the solver (k_mech3_kpx) or z = M r through the Green passes every solve
// starts with (x rows, y lines, z tiles with the Green symbol, y lines, x
// rows writing p = z), in the context's precision.
template <typename T> int debug_apply3_t(fgcg_ctx* c, int op, const MechMat& m, const double* in, double* out) {
  const long long n3 = 3 * c->n;
  int rc;
  resolve_reference(c, m);
  if (op == FGCG_OP_MECH_K) {
    if ((rc = running_state(c))) return rc;
    const int nkp = std::min(kp3_chunks(c->nx, c->ny, c->nz), KP3_MAX_BLOCKS);
    hipLaunchKernelGGL((k_convert<T, double>), dim3(c->npost), dim3(PT), 0, c->stream, (T*)c->p, in, n3);
    hipLaunchKernelGGL((k_mech3_kpx<T, T, false>), dim3(nkp), dim3(NT), 0, c->stream, m, (const T*)c->p, (T*)c->tmp,
                       (const double*)nullptr, grid3(c), (T)(1.0 / c->h), c->st, c->part_a);
    hipLaunchKernelGGL((k_convert<double, T>), dim3(c->npost), dim3(PT), 0, c->stream, out, (const T*)c->tmp, n3);
    HIPCHK(hipGetLastError());
    return 0;
  }
  if ((rc = tune3(c))) return rc;  // (overwrites the workspace)
  hipLaunchKernelGGL((k_convert<T, double>), dim3(c->npost), dim3(PT), 0, c->stream, (T*)c->r, in, n3);
  HIPCHK(hipMemsetAsync(c->p, 0, sizeof(T) * n3, c->stream));  // z = 0 stays if r = 0
  if ((rc = mech3_init<T>(c, 0.0, 1))) return rc;
  hipLaunchKernelGGL((k_convert<double, T>), dim3(c->npost), dim3(PT), 0, c->stream, out, (const T*)c->p, n3);
  HIPCHK(hipGetLastError());
  return 0;
}

int debug_apply3(fgcg_ctx* c, int op, const MechMat& m, const double* in, double* out) {
  return c->prec == FGCG_FP64 ? debug_apply3_t<double>(c, op, m, in, out) : debug_apply3_t<float>(c, op, m, in, out);
}

int history3(fgcg_ctx* c, const MechMat& m0, const double* strain, const double* e, double* H) {
  hipLaunchKernelGGL(k_history3, dim3(c->npost), dim3(NT), 0, c->stream, m0, strain, e, H, c->n);
  HIPCHK(hipGetLastError());
  return 0;
}

// Real-input transform of one field, FP64, through the passes the solvers use.
// dir > 0: in real [N] -> out half spectrum [nz][ny][nx/2+1] (complex,
// unnormalised); dir < 0: the inverse with the 1/N factor.
int debug_fft(fgcg_ctx* c, int dir, const double* in, double* out) {
  CT<double>* spec = (CT<double>*)c->spec;
  const long long nh = (long long)c->nxh * c->ny * c->nz;
  const int nb = (int)std::min<long long>((nh + NT - 1) / NT, 4096);
  int rc = 0;
  bool ok = true;
  auto ypass = [&](bool inv) {
    const int nlines = c->nxh * c->nz;
    ok &= with_n(c->ny, [&](auto NYc) {
      constexpr int NY = decltype(NYc)::value;
      constexpr int LPB = ylines_for(NY, 1);
      const dim3 g((nlines + LPB - 1) / LPB);
      if (inv)
        rc |= launch(c, -1, (const void*)&k_ypass<double, NY, 1, true>, g, (const CgState*)nullptr, spec, nlines,
                     tw_y<double>(c));
      else
        rc |= launch(c, -1, (const void*)&k_ypass<double, NY, 1, false>, g, (const CgState*)nullptr, spec, nlines,
                     tw_y<double>(c));
    });
  };
  if (dir > 0) {
    const CopyProN<double, 1> cp{Field<double>{(double*)in, c->n, 0}, c->nx};
    rc |= launch_row_fwd<double, 1>(c, -1, cp, spec);
    ypass(false);
    if (c->ndim == 3) rc |= launch_zpass<double, true, false>(c, -1, NoSym{}, spec, 1);
    hipLaunchKernelGGL(k_spec_out, dim3(nb), dim3(NT), 0, c->stream, (const double2*)spec, (double2*)out, c->nxh,
                       c->ny, c->nz);
  } else {
    hipLaunchKernelGGL(k_spec_in, dim3(nb), dim3(NT), 0, c->stream, (const double2*)in, (double2*)spec, c->nxh,
                       c->ny, c->nz);
    if (c->ndim == 3) rc |= launch_zpass<double, false, true>(c, -1, NoSym{}, spec, 1);
    ypass(true);
    const StoreEpi<double, 1> st{Field<double>{out, c->n, 0}, Field<double>{nullptr, c->n, 0},
                                 1.0 / (double)c->n, c->nx, nullptr, 0};
    rc |= launch_row_inv<double, 1>(c, -1, st, spec);
  }
  if (!ok) return fail(FGCG_EUNSUPPORTED, "axis length without a transform kernel");
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return rc;
}

}  // namespace fgcg
