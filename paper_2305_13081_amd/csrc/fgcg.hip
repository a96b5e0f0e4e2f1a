// Entry points of the fgcg C ABI declared in include/fgcg.h and the 2D
// solvers (3D grids are handled in fgcg3d.hip).
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>

#include "adjoint.hpp"
#include "engine.hpp"
#include "sr2d.hpp"
#include "strain_form.hpp"

using namespace fgcg;

namespace {

// ---------------------------------------------------------- mechanics
// Every context holds nsamp samples of one grid size (1 outside a batch);
// sample s of a 2-component field starts at s * 2n, of a spectrum at
// s * 2 nxh ny, and kernels take the sample, or for the one-component passes
// the (sample, component) pair, from blockIdx.y.
constexpr int RELIABLE_EVERY = 10;  // FP32-mixed: true residual every tenth iteration

template <typename T> Field<T> fld(void* p, const fgcg_ctx* c) { return Field<T>{(T*)p, c->n, 2 * c->n}; }
inline long long spec_ss(const fgcg_ctx* c) { return 2LL * c->nxh * c->ny; }

// The 2D inverse row pass of the mechanics (one component per block): the
// p prefetch goes before the CG-state check for a single sample, after it in
// batches (blocks of converged samples then read nothing).
template <typename T>
int launch_mech_row_inv(fgcg_ctx* c, int kind, const MechUEpi<T, 2>& e, CT<T>* spec, int ns, long long ss) {
  if (ns == 1) {
    const MechUEpiC<T, 2, true> ec{e};
    return launch_row_inv<T, 1, MechUEpiC<T, 2, true>, true>(c, kind, ec, spec, 2 * ns, ss / 2);
  }
  const MechUEpiC<T, 2, false> ec{e};
  return launch_row_inv<T, 1, MechUEpiC<T, 2, false>, true>(c, kind, ec, spec, 2 * ns, ss / 2);
}

// The Green pass of the mechanics PCG (partial sums of r.z into part_rr):
// the unit Green operator one component per block, or the reference medium
// with both components of a column per block.  st nullable (no state check).
template <typename T> int launch_green(fgcg_ctx* c, int kind, const CgState* st, int ns, long long ss) {
  CT<T>* spec = (CT<T>*)c->spec;
  if (c->precond == 1) {
    const MechRefGreen<T> g{c->Dx, c->Dy, 1.0 / (double)c->n, c->use_lam, c->use_mu, c->nx, st, c->part_rr};
    return launch_col<T, 2, 2, MechRefGreen<T>, true>(c, kind, g, spec, spec, ns, ss);
  }
  const MechGreen<T> g{c->Dx, c->Dy, 1.0 / (double)c->n, c->nx, st, c->part_rr};
  return launch_col<T, 1, 1, MechGreen<T>, true>(c, kind, g, spec, spec, 2 * ns, ss / 2);
}

// Partial sums of r.z per sample left by the Green pass.
inline int green_parts(const fgcg_ctx* c) { return c->precond == 1 ? c->ncol : 2 * c->ncol; }

// ---------------------------------------------- residual-spectrum PCG (2D FP64)
inline int ensure_rhat(fgcg_ctx* c) {
  if (!c->rhat) {
    const size_t bytes = sizeof(double2) * 2 * (size_t)c->nxh * c->rows * c->nsamp;
    if (hipMalloc(&c->rhat, bytes) != hipSuccess) return fail(FGCG_ENOMEM, "residual spectra");
  }
  if (fused_active(c) && !c->p_odd) {
    if (hipMalloc(&c->p_odd, sizeof(double) * 2 * (size_t)c->n * c->nsamp) != hipSuccess ||
        hipMalloc(&c->spec_q, sizeof(double2) * 2 * (size_t)c->nxh * c->rows * c->nsamp) != hipSuccess)
      return fail(FGCG_ENOMEM, "two-pass form buffers");
  }
  return 0;
}

// The fused row stage of the two-pass form (k_sr_row): init (p_0 = z_0 into
// p) or iteration k with parity k & 1 (p_k from p or p_odd, p_{k+1} into the
// other).
inline int launch_sr_row(fgcg_ctx* c, int kind, const MechMat& m, int init, double tol, int maxit, int parity,
                         int ns) {
  int rc = 0;
  with_n(c->nx, [&](auto NXc) {
    constexpr int NX = decltype(NXc)::value;
    if constexpr (NX % 64 == 0) {
      double* pe = (double*)c->p;
      double* po = (double*)c->p_odd;
      const SrRowArgs<double> a{(const double2*)c->spec, (double2*)c->spec_q, parity ? po : pe,
                                init ? pe : (parity ? pe : po), (double*)c->x, c->st, c->part_rr, green_parts(c),
                                c->part_a, c->rows, (long long)c->nxh * c->rows, 1.0 / c->h, init, tol, maxit};
      with_plan<NX>(c->plan_row, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        dim3 g((c->rows + SR_ROWS - 1) / SR_ROWS, ns);
        if (kind >= 0) set_kname(c, kind, "k_sr_row<%s, %d", "double", NX);
        const void* fn = m.Efield ? (const void*)&k_sr_row<double, NX, P, true>
                                  : (const void*)&k_sr_row<double, NX, P, false>;
        rc = launch_b(c, kind, fn, g, dim3(sr_threads(NX)), a, m, tw_x<double>(c));
      });
    } else {
      rc = fail(FGCG_EUNSUPPORTED, "the two-pass form needs nx a multiple of 64");
    }
  });
  return rc;
}

// q = K p, its x transforms and the p.Kp partial sums (k_kp_fwd), tuned rows
// per block and radix plan.
template <typename T> int launch_kp_fwd(fgcg_ctx* c, int kind, const MechMat& m, const T* p, int ns) {
  int rc = 0;
  with_n(c->nx, [&](auto NXc) {
    constexpr int NX = decltype(NXc)::value;
    if constexpr (NX % NT == 0) {
      if (c->kp_both) {
        // both components per block, rows_for(NX) rows (the partial sums are
        // per grid row, so this need not match the inverse pass's rows)
        constexpr int R = rows_for(NX);
        with_plan<NX>(c->plan_row, [&](auto Pc) {
          constexpr int P = decltype(Pc)::value;
          dim3 g((c->rows + R - 1) / R, ns);
          if (kind >= 0) set_kname(c, kind, "k_kp_fwd2<%s, %d", tname<T>(), NX);
          const void* fn = m.Efield ? (const void*)&k_kp_fwd2<T, NX, R, P, true>
                                    : (const void*)&k_kp_fwd2<T, NX, R, P, false>;
          rc = launch_b(c, kind, fn, g, dim3(kp_threads(NX)), m, p, c->st, c->part_a, (CT<T>*)c->spec, c->rows,
                        (long long)c->nxh * c->rows, (T)(1.0 / c->h), tw_x<T>(c));
        });
        return;
      }
      with_rows<NX>(c->rows_pick, [&](auto Rc) {
        with_plan<NX>(c->plan_row, [&](auto Pc) {
          constexpr int R = decltype(Rc)::value, P = decltype(Pc)::value;
          dim3 g((c->rows + R - 1) / R, 2 * ns);
          if (kind >= 0) set_kname(c, kind, "k_kp_fwd<%s, %d", tname<T>(), NX);
          const void* fn = m.Efield ? (const void*)&k_kp_fwd<T, NX, R, P, true>
                                    : (const void*)&k_kp_fwd<T, NX, R, P, false>;
          rc = launch_b(c, kind, fn, g, dim3(kp_threads(NX)), m, p, c->st, c->part_a, (CT<T>*)c->spec, c->rows,
                        (long long)c->nxh * c->rows, (T)(1.0 / c->h), tw_x<T>(c));
        });
      });
    } else {
      rc = fail(FGCG_EUNSUPPORTED, "residual-spectrum PCG needs nx a multiple of 256");
    }
  });
  return rc;
}

// The Green pass on the residual spectrum (init: r_hat = FFT(f)).
template <typename T> int launch_green_sr(fgcg_ctx* c, int kind, int init, int ns) {
  const MechGreenSR<T> g{c->Dx,     c->Dy,      1.0 / (double)c->n, c->nx, c->st, c->part_rr, c->part_a,
                         (c->kp_both ? 1 : 2) * c->rows, (CT<T>*)c->rhat, (long long)c->nxh * c->rows, c->rows,
                         init};
  CT<T>* spec = (CT<T>*)c->spec;
  // the two-pass form's row stage leaves the x spectra of K p in spec_q
  CT<T>* in = fused_active(c) && !init ? (CT<T>*)c->spec_q : spec;
  return launch_col<T, 1, 1, MechGreenSR<T>, true>(c, kind, g, in, spec, 2 * ns, (long long)c->nxh * c->rows);
}

// The inverse pass with the direction and the (deferred) solution update.
template <typename T>
int launch_sr_row_inv(fgcg_ctx* c, int kind, const MechUEpi<T, 2>& e, const Field<T>& X, int ns) {
  CT<T>* spec = (CT<T>*)c->spec;
  const long long ss = (long long)c->nxh * c->rows;
  if (ns == 1) {
    const MechUEpiSRC<T, true> ec{e, X};
    return launch_row_inv<T, 1, MechUEpiSRC<T, true>, true>(c, kind, ec, spec, 2 * ns, ss);
  }
  const MechUEpiSRC<T, false> ec{e, X};
  return launch_row_inv<T, 1, MechUEpiSRC<T, false>, true>(c, kind, ec, spec, 2 * ns, ss);
}

// The last solution update, when the stop test ended the solve in the inverse pass.
inline int sr_finish(fgcg_ctx* c) {
  if (!sr_active(c)) return 0;
  const double* po = (const double*)(fused_active(c) ? c->p_odd : c->p);
  hipLaunchKernelGGL((k_sr_finish<double>), dim3(c->npost, c->nsamp), dim3(PT), 0, c->stream, (double*)c->x,
                     (const double*)c->p, po, (const CgState*)c->st, 2 * c->n);
  HIPCHK(hipGetLastError());
  return 0;
}

// z = M r, p = z, r.z and the CG state of every sample (R holds f, X holds 0).
template <typename T> int mech_init(fgcg_ctx* c, const MechMat& m, double tol, int maxit) {
  CT<T>* spec = (CT<T>*)c->spec;
  const int ns = c->nsamp;
  const long long ss = spec_ss(c);
  int rc;
  const CopyProN<T, 2> cp{fld<T>(c->r, c), c->nx};
  if ((rc = launch_row_fwd<T, 2, CopyProN<T, 2>, true>(c, -1, cp, spec, ns, ss))) return rc;
  if constexpr (std::is_same<T, double>::value) if (sr_active(c)) {
    // r_hat = FFT(f) stored, z = M r, p = z
    if ((rc = ensure_rhat(c)) || (rc = launch_green_sr<T>(c, -1, 1, ns))) return rc;
    if (fused_active(c)) {
      // p_0 = z_0, and the stiffness and forward transforms of p_0
      if ((rc = launch_sr_row(c, -1, m, 1, tol, maxit, 0, ns))) return rc;
      HIPCHK(hipGetLastError());
      return 0;
    }
    MechUEpi<T, 2> e0{fld<T>(c->p, c), c->nx, c->st, c->part_rr, green_parts(c), 1, tol, maxit};
    e0.sr = 1;
    if ((rc = launch_sr_row_inv<T>(c, -1, e0, fld<T>(c->x, c), ns))) return rc;
    HIPCHK(hipGetLastError());
    return 0;
  }
  if ((rc = launch_green<T>(c, -1, nullptr, ns, ss))) return rc;
  const MechUEpi<T, 2> e0{fld<T>(c->p, c), c->nx, c->st, c->part_rr, green_parts(c), 1, tol, maxit};
  if ((rc = launch_mech_row_inv<T>(c, -1, e0, spec, ns, ss))) return rc;
  HIPCHK(hipGetLastError());
  return 0;
}

// The launches of one CG iteration (all samples).  reliable: FP32-mixed
// reliable update (fold into the FP64 solution, FP64 true residual).
// parity: k & 1 of the iteration (the two-pass form's direction buffers).
template <typename T>
int mech_iter(fgcg_ctx* c, const MechMat& m, double tol, int maxit, bool reliable, int parity) {
  CT<T>* spec = (CT<T>*)c->spec;
  const int ns = c->nsamp;
  const long long ss = spec_ss(c);
  const Field<T> X = fld<T>(c->x, c), R = fld<T>(c->r, c), P = fld<T>(c->p, c), Q = fld<T>(c->tmp, c);
  if constexpr (std::is_same<T, double>::value) if (fused_active(c)) {
    int r = launch_green_sr<T>(c, FGCG_K_MECH_COL, 0, ns);
    r |= launch_sr_row(c, FGCG_K_MECH_ROW_FWD, m, 0, tol, maxit, parity, ns);
    return r;
  }
  if constexpr (std::is_same<T, double>::value) if (sr_active(c)) {
    int r = launch_kp_fwd<T>(c, FGCG_K_MECH_ROW_FWD, m, (const T*)P.p, ns);
    r |= launch_green_sr<T>(c, FGCG_K_MECH_COL, 0, ns);
    MechUEpi<T, 2> epi{P, c->nx, c->st, c->part_rr, green_parts(c), 0, tol, maxit};
    epi.sr = 1;
    r |= launch_sr_row_inv<T>(c, FGCG_K_MECH_ROW_INV, epi, X, ns);
    return r;
  }
  set_kname(c, FGCG_K_MECH_KP, "k_mech_kp<%s%.0d", tname<T>(), 0);
  int r = launch(c, FGCG_K_MECH_KP, (const void*)&k_mech_kp<T>, dim3(c->nkpt, ns), m, (const T*)P.p, Q.p, c->n,
                 c->nx, c->ny, (T)(1.0 / c->h), c->st, c->part_a);
  if (!reliable) {
    const MechUProC<T, 2> pro{{X, R, P, Q, c->nx, c->st, c->part_a, c->nkpt}};
    r |= launch_row_fwd<T, 1, MechUProC<T, 2>, true>(c, FGCG_K_MECH_ROW_FWD, pro, spec, 2 * ns, ss / 2);
  } else {
    r |= launch(c, -1, (const void*)&k_mech_fold<T>, dim3(c->npost, ns), X.p, c->xh, (const T*)P.p, 2 * c->n, c->st,
                (const double*)c->part_a, c->nkpt);
    r |= launch(c, -1, (const void*)&k_mech_true_res<T>, dim3(c->nkp, ns), m, (const double*)c->xh,
                (const double*)c->fh, R.p, c->n, c->nx, c->ny, 1.0 / c->h, (const CgState*)c->st);
    const CopyProN<T, 2> cp{R, c->nx};
    r |= launch_row_fwd<T, 2, CopyProN<T, 2>, true>(c, -1, cp, spec, ns, ss);
  }
  r |= launch_green<T>(c, FGCG_K_MECH_COL, c->st, ns, ss);
  const MechUEpi<T, 2> epi{P, c->nx, c->st, c->part_rr, green_parts(c), 0, tol, maxit};
  r |= launch_mech_row_inv<T>(c, FGCG_K_MECH_ROW_INV, epi, spec, ns, ss);
  return r;
}

// r = f = -grad^H g C : (eps_mac_s - e I), x = 0 for every sample (FP64
// right-hand side and solution in FP32-mixed contexts, with r rounded to FP32).
int mech_rhs(fgcg_ctx* c, const MechMat& m, const double* eig) {
  const int ns = c->nsamp;
  if (c->prec == FGCG_FP64) {
    hipLaunchKernelGGL((k_mech_rhs<double>), dim3(c->nkp, ns), dim3(NT), 0, c->stream, m, eig, (const double*)c->ems,
                       (double*)c->r, (double*)c->x, c->n, c->nx, c->ny, 1.0 / c->h);
  } else {
    hipLaunchKernelGGL((k_mech_rhs<double>), dim3(c->nkp, ns), dim3(NT), 0, c->stream, m, eig, (const double*)c->ems,
                       c->fh, c->xh, c->n, c->nx, c->ny, 1.0 / c->h);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(c->npost), dim3(PT), 0, c->stream, (float*)c->r,
                       (const double*)c->fh, 2 * c->n * ns);
    HIPCHK(hipMemsetAsync(c->x, 0, sizeof(float) * 2 * c->n * ns, c->stream));
  }
  HIPCHK(hipGetLastError());
  return 0;
}

Key mech_key(const fgcg_ctx* c, const MechMat& m, double tol, int maxit) {
  Key key;
  key.add(m.phase).add(m.d).add(m.Efield).add(m.lm_dev).add(m.kappa).add(m.lam_per_E).add(m.mu_per_E).add(m.lm);
  key.add(c->prec).add(c->precond).add(c->use_lam).add(c->use_mu).add(tol).add(maxit).add(c->rows_pick).add(c->plan_row).add(c->plan_col);
  key.add(sr_active(c)).add(fused_active(c));
  return key;
}

// Timing workspace of the 2D mechanics passes: zero fields and spectra, a
// running CG state per sample (unit r.z, no stop test) and unit partial sums,
// so that every pass does its full work.
template <typename T> int timing_workspace(fgcg_ctx* c) {
  const int ns = c->nsamp;
  int rc = running_state(c);
  if (rc) return rc;
  const size_t nv = sizeof(T) * c->ncw * (size_t)c->n * ns;
  for (void* b : {c->x, c->r, c->p, c->tmp}) HIPCHK(hipMemsetAsync(b, 0, nv, c->stream));
  HIPCHK(hipMemsetAsync(c->spec, 0, sizeof(CT<T>) * c->ncw * (size_t)c->nxh * c->rows * ns, c->stream));
  if (sr_active(c)) {
    if ((rc = ensure_rhat(c))) return rc;
    const size_t sb = sizeof(CT<T>) * 2 * (size_t)c->nxh * c->rows * ns;
    HIPCHK(hipMemsetAsync(c->rhat, 0, sb, c->stream));
    if (fused_active(c)) {
      HIPCHK(hipMemsetAsync(c->spec_q, 0, sb, c->stream));
      HIPCHK(hipMemsetAsync(c->p_odd, 0, nv, c->stream));
    }
  }
  // (k_kp_fwd leaves two partial sums per grid row and sample)
  const int npa = std::max(c->nkpt, 2 * c->rows), nprz = 2 * c->ncol;
  std::vector<double> ones((size_t)std::max(npa, nprz) * ns, 1.0);
  HIPCHK(hipMemcpyAsync(c->part_a, ones.data(), sizeof(double) * npa * ns, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->part_rr, ones.data(), sizeof(double) * nprz * ns, hipMemcpyHostToDevice, c->stream));
  // the host vectors are read by the copies: wait before they go out of scope
  HIPCHK(hipStreamSynchronize(c->stream));
  return 0;
}

// Autotuning of the 2D mechanics passes: the rows per block and the radix
// plan of the row passes (the forward pass with the CG update and the inverse
// pass with the direction update, timed as a pair) and the radix plan of the
// Green column pass.  Each candidate is timed with HIP events on the context's
// own workspace and samples, 3 + 10 launches; the fastest rows choice is kept,
// and radix 16 replaces radix 8 only when more than 3 % faster (plans are
// timed on grids of at least 2^18 voxels, radix 8 below).  Values fixed
// through the options are not tuned.  The rows choice does not change any
// result (rows are paired and transformed identically; these passes carry no
// partial sums); the plan changes the rounding of the transforms only.  The
// workspace and the CG state are overwritten, so this runs before the
// right-hand side is formed.
// Material of the pass and iteration timings: phase 0 everywhere with unit
// Lame constants and zero damage (the phase-table and damage paths of the
// staggered solves), from zeroed buffers allocated on first use.
inline int timing_material(fgcg_ctx* c, MechMat* m) {
  const size_t nv = (size_t)c->n * c->nsamp;
  if (!c->timing_E) {
    if (hipMalloc(&c->timing_E, sizeof(double) * nv + nv) != hipSuccess) return fail(FGCG_ENOMEM, "timing fields");
    HIPCHK(hipMemsetAsync(c->timing_E, 0, sizeof(double) * nv + nv, c->stream));
  }
  std::memset(m, 0, sizeof *m);
  m->phase = (const uint8_t*)(c->timing_E + nv);
  m->d = c->timing_E;
  m->ss = c->n;
  m->nphase = 1;
  m->lm.a[0] = m->lm.b[0] = 1.0;
  return 0;
}

template <typename T> int tune_passes_t(fgcg_ctx* c) {
  std::vector<int> rows_c, prow_c, pcol_c;
  with_n(c->nx, [&](auto NXc) {
    constexpr int NX = decltype(NXc)::value;
    rows_c = rows_candidates<NX>();
    prow_c = plan1_differs(NX) ? std::vector<int>{1, 2} : std::vector<int>{1};
  });
  with_n(c->ny, [&](auto NYc) {
    constexpr int NY = decltype(NYc)::value;
    pcol_c = plan1_differs(NY) ? std::vector<int>{1, 2} : std::vector<int>{1};
    // one wavefront per column: the one-component (unit) Green pass
    if (wave_col_ok(NY) && c->precond == 0) pcol_c.push_back(3);
  });
  // below 2^18 voxels the passes are launch-bound and plan timings are
  // noise: radix 8 (so every context of a small size has the same schedule)
  if (c->n < (1LL << 18)) prow_c = pcol_c = {1};
  if (c->rows_pick) rows_c = {c->rows_pick};
  if (c->plan_row) prow_c = {c->plan_row};
  if (c->plan_col) pcol_c = {c->plan_col};
  if (fused_active(c)) rows_c = {rows_c[0]};  // the fused row stage has a fixed tile
  const int ns = c->nsamp;
  const long long ss = spec_ss(c);
  int rc = timing_workspace<T>(c);
  if (rc) return rc;
  const int npa = c->nkpt, nprz = green_parts(c);
  CT<T>* spec = (CT<T>*)c->spec;
  const Field<T> X = fld<T>(c->x, c), R = fld<T>(c->r, c), P = fld<T>(c->p, c), Q = fld<T>(c->tmp, c);
  const MechUProC<T, 2> pro{{X, R, P, Q, c->nx, c->st, c->part_a, npa}};
  const MechUEpi<T, 2> epi{P, c->nx, c->st, c->part_rr, nprz, 0, 0.0, 1 << 30};
  const bool sr = sr_active(c);
  MechUEpi<T, 2> epi_sr = epi;
  epi_sr.sr = 1;
  MechMat tmat;
  if ((rc = timing_material(c, &tmat))) return rc;
  // the Green pass (of the context's preconditioner) without a CG state,
  // timed after the row passes, whose direction update reads part_rr
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // times 3 + 10 launches of f, the last 10 between events
  auto time_it = [&](auto&& f) -> float {
    for (int rep = 0; rep < 13 && !rc; ++rep) {
      if (rep == 3 && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(FGCG_EHIP, "hipEventRecord");
      rc |= f();
    }
    float ms = 0.f;
    if (!rc && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = fail(FGCG_EHIP, "timing a pass candidate failed");
    return ms;
  };
  // The rows choice keeps the fastest candidate (it never changes results).
  // A radix plan other than the first candidate must win by more than 3 %:
  // the plan changes rounding, so near-ties (timing noise) keep one schedule
  // and contexts of the same size agree.
  constexpr float PLAN_MARGIN = 0.97f;
  std::vector<float> best_p(prow_c.size(), 0.f);
  std::vector<int> rows_p(prow_c.size(), rows_c[0]);
  if (rows_c.size() * prow_c.size() > 1) {
    for (int R_ : rows_c)
      for (size_t ip = 0; ip < prow_c.size(); ++ip) {
        if (rc) break;
        c->rows_pick = R_;
        c->plan_row = prow_c[ip];
        const float ms = time_it([&] {
          if constexpr (std::is_same<T, double>::value) {
            if (fused_active(c)) return launch_sr_row(c, -1, tmat, 0, 0.0, 1 << 30, 0, ns);
            if (sr)
              return launch_kp_fwd<T>(c, -1, tmat, (const T*)P.p, ns) | launch_sr_row_inv<T>(c, -1, epi_sr, X, ns);
          }
          return launch_row_fwd<T, 1, MechUProC<T, 2>, true>(c, -1, pro, spec, 2 * ns, ss / 2) |
                 launch_mech_row_inv<T>(c, -1, epi, spec, ns, ss);
        });
        if (R_ == rows_c[0] || ms < best_p[ip]) {
          best_p[ip] = ms;
          rows_p[ip] = R_;
        }
      }
  }
  size_t ip_pick = 0;
  for (size_t ip = 1; ip < prow_c.size(); ++ip)
    if (best_p[ip] < PLAN_MARGIN * best_p[ip_pick]) ip_pick = ip;
  const int pick_r = rows_p[ip_pick], pick_p = prow_c[ip_pick];
  int pick_c = pcol_c[0];
  if (pcol_c.size() > 1) {
    std::vector<float> tc(pcol_c.size(), 0.f);
    if (sr) {
      // the residual-spectrum Green pass forms alpha from the stiffness
      // pass's partial sums, which the row timings left at zero: unit sums
      std::vector<double> ones((size_t)2 * c->rows * ns, 1.0);
      HIPCHK(hipMemcpyAsync(c->part_a, ones.data(), sizeof(double) * ones.size(), hipMemcpyHostToDevice, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    }
    for (size_t ip = 0; ip < pcol_c.size() && !rc; ++ip) {
      c->plan_col = pcol_c[ip];
      tc[ip] = time_it([&] {
        if constexpr (std::is_same<T, double>::value)
          if (sr) return launch_green_sr<T>(c, -1, 0, ns);
        return launch_green<T>(c, -1, nullptr, ns, ss);
      });
    }
    size_t ic = 0;
    for (size_t ip = 1; ip < pcol_c.size(); ++ip)
      if (tc[ip] < PLAN_MARGIN * tc[ic]) ic = ip;
    pick_c = pcol_c[ic];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipGetLastError());
  c->rows_pick = pick_r;
  c->plan_row = pick_p;
  c->plan_col = pick_c;
  return rc;
}

// A fixed, mean-free-ish pattern for the direction of the iteration timings.
template <typename T>
__global__ void __launch_bounds__(PT) k_pattern(T* __restrict__ v, long long n) {
  for (long long i = blockIdx.x * (long long)PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT)
    v[i] = (T)((double)((unsigned long long)(i * 2654435761ULL) & 0xffffULL) / 65536.0 - 0.5);
}

// Average time of one whole mechanics CG iteration (form 1: residual
// spectrum, 2: four passes, 3: residual spectrum in two passes) launched back
// to back, 3 + 10 iterations between
// HIP events, on a workspace that runs genuine CG steps: the timing material
// (unit Lame constants), a fixed pattern as the first direction, zero x and
// r, a state that never converges (threshold -1).  Overwrites the workspace
// and the CG state.
template <typename T> int time_iteration(fgcg_ctx* c, int form, float* ms_per_iter) {
  int rc = timing_workspace<T>(c);
  if (rc) return rc;
  const int ns = c->nsamp;
  const long long ss = spec_ss(c);
  std::vector<CgState> hs(ns);
  for (CgState& t : hs) {
    std::memset(&t, 0, sizeof t);
    t.rz[0] = t.rz[1] = 1.0;
    t.bnorm2 = 1.0;
    t.thr = -1.0;
    t.maxit = 1 << 30;
  }
  HIPCHK(hipMemcpyAsync(c->st, hs.data(), sizeof(CgState) * ns, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL((k_pattern<T>), dim3(c->npost), dim3(PT), 0, c->stream, (T*)c->p, 2 * c->n * ns);
  // the two-pass form starts an iteration at the Green pass, whose input
  // q_hat is zero here: a residual spectrum to work on (else r = 0 after the
  // first iteration, and the second ends the solve on p.Kp = 0)
  if (form == 3)
    hipLaunchKernelGGL((k_pattern<double>), dim3(c->npost), dim3(PT), 0, c->stream, (double*)c->rhat,
                       4LL * c->nxh * c->rows * ns);
  HIPCHK(hipStreamSynchronize(c->stream));
  MechMat tm;
  if ((rc = timing_material(c, &tm))) return rc;
  const Field<T> X = fld<T>(c->x, c), R = fld<T>(c->r, c), P = fld<T>(c->p, c), Q = fld<T>(c->tmp, c);
  MechUEpi<T, 2> epi{P, c->nx, c->st, c->part_rr, green_parts(c), 0, 0.0, 1 << 30};
  int par = 0;
  auto one = [&]() -> int {
    if constexpr (std::is_same<T, double>::value) {
      if (form == 3) {
        const int r = launch_green_sr<T>(c, -1, 0, ns) | launch_sr_row(c, -1, tm, 0, 0.0, 1 << 30, par, ns);
        par ^= 1;
        return r;
      }
      if (form == 1) {
        MechUEpi<T, 2> e = epi;
        e.sr = 1;
        return launch_kp_fwd<T>(c, -1, tm, (const T*)P.p, ns) | launch_green_sr<T>(c, -1, 0, ns) |
               launch_sr_row_inv<T>(c, -1, e, X, ns);
      }
    }
    const MechUProC<T, 2> pro{{X, R, P, Q, c->nx, c->st, c->part_a, c->nkpt}};
    return launch(c, -1, (const void*)&k_mech_kp<T>, dim3(c->nkpt, ns), tm, (const T*)P.p, Q.p, c->n, c->nx, c->ny,
                  (T)(1.0 / c->h), c->st, c->part_a) |
           launch_row_fwd<T, 1, MechUProC<T, 2>, true>(c, -1, pro, (CT<T>*)c->spec, 2 * ns, ss / 2) |
           launch_green<T>(c, -1, c->st, ns, ss) | launch_mech_row_inv<T>(c, -1, epi, (CT<T>*)c->spec, ns, ss);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(FGCG_EHIP, "hipEventCreate");
  for (int i = 0; i < 3 && !rc; ++i) rc = one();
  if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(FGCG_EHIP, "hipEventRecord");
  for (int i = 0; i < 10 && !rc; ++i) rc = one();
  float ms = 0.f;
  if (!rc && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = fail(FGCG_EHIP, "timing an iteration failed");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!rc) *ms_per_iter = ms / 10.f;
  return rc;
}

// Tuned picks are kept per process, keyed by the device and everything the
// timings depend on (grid, precision, preconditioner, iteration form, samples
// and the values pinned through the options), so later contexts of the same
// shape take them without timing again.
struct TuneKey {
  int dev, nx, ny, prec, precond, sr, nsamp, rows, prow, pcol;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, nx, ny, prec, precond, sr, nsamp, rows, prow, pcol) <
           std::tie(o.dev, o.nx, o.ny, o.prec, o.precond, o.sr, o.nsamp, o.rows, o.prow, o.pcol);
  }
};
std::mutex tune_mu;

std::map<TuneKey, std::array<int, 4>> tune_cache;

// The passes of the context's mechanics form, and on grids of at least 2^18
// voxels where the residual-spectrum form applies, the form itself: each
// form's passes are tuned, one whole iteration of each is timed and the
// fastest is kept (smaller grids take SR_DEFAULT_FORM).
constexpr int SR_DEFAULT_FORM = 3;
inline int tune_passes(fgcg_ctx* c) {
  const bool forms = sr_eligible(c) && c->sr_pick == 0;
  if (c->rows_pick && c->plan_row && c->plan_col) {
    if (forms) c->sr_pick = SR_DEFAULT_FORM;
    return 0;
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const TuneKey key{dev, c->nx, c->ny, c->prec, c->precond, forms ? 1 : (sr_eligible(c) ? 10 + c->sr_pick : 0), c->nsamp,
                    c->rows_pick, c->plan_row, c->plan_col};
  {
    std::lock_guard<std::mutex> g(tune_mu);
    auto it = tune_cache.find(key);
    if (it != tune_cache.end()) {
      c->rows_pick = it->second[0];
      c->plan_row = it->second[1];
      c->plan_col = it->second[2];
      if (forms) c->sr_pick = it->second[3];
      return 0;
    }
  }
  auto tune = [&]() { return c->prec == FGCG_FP64 ? tune_passes_t<double>(c) : tune_passes_t<float>(c); };
  int rc;
  if (forms && c->n >= (1LL << 18)) {
    const int r0 = c->rows_pick, p0 = c->plan_row, q0 = c->plan_col;
    float t[3] = {0.f, 0.f, 0.f};
    std::array<int, 3> pk[3];
    for (int f = 1; f <= 3; ++f) {
      if (f == 1 && !sr3_ok(c)) {
        t[0] = 3.0e38f;  // no three-pass form on these rows
        continue;
      }
      c->rows_pick = r0;
      c->plan_row = p0;
      c->plan_col = q0;
      c->sr_pick = f;
      if ((rc = ensure_rhat(c)) || (rc = tune()) || (rc = time_iteration<double>(c, f, &t[f - 1]))) return rc;
      pk[f - 1] = {c->rows_pick, c->plan_row, c->plan_col};
    }
    int f = SR_DEFAULT_FORM;
    for (int g = 1; g <= 3; ++g)
      if (t[g - 1] < t[f - 1]) f = g;
    c->sr_pick = f;
    c->rows_pick = pk[f - 1][0];
    c->plan_row = pk[f - 1][1];
    c->plan_col = pk[f - 1][2];
  } else {
    if (forms) c->sr_pick = SR_DEFAULT_FORM;
    if (forms && (rc = ensure_rhat(c))) return rc;
    if ((rc = tune())) return rc;
  }
  std::lock_guard<std::mutex> g(tune_mu);
  tune_cache[key] = {c->rows_pick, c->plan_row, c->plan_col, c->sr_pick};
  return 0;
}

// Average duration of one 2D mechanics pass launched reps times back to back
// (after 3 untimed launches) between two HIP events on the context's stream,
// with the tuned rows per block and radix plans, on the timing workspace.
template <typename T> int time_pass_t(fgcg_ctx* c, int kind, int reps, double* us) {
  int rc = timing_workspace<T>(c);
  if (rc) return rc;
  const int ns = c->nsamp;
  const long long ss = spec_ss(c);
  CT<T>* spec = (CT<T>*)c->spec;
  const Field<T> X = fld<T>(c->x, c), R = fld<T>(c->r, c), P = fld<T>(c->p, c), Q = fld<T>(c->tmp, c);
  const MechUProC<T, 2> pro{{X, R, P, Q, c->nx, c->st, c->part_a, c->nkpt}};
  const MechUEpi<T, 2> epi{P, c->nx, c->st, c->part_rr, green_parts(c), 0, 0.0, 1 << 30};
  // (only one kind is launched: the Green pass's partial sums may overwrite
  // the unit sums the direction update would read)
  const bool sr = sr_active(c);
  MechUEpi<T, 2> epi_sr = epi;
  epi_sr.sr = 1;
  MechMat tmat;
  if ((rc = timing_material(c, &tmat))) return rc;
  auto one = [&]() -> int {
    if constexpr (std::is_same<T, double>::value) {
      if (fused_active(c)) {
        if (kind == FGCG_K_MECH_ROW_FWD) return launch_sr_row(c, -1, tmat, 0, 0.0, 1 << 30, 0, ns);
        if (kind == FGCG_K_MECH_ROW_INV) return fail(FGCG_EUNSUPPORTED, "the two-pass form has no inverse row pass");
        return launch_green_sr<T>(c, -1, 0, ns);
      }
    }
    if constexpr (std::is_same<T, double>::value)
      if (sr) {
        if (kind == FGCG_K_MECH_ROW_FWD) return launch_kp_fwd<T>(c, -1, tmat, (const T*)P.p, ns);
        if (kind == FGCG_K_MECH_ROW_INV) return launch_sr_row_inv<T>(c, -1, epi_sr, X, ns);
        return launch_green_sr<T>(c, -1, 0, ns);
      }
    if (kind == FGCG_K_MECH_ROW_FWD)
      return launch_row_fwd<T, 1, MechUProC<T, 2>, true>(c, -1, pro, spec, 2 * ns, ss / 2);
    if (kind == FGCG_K_MECH_ROW_INV)
      return launch_mech_row_inv<T>(c, -1, epi, spec, ns, ss);
    return launch_green<T>(c, -1, nullptr, ns, ss);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(FGCG_EHIP, "hipEventCreate");
  for (int i = 0; i < 3 && !rc; ++i) rc = one();
  if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(FGCG_EHIP, "hipEventRecord");
  for (int i = 0; i < reps && !rc; ++i) rc = one();
  float ms = 0.f;
  if (!rc && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = fail(FGCG_EHIP, "timing the pass failed");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!rc) *us = 1e3 * (double)ms / reps;
  return rc;
}

// Kernel-level hook: q = K p through the stiffness pass of the solver
// (k_mech_kp) or z = M r through the Green passes the solver starts every
// solve with (row transform, k_col<MechGreen> with the tuned radix plan,
// inverse row transform writing p = z), in the context's precision.
template <typename T> int debug_apply_t(fgcg_ctx* c, int op, const MechMat& m, const double* in, double* out) {
  const long long n2 = 2 * c->n;
  int rc;
  if (op == FGCG_OP_MECH_K) {
    if ((rc = running_state(c))) return rc;
    hipLaunchKernelGGL((k_convert<T, double>), dim3(c->npost), dim3(PT), 0, c->stream, (T*)c->p, in, n2);
    bool via_sr = false;
    if constexpr (std::is_same<T, double>::value) {
      if (fused_active(c)) {
        // the two-pass form's row stage in its init mode: z_hat = FFT_x(u) / nx
        // (x transforms, then the identity symbol with 1/N between the y
        // transforms) gives p_0 = u and the x spectra of K u in spec_q, which
        // the column and row passes bring back to real space
        if ((rc = ensure_rhat(c))) return rc;  // (allocates spec_q on first use)
        if (!c->spec_q || !c->p_odd) return fail(FGCG_EHIP, "two-pass form buffers missing");
        CT<T>* spec = (CT<T>*)c->spec;
        CT<T>* sq = (CT<T>*)c->spec_q;
        const long long ss = (long long)c->nxh * c->rows;
        const ScaleSym<T> id{1.0 / (double)c->n};
        const CopyProN<T, 2> cp{fld<T>(c->p, c), c->nx};
        const StoreCompEpi<T> store{fld<T>(c->tmp, c), c->nx};
        std::vector<double> ones((size_t)green_parts(c), 1.0);  // r.z > 0: the init does not stop
        HIPCHK(hipMemcpyAsync(c->part_rr, ones.data(), sizeof(double) * ones.size(), hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if ((rc = launch_row_fwd<T, 2, CopyProN<T, 2>, true>(c, -1, cp, spec, 1, 2 * ss)) ||
            (rc = launch_col<T, 1, 1, ScaleSym<T>>(c, -1, id, spec, spec, 2, ss)) ||
            (rc = launch_sr_row(c, -1, m, 1, 0.0, 1, 0, 1)) ||
            (rc = launch_col<T, 1, 1, ScaleSym<T>>(c, -1, id, sq, sq, 2, ss)) ||
            (rc = launch_row_inv<T, 1, StoreCompEpi<T>>(c, -1, store, sq, 2, ss)))
          return rc;
        via_sr = true;
      } else if (sr_active(c)) {
        // the stiffness of the residual-spectrum PCG (k_kp_fwd) returns x
        // transforms of q: back to real space through the column and row passes
        CT<T>* spec = (CT<T>*)c->spec;
        const long long ss = (long long)c->nxh * c->rows;
        const ScaleSym<T> id{1.0 / (double)c->n};
        const StoreCompEpi<T> store{fld<T>(c->tmp, c), c->nx};
        if ((rc = launch_kp_fwd<T>(c, -1, m, (const T*)c->p, 1)) ||
            (rc = launch_col<T, 1, 1, ScaleSym<T>>(c, -1, id, spec, spec, 2, ss)) ||
            (rc = launch_row_inv<T, 1, StoreCompEpi<T>>(c, -1, store, spec, 2, ss)))
          return rc;
        via_sr = true;
      }
    }
    if (!via_sr)
      hipLaunchKernelGGL((k_mech_kp<T>), dim3(c->nkpt, 1), dim3(NT), 0, c->stream, m, (const T*)c->p, (T*)c->tmp,
                         c->n, c->nx, c->ny, (T)(1.0 / c->h), c->st, c->part_a);
    hipLaunchKernelGGL((k_convert<double, T>), dim3(c->npost), dim3(PT), 0, c->stream, out, (const T*)c->tmp, n2);
    HIPCHK(hipGetLastError());
    return 0;
  }
  resolve_reference(c, m);
  if ((rc = tune_passes(c))) return rc;
  hipLaunchKernelGGL((k_convert<T, double>), dim3(c->npost), dim3(PT), 0, c->stream, (T*)c->r, in, n2);
  HIPCHK(hipMemsetAsync(c->p, 0, sizeof(T) * n2, c->stream));  // z = 0 stays if r = 0
  if ((rc = mech_init<T>(c, m, 0.0, 1))) return rc;
  hipLaunchKernelGGL((k_convert<double, T>), dim3(c->npost), dim3(PT), 0, c->stream, out, (const T*)c->p, n2);
  HIPCHK(hipGetLastError());
  return 0;
}

// Builds the iteration closure of a context (period RELIABLE_EVERY in FP32-mixed).
// Called once per iteration, from k = 0 (graph chunks have an even length,
// so a chunk always starts at an even k and the parity baked into it holds).
struct MechIterFn {
  fgcg_ctx* c;
  MechMat m;
  double tol;
  int maxit;
  int j = 0;
  int par = 0;
  int operator()() {
    const int parity = par;
    par ^= 1;
    if (c->prec == FGCG_FP64) return mech_iter<double>(c, m, tol, maxit, false, parity);
    const bool rel = j == RELIABLE_EVERY - 1;
    j = rel ? 0 : j + 1;
    return mech_iter<float>(c, m, tol, maxit, rel, parity);
  }
};

// Solve from the right-hand side in R (X = 0); the result stays in X (FP64)
// or X + XH (FP32-mixed, folded into XH at the end).
// (The rows per block must have been tuned already: tuning overwrites the workspace.)
int mech_pcg(fgcg_ctx* c, const MechMat& m, double tol, int maxit, CgState* out) {
  int rc = c->prec == FGCG_FP64 ? mech_init<double>(c, m, tol, maxit) : mech_init<float>(c, m, tol, maxit);
  if (rc) return rc;
  MechIterFn it{c, m, tol, maxit};
  const int K = c->prec == FGCG_FP64 ? c->chunk : 2 * RELIABLE_EVERY;
  if ((rc = run_cg(c, c->prec == FGCG_FP64 ? 0 : 5, mech_key(c, m, tol, maxit), c->st, c->h_st, it, maxit, K)))
    return rc;
  *out = *c->h_st;
  if ((rc = sr_finish(c))) return rc;
  if (c->prec != FGCG_FP64) {
    hipLaunchKernelGGL((k_fold_final<float>), dim3(c->npost, c->nsamp), dim3(PT), 0, c->stream,
                       (const float*)c->x, c->xh, 2 * c->n);
    HIPCHK(hipGetLastError());
  }
  return 0;
}

// eps = eps_mac + sym(grad u), sigma, and per sample the mean stress and the
// energy (host arrays [nsamp][3], [nsamp]) from the final displacement.
int mech_post(fgcg_ctx* c, const MechMat& m, const double* eig, double* strain, double* stress,
              double* mean_stress, double* energy) {
  const int ns = c->nsamp;
  if (c->prec == FGCG_FP64)
    hipLaunchKernelGGL((k_mech_post_u<double>), dim3(c->npost, ns), dim3(NT), 0, c->stream, m,
                       (const double*)c->x, c->n, c->nx, c->ny, 1.0 / c->h, eig, (const double*)c->ems, strain,
                       stress, c->part_post);
  else
    hipLaunchKernelGGL((k_mech_post_u<double>), dim3(c->npost, ns), dim3(NT), 0, c->stream, m,
                       (const double*)c->xh, c->n, c->nx, c->ny, 1.0 / c->h, eig, (const double*)c->ems, strain,
                       stress, c->part_post);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_part, c->part_post, sizeof(double) * 4 * c->npost * ns, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int s = 0; s < ns; ++s) {
    double acc[4] = {0, 0, 0, 0};
    const double* pp = c->h_part + 4LL * c->npost * s;
    for (int b = 0; b < c->npost; ++b)
      for (int j = 0; j < 4; ++j) acc[j] += pp[4 * b + j];
    if (mean_stress)
      for (int j = 0; j < 3; ++j) mean_stress[3 * s + j] = acc[j] / (double)c->n;
    if (energy) energy[s] = 0.5 * c->h * c->h * acc[3];
  }
  return 0;
}

// ---------------------------------------------------- strain form (2D, FP64)
// The paper's projected CG on the symmetric strain (any gradient operator):
// b = -G[g C : (eps_mac - e I)], then three passes per iteration (see
// strain_form.hpp), then the post-processing of the strain.
int mech_sf_solve(fgcg_ctx* c, const MechMat& m, const double* eig, const double* em, double tol, int maxit,
                  double* strain, double* stress, double* mean_stress, double* energy, fgcg_info* info) {
  const double t0 = now();
  const long long n = c->n;
  CT<double>* spec = (CT<double>*)c->sf_spec;
  const Field<double> X{c->sf_buf, n, 0}, R{c->sf_buf + 3 * n, n, 0}, P{c->sf_buf + 6 * n, n, 0};
  int rc;
  const VecSrcPro<double, 3, StrainLaw> src{{m}, eig, {em[0], em[1], em[2]}, c->nx, n};
  if ((rc = launch_row_fwd<double, 3>(c, -1, src, spec))) return rc;
  const SymProj<double> pj0{c->Dx, c->Dy, 1.0 / (double)n, nullptr};
  if ((rc = launch_col<double, 3, 3>(c, -1, pj0, spec, spec))) return rc;
  const VecRhsEpi<double, 3> rhs{X, R, c->nx, c->part_rr, c->part_b};
  if ((rc = launch_row_inv<double, 3>(c, -1, rhs, spec))) return rc;
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(NT), 0, c->stream, c->st, c->part_b, c->nrow, 0, tol, maxit);
  HIPCHK(hipGetLastError());
  const CgCtl cc{c->st, c->part_a, c->part_rr, c->nrow, c->nrow, 0, 0};
  const VecCgPro<double, 3, StrainLaw> pro{P, R, {m}, c->nx, cc};
  const SymProj<double> pj{c->Dx, c->Dy, 1.0 / (double)n, c->st};
  const VecCgEpi<double, 3> epi{X, R, P, c->nx, cc};
  auto iter = [&]() -> int {
    int r = launch_row_fwd<double, 3>(c, FGCG_K_MECH_ROW_FWD, pro, spec);
    r |= launch_col<double, 3, 3>(c, FGCG_K_MECH_COL, pj, spec, spec);
    r |= launch_row_inv<double, 3>(c, FGCG_K_MECH_ROW_INV, epi, spec);
    return r;
  };
  Key key;
  key.add(m.phase).add(m.d).add(m.Efield).add(m.kappa).add(m.lam_per_E).add(m.mu_per_E).add(m.lm).add(c->gradop);
  key.add(tol).add(maxit);
  if ((rc = run_cg(c, 8, key, c->st, c->h_st, iter, maxit))) return rc;
  const CgState s = *c->h_st;
  hipLaunchKernelGGL(k_sf_post, dim3(c->npost), dim3(NT), 0, c->stream, m, (const double*)X.p, n, eig, em[0], em[1],
                     em[2], strain, stress, c->part_post);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_part, c->part_post, sizeof(double) * 4 * c->npost, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double acc[4] = {0, 0, 0, 0};
  for (int b = 0; b < c->npost; ++b)
    for (int j = 0; j < 4; ++j) acc[j] += c->h_part[4 * b + j];
  if (mean_stress)
    for (int j = 0; j < 3; ++j) mean_stress[j] = acc[j] / (double)n;
  if (energy) *energy = 0.5 * c->h * c->h * acc[3];
  fill_info(info, s, now() - t0);
  return status_of(s);
}

// The paths that need the forward difference's local stencil.
inline bool forward_only(const fgcg_ctx* c) { return c->gradop != 0; }

int upload_ems(fgcg_ctx* c, const double* em_host) {
  HIPCHK(hipMemcpyAsync(c->ems, em_host, sizeof(double) * 3 * c->nsamp, hipMemcpyHostToDevice, c->stream));
  return 0;
}

int mech_solve_single(fgcg_ctx* c, const MechMat& m, const double* eig, const double* em, double tol, int maxit,
                      double* strain, double* stress, double* mean_stress, double* energy, fgcg_info* info) {
  const double t0 = now();
  int rc;
  resolve_reference(c, m);
  if ((rc = tune_passes(c)) || (rc = upload_ems(c, em)) || (rc = mech_rhs(c, m, eig))) return rc;
  CgState s;
  if ((rc = mech_pcg(c, m, tol, maxit, &s))) return rc;
  double e;
  if ((rc = mech_post(c, m, eig, strain, stress, mean_stress, energy ? energy : &e))) return rc;
  fill_info(info, s, now() - t0);
  return status_of(s);
}

// Adjoint gradient dJ/dE_x (FP64): forward solve (strain recomputed), the
// objective's G = dJ/deps, a second PCG solve K lam = grad^H G (skipped for
// the energy, where lam = 0), and the gradient assembly.
int mech_adjoint_t(fgcg_ctx* c, const MechMat& m, const double* eig, const double* em, const double* dJ,
                   int objective, double tol, int maxit, double* grad, double* J, fgcg_info* info_fwd,
                   fgcg_info* info_adj) {
  double* strain = c->aux;
  double* G = c->aux + 3 * c->n;
  double mean[3], energy;
  int rc = mech_solve_single(c, m, eig, em, tol, maxit, strain, nullptr, mean, &energy, info_fwd);
  if (rc < 0) return rc;
  const int fwd_status = rc;
  const double N = (double)c->n;
  double scale = 0.0;
  if (objective == ADJ_ENERGY) scale = c->h * c->h;
  if (objective == ADJ_C11) scale = 1.0 / (N * em[0]);
  if (J) *J = objective == ADJ_ENERGY ? energy : (objective == ADJ_C11 ? mean[0] / em[0] : 0.0);
  if (!grad) {  // the objective only
    if (info_adj) std::memset(info_adj, 0, sizeof *info_adj);
    return fwd_status;
  }
  const double t0 = now();
  CgState s{};
  int have_lam = 0;
  if (objective != ADJ_ENERGY) {
    hipLaunchKernelGGL(k_adj_g, dim3(c->nkp), dim3(NT), 0, c->stream, m, (const double*)strain, eig, dJ, objective,
                       scale, c->n, G);
    hipLaunchKernelGGL(k_adj_rhs, dim3(c->nkp), dim3(NT), 0, c->stream, (const double*)G, (double*)c->r,
                       (double*)c->x, c->n, c->nx, c->ny, 1.0 / c->h);
    HIPCHK(hipGetLastError());
    if ((rc = mech_pcg(c, m, tol, maxit, &s))) return rc;
    have_lam = 1;
  } else {
    s.done = 1;
  }
  hipLaunchKernelGGL(k_adj_grad, dim3(c->nkp), dim3(NT), 0, c->stream, m, (const double*)strain, eig,
                     (const double*)c->x, objective, objective == ADJ_ENERGY ? c->h * c->h : scale, have_lam, c->n,
                     c->nx, c->ny, 1.0 / c->h, grad);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  fill_info(info_adj, s, now() - t0);
  const int adj_status = status_of(s);
  if (adj_status < 0) return adj_status;
  return (fwd_status == FGCG_NOT_CONVERGED || adj_status == FGCG_NOT_CONVERGED) ? FGCG_NOT_CONVERGED : FGCG_OK;
}

// ------------------------------------------------------------ phase field
template <typename T> struct PfApplyEpi {
  Field<T> v, q;
  const double* H;
  double a;
  int nx;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int xx, const T* l, double&, double) const {
    const long long i = (long long)y * nx + xx;
    q.at(s, 0, i) = (T)(a + H[i]) * v.at(s, 0, i) + l[0];
  }
  __device__ void partial(int, double) const {}
};

template <typename T>
int pf_solve_t(fgcg_ctx* c, const double* H, double Gc, double l0, double* d, double tol, int maxit,
               fgcg_info* info) {
  const double t0 = now();
  CT<T>* spec = (CT<T>*)c->spec;
  Field<T> X{(T*)c->x, c->n, 0}, R{(T*)c->r, c->n, 0}, P{(T*)c->p, c->n, 0};
  const double a = Gc / (2.0 * l0);
  const double cl = 0.5 * Gc * l0 / (double)c->n;
  int rc;
  hipLaunchKernelGGL((k_convert<T, double>), dim3(c->npost), dim3(PT), 0, c->stream, (T*)c->x, d, c->n);
  hipLaunchKernelGGL(k_norm2, dim3(c->npost), dim3(PT), 0, c->stream, H, c->n, c->part_b);
  // r = H - A x0
  CopyPro<T> cp{X, c->nx};
  if ((rc = launch_row_fwd<T, 1>(c, -1, cp, spec))) return rc;
  PfLap<T> lap0{c->Dx, c->Dy, cl, c->nx, nullptr, nullptr, 0, 0};
  if ((rc = launch_col<T, 1, 1>(c, -1, lap0, spec, spec))) return rc;
  PfResEpi<T> res{X, R, H, 0, a, c->nx, c->part_rr, 0};
  if ((rc = launch_row_inv<T, 1>(c, -1, res, spec))) return rc;
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(NT), 0, c->stream, c->st, c->part_b, c->npost, 0, tol, maxit);
  const CgCtl cc{c->st, c->part_a, c->part_rr, c->nrow + c->ncol, c->nrow, 0, 0};
  const PfCgPro<T> pro{P, R, H, 0, a, c->nx, cc};
  const PfLap<T> lap{c->Dx, c->Dy, cl, c->nx, c->st, c->part_a, 0, c->nrow};
  const PfCgEpi<T> epi{X, R, P, H, 0, a, c->nx, cc};
  auto iter = [&]() -> int {
    int r = launch_row_fwd<T, 1>(c, FGCG_K_PF_ROW_FWD, pro, spec);
    r |= launch_col<T, 1, 1>(c, FGCG_K_PF_COL, lap, spec, spec);
    r |= launch_row_inv<T, 1>(c, FGCG_K_PF_ROW_INV, epi, spec);
    return r;
  };
  Key key;
  key.add(H).add(a).add(cl);
  if ((rc = run_cg(c, 1, key, c->st, c->h_st, iter, maxit))) return rc;
  const CgState s = *c->h_st;
  if (s.zero_rhs) HIPCHK(hipMemsetAsync(c->x, 0, sizeof(T) * c->n, c->stream));
  hipLaunchKernelGGL((k_convert<double, T>), dim3(c->npost), dim3(PT), 0, c->stream, d, (const T*)c->x, c->n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  fill_info(info, s, now() - t0);
  return status_of(s);
}

// -------------------------------------------------------------- diffusion
template <typename T> struct DiffApplyEpi {
  Field<T> v, q;
  DiffCoef co;
  int nx;
  __device__ bool begin(int, double*, double&) const { return true; }
  __device__ void point(int s, int y, int xx, const T* l, double&, double) const {
    const long long i = (long long)y * nx + xx;
    double D, kr;
    pick(co.dk, co.phase[i], D, kr);
    q.at(s, 0, i) = (T)(co.inv_dt + kr) * v.at(s, 0, i) + l[0];
  }
  __device__ void partial(int, double) const {}
};

int make_diff_coef(const uint8_t* phase, int nphase, const double* D_tab, const double* k_tab, double dt,
                   int band, long long n, DiffCoef* co) {
  if (!phase || !D_tab || !k_tab) return fail(FGCG_EINVAL, "phase/D_tab/k_tab is NULL");
  if (nphase < 1 || nphase > FGCG_MAX_PHASES) return fail(FGCG_EINVAL, "nphase outside 1..8");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FGCG_EDOMAIN, "dt <= 0");
  std::memset(co, 0, sizeof *co);
  co->phase = phase;
  co->ss = n;
  co->inv_dt = 1.0 / dt;
  co->band = band;
  for (int i = 0; i < nphase; ++i) {
    if (!(D_tab[i] >= 0.0) || !std::isfinite(D_tab[i])) return fail(FGCG_EDOMAIN, "D < 0");
    if (!(k_tab[i] >= 0.0) || !std::isfinite(k_tab[i])) return fail(FGCG_EDOMAIN, "k < 0");
    co->dk.a[i] = D_tab[i];
    co->dk.b[i] = k_tab[i];
  }
  return 0;
}

template <typename T>
int diff_pipeline_apply(fgcg_ctx* c, const DiffCoef& co, CT<T>* spec, const CgState* st, double* part_mid,
                        int poff, const int* kinds) {
  const double inv_n = 1.0 / (double)c->n;
  int rc = 0;
  DiffGrad<T> grad{c->Dx, c->Dy, inv_n, st};
  rc |= launch_col<T, 1, 2>(c, kinds ? kinds[0] : -1, grad, spec, spec);
  DiffMid<T> mid{co, c->nx, st, part_mid, 0, poff};
  rc |= launch_row_mid<T, 2, 2>(c, kinds ? kinds[1] : -1, mid, spec);
  DiffDiv<T> div{c->Dx, c->Dy, inv_n, st};
  rc |= launch_col<T, 2, 1>(c, kinds ? kinds[2] : -1, div, spec, spec);
  return rc;
}

template <typename T>
int diff_step_t(fgcg_ctx* c, const DiffCoef& co, double c_dir, double* cfield, double tol, int maxit,
                fgcg_info* info) {
  const double t0 = now();
  CT<T>* spec = (CT<T>*)c->spec;
  Field<T> X{(T*)c->x, c->n, 0}, R{(T*)c->r, c->n, 0}, P{(T*)c->p, c->n, 0}, TM{(T*)c->tmp, c->n, 0};
  int rc;
  // b_F = M (c^n/dt - A c_B): only its norm is needed
  BandSrcPro<T> sb{nullptr, 0, co.band, c_dir, c->nx};
  if ((rc = launch_row_fwd<T, 1>(c, -1, sb, spec))) return rc;
  if ((rc = diff_pipeline_apply<T>(c, co, spec, nullptr, nullptr, 0, nullptr))) return rc;
  DiffResEpi<T> eb{TM, Field<T>{nullptr, c->n, 0}, cfield, nullptr, 0, co, c_dir, c->nx, c->part_b, 0};
  if ((rc = launch_row_inv<T, 1>(c, -1, eb, spec))) return rc;
  // r0 = M (c^n/dt - A c~), x0 = M c^n, c~ = c^n with the band set to c_dir
  BandSrcPro<T> sc{cfield, 0, co.band, c_dir, c->nx};
  if ((rc = launch_row_fwd<T, 1>(c, -1, sc, spec))) return rc;
  if ((rc = diff_pipeline_apply<T>(c, co, spec, nullptr, nullptr, 0, nullptr))) return rc;
  DiffResEpi<T> er{R, X, cfield, cfield, 0, co, c_dir, c->nx, c->part_rr, 0};
  if ((rc = launch_row_inv<T, 1>(c, -1, er, spec))) return rc;
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(NT), 0, c->stream, c->st, c->part_b, c->nrow, 0, tol, maxit);
  static const int kinds[3] = {FGCG_K_DIFF_COL_GRAD, FGCG_K_DIFF_ROW_MID, FGCG_K_DIFF_COL_DIV};
  const CgCtl cc{c->st, c->part_a, c->part_rr, 2 * c->nrow, c->nrow, 0, 0};
  const DiffCgPro<T> pro{P, R, co, c->nx, cc};
  const DiffCgEpi<T> epi{X, R, P, co, c->nx, cc};
  auto iter = [&]() -> int {
    int r = launch_row_fwd<T, 1>(c, FGCG_K_DIFF_ROW_FWD, pro, spec);
    r |= diff_pipeline_apply<T>(c, co, spec, c->st, c->part_a, c->nrow, kinds);
    r |= launch_row_inv<T, 1>(c, FGCG_K_DIFF_ROW_INV, epi, spec);
    return r;
  };
  Key key;
  key.add(co.phase).add(co.dk).add(co.inv_dt).add(co.band);
  if ((rc = run_cg(c, 2, key, c->st, c->h_st, iter, maxit))) return rc;
  const CgState s = *c->h_st;
  if (s.zero_rhs) HIPCHK(hipMemsetAsync(c->x, 0, sizeof(T) * c->n, c->stream));
  hipLaunchKernelGGL((k_diff_finish<T>), dim3(c->npost), dim3(PT), 0, c->stream, cfield, (const T*)c->x, c->n,
                     c->nx, co.band, c_dir);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  fill_info(info, s, now() - t0);
  return status_of(s);
}

// ------------------------------------------------- stencil scalar CG
template <typename T, class Op>
int scg_solve(fgcg_ctx* c, int which, const Key& key, const Op& op, const double* xin, double bscale,
              const double* bsrc, double c_dir, double tol, int maxit, int kind_dir, int kind_upd, CgState* out) {
  T* X = (T*)c->x;
  T* R = (T*)c->r;
  T* P0 = (T*)c->p;
  T* P1 = P0 + c->n;  // second direction buffer (p holds at least 2 components of room)
  T* Q = (T*)c->tmp;
  int parity = 0;     // iteration k reads P[k & 1] and writes P[(k + 1) & 1]
  const int nsb = (int)(c->sgrid.x * c->sgrid.y);
  hipLaunchKernelGGL((k_scg_init<T, Op>), c->sgrid, dim3(NT), 0, c->stream, op, xin, bscale, bsrc, c_dir, X, R,
                     c->nx, c->ny, c->nz, c->part_b, c->part_rr);
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(NT), 0, c->stream, c->st, c->part_b, nsb, 0, tol, maxit);
  HIPCHK(hipGetLastError());
  if (c->ndim == 2 && c->scg_onered) {
    // one-reduction form: x, p in the two components of x; r, w, s double-buffered
    // by iteration parity in r, p and tmp
    T* Px = X + c->n;
    T* Rb[2] = {R, R + c->n};
    T* Wb[2] = {P0, P1};
    T* Sb[2] = {Q, Q + c->n};
    const int np = std::min(scg_chunks(c->nx, c->ny, 1), 1024);
    Key k2 = key;
    k2.add(1);
    int rc = launch(c, -1, (const void*)&k_scg_cg<T, Op>, dim3(np), op, X, Px, (const T*)Rb[0], Rb[1],
                    (const T*)Wb[0], Wb[0], (const T*)Sb[0], Sb[1], c->nx, c->ny, c->st, c->part_a, np, 0, 1);
    if (rc) return rc;
    auto iter1 = [&]() -> int {
      set_kname(c, kind_dir, "k_scg_cg<%s%.0d", tname<T>(), 0);
      const int q = parity;
      parity ^= 1;
      return launch(c, kind_dir, (const void*)&k_scg_cg<T, Op>, dim3(np), op, X, Px, (const T*)Rb[q], Rb[q ^ 1],
                    (const T*)Wb[q], Wb[q ^ 1], (const T*)Sb[q], Sb[q ^ 1], c->nx, c->ny, c->st, c->part_a, np, q,
                    0);
    };
    if ((rc = run_cg(c, which, k2, c->st, c->h_st, iter1, maxit))) return rc;
    *out = c->h_st[0];
    return 0;
  }
  const int ndir = std::min(scg_chunks(c->nx, c->ny, c->nz), 2048);  // p.q partial sums in part_a
  const CgCtl cc{c->st, c->part_a, c->part_rr, ndir, nsb, 0, 0};
  auto iter = [&]() -> int {
    set_kname(c, kind_dir, "k_scg_dir<%s%.0d", tname<T>(), 0);
    set_kname(c, kind_upd, "k_scg_upd<%s%.0d", tname<T>(), 0);
    T* pin = parity ? P1 : P0;
    T* pout = parity ? P0 : P1;
    parity ^= 1;
    int r = launch(c, kind_dir, (const void*)&k_scg_dir<T, Op>, dim3(ndir), op, (const T*)R, (const T*)pin, pout, Q,
                   c->nx, c->ny, c->nz, cc);
    r |= launch(c, kind_upd, (const void*)&k_scg_upd<T>, c->sgrid, X, R, (const T*)pout, (const T*)Q, c->nx,
                c->rows, cc);
    return r;
  };
  int rc = run_cg(c, which, key, c->st, c->h_st, iter, maxit);
  if (rc) return rc;
  *out = c->h_st[0];
  return 0;
}

template <typename T>
int pf_solve_stencil(fgcg_ctx* c, const double* H, double Gc, double l0, double* d, double tol, int maxit,
                     fgcg_info* info) {
  const double t0 = now();
  const PfStencil op{H, Gc / (2.0 * l0), 0.5 * Gc * l0 / (c->h * c->h)};
  Key key;
  key.add(op.H).add(op.a).add(op.cih2);
  CgState s;
  int rc = scg_solve<T>(c, 3, key, op, d, 1.0, H, 0.0, tol, maxit, FGCG_K_PF_ROW_FWD, FGCG_K_PF_ROW_INV, &s);
  if (rc) return rc;
  if (s.zero_rhs) HIPCHK(hipMemsetAsync(c->x, 0, sizeof(T) * c->n, c->stream));
  hipLaunchKernelGGL((k_convert<double, T>), dim3(c->npost), dim3(PT), 0, c->stream, d, (const T*)c->x, c->n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  fill_info(info, s, now() - t0);
  return status_of(s);
}

// Diffusion step with the stencil CG; Op is DiffStencil (phase tables, band)
// or DiffFieldStencil (per-voxel fields, mask).  which: the graph slot.
template <typename T, class Op>
int diff_step_stencil(fgcg_ctx* c, const Op& op, double inv_dt, int which, const Key& key, double c_dir,
                      double* cfield, double tol, int maxit, fgcg_info* info) {
  const double t0 = now();
  CgState s;
  int rc = scg_solve<T>(c, which, key, op, cfield, inv_dt, cfield, c_dir, tol, maxit, FGCG_K_DIFF_ROW_FWD,
                        FGCG_K_DIFF_ROW_INV, &s);
  if (rc) return rc;
  if (s.zero_rhs) HIPCHK(hipMemsetAsync(c->x, 0, sizeof(T) * c->n, c->stream));
  hipLaunchKernelGGL((k_scg_finish<T, Op>), dim3(c->npost), dim3(NT), 0, c->stream, op, cfield, (const T*)c->x,
                     c->n, c->nx, c_dir);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  fill_info(info, s, now() - t0);
  return status_of(s);
}

template <typename T> int make_twiddles(int n, void** out) {
  std::vector<CT<T>> t(n);
  for (int k = 0; k < n; ++k) {
    const double th = 2.0 * M_PI * (double)k / (double)n;
    t[k] = CT<T>{(T)std::cos(th), (T)-std::sin(th)};
  }
  HIPCHK(hipMalloc(out, sizeof(CT<T>) * n));
  HIPCHK(hipMemcpy(*out, t.data(), sizeof(CT<T>) * n, hipMemcpyHostToDevice));
  return 0;
}

template <typename T> int alloc_workspace(fgcg_ctx* c) {
  const size_t ns = (size_t)c->nsamp;
  const size_t nr = sizeof(T) * c->ncw * (size_t)c->n * ns;
  HIPCHK(hipMalloc(&c->x, nr));
  HIPCHK(hipMalloc(&c->r, nr));
  HIPCHK(hipMalloc(&c->p, nr));
  HIPCHK(hipMalloc(&c->tmp, nr));
  HIPCHK(hipMalloc(&c->spec, sizeof(CT<T>) * c->ncw * (size_t)c->nxh * c->rows * ns));
  HIPCHK(hipMalloc(&c->ems, sizeof(double) * 3 * ns));
  if (c->batch) {
    HIPCHK(hipMalloc(&c->phase_buf, (size_t)c->n * ns));
    HIPCHK(hipMalloc(&c->strain_buf, sizeof(double) * 3 * (size_t)c->n * ns));
    HIPCHK(hipMalloc(&c->lm_dev, sizeof(double) * 16 * ns));
  }
  int rc;
  if ((rc = make_twiddles<double>(c->nx, &c->twx)) || (rc = make_twiddles<double>(c->ny, &c->twy))) return rc;
  if (c->prec == FGCG_FP32_MIXED) {
    if ((rc = make_twiddles<float>(c->nx, &c->twx32)) || (rc = make_twiddles<float>(c->ny, &c->twy32))) return rc;
    const size_t nu = c->ndim == 3 ? 3 : 2;  // displacement components
    HIPCHK(hipMalloc(&c->xh, sizeof(double) * nu * (size_t)c->n * ns));
    HIPCHK(hipMalloc(&c->fh, sizeof(double) * nu * (size_t)c->n * ns));
  } else if (ns == 1 && c->ndim == 2) {
    HIPCHK(hipMalloc(&c->aux, sizeof(double) * 6 * (size_t)c->n));
  }
  return 0;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* fgcg_strerror(int status) {
  switch (status) {
    case FGCG_OK: return "ok";
    case FGCG_NOT_CONVERGED: return "not converged within maxit";
    case FGCG_EINVAL: return "invalid argument";
    case FGCG_EDOMAIN: return "argument outside its domain";
    case FGCG_EBREAKDOWN: return "CG breakdown";
    case FGCG_ENOMEM: return "out of memory";
    case FGCG_EHIP: return "HIP runtime error";
    case FGCG_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* fgcg_last_error(void) { return g_err.c_str(); }

static int create_ctx(const fgcg_grid* grid, void* hip_stream, int nsamp, bool batch, fgcg_ctx** out);

int fgcg_create(const fgcg_grid* grid, void* hip_stream, fgcg_ctx** out) {
  return create_ctx(grid, hip_stream, 1, false, out);
}

static int create_ctx(const fgcg_grid* grid, void* hip_stream, int nsamp, bool batch, fgcg_ctx** out) {
  if (!grid || !out) return fail(FGCG_EINVAL, "grid/out is NULL");
  *out = nullptr;
  if (grid->ndim != 2 && grid->ndim != 3) return fail(FGCG_EINVAL, "ndim must be 2 or 3");
  if (grid->ndim == 3 && (nsamp != 1 || batch)) return fail(FGCG_EUNSUPPORTED, "batches are 2D");
  if (!(grid->h > 0.0) || !std::isfinite(grid->h)) return fail(FGCG_EDOMAIN, "h <= 0");
  if (grid->ndim == 2 && (!size_supported(grid->n[0]) || !size_supported(grid->n[1])))
    return fail(FGCG_EINVAL, "axis length must be one of 8..2048 of the form 2^a 3^b");
  if (grid->ndim == 3 &&
      (!size3_supported(grid->n[0]) || !size3_supported(grid->n[1]) || !size3_supported(grid->n[2])))
    return fail(FGCG_EINVAL, "3D axis length must be one of 8..512 of the form 2^a 3^b");
  if (grid->precision != FGCG_FP64 && grid->precision != FGCG_FP32_MIXED)
    return fail(FGCG_EINVAL, "unknown precision");
  fgcg_ctx* c = new fgcg_ctx();
  c->ndim = grid->ndim;
  c->nx = grid->n[0];
  c->ny = grid->n[1];
  c->nz = grid->ndim == 3 ? grid->n[2] : 1;
  c->rows = c->ny * c->nz;
  c->nxh = c->nx / 2 + 1;
  c->n = (long long)c->nx * c->rows;
  c->h = grid->h;
  c->prec = grid->precision;
  c->nsamp = nsamp;
  c->ncw = c->ndim == 3 ? 3 : 2;
  c->batch = batch;
  c->user_stream = (hipStream_t)hip_stream;
  {
    const char* ng = std::getenv("FGCG_NO_GRAPH");
    c->use_graphs = !(ng && ng[0] == '1');
  }
  with_n(c->nx, [&](auto NXc) {
    constexpr int R = rows_for(decltype(NXc)::value);
    c->nrow = (c->rows + R - 1) / R;
  });
  c->ncol = c->nxh;
  c->npost = (int)std::min<long long>((c->n + PT - 1) / PT, 1024);
  // slab-walking kernels: a multiple of 8 blocks (one slab per XCD)
  const auto slab_blocks = [&](long long cap) {
    return (int)std::max<long long>(8, std::min<long long>((c->n + NT - 1) / NT, cap) & ~7LL);
  };
  c->nkp = slab_blocks(1024);
  c->nkpt = std::min(kp_tiles(c->nx, c->rows), 1024);
  int rc = 0;
  auto chk = [&](hipError_t e) {
    if (e != hipSuccess && !rc) rc = fail(FGCG_ENOMEM, std::string("allocation failed: ") + hipGetErrorString(e));
  };
  chk(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  chk(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
  chk(hipEventCreateWithFlags(&c->ev_done[0], hipEventDisableTiming));
  chk(hipEventCreateWithFlags(&c->ev_done[1], hipEventDisableTiming));
  if (!rc) rc = alloc_workspace<double>(c);
  if (!rc) {
    chk(hipMalloc(&c->Dx, sizeof(double2) * c->nxh));
    chk(hipMalloc(&c->Dy, sizeof(double2) * c->ny));
    const size_t ns = (size_t)nsamp;
    chk(hipMalloc(&c->st, sizeof(CgState) * ns));
    chk(hipHostMalloc(&c->h_st, sizeof(CgState) * 2 * ns, hipHostMallocDefault));
    const int npa = std::max(std::max(c->nrow + std::max(c->ncol, c->nrow), c->nkp), 4096);
    chk(hipMalloc(&c->part_a, sizeof(double) * npa * ns));
    chk(hipMalloc(&c->part_rr, sizeof(double) * std::max(std::max(c->nrow, 2 * c->ncol), 512) * ns));
    chk(hipMalloc(&c->part_b, sizeof(double) * std::max(std::max(c->nrow, c->npost), 512)));
    // post-processing partials: 4-5 per block (2D), 7 per stencil block (3D, at most 1024 blocks)
    const size_t npp = std::max<size_t>(5 * (size_t)c->npost * ns, 7 * 1024);
    chk(hipMalloc(&c->part_post, sizeof(double) * npp));
    c->sgrid = dim3(slab_blocks(512));
    chk(hipHostMalloc(&c->h_part, sizeof(double) * npp, hipHostMallocDefault));
  }
  if (!rc) {
    // gradient symbols, the forward difference by default:
    // D(k) = (exp(i theta) - 1)/h = (-2 sin^2(theta/2) + i sin theta)/h
    const std::vector<double2> dx = grad_symbol(c->nx, c->h, 0), dy = grad_symbol(c->ny, c->h, 0);
    chk(hipMemcpy(c->Dx, dx.data(), sizeof(double2) * c->nxh, hipMemcpyHostToDevice));
    chk(hipMemcpy(c->Dy, dy.data(), sizeof(double2) * c->ny, hipMemcpyHostToDevice));
  }
  if (!rc && c->ndim == 3) rc = alloc3d(c);
  if (rc) {
    fgcg_destroy(c);
    return rc;
  }
  *out = c;
  return FGCG_OK;
}

void fgcg_destroy(fgcg_ctx* c) {
  if (!c) return;
  void* dev[] = {c->timing_E, c->rhat, c->p_odd, c->spec_q, c->sf_buf, c->sf_spec, c->lm_dev, c->ems,  c->phase_buf, c->strain_buf, c->twx,    c->twy,    c->twx32,  c->twy32, c->twz,
                 c->twz32, c->Dz,       c->red,        c->part_z, c->xh,     c->fh,     c->aux,   c->Dx,
                 c->Dy,   c->x,         c->r,          c->p,      c->tmp,    c->spec,   c->st,    c->part_a,
                 c->part_rr, c->part_b, c->part_post};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (c->h_st) (void)hipHostFree(c->h_st);
  if (c->h_part) (void)hipHostFree(c->h_part);
  for (auto& g : c->graphs) release_graph(c, g);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : {c->ev_in, c->ev_done[0], c->ev_done[1]})
    if (e) (void)hipEventDestroy(e);
  if (c->stream && c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int fgcg_set_stream(fgcg_ctx* c, void* s) {
  if (!c) return fail(FGCG_EINVAL, "ctx is NULL");
  c->user_stream = (hipStream_t)s;
  return FGCG_OK;
}

int fgcg_set_option(fgcg_ctx* c, int option, int value) {
  if (!c) return fail(FGCG_EINVAL, "ctx is NULL");
  switch (option) {
    case FGCG_OPT_SCALAR_SPECTRAL:
      c->scalar_spectral = value != 0;
      return FGCG_OK;
    case FGCG_OPT_GRAPHS:
      c->use_graphs = value != 0;
      return FGCG_OK;
    case FGCG_OPT_CHUNK:
      // even, so every chunk starts at an even iteration (double-buffered directions)
      if (value < 2 || value > 256 || (value & 1)) return fail(FGCG_EINVAL, "chunk must be even, 2..256");
      c->chunk = value;
      for (auto& g : c->graphs) release_graph(c, g);
      return FGCG_OK;
    case FGCG_OPT_ROWS: {
      if (c->ndim != 2) return fail(FGCG_EUNSUPPORTED, "rows per block are tuned on 2D grids");
      std::vector<int> cand;
      with_n(c->nx, [&](auto NXc) { cand = rows_candidates<decltype(NXc)::value>(); });
      if (value != 0 && std::find(cand.begin(), cand.end(), value) == cand.end())
        return fail(FGCG_EINVAL, "rows per block must be 0 or one of the candidates for this nx");
      c->rows_pick = value;
      return FGCG_OK;
    }
    case FGCG_OPT_GRADIENT:
    case FGCG_OPT_STRAIN_FORM: {
      const int top = option == FGCG_OPT_GRADIENT ? 3 : 1;
      if (value < 0 || value > top) return fail(FGCG_EINVAL, "gradient 0..3, strain form 0 or 1");
      if (c->batch) return fail(FGCG_EUNSUPPORTED, "batch groups take the forward difference");
      if (option == FGCG_OPT_GRADIENT && value != 0 && c->ndim == 3)
        return fail(FGCG_EUNSUPPORTED, "3D grids take the forward difference");
      if (option == FGCG_OPT_STRAIN_FORM && value != 0 && c->ndim == 3)
        return fail(FGCG_EUNSUPPORTED, "the strain form is 2D");
      const int grad = option == FGCG_OPT_GRADIENT ? value : c->gradop;
      const int sf = option == FGCG_OPT_STRAIN_FORM ? value : c->strain_form;
      if ((grad != 0 || sf) && !c->sf_buf) {
        // the strain form's own workspace: x, r, p of 3 components and 3 spectra
        if (hipMalloc(&c->sf_buf, sizeof(double) * 9 * (size_t)c->n) != hipSuccess ||
            hipMalloc(&c->sf_spec, sizeof(double2) * 3 * (size_t)c->nxh * c->ny) != hipSuccess)
          return fail(FGCG_ENOMEM, "strain-form workspace");
      }
      if (option == FGCG_OPT_GRADIENT && value != c->gradop) {
        const std::vector<double2> dx = grad_symbol(c->nx, c->h, value), dy = grad_symbol(c->ny, c->h, value);
        HIPCHK(hipMemcpy(c->Dx, dx.data(), sizeof(double2) * c->nxh, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->Dy, dy.data(), sizeof(double2) * c->ny, hipMemcpyHostToDevice));
        for (auto& g : c->graphs) release_graph(c, g);
      }
      (option == FGCG_OPT_GRADIENT ? c->gradop : c->strain_form) = value;
      return FGCG_OK;
    }
    case FGCG_OPT_SPECTRAL_RES:
      if (value != 0 && value != 1) return fail(FGCG_EINVAL, "spectral residual must be 0 or 1");
      c->sr_opt = value;
      return FGCG_OK;
    case FGCG_OPT_MECH_PASSES:
      return fail(FGCG_EINVAL, "the number of mechanics passes is read-only");
    case FGCG_OPT_MECH_FORM: {
      if (value != 0 && (value < 2 || value > 4)) return fail(FGCG_EINVAL, "mechanics form 0 (tune), 2, 3 or 4");
      if (value != 0 && value != 4 && !sr_eligible(c))
        return fail(FGCG_EUNSUPPORTED, "the residual-spectrum forms need a 2D FP64 context with nx a multiple of 64");
      if (value == 3 && !sr3_ok(c)) return fail(FGCG_EUNSUPPORTED, "the three-pass form needs nx a multiple of 256");
      const int pick = value == 0 ? 0 : value == 2 ? 3 : value == 3 ? 1 : 2;
      if (pick != c->sr_pick) {
        c->sr_pick = pick;
        c->rows_pick = c->plan_row = c->plan_col = 0;  // the passes change: tune them again
      }
      return FGCG_OK;
    }
    case FGCG_OPT_SCALAR_CG:
      if (value != 0 && value != 1) return fail(FGCG_EINVAL, "scalar CG form must be 0 or 1");
      c->scg_onered = value;
      return FGCG_OK;
    case FGCG_OPT_PRECOND:
      if (value != 0 && value != 1) return fail(FGCG_EINVAL, "preconditioner must be 0 (unit) or 1 (reference)");
      if (c->batch) return fail(FGCG_EUNSUPPORTED, "batch groups take the unit Green operator");
      if (value != c->precond && c->ndim == 2) c->plan_col = 0;  // the column pass changes: tune it again
      c->precond = value;
      return FGCG_OK;
    case FGCG_OPT_ROW_SPLIT:
    case FGCG_OPT_ZTILES: {
      if (c->ndim != 3) return fail(FGCG_EUNSUPPORTED, "row splits and z tiles are tuned on 3D grids");
      const int top = option == FGCG_OPT_ROW_SPLIT ? 4 : 2;
      if (value < 0 || value > top) return fail(FGCG_EINVAL, "row split 0..4, z tiles 0..2");
      int& v = option == FGCG_OPT_ROW_SPLIT ? c->split3 : c->zpt_pick;
      if (v != value)
        for (auto& g : c->graphs) release_graph(c, g);  // captured launches use the old choice
      v = value;
      return FGCG_OK;
    }
    case FGCG_OPT_ROW_PLAN:
    case FGCG_OPT_COL_PLAN:
      if (c->ndim != 2) return fail(FGCG_EUNSUPPORTED, "radix plans are tuned on 2D grids");
      if (value < 0 || value > (option == FGCG_OPT_COL_PLAN ? 3 : 2))
        return fail(FGCG_EINVAL, "plan must be 0 (tune), 1 or 2 (3 for the column pass)");
      (option == FGCG_OPT_ROW_PLAN ? c->plan_row : c->plan_col) = value;
      return FGCG_OK;
    default:
      return fail(FGCG_EINVAL, "unknown option");
  }
}

int fgcg_set_reference(fgcg_ctx* c, double lam0, double mu0) {
  if (!c) return fail(FGCG_EINVAL, "ctx is NULL");
  const bool automatic = lam0 == 0.0 && mu0 == 0.0;
  if (!automatic && !(mu0 > 0.0 && lam0 > -2.0 * mu0 / 3.0 && std::isfinite(lam0) && std::isfinite(mu0)))
    return fail(FGCG_EDOMAIN, "reference medium needs mu0 > 0 and a positive bulk modulus");
  c->ref_lam = lam0;
  c->ref_mu = mu0;
  return FGCG_OK;
}

int fgcg_get_option(fgcg_ctx* c, int option, int* value) {
  if (!c || !value) return fail(FGCG_EINVAL, "ctx/value is NULL");
  switch (option) {
    case FGCG_OPT_SCALAR_SPECTRAL: *value = c->scalar_spectral; return FGCG_OK;
    case FGCG_OPT_GRAPHS: *value = c->use_graphs ? 1 : 0; return FGCG_OK;
    case FGCG_OPT_CHUNK: *value = c->chunk; return FGCG_OK;
    case FGCG_OPT_ROWS: *value = c->rows_pick; return FGCG_OK;
    case FGCG_OPT_ROW_PLAN: *value = c->plan_row; return FGCG_OK;
    case FGCG_OPT_COL_PLAN: *value = c->plan_col; return FGCG_OK;
    case FGCG_OPT_PRECOND: *value = c->precond; return FGCG_OK;
    case FGCG_OPT_GRADIENT: *value = c->gradop; return FGCG_OK;
    case FGCG_OPT_STRAIN_FORM: *value = c->strain_form; return FGCG_OK;
    case FGCG_OPT_SPECTRAL_RES: *value = c->sr_opt; return FGCG_OK;
    case FGCG_OPT_SCALAR_CG: *value = c->scg_onered; return FGCG_OK;
    case FGCG_OPT_MECH_PASSES: *value = c->ndim != 2 ? 0 : (fused_active(c) ? 2 : sr_active(c) ? 3 : 4); return FGCG_OK;
    case FGCG_OPT_MECH_FORM:
      *value = c->ndim != 2 || !sr_eligible(c) ? (c->ndim == 2 ? 4 : 0)
                                                : (c->sr_pick == 0 ? 0 : c->sr_pick == 3 ? 2 : c->sr_pick == 1 ? 3 : 4);
      return FGCG_OK;
    case FGCG_OPT_ROW_SPLIT: *value = c->split3; return FGCG_OK;
    case FGCG_OPT_ZTILES: *value = c->zpt_pick; return FGCG_OK;
    default: return fail(FGCG_EINVAL, "unknown option");
  }
}

int fgcg_mech_solve(fgcg_ctx* c, const fgcg_material* mat, const double* d, double kappa, const double* eig,
                    const double* eps_mac, double tol, int maxit, double* strain, double* stress,
                    double* mean_stress, double* energy, fgcg_info* info) {
  if (!c || !eps_mac || !strain) return fail(FGCG_EINVAL, "ctx/eps_mac/strain is NULL");
  int rc;
  if ((rc = check_solver_args(tol, maxit))) return rc;
  const int ns = c->ndim == 3 ? 6 : 3;
  for (int j = 0; j < ns; ++j)
    if (!std::isfinite(eps_mac[j])) return fail(FGCG_EDOMAIN, "eps_mac not finite");
  MechMat m;
  if ((rc = make_mech_mat(c, mat, d, kappa, &m))) return rc;
  if ((rc = enter(c))) return rc;
  if (c->ndim == 3) {
    if (m.Efield) return fail(FGCG_EUNSUPPORTED, "per-voxel E fields are 2D only");
    if (c->gradop != 0 || c->strain_form) return fail(FGCG_EUNSUPPORTED, "3D mechanics takes the forward difference");
    return mech3_solve(c, m, eig, eps_mac, tol, maxit, strain, stress, mean_stress, energy, info);
  }
  if (c->gradop != 0 || c->strain_form) {
    if (c->prec != FGCG_FP64) return fail(FGCG_EUNSUPPORTED, "the strain-form solver runs in FP64 contexts");
    return mech_sf_solve(c, m, eig, eps_mac, tol, maxit, strain, stress, mean_stress, energy, info);
  }
  return mech_solve_single(c, m, eig, eps_mac, tol, maxit, strain, stress, mean_stress, energy, info);
}

int fgcg_mech_adjoint(fgcg_ctx* c, const fgcg_material* mat, const double* d, double kappa, const double* eig,
                      const double* eps_mac, const double* dJ_dstrain, int objective, double tol, int maxit,
                      double* grad_E, double* J, fgcg_info* info_fwd, fgcg_info* info_adj) {
  if (!c || !eps_mac) return fail(FGCG_EINVAL, "ctx/eps_mac is NULL");
  if (c->prec != FGCG_FP64) return fail(FGCG_EUNSUPPORTED, "the adjoint runs in FP64 contexts");
  if (c->ndim != 2) return fail(FGCG_EUNSUPPORTED, "the adjoint is 2D only");
  if (objective != ADJ_USER && objective != ADJ_ENERGY && objective != ADJ_C11)
    return fail(FGCG_EINVAL, "unknown objective");
  if (objective == ADJ_USER && !dJ_dstrain) return fail(FGCG_EINVAL, "dJ_dstrain is NULL");
  if (forward_only(c) || c->strain_form) return fail(FGCG_EUNSUPPORTED, "the adjoint takes the forward difference");
  if (objective == ADJ_C11 && !(eps_mac[0] != 0.0)) return fail(FGCG_EDOMAIN, "C11 needs eps_mac[0] != 0");
  int rc;
  if ((rc = check_solver_args(tol, maxit))) return rc;
  MechMat m;
  if ((rc = make_mech_mat(c, mat, d, kappa, &m))) return rc;
  if ((rc = enter(c))) return rc;
  return mech_adjoint_t(c, m, eig, eps_mac, dJ_dstrain, objective, tol, maxit, grad_E, J, info_fwd, info_adj);
}

int fgcg_phasefield_solve(fgcg_ctx* c, const double* H, double Gc, double l0, double* d, double tol, int maxit,
                          fgcg_info* info) {
  if (!c || !H || !d) return fail(FGCG_EINVAL, "ctx/H/d is NULL");
  int rc;
  if ((rc = check_solver_args(tol, maxit))) return rc;
  if (!(Gc > 0.0) || !std::isfinite(Gc)) return fail(FGCG_EDOMAIN, "Gc <= 0");
  if (!(l0 > 0.0) || !std::isfinite(l0)) return fail(FGCG_EDOMAIN, "l0 <= 0");
  if ((rc = enter(c))) return rc;
  const bool spectral = c->scalar_spectral || forward_only(c);
  if (spectral && c->ndim == 3) return fail(FGCG_EUNSUPPORTED, "spectral scalar operators are 2D only");
  if (!spectral) return pf_solve_stencil<double>(c, H, Gc, l0, d, tol, maxit, info);
  return pf_solve_t<double>(c, H, Gc, l0, d, tol, maxit, info);
}

int fgcg_diffusion_step_phases(fgcg_ctx* c, const uint8_t* phase, int nphase, const double* D_tab,
                               const double* k_tab, int band_width, double c_dir, double dt, double* cfield,
                               double tol, int maxit, fgcg_info* info) {
  if (!c || !cfield) return fail(FGCG_EINVAL, "ctx/c is NULL");
  int rc;
  if ((rc = check_solver_args(tol, maxit))) return rc;
  if (band_width < 0 || band_width >= c->nx) return fail(FGCG_EINVAL, "band_width outside [0, nx)");
  if (!std::isfinite(c_dir)) return fail(FGCG_EDOMAIN, "c_dir not finite");
  DiffCoef co;
  if ((rc = make_diff_coef(phase, nphase, D_tab, k_tab, dt, band_width, c->n, &co))) return rc;
  if ((rc = enter(c))) return rc;
  const bool spectral = c->scalar_spectral || forward_only(c);
  if (spectral && c->ndim == 3) return fail(FGCG_EUNSUPPORTED, "spectral scalar operators are 2D only");
  if (!spectral) {
    const DiffStencil op{co, co.phase, 1.0 / (c->h * c->h)};
    Key key;
    key.add(co.phase).add(co.dk).add(co.inv_dt).add(co.band).add(op.ih2);
    return diff_step_stencil<double>(c, op, co.inv_dt, 4, key, c_dir, cfield, tol, maxit, info);
  }
  return diff_step_t<double>(c, co, c_dir, cfield, tol, maxit, info);
}

int fgcg_diffusion_step(fgcg_ctx* c, double* cfield, const double* Dfield, const double* krate,
                        const uint8_t* dirichlet_mask, double c_dir, double dt, double tol, int maxit,
                        fgcg_info* info) {
  if (!c || !cfield || !Dfield) return fail(FGCG_EINVAL, "ctx/c/D is NULL");
  int rc;
  if ((rc = check_solver_args(tol, maxit))) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FGCG_EDOMAIN, "dt <= 0");
  if (!std::isfinite(c_dir)) return fail(FGCG_EDOMAIN, "c_dir not finite");
  if (forward_only(c)) return fail(FGCG_EUNSUPPORTED, "the per-voxel diffusion step takes the forward difference");
  if ((rc = enter(c))) return rc;
  const DiffFieldStencil op{Dfield, krate, dirichlet_mask, 1.0 / dt, 1.0 / (c->h * c->h)};
  Key key;
  key.add(op.D).add(op.kr).add(op.mask).add(op.inv_dt).add(op.ih2);
  return diff_step_stencil<double>(c, op, op.inv_dt, 6, key, c_dir, cfield, tol, maxit, info);
}

int fgcg_staggered_step(fgcg_ctx* c, fgcg_state* s, const fgcg_params* p, fgcg_step_info* info) {
  if (!c || !s || !p || !info) return fail(FGCG_EINVAL, "ctx/state/params/info is NULL");
  if (!s->c || !s->f || !s->e || !s->H || !s->d || !s->strain) return fail(FGCG_EINVAL, "state field is NULL");
  if (!p->mat.phase) return fail(FGCG_EINVAL, "params.mat.phase is NULL");
  if (!(p->dt > 0.0)) return fail(FGCG_EDOMAIN, "dt <= 0");
  std::memset(info, 0, sizeof *info);
  int rc;
  if ((rc = enter(c))) return rc;
  if (p->diffuse) {
    rc = fgcg_diffusion_step_phases(c, p->mat.phase, p->mat.nphase, p->D_tab, p->k_tab, p->band_width, p->c_dir,
                                    p->dt, s->c, p->tol_diff, p->maxit, &info->diff);
    if (rc < 0) return rc;
  }
  const double e_pres = p->n_ramp > 0 ? p->e_ramp * (double)(s->step + 1) / (double)p->n_ramp : 0.0;
  PhaseTab dtk{};
  if (p->diffuse && p->k_tab)
    for (int i = 0; i < p->mat.nphase && i < FGCG_MAX_PHASES; ++i) dtk.a[i] = p->dt * p->k_tab[i];
  hipLaunchKernelGGL(k_precip, dim3(c->npost), dim3(PT), 0, c->stream, p->mat.phase, s->c, s->f, s->e, c->n, dtk,
                     p->e_per_f, p->diffuse, e_pres);
  HIPCHK(hipGetLastError());
  rc = fgcg_mech_solve(c, &p->mat, s->d, p->kappa, s->e, p->eps_mac, p->tol_mech, p->maxit, s->strain, nullptr,
                       info->mean_stress, &info->energy, &info->mech);
  if (rc < 0) return rc;
  MechMat m0;
  if ((rc = make_mech_mat(c, &p->mat, nullptr, 0.0, &m0))) return rc;
  if (c->ndim == 3) {
    if ((rc = history3(c, m0, s->strain, s->e, s->H))) return rc;
  } else {
    hipLaunchKernelGGL(k_history, dim3(c->npost), dim3(PT), 0, c->stream, m0, s->strain, s->e, s->H, c->n);
    HIPCHK(hipGetLastError());
  }
  rc = fgcg_phasefield_solve(c, s->H, p->Gc, p->l0, s->d, p->tol_pf, p->maxit, &info->pf);
  if (rc < 0) return rc;
  hipLaunchKernelGGL(k_observe, dim3(c->npost), dim3(PT), 0, c->stream, p->mat.phase, s->d, s->f, c->n,
                     c->part_post);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_part, c->part_post, sizeof(double) * 5 * c->npost, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double mx = 0, cnt = 0, sd = 0, sf = 0, ns = 0;
  for (int b = 0; b < c->npost; ++b) {
    mx = std::max(mx, c->h_part[5 * b]);
    cnt += c->h_part[5 * b + 1];
    sd += c->h_part[5 * b + 2];
    sf += c->h_part[5 * b + 3];
    ns += c->h_part[5 * b + 4];
  }
  info->max_d = mx;
  info->damaged_fraction = ns > 0 ? cnt / ns : 0.0;
  info->porosity_increase = sd / (double)c->n;
  info->total_precipitate = sf;
  s->step += 1;
  int worst = FGCG_OK;
  for (const fgcg_info* i : {&info->diff, &info->mech, &info->pf})
    if (i->status == FGCG_NOT_CONVERGED) worst = FGCG_NOT_CONVERGED;
  return worst;
}

int fgcg_debug_apply(fgcg_ctx* c, int op, const fgcg_material* mat, const double* d, double kappa,
                     const double* in, double* out) {
  if (!c || !in || !out) return fail(FGCG_EINVAL, "ctx/in/out is NULL");
  if (op != FGCG_OP_MECH_K && op != FGCG_OP_MECH_M) return fail(FGCG_EINVAL, "unknown operator");
  if (forward_only(c)) return fail(FGCG_EUNSUPPORTED, "the solver operators take the forward difference");
  MechMat m;
  int rc;
  if ((rc = make_mech_mat(c, mat, d, kappa, &m))) return rc;
  if (c->ndim == 3 && m.Efield) return fail(FGCG_EUNSUPPORTED, "per-voxel E fields are 2D only");
  if ((rc = enter(c))) return rc;
  if (c->ndim == 3) rc = debug_apply3(c, op, m, in, out);
  else rc = c->prec == FGCG_FP64 ? debug_apply_t<double>(c, op, m, in, out) : debug_apply_t<float>(c, op, m, in, out);
  if (rc) return rc;
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return FGCG_OK;
}

int fgcg_phasefield_apply(fgcg_ctx* c, const double* H, double Gc, double l0, const double* v, double* q) {
  if (!c || !H || !v || !q) return fail(FGCG_EINVAL, "ctx/H/v/q is NULL");
  if (c->ndim != 2) return fail(FGCG_EUNSUPPORTED, "the apply hooks are 2D only");
  if (!(Gc > 0.0) || !(l0 > 0.0)) return fail(FGCG_EDOMAIN, "Gc/l0 <= 0");
  CT<double>* spec = (CT<double>*)c->spec;
  int rc;
  if ((rc = enter(c))) return rc;
  CopyPro<double> cp{Field<double>{(double*)v, c->n, 0}, c->nx};
  if ((rc = launch_row_fwd<double, 1>(c, -1, cp, spec))) return rc;
  PfLap<double> lap{c->Dx, c->Dy, 0.5 * Gc * l0 / (double)c->n, c->nx, nullptr, nullptr, 0, 0};
  if ((rc = launch_col<double, 1, 1>(c, -1, lap, spec, spec))) return rc;
  PfApplyEpi<double> ep{Field<double>{(double*)v, c->n, 0}, Field<double>{q, c->n, 0}, H, Gc / (2.0 * l0), c->nx};
  if ((rc = launch_row_inv<double, 1>(c, -1, ep, spec))) return rc;
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return FGCG_OK;
}

int fgcg_diffusion_apply(fgcg_ctx* c, const uint8_t* phase, int nphase, const double* D_tab, const double* k_tab,
                         double dt, const double* v, double* q) {
  if (!c || !v || !q) return fail(FGCG_EINVAL, "ctx/v/q is NULL");
  if (c->ndim != 2) return fail(FGCG_EUNSUPPORTED, "the apply hooks are 2D only");
  DiffCoef co;
  int rc;
  if ((rc = make_diff_coef(phase, nphase, D_tab, k_tab, dt, 0, c->n, &co))) return rc;
  if ((rc = enter(c))) return rc;
  CT<double>* spec = (CT<double>*)c->spec;
  CopyPro<double> cp{Field<double>{(double*)v, c->n, 0}, c->nx};
  if ((rc = launch_row_fwd<double, 1>(c, -1, cp, spec))) return rc;
  if ((rc = diff_pipeline_apply<double>(c, co, spec, nullptr, nullptr, 0, nullptr))) return rc;
  DiffApplyEpi<double> ep{Field<double>{(double*)v, c->n, 0}, Field<double>{q, c->n, 0}, co, c->nx};
  if ((rc = launch_row_inv<double, 1>(c, -1, ep, spec))) return rc;
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return FGCG_OK;
}

int fgcg_debug_fft(fgcg_ctx* c, int dir, const double* in, double* out) {
  if (!c || !in || !out) return fail(FGCG_EINVAL, "ctx/in/out is NULL");
  if (dir == 0) return fail(FGCG_EINVAL, "dir must be nonzero");
  int rc;
  if ((rc = enter(c))) return rc;
  return debug_fft(c, dir, in, out);
}

int fgcg_time_pass(fgcg_ctx* c, int kind, int reps, double* us_per_launch) {
  if (!c || !us_per_launch) return fail(FGCG_EINVAL, "ctx/us_per_launch is NULL");
  if (c->ndim != 2) return fail(FGCG_EUNSUPPORTED, "pass timing covers the 2D mechanics passes");
  if (kind != FGCG_K_MECH_ROW_FWD && kind != FGCG_K_MECH_ROW_INV && kind != FGCG_K_MECH_COL)
    return fail(FGCG_EINVAL, "kind must be FGCG_K_MECH_ROW_FWD, _ROW_INV or _COL");
  if (reps < 1 || reps > 100000) return fail(FGCG_EINVAL, "reps must be 1..100000");
  int rc;
  if ((rc = enter(c)) || (rc = tune_passes(c))) return rc;
  rc = c->prec == FGCG_FP64 ? time_pass_t<double>(c, kind, reps, us_per_launch)
                            : time_pass_t<float>(c, kind, reps, us_per_launch);
  if (rc) return rc;
  HIPCHK(hipGetLastError());
  return FGCG_OK;
}

int fgcg_profile(fgcg_ctx* c, unsigned mask) {
  if (!c) return fail(FGCG_EINVAL, "ctx is NULL");
  HIPCHK(hipStreamSynchronize(c->stream));
  int rc = prof_flush(c);
  if (rc) return rc;
  c->prof_mask = mask;
  for (int k = 0; k < FGCG_K_NKINDS; ++k) {
    c->prof_ms[k] = 0;
    c->prof_n[k] = 0;
  }
  return FGCG_OK;
}

int fgcg_profile_read(fgcg_ctx* c, int kind, double* ms, long long* launches) {
  if (!c || kind < 0 || kind >= FGCG_K_NKINDS) return fail(FGCG_EINVAL, "bad ctx/kind");
  HIPCHK(hipStreamSynchronize(c->stream));
  int rc = prof_flush(c);
  if (rc) return rc;
  if (ms) *ms = c->prof_ms[kind];
  if (launches) *launches = c->prof_n[kind];
  return FGCG_OK;
}

const char* fgcg_kernel_name(fgcg_ctx* c, int kind) {
  if (!c || kind < 0 || kind >= FGCG_K_NKINDS) return "";
  return c->kname[kind].c_str();
}


// ------------------------------------------------------------ batches
struct fgcg_batch {
  int nb = 0;
  std::vector<fgcg_ctx*> groups;
  std::vector<std::vector<int>> members;  // sample ids of each group
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::vector<char> key;
  hipEvent_t ev_done[2] = {nullptr, nullptr};
};

void fgcg_batch_destroy(fgcg_batch* b) {
  if (!b) return;
  for (auto& e : b->exec)
    if (e) (void)hipGraphExecDestroy(e);
  for (auto& e : b->ev_done)
    if (e) (void)hipEventDestroy(e);
  for (fgcg_ctx* c : b->groups) fgcg_destroy(c);
  delete b;
}

int fgcg_batch_create(int nb, const int* nx, const int* ny, double h, int precision, void* hip_stream,
                      fgcg_batch** out) {
  if (!out || !nx || !ny || nb < 1) return fail(FGCG_EINVAL, "nb < 1 or NULL arrays");
  *out = nullptr;
  fgcg_batch* b = new fgcg_batch();
  b->nb = nb;
  std::vector<std::pair<int, int>> sizes;
  for (int i = 0; i < nb; ++i) {
    int g = -1;
    for (size_t k = 0; k < sizes.size(); ++k)
      if (sizes[k].first == nx[i] && sizes[k].second == ny[i]) g = (int)k;
    if (g < 0) {
      sizes.push_back({nx[i], ny[i]});
      b->members.push_back({});
      g = (int)sizes.size() - 1;
    }
    b->members[g].push_back(i);
  }
  int rc = 0;
  for (size_t g = 0; g < sizes.size() && !rc; ++g) {
    fgcg_grid grid{2, {sizes[g].first, sizes[g].second, 1}, h, precision};
    fgcg_ctx* c = nullptr;
    rc = create_ctx(&grid, hip_stream, (int)b->members[g].size(), true, &c);
    if (!rc) {
      if (g > 0) {  // every group runs on the first group's stream
        (void)hipStreamDestroy(c->stream);
        c->stream = b->groups[0]->stream;
        c->own_stream = false;
      }
      b->groups.push_back(c);
    }
  }
  if (!rc && hipEventCreateWithFlags(&b->ev_done[0], hipEventDisableTiming) != hipSuccess) rc = FGCG_EHIP;
  if (!rc && hipEventCreateWithFlags(&b->ev_done[1], hipEventDisableTiming) != hipSuccess) rc = FGCG_EHIP;
  if (rc) {
    fgcg_batch_destroy(b);
    return rc;
  }
  *out = b;
  return FGCG_OK;
}

int fgcg_mech_solve_batched(fgcg_batch* b, const uint8_t* const* phases, int nphase, const double* E_tab,
                            const double* nu_tab, const double* eps_mac, double tol, int maxit,
                            double* const* strains, double* mean_stress, double* energy, fgcg_info* infos) {
  if (!b || !phases || !eps_mac || !E_tab || !nu_tab) return fail(FGCG_EINVAL, "batch/phases/tables/eps_mac is NULL");
  int rc;
  if ((rc = check_solver_args(tol, maxit))) return rc;
  if (nphase < 1 || nphase > FGCG_MAX_PHASES) return fail(FGCG_EINVAL, "nphase outside 1..8");
  for (int i = 0; i < b->nb; ++i)
    if (!phases[i]) return fail(FGCG_EINVAL, "phase pointer is NULL");
  const double t0 = now();
  fgcg_ctx* c0 = b->groups[0];
  hipStream_t st = c0->stream;
  if ((rc = enter(c0))) return rc;
  std::vector<MechMat> mats(b->groups.size());
  std::vector<std::vector<double>> lm_host(b->groups.size());
  for (size_t g = 0; g < b->groups.size(); ++g) {
    fgcg_ctx* c = b->groups[g];
    const std::vector<int>& mem = b->members[g];
    // tables of the group's first sample go into the kernel arguments; when the
    // members' tables differ, each sample's table is read from device memory
    fgcg_material mat{c->phase_buf, nphase, E_tab + (size_t)nphase * mem[0], nu_tab + (size_t)nphase * mem[0],
                      nullptr, 0.0};
    if ((rc = make_mech_mat(c, &mat, nullptr, 0.0, &mats[g]))) return rc;
    bool same = true;
    std::vector<double>& lh = lm_host[g];
    lh.assign(16 * mem.size(), 0.0);
    for (size_t s = 0; s < mem.size(); ++s) {
      MechMat ms;
      fgcg_material mi{c->phase_buf, nphase, E_tab + (size_t)nphase * mem[s], nu_tab + (size_t)nphase * mem[s],
                       nullptr, 0.0};
      if ((rc = make_mech_mat(c, &mi, nullptr, 0.0, &ms))) return rc;
      for (int q = 0; q < FGCG_MAX_PHASES; ++q) {
        lh[16 * s + q] = ms.lm.a[q];
        lh[16 * s + 8 + q] = ms.lm.b[q];
        same = same && ms.lm.a[q] == mats[g].lm.a[q] && ms.lm.b[q] == mats[g].lm.b[q];
      }
    }
    if (!same) {
      HIPCHK(hipMemcpyAsync(c->lm_dev, lh.data(), sizeof(double) * lh.size(), hipMemcpyHostToDevice, st));
      mats[g].lm_dev = c->lm_dev;
    }
    std::vector<double> em(3 * mem.size());
    for (size_t s = 0; s < mem.size(); ++s) {
      HIPCHK(hipMemcpyAsync(c->phase_buf + (size_t)c->n * s, phases[mem[s]], (size_t)c->n, hipMemcpyDeviceToDevice,
                            st));
      for (int j = 0; j < 3; ++j) em[3 * s + j] = eps_mac[3 * mem[s] + j];
    }
    resolve_reference(c, mats[g]);
    if ((rc = tune_passes(c)) || (rc = upload_ems(c, em.data())) || (rc = mech_rhs(c, mats[g], nullptr))) return rc;
    rc = c->prec == FGCG_FP64 ? mech_init<double>(c, mats[g], tol, maxit) : mech_init<float>(c, mats[g], tol, maxit);
    if (rc) return rc;
  }
  auto all_done = [&](int slot) {
    for (fgcg_ctx* c : b->groups)
      for (int s = 0; s < c->nsamp; ++s)
        if (!c->h_st[slot * c->nsamp + s].done) return false;
    return true;
  };
  auto copy_states = [&](int slot) -> int {
    for (fgcg_ctx* c : b->groups)
      HIPCHK(hipMemcpyAsync(c->h_st + slot * c->nsamp, c->st, sizeof(CgState) * c->nsamp, hipMemcpyDeviceToHost, st));
    return 0;
  };
  if ((rc = copy_states(0))) return rc;
  HIPCHK(hipStreamSynchronize(st));
  int last = 0;
  if (!all_done(0)) {
    const int K = c0->prec == FGCG_FP64 ? c0->chunk : 2 * RELIABLE_EVERY;
    Key key = mech_key(c0, mats[0], tol, maxit);
    key.add(K);
    for (const MechMat& mg : mats) key.add(mg.lm).add(mg.lm_dev);
    for (fgcg_ctx* cg : b->groups) key.add(cg->rows_pick).add(cg->plan_row).add(cg->plan_col);
    if (key.b != b->key || !b->exec[0] || !b->exec[1]) {
      for (auto& e : b->exec)
        if (e) (void)hipGraphExecDestroy(e);
      b->exec[0] = b->exec[1] = nullptr;
      for (int i = 0; i < 2; ++i) {
        hipGraph_t graph;
        HIPCHK(hipGraphCreate(&graph, 0));
        for (size_t g = 0; g < b->groups.size() && !rc; ++g) {
          fgcg_ctx* c = b->groups[g];
          c->graph = graph;
          c->building = true;
          c->build_timed = false;
          c->last = nullptr;  // an independent chain per size group
          MechIterFn it{c, mats[g], tol, maxit};
          for (int j = 0; j < K && !rc; ++j) rc = it();
          c->building = false;
          c->graph = nullptr;
          c->pending.clear();
        }
        if (!rc && hipGraphInstantiate(&b->exec[i], graph, nullptr, nullptr, 0) != hipSuccess)
          rc = fail(FGCG_EHIP, "hipGraphInstantiate failed");
        (void)hipGraphDestroy(graph);
        if (rc) return rc;
      }
      b->key = key.b;
    }
    long long launched = 0;
    auto go = [&](int i) -> int {
      HIPCHK(hipGraphLaunch(b->exec[i], st));
      int r = copy_states(i);
      if (r) return r;
      HIPCHK(hipEventRecord(b->ev_done[i], st));
      launched += K;
      return 0;
    };
    if ((rc = go(0)) || (rc = go(1))) return rc;
    int i = 0;
    for (;;) {
      HIPCHK(hipEventSynchronize(b->ev_done[i]));
      if (all_done(i)) break;
      if (launched > (long long)maxit + 4LL * K) return fail(FGCG_EHIP, "batched CG driver overran the iteration limit");
      if ((rc = go(i))) return rc;
      i ^= 1;
    }
    HIPCHK(hipStreamSynchronize(st));
    last = i;
  }
  int worst = FGCG_OK;
  std::vector<double> means, ens;
  for (size_t g = 0; g < b->groups.size(); ++g) {
    fgcg_ctx* c = b->groups[g];
    const std::vector<int>& mem = b->members[g];
    if ((rc = sr_finish(c))) return rc;
    if (c->prec != FGCG_FP64) {
      hipLaunchKernelGGL((k_fold_final<float>), dim3(c->npost, c->nsamp), dim3(PT), 0, st, (const float*)c->x, c->xh,
                         2 * c->n);
      HIPCHK(hipGetLastError());
    }
    means.assign(3 * mem.size(), 0.0);
    ens.assign(mem.size(), 0.0);
    if ((rc = mech_post(c, mats[g], nullptr, c->strain_buf, nullptr, means.data(), ens.data()))) return rc;
    for (size_t s = 0; s < mem.size(); ++s) {
      const int id = mem[s];
      if (strains && strains[id])
        HIPCHK(hipMemcpyAsync(strains[id], c->strain_buf + 3 * (size_t)c->n * s, sizeof(double) * 3 * c->n,
                              hipMemcpyDeviceToDevice, st));
      if (mean_stress)
        for (int j = 0; j < 3; ++j) mean_stress[3 * id + j] = means[3 * s + j];
      if (energy) energy[id] = ens[s];
      const CgState& cs = c->h_st[last * c->nsamp + s];
      if (infos) fill_info(&infos[id], cs, now() - t0);
      const int stt = status_of(cs);
      if (stt < 0 && worst >= 0) worst = stt;
      if (stt == FGCG_NOT_CONVERGED && worst == FGCG_OK) worst = FGCG_NOT_CONVERGED;
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  return worst;
}

}  // extern "C"
