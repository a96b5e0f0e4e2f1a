// Entry points of the static diffusion homogenisation (Sec. 2.1, the
// diffusion block of Alg. 1), the concentration reconstruction and the
// effective diffusivity (App. B), 2D and 3D grids, FP64 contexts.  The CG is
// the displacement-form engine of the mechanics with one component: per
// iteration the flux stencil pass (q = K p, p.Kp partial sums), the forward x
// transform with the CG update, the Green passes (column in 2D; y, z, y in 3D)
// and the inverse x transform with the direction update.
#include "homog.hpp"
#include "launch3d.hpp"
#include "strain_form.hpp"

using namespace fgcg;

namespace {

constexpr int GRAPH_SLOT = 7;  // chunk graphs of the homogenisation CG

Field<double> fld1(void* p, const fgcg_ctx* c) { return Field<double>{(double*)p, c->n, c->n}; }

Vec3 vec3(const fgcg_ctx* c, const double* g) {
  Vec3 v{{g[0], g[1], c->ndim == 3 ? g[2] : 0.0}};
  return v;
}

int nkp2(const fgcg_ctx* c) { return std::min(fk_tiles(c->nx, c->ny), 1024); }
int nkp3(const fgcg_ctx* c) { return std::min(f3_chunks(c->nx, c->ny, c->nz), KP3_MAX_BLOCKS); }

// ---------------------------------------------------------------- 2D
// z = M r, p = z, r.z and the CG state (r holds f, x holds 0).
int init2(fgcg_ctx* c, double tol, int maxit) {
  CT<double>* spec = (CT<double>*)c->spec;
  int rc;
  const CopyProN<double, 1> cp{fld1(c->r, c), c->nx};
  if ((rc = launch_row_fwd<double, 1>(c, -1, cp, spec))) return rc;
  const MechGreen<double, 1> g0{c->Dx, c->Dy, 1.0 / (double)c->n, c->nx, nullptr, c->part_rr};
  if ((rc = launch_col<double, 1, 1>(c, -1, g0, spec, spec))) return rc;
  const MechUEpi<double, 1> e0{fld1(c->p, c), c->nx, c->st, c->part_rr, c->ncol, 1, tol, maxit};
  if ((rc = launch_row_inv<double, 1>(c, -1, e0, spec))) return rc;
  HIPCHK(hipGetLastError());
  return 0;
}

int iter2(fgcg_ctx* c, const double* Df, double tol, int maxit) {
  CT<double>* spec = (CT<double>*)c->spec;
  const Field<double> X = fld1(c->x, c), R = fld1(c->r, c), P = fld1(c->p, c), Q = fld1(c->tmp, c);
  const int nkp = nkp2(c);
  int r = launch(c, -1, (const void*)&k_flux_kp<double>, dim3(nkp), Df, (const double*)P.p, Q.p, c->nx, c->ny,
                 1.0 / c->h, c->st, c->part_a);
  const MechUProC<double, 1> pro{{X, R, P, Q, c->nx, c->st, c->part_a, nkp}};
  r |= launch_row_fwd<double, 1>(c, -1, pro, spec);
  const MechGreen<double, 1> green{c->Dx, c->Dy, 1.0 / (double)c->n, c->nx, c->st, c->part_rr};
  r |= launch_col<double, 1, 1>(c, -1, green, spec, spec);
  const MechUEpiC<double, 1, false> epi{{P, c->nx, c->st, c->part_rr, c->ncol, 0, tol, maxit}};
  r |= launch_row_inv<double, 1>(c, -1, epi, spec);
  return r;
}

// ---------------------------------------------------------------- 3D
// x rows, y lines, z tiles with the Green symbol (r.z into red[1]), y lines.
template <class Pro> int green3_1(fgcg_ctx* c, const Pro& pro, const CgState* st) {
  CT<double>* spec = (CT<double>*)c->spec;
  int r = launch_row_fwd<double, 1>(c, -1, pro, spec);
  r |= launch_ypass<double, 1>(c, -1, false, st, spec);
  const Green3<double> g{c->Dx, c->Dy, c->Dz, 1.0 / (double)c->n, c->nx, st, c->part_z};
  r |= launch_zpass<double, true, true>(c, -1, g, spec, 1);
  r |= launch_reduce(c, c->part_z, zblocks<double>(c, 1), c->red + 1);
  r |= launch_ypass<double, 1>(c, -1, true, st, spec);
  return r;
}

int init3(fgcg_ctx* c, double tol, int maxit) {
  const CopyProN<double, 1> cp{fld1(c->r, c), c->nx};
  int r = green3_1(c, cp, nullptr);
  const MechUEpi<double, 1> e0{fld1(c->p, c), c->nx, c->st, c->red + 1, 1, 1, tol, maxit};
  r |= launch_row_inv<double, 1>(c, -1, e0, (const CT<double>*)c->spec);
  HIPCHK(hipGetLastError());
  return r;
}

int iter3(fgcg_ctx* c, const double* Df, double tol, int maxit) {
  const Field<double> X = fld1(c->x, c), R = fld1(c->r, c), P = fld1(c->p, c), Q = fld1(c->tmp, c);
  const int nkp = nkp3(c);
  int r = launch(c, -1, (const void*)&k_flux3_kp<double>, dim3(nkp), Df, (const double*)P.p, Q.p, grid3(c),
                 1.0 / c->h, c->st, c->part_a);
  r |= launch_reduce(c, c->part_a, nkp, c->red);
  const MechUPro<double, 1> pro{X, R, P, Q, c->nx, c->st, c->red, 1};
  r |= green3_1(c, pro, c->st);
  const MechUEpi<double, 1> epi{P, c->nx, c->st, c->red + 1, 1, 0, tol, maxit};
  r |= launch_row_inv<double, 1>(c, -1, epi, (const CT<double>*)c->spec);
  return r;
}

// The paper's projected CG on the concentration-gradient fluctuation (2D,
// any gradient operator): b = -G[D grad c_mac], three passes per iteration.
// x (2 components) in c->x; phi (optional) by the inverse gradient of x.
int homogenize_gf(fgcg_ctx* c, const double* Df, const double* gmac, double tol, int maxit, double* grad_c,
                  double* phi, double* mean_flux, fgcg_info* info) {
  const double t0 = now();
  const long long n = c->n;
  CT<double>* spec = (CT<double>*)c->spec;
  const Field<double> X{(double*)c->x, n, 0}, R{(double*)c->r, n, 0}, P{(double*)c->p, n, 0};
  int rc;
  const VecSrcPro<double, 2, FluxLaw> src{{Df}, nullptr, {gmac[0], gmac[1], 0.0}, c->nx, n};
  if ((rc = launch_row_fwd<double, 2>(c, -1, src, spec))) return rc;
  const VecProj<double> pj0{c->Dx, c->Dy, 1.0 / (double)n, nullptr};
  if ((rc = launch_col<double, 2, 2>(c, -1, pj0, spec, spec))) return rc;
  const VecRhsEpi<double, 2> rhs{X, R, c->nx, c->part_rr, c->part_b};
  if ((rc = launch_row_inv<double, 2>(c, -1, rhs, spec))) return rc;
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(NT), 0, c->stream, c->st, c->part_b, c->nrow, 0, tol, maxit);
  HIPCHK(hipGetLastError());
  const CgCtl cc{c->st, c->part_a, c->part_rr, c->nrow, c->nrow, 0, 0};
  const VecCgPro<double, 2, FluxLaw> pro{P, R, {Df}, c->nx, cc};
  const VecProj<double> pj{c->Dx, c->Dy, 1.0 / (double)n, c->st};
  const VecCgEpi<double, 2> epi{X, R, P, c->nx, cc};
  auto iter = [&]() -> int {
    int r = launch_row_fwd<double, 2>(c, -1, pro, spec);
    r |= launch_col<double, 2, 2>(c, -1, pj, spec, spec);
    r |= launch_row_inv<double, 2>(c, -1, epi, spec);
    return r;
  };
  Key key;
  key.add(Df).add(tol).add(maxit).add(c->gradop);
  if ((rc = run_cg(c, 9, key, c->st, c->h_st, iter, maxit))) return rc;
  const CgState s = *c->h_st;
  hipLaunchKernelGGL(k_hg_post, dim3(c->npost), dim3(NT), 0, c->stream, Df, (const double*)X.p, n, gmac[0], gmac[1],
                     grad_c, c->part_post);
  HIPCHK(hipGetLastError());
  if (phi) {
    const CopyProN<double, 1> cp{Field<double>{X.p, n, n}, c->nx};
    const long long cs = (long long)c->nxh * c->rows;
    if ((rc = launch_row_fwd<double, 1>(c, -1, cp, spec, 2, cs))) return rc;
    const InvGradSym<double> ig{c->Dx, c->Dy, 1.0 / (double)n};
    if ((rc = launch_col<double, 2, 1>(c, -1, ig, spec, spec))) return rc;
    const StoreEpi<double, 1> st{Field<double>{phi, n, 0}, Field<double>{nullptr, n, 0}, 1.0, c->nx, nullptr, 0};
    if ((rc = launch_row_inv<double, 1>(c, -1, st, spec))) return rc;
  }
  HIPCHK(hipMemcpyAsync(c->h_part, c->part_post, sizeof(double) * 4 * c->npost, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double acc[4] = {0, 0, 0, 0};
  for (int b = 0; b < c->npost; ++b)
    for (int j = 0; j < 4; ++j) acc[j] += c->h_part[4 * b + j];
  if (mean_flux)
    for (int j = 0; j < 2; ++j) mean_flux[j] = acc[j] / (double)n;
  fill_info(info, s, now() - t0);
  return status_of(s);
}

// One homogenisation solve: phi in c->x.  Writes the mean flux (host [dim])
// and optional grad c / phi fields.
int homogenize(fgcg_ctx* c, const double* Df, const double* gmac, double tol, int maxit, double* grad_c,
               double* phi, double* mean_flux, double* energy_density, fgcg_info* info) {
  if (c->ndim == 2 && (c->gradop != 0 || c->strain_form))
    return homogenize_gf(c, Df, gmac, tol, maxit, grad_c, phi, mean_flux, info);
  const double t0 = now();
  const Vec3 gm = vec3(c, gmac);
  const int nb = c->ndim == 3 ? nslab(c) : (int)c->sgrid.x;
  hipLaunchKernelGGL(k_flux_rhs, dim3(nb), dim3(NT), 0, c->stream, Df, gm, (double*)c->r, (double*)c->x, c->nx,
                     c->ny, c->nz, 1.0 / c->h);
  HIPCHK(hipGetLastError());
  int rc = c->ndim == 3 ? init3(c, tol, maxit) : init2(c, tol, maxit);
  if (rc) return rc;
  auto it = [&]() -> int { return c->ndim == 3 ? iter3(c, Df, tol, maxit) : iter2(c, Df, tol, maxit); };
  Key key;
  key.add(Df).add(tol).add(maxit);
  if ((rc = run_cg(c, GRAPH_SLOT, key, c->st, c->h_st, it, maxit))) return rc;
  const CgState s = *c->h_st;
  hipLaunchKernelGGL(k_flux_post, dim3(nb), dim3(NT), 0, c->stream, Df, (const double*)c->x, gm, c->nx, c->ny, c->nz,
                     1.0 / c->h, grad_c, phi, c->part_post);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_part, c->part_post, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double acc[4] = {0, 0, 0, 0};
  for (int b = 0; b < nb; ++b)
    for (int j = 0; j < 4; ++j) acc[j] += c->h_part[4 * b + j];
  if (mean_flux)
    for (int j = 0; j < c->ndim; ++j) mean_flux[j] = acc[j] / (double)c->n;
  if (energy_density) *energy_density = acc[3] / (double)c->n;
  fill_info(info, s, now() - t0);
  return status_of(s);
}

int check_ctx(fgcg_ctx* c) {
  if (c->prec != FGCG_FP64) return fail(FGCG_EUNSUPPORTED, "the diffusion homogenisation runs in FP64 contexts");
  if (c->nsamp != 1) return fail(FGCG_EUNSUPPORTED, "batch contexts are not supported");
  return 0;
}

}  // namespace

extern "C" {

int fgcg_diffusion_homogenize(fgcg_ctx* c, const double* Dfield, const double* grad_cmac, double tol, int maxit,
                              double* grad_c, double* phi, double* mean_flux, fgcg_info* info) {
  if (!c || !Dfield || !grad_cmac) return fail(FGCG_EINVAL, "ctx/Dfield/grad_cmac is NULL");
  int rc;
  if ((rc = check_ctx(c)) || (rc = check_solver_args(tol, maxit))) return rc;
  for (int a = 0; a < c->ndim; ++a)
    if (!std::isfinite(grad_cmac[a])) return fail(FGCG_EDOMAIN, "grad_cmac not finite");
  if ((rc = enter(c))) return rc;
  return homogenize(c, Dfield, grad_cmac, tol, maxit, grad_c, phi, mean_flux, nullptr, info);
}

int fgcg_diffusivity_eff(fgcg_ctx* c, const double* Dfield, double tol, int maxit, double* Deff,
                         fgcg_info* infos) {
  if (!c || !Dfield || !Deff) return fail(FGCG_EINVAL, "ctx/Dfield/Deff is NULL");
  int rc;
  if ((rc = check_ctx(c)) || (rc = check_solver_args(tol, maxit))) return rc;
  if ((rc = enter(c))) return rc;
  const int dim = c->ndim;
  int worst = FGCG_OK;
  for (int a = 0; a < dim; ++a) {
    double g[3] = {0.0, 0.0, 0.0}, mf[3] = {0.0, 0.0, 0.0};
    g[a] = 1.0;
    rc = homogenize(c, Dfield, g, tol, maxit, nullptr, nullptr, mf, nullptr, infos ? &infos[a] : nullptr);
    if (rc < 0) return rc;
    if (rc == FGCG_NOT_CONVERGED) worst = rc;
    for (int b = 0; b < dim; ++b) Deff[b * dim + a] = -mf[b];
  }
  return worst;
}

int fgcg_concentration(fgcg_ctx* c, const uint8_t* phase, const double* grad_c, const double* grad_cmac,
                       double c_mac, double* cout, double* beta) {
  if (!c || !phase || !grad_c || !grad_cmac || !cout) return fail(FGCG_EINVAL, "ctx/phase/grad_c/grad_cmac/c is NULL");
  int rc;
  if ((rc = check_ctx(c))) return rc;
  if (!std::isfinite(c_mac)) return fail(FGCG_EDOMAIN, "c_mac not finite");
  if ((rc = enter(c))) return rc;
  CT<double>* spec = (CT<double>*)c->spec;
  const long long cs = (long long)c->nxh * c->rows;  // spectrum stride of one component
  const CopyProN<double, 1> cp{Field<double>{(double*)grad_c, c->n, c->n}, c->nx};
  double* phi = (double*)c->x;
  const StoreEpi<double, 1> st{Field<double>{phi, c->n, 0}, Field<double>{nullptr, c->n, 0}, 1.0, c->nx, nullptr, 0};
  if (c->ndim == 2) {
    // row transforms of both components, phi_hat = (i xi)^-1 . g_hat in the column pass, inverse rows
    if ((rc = launch_row_fwd<double, 1>(c, -1, cp, spec, 2, cs))) return rc;
    const InvGradSym<double> sym{c->Dx, c->Dy, 1.0 / (double)c->n};
    if ((rc = launch_col<double, 2, 1>(c, -1, sym, spec, spec))) return rc;
    if ((rc = launch_row_inv<double, 1>(c, -1, st, spec))) return rc;
  } else {
    // forward x, y, z transforms of the three components, the inverse gradient
    // mode by mode, inverse z, y, x transforms of phi
    if ((rc = launch_row_fwd<double, 1>(c, -1, cp, spec, 3, cs))) return rc;
    if ((rc = launch_ypass<double, 3>(c, -1, false, nullptr, spec))) return rc;
    if ((rc = launch_zpass<double, true, false>(c, -1, NoSym{}, spec, 3))) return rc;
    const int nb = (int)std::min<long long>((cs + NT - 1) / NT, 4096);
    hipLaunchKernelGGL(k_invgrad3, dim3(nb), dim3(NT), 0, c->stream, (double2*)spec, c->Dx, c->Dy, c->Dz, c->nxh,
                       c->ny, c->nz, 1.0 / (double)c->n);
    if ((rc = launch_zpass<double, false, true>(c, -1, NoSym{}, spec, 1))) return rc;
    if ((rc = launch_ypass<double, 1>(c, -1, true, nullptr, spec))) return rc;
    if ((rc = launch_row_inv<double, 1>(c, -1, st, spec))) return rc;
  }
  const Vec3 gm = vec3(c, grad_cmac);
  const int nb = c->ndim == 3 ? nslab(c) : (int)c->sgrid.x;
  hipLaunchKernelGGL(k_conc_sums, dim3(nb), dim3(NT), 0, c->stream, phase, (const double*)phi, gm, c->h, c->nx, c->ny,
                     c->nz, c->part_post);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_part, c->part_post, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int b = 0; b < nb; ++b)
    for (int j = 0; j < 6; ++j) a[j] += c->h_part[6 * b + j];
  // eq. psi-two-values: pore mean c_mac / eta, solid mean 0
  const double npore = a[2], nsolid = a[5];
  const double eta = npore / (double)c->n;
  const double bp = npore > 0 ? c_mac / eta - a[1] / npore - a[0] / npore : 0.0;
  const double bs = nsolid > 0 ? -a[4] / nsolid - a[3] / nsolid : 0.0;
  hipLaunchKernelGGL(k_conc_write, dim3(nb), dim3(NT), 0, c->stream, phase, (const double*)phi, gm, c->h, c->nx, c->ny,
                     c->nz, bp, bs, cout);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  if (beta) {
    beta[0] = bp;
    beta[1] = bs;
  }
  return FGCG_OK;
}

}  // extern "C"
