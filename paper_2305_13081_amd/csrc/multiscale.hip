// Multiscale coupling of the diffusion (Sec. 3.2): a macroscopic bar whose
// material points carry representative volumes.
//
// The volume problem of Sec. 2.1 is linear in grad c_mac: its upscaled flux is
// <j> = -D_eff grad c_mac (D_eff from one homogenisation per axis), and for
// grad c_mac = g e_y (the bar runs along the volume's y axis) its local
// concentration (eq. concentration-correct) is
//   c(x) = g u(x) + [pore] c_mac / eta,
// u the concentration of the unit gradient with c_mac = 0 (its pore and solid
// means are zero, eq. psi-two-values), eta the pore share.  D_eff and u are
// computed once, on the GPU, when the object is created.  A time step then
//   1. advances the bar: finite volumes, backward Euler, influx J_in through
//      the face at Y = 0, none at Y = L, the face conductance D_eff,yy / dY
//      (one microstructure along the bar); a tridiagonal solve of ncell
//      unknowns on the host;
//   2. hands each coupled volume its cell's concentration c_mac and gradient
//      g (the mean of the cell's two face gradients; the face at Y = 0 takes
//      -J_in / D_eff,yy) and updates it on the GPU: local concentration,
//      irreversible precipitation c_ppt = max(c_ppt, (c - S)_+) in the pores,
//      eigenstrain e = (c_ppt M_ppt - 1)_+ (eq. eigen-simplify) in one fused
//      kernel, then the mechanics (eps_mac = 0) with the previous damage, the
//      history and the phase field (Alg. 1's blocks, the context's solvers).
#include <algorithm>
#include <vector>

#include "engine.hpp"

using namespace fgcg;

namespace {

// Local concentration, precipitate and eigenstrain of one volume; per-block
// partial sums [sum c_ppt, max e].
__global__ void __launch_bounds__(NT) k_ms_precip(const uint8_t* __restrict__ phase, const double* __restrict__ u,
                                                  double g, double c_pore, double solubility, double molar_volume,
                                                  long long n, double* __restrict__ conc, double* __restrict__ cppt,
                                                  double* __restrict__ e, double* __restrict__ part) {
  __shared__ double red[NT / 64];
  __shared__ double redm[NT];
  double sum = 0.0, mx = 0.0;
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const bool pore = phase[i] == 0;
    const double cv = g * u[i] + (pore ? c_pore : 0.0);
    const double p = pore ? fmax(cppt[i], fmax(cv - solubility, 0.0)) : 0.0;
    const double ev = pore ? fmax(p * molar_volume - 1.0, 0.0) : 0.0;
    conc[i] = cv;
    cppt[i] = p;
    e[i] = ev;
    sum += p;
    mx = fmax(mx, ev);
  }
  redm[threadIdx.x] = mx;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) redm[threadIdx.x] = fmax(redm[threadIdx.x], redm[threadIdx.x + w]);
    __syncthreads();
  }
  const double t = block_sum(sum, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t;
    part[2 * blockIdx.x + 1] = redm[0];
  }
}

// State fields of one volume, in this order; each N doubles except the strain
// (n_s N).
enum { F_C = 0, F_CPPT, F_E, F_H, F_D, F_STRAIN, F_COUNT };

}  // namespace

struct fgcg_ms {
  fgcg_ctx* c = nullptr;
  fgcg_ms_params prm{};
  fgcg_material mat{};
  std::vector<double> E_tab, nu_tab;
  double Deff[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double Dbar = 0.0;    // D_eff along the bar (the yy entry)
  double eta = 0.0;     // pore share of the volume
  double* u = nullptr;  // device [N] unit-gradient concentration
  std::vector<int> cells;
  std::vector<double*> fields;  // F_COUNT device buffers per volume
  double* part = nullptr;       // device partial sums of k_ms_precip
  int npart = 0;
  std::vector<double> hpart, cbar, gbar;
  double time = 0.0;
};

namespace {

// Backward-Euler step of the bar (Thomas algorithm), then the cell gradients.
void bar_step(fgcg_ms* ms) {
  const int n = ms->prm.ncell;
  const double dY = ms->prm.length / n, dt = ms->prm.dt, D = ms->Dbar;
  const double k = D / dY;  // face conductance
  std::vector<double> lo(n, 0.0), di(n, dY / dt), up(n, 0.0), r(n);
  for (int i = 0; i < n; ++i) r[i] = ms->cbar[i] * dY / dt;
  r[0] += ms->prm.J_in;
  for (int f = 0; f + 1 < n; ++f) {  // face between cells f and f + 1
    di[f] += k;
    di[f + 1] += k;
    up[f] = -k;
    lo[f + 1] = -k;
  }
  for (int i = 1; i < n; ++i) {
    const double w = lo[i] / di[i - 1];
    di[i] -= w * up[i - 1];
    r[i] -= w * r[i - 1];
  }
  ms->cbar[n - 1] = r[n - 1] / di[n - 1];
  for (int i = n - 2; i >= 0; --i) ms->cbar[i] = (r[i] - up[i] * ms->cbar[i + 1]) / di[i];
  std::vector<double> face(n + 1, 0.0);
  face[0] = -ms->prm.J_in / D;
  for (int f = 1; f < n; ++f) face[f] = (ms->cbar[f] - ms->cbar[f - 1]) / dY;
  for (int i = 0; i < n; ++i) ms->gbar[i] = 0.5 * (face[i] + face[i + 1]);
}

int ms_check_ctx(const fgcg_ctx* c) {
  if (c->prec != FGCG_FP64 || c->nsamp != 1)
    return fail(FGCG_EUNSUPPORTED, "multiscale volumes are single FP64 contexts");
  return 0;
}

}  // namespace

extern "C" {

void fgcg_ms_destroy(fgcg_ms* ms) {
  if (!ms) return;
  if (ms->c) (void)hipStreamSynchronize(ms->c->stream);
  for (double* f : ms->fields)
    if (f) (void)hipFree(f);
  if (ms->u) (void)hipFree(ms->u);
  if (ms->part) (void)hipFree(ms->part);
  delete ms;
}

int fgcg_ms_create(fgcg_ctx* c, const fgcg_material* mat, const double* D_rve, const fgcg_ms_params* prm, int nrve,
                   const int* rve_cells, fgcg_ms** out) {
  if (!c || !mat || !mat->phase || !mat->E_tab || !mat->nu_tab || !D_rve || !prm || !out ||
      (nrve > 0 && !rve_cells))
    return fail(FGCG_EINVAL, "ctx/material/phase/tables/D/params/out/cells is NULL");
  *out = nullptr;
  int rc;
  if ((rc = ms_check_ctx(c))) return rc;
  if (mat->E_field) return fail(FGCG_EUNSUPPORTED, "multiscale volumes take phase tables");
  if (mat->nphase < 1 || mat->nphase > FGCG_MAX_PHASES) return fail(FGCG_EINVAL, "nphase outside 1..max");
  if (nrve < 0 || prm->ncell < 2 || !(prm->length > 0) || !(prm->dt > 0) || !(prm->J_in >= 0) ||
      !(prm->solubility >= 0) || !(prm->molar_volume >= 0) || !(prm->Gc > 0) || !(prm->l0 > 0) ||
      !(prm->kappa >= 0) || !(prm->tol >= 0) || !(prm->tol_homog >= 0) || prm->maxit < 1)
    return fail(FGCG_EDOMAIN, "bar or volume parameter outside its domain");
  for (int i = 0; i < nrve; ++i)
    if (rve_cells[i] < 0 || rve_cells[i] >= prm->ncell) return fail(FGCG_EINVAL, "volume cell outside the bar");
  if ((rc = enter(c))) return rc;
  fgcg_ms* ms = new fgcg_ms();
  ms->c = c;
  ms->prm = *prm;
  ms->E_tab.assign(mat->E_tab, mat->E_tab + mat->nphase);
  ms->nu_tab.assign(mat->nu_tab, mat->nu_tab + mat->nphase);
  ms->mat = *mat;
  ms->mat.E_tab = ms->E_tab.data();
  ms->mat.nu_tab = ms->nu_tab.data();
  ms->cells.assign(rve_cells, rve_cells + nrve);
  ms->cbar.assign(prm->ncell, 0.0);
  ms->gbar.assign(prm->ncell, 0.0);
  const long long n = c->n;
  const int dim = c->ndim, ns = dim == 2 ? 3 : 6;
  auto bail = [&](int r) {
    fgcg_ms_destroy(ms);
    return r;
  };
  ms->npart = (int)std::min<long long>((n + NT - 1) / NT, 1024);
  ms->hpart.resize(2 * ms->npart);
  if (hipMalloc(&ms->u, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&ms->part, sizeof(double) * 2 * ms->npart) != hipSuccess)
    return bail(fail(FGCG_ENOMEM, "multiscale workspace"));
  for (int i = 0; i < nrve; ++i)
    for (int k = 0; k < F_COUNT; ++k) {
      double* f = nullptr;
      const size_t sz = sizeof(double) * (k == F_STRAIN ? ns : 1) * (size_t)n;
      if (hipMalloc(&f, sz) != hipSuccess) return bail(fail(FGCG_ENOMEM, "volume state"));
      ms->fields.push_back(f);
      if (hipMemsetAsync(f, 0, sz, c->stream) != hipSuccess) return bail(fail(FGCG_EHIP, "hipMemsetAsync"));
    }
  // D_eff, then u: the gradient field of the unit solve along y and its
  // concentration with c_mac = 0
  fgcg_info infos[3];
  if ((rc = fgcg_diffusivity_eff(c, D_rve, prm->tol_homog, prm->maxit, ms->Deff, infos)) < 0) return bail(rc);
  ms->Dbar = ms->Deff[dim * 1 + 1];
  if (!(ms->Dbar > 0.0)) return bail(fail(FGCG_EDOMAIN, "D_eff along the bar is not positive"));
  double* grad = nullptr;
  if (hipMalloc(&grad, sizeof(double) * dim * n) != hipSuccess) return bail(fail(FGCG_ENOMEM, "unit gradient"));
  const double gy[3] = {0.0, 1.0, 0.0};
  rc = fgcg_diffusion_homogenize(c, D_rve, gy, prm->tol_homog, prm->maxit, grad, nullptr, nullptr, infos);
  if (rc >= 0) rc = fgcg_concentration(c, mat->phase, grad, gy, 0.0, ms->u, nullptr);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(grad);
  if (rc < 0) return bail(rc);
  std::vector<uint8_t> ph(n);
  if (hipMemcpy(ph.data(), mat->phase, n, hipMemcpyDeviceToHost) != hipSuccess)
    return bail(fail(FGCG_EHIP, "hipMemcpy"));
  long long np = 0;
  for (long long i = 0; i < n; ++i) np += ph[i] == 0;
  if (np == 0) return bail(fail(FGCG_EDOMAIN, "the volume has no pores (phase 0)"));
  ms->eta = (double)np / (double)n;
  *out = ms;
  return FGCG_OK;
}

int fgcg_ms_step(fgcg_ms* ms, fgcg_ms_info* infos) {
  if (!ms) return fail(FGCG_EINVAL, "multiscale object is NULL");
  fgcg_ctx* c = ms->c;
  int rc;
  if ((rc = enter(c))) return rc;
  bar_step(ms);
  const long long n = c->n;
  MechMat m0;
  if ((rc = make_mech_mat(c, &ms->mat, nullptr, 0.0, &m0))) return rc;
  const double zero[6] = {0, 0, 0, 0, 0, 0};
  int worst = FGCG_OK;
  for (size_t r = 0; r < ms->cells.size(); ++r) {
    double* const* f = ms->fields.data() + F_COUNT * r;
    const int k = ms->cells[r];
    fgcg_ms_info inf{};
    inf.c_mac = ms->cbar[k];
    inf.grad_mac = ms->gbar[k];
    hipLaunchKernelGGL(k_ms_precip, dim3(ms->npart), dim3(NT), 0, c->stream, ms->mat.phase, (const double*)ms->u,
                       inf.grad_mac, inf.c_mac / ms->eta, ms->prm.solubility, ms->prm.molar_volume, n, f[F_C],
                       f[F_CPPT], f[F_E], ms->part);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ms->hpart.data(), ms->part, sizeof(double) * 2 * ms->npart, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (int b = 0; b < ms->npart; ++b) {
      sum += ms->hpart[2 * b];
      inf.max_e = std::max(inf.max_e, ms->hpart[2 * b + 1]);
    }
    inf.mean_cppt = sum / (double)n;
    rc = fgcg_mech_solve(c, &ms->mat, f[F_D], ms->prm.kappa, f[F_E], zero, ms->prm.tol, ms->prm.maxit, f[F_STRAIN],
                         nullptr, inf.mean_stress, &inf.energy, &inf.mech);
    if (rc < 0) return rc;
    if (rc != FGCG_OK) worst = rc;
    if (c->ndim == 3) {
      if ((rc = history3(c, m0, f[F_STRAIN], f[F_E], f[F_H]))) return rc;
    } else {
      hipLaunchKernelGGL(k_history, dim3(c->npost), dim3(PT), 0, c->stream, m0, (const double*)f[F_STRAIN],
                         (const double*)f[F_E], f[F_H], n);
      HIPCHK(hipGetLastError());
    }
    rc = fgcg_phasefield_solve(c, f[F_H], ms->prm.Gc, ms->prm.l0, f[F_D], ms->prm.tol, ms->prm.maxit, &inf.pf);
    if (rc < 0) return rc;
    if (rc != FGCG_OK) worst = rc;
    hipLaunchKernelGGL(k_observe, dim3(c->npost), dim3(PT), 0, c->stream, ms->mat.phase, (const double*)f[F_D],
                       (const double*)f[F_CPPT], n, c->part_post);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->h_part, c->part_post, sizeof(double) * 5 * c->npost, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int b = 0; b < c->npost; ++b) inf.max_d = std::max(inf.max_d, c->h_part[5 * b]);
    if (infos) infos[r] = inf;
  }
  ms->time += ms->prm.dt;
  return worst;
}

int fgcg_ms_read(const fgcg_ms* ms, double* c_bar, double* grad_bar, double* D_eff, double* time) {
  if (!ms) return fail(FGCG_EINVAL, "multiscale object is NULL");
  if (c_bar) std::copy(ms->cbar.begin(), ms->cbar.end(), c_bar);
  if (grad_bar) std::copy(ms->gbar.begin(), ms->gbar.end(), grad_bar);
  if (D_eff) std::copy(ms->Deff, ms->Deff + ms->c->ndim * ms->c->ndim, D_eff);
  if (time) *time = ms->time;
  return FGCG_OK;
}

int fgcg_ms_volume(const fgcg_ms* ms, int rve, double* conc, double* cppt, double* e, double* H, double* d,
                   double* strain) {
  if (!ms) return fail(FGCG_EINVAL, "multiscale object is NULL");
  if (rve < 0 || rve >= (int)ms->cells.size()) return fail(FGCG_EINVAL, "no such volume");
  fgcg_ctx* c = ms->c;
  const size_t nb = sizeof(double) * (size_t)c->n;
  const int ns = c->ndim == 2 ? 3 : 6;
  double* dst[F_COUNT] = {conc, cppt, e, H, d, strain};
  for (int k = 0; k < F_COUNT; ++k)
    if (dst[k])
      HIPCHK(hipMemcpyAsync(dst[k], ms->fields[F_COUNT * rve + k], (k == F_STRAIN ? ns : 1) * nb,
                            hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return FGCG_OK;
}

}  // extern "C"
