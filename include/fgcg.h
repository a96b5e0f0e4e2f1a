/*
 * fgcg -- Fourier-Galerkin projected conjugate gradients on MI355X (gfx950).
 *
 * C ABI of the hot path of the FFT-based corrosion-fracture framework of
 * Pundir, Kammer and Angst (arXiv 2305.13081):
 *
 *   mechanics   Sec. 2.3, eq. solid / eq. solid-final, projection of App. A:
 *               div( g(d) C(x) : (eps - e I) ) = 0, <eps> = eps_mac
 *   phase field Sec. 2.4, eq. crack / eq. crack-fft (AT2, history field H)
 *   diffusion   Sec. 2.1 (Fick's law, D defined voxel by voxel): the static
 *               homogenisation in gradient-primary form with the
 *               concentration reconstruction, and one implicit time step with
 *               a first-order sink and Dirichlet voxels
 *   staggered   Alg. 1: diffusion -> precipitation/eigenstrain -> mechanics ->
 *               history -> phase field
 *
 * Every gradient is the forward difference of Sec. 2.6,
 * D_a(k) = (exp(2 pi i k_a / n_a) - 1) / h.
 *
 * Conventions
 *   - Grids are periodic, 2D with n[0] = nx (fastest) and n[1] = ny, or 3D
 *     with n[2] = nz as well; every axis length is 2^a 3^b, 8..2048 in 2D and
 *     8..512 in 3D.  N is the number of voxels.
 *   - Field pointers are DEVICE pointers owned by the caller, contiguous,
 *     component-major: [comp][ny][nx] or [comp][nz][ny][nx].  Host pointers
 *     are marked "host".
 *   - Strain and stress use Voigt order with TENSOR shear (eps_12, not
 *     gamma_12): n_s = 3 components (11, 22, 12) in 2D (plane strain), n_s = 6
 *     components (11, 22, 33, 23, 13, 12) in 3D.  Index 1 is the x axis.
 *     Phase ids are uint8 (0 = pore, 1 = solid, up to FGCG_MAX_PHASES phases).
 *   - All work is enqueued on the context's HIP stream; calls that return an
 *     fgcg_info or host scalars return after the stream has finished them.
 *   - The context owns every workspace buffer; solves allocate nothing.
 *   - Errors are returned as status codes, never thrown.  A detail string for
 *     the last error of the calling thread is available from fgcg_last_error.
 *   - A context may be used by one thread at a time.
 */
#ifndef FGCG_H
#define FGCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGCG_MAX_PHASES 8

typedef enum {
  FGCG_OK = 0,
  FGCG_NOT_CONVERGED = 1, /* warning: outputs hold the last iterate */
  FGCG_EINVAL = -1,       /* null required pointer, bad size, tol < 0, ... */
  FGCG_EDOMAIN = -2,      /* E <= 0, nu outside (-1, 0.5), dt/l0/Gc/h <= 0, non-finite input */
  FGCG_EBREAKDOWN = -3,   /* CG breakdown: p.Ap <= 0 or a non-finite scalar */
  FGCG_ENOMEM = -4,
  FGCG_EHIP = -5,         /* a HIP runtime call failed */
  FGCG_EUNSUPPORTED = -6  /* valid request the library does not implement */
} fgcg_status;

typedef enum { FGCG_FP64 = 0, FGCG_FP32_MIXED = 1 } fgcg_precision;

typedef struct {
  int ndim;      /* 2 or 3 */
  int n[3];      /* n[0] = nx, n[1] = ny, n[2] = nz (unused in 2D) */
  double h;      /* voxel size, > 0 */
  int precision; /* fgcg_precision */
} fgcg_grid;

/* Isotropic elastic material mixed voxel by voxel (Sec. 2.3):
 * C(x) = lambda(x) I (x) I + 2 mu(x) II, plane strain in 2D. */
typedef struct {
  const uint8_t* phase;  /* device [N], phase id per voxel, 0..nphase-1 (not checked; other
                            values give undefined moduli) */
  int nphase;            /* 1..FGCG_MAX_PHASES */
  const double* E_tab;   /* host [nphase], Young's modulus per phase (Pa) */
  const double* nu_tab;  /* host [nphase], Poisson ratio per phase */
  const double* E_field; /* device [N] or NULL: per-voxel Young's modulus, overrides E_tab */
  double nu_field;       /* uniform Poisson ratio used with E_field */
} fgcg_material;

typedef struct {
  int iters;           /* CG iterations taken */
  int status;          /* fgcg_status of this solve */
  double rel_res;      /* ||r_k|| / ||b|| from the CG recurrence */
  double bnorm;        /* ||b|| */
  double seconds;      /* wall time of the solve (host clock) */
} fgcg_info;

typedef struct fgcg_ctx fgcg_ctx;

/* Create a context for one grid.  hip_stream: a hipStream_t or NULL (the
 * null stream).  Allocates all workspace.  Returns EINVAL for unsupported
 * sizes, EDOMAIN for h <= 0. */
int fgcg_create(const fgcg_grid* grid, void* hip_stream, fgcg_ctx** out);
void fgcg_destroy(fgcg_ctx* ctx);
int fgcg_set_stream(fgcg_ctx* ctx, void* hip_stream);
const char* fgcg_strerror(int status);
const char* fgcg_last_error(void);

/* Context options.
 *   FGCG_OPT_SCALAR_SPECTRAL  0 (default): the phase-field and diffusion
 *       operators are applied as real-space stencils (the forward-difference
 *       gradient of Sec. 2.6 is local, so this is the same operator); 1: they
 *       are applied in Fourier space as eq. crack-fft writes them.
 *   FGCG_OPT_GRAPHS           1 (default): CG iterations are replayed as HIP
 *       graphs of FGCG_OPT_CHUNK iterations; 0: plain launches.
 *   FGCG_OPT_CHUNK            iterations per graph chunk, even, 2..256 (default 16).
 *   FGCG_OPT_ROWS             2D grids: rows per block of the mechanics row
 *       passes (the forward pass with the CG update, the inverse pass with the
 *       direction update).  0 (default): autotune, i.e. time every candidate
 *       (the default for nx times 1/2, 1 and 2, even, 2..16, at most 4096
 *       voxels per block) on the context's own workspace before the next
 *       mechanics solve and keep the fastest; or a candidate value, fixed.
 *       The choice changes timing only, never results.  EUNSUPPORTED in 3D.
 *   FGCG_OPT_ROW_PLAN, FGCG_OPT_COL_PLAN   2D grids: radix plan of the LDS
 *       transforms in the mechanics row passes (timed jointly with the rows
 *       per block) and in the Green column pass.  1: radix 8 (with a trailing
 *       4); 2: radix 16 where it fits (fewer stages, larger butterflies); the
 *       same as 1 for lengths where radix 16 does not fit; column pass only,
 *       3: one 64-lane wavefront per column holding the column in registers
 *       (lengths 256..2048, unit Green operator; plan 1 otherwise).  0 (default):
 *       autotune before the next mechanics solve, as for FGCG_OPT_ROWS, on
 *       grids of at least 2^18 voxels (radix 8 below; radix 16 is kept only
 *       when more than 3 % faster, so near-ties give the same schedule in
 *       every context of a size).  The plan changes the rounding of the
 *       transforms only.  EUNSUPPORTED in 3D.
 *   FGCG_OPT_PRECOND          preconditioner of the mechanics CG (Sec. 5 names
 *       the property contrast as what limits the solver's efficiency).
 *       0 (default): the Green operator (grad^H grad)^-1 of a unit medium,
 *       i.e. the projected CG of eq. solid-final iterate by iterate; 1: the
 *       Green operator K0^-1 of a homogeneous isotropic reference medium,
 *       K0(k) = mu0 |D|^2 I + lam0 conj(D) D^T + mu0 D D^H, inverted mode by
 *       mode (a 2 x 2 closed form in the 2D column pass with both displacement
 *       components per block; a 3 x 3 Cholesky solve between the forward and
 *       inverse z transforms in 3D).  Same discrete solution; the stop test
 *       then measures r.K0^-1 r instead of the projected residual.  The
 *       reference is fgcg_set_reference's, else the Lame ratio of the stiffest
 *       phase (of nu_field with a per-voxel E field).  Changing it re-tunes
 *       the 2D column plan.  EUNSUPPORTED for the groups of a batch.
 *   FGCG_OPT_GRADIENT         the gradient operator of every solve (Sec. 2.6):
 *       0 (default) forward difference (exp(i theta) - 1)/h; 1 central
 *       difference i sin(theta)/h; 2 eighth-order central difference
 *       (2 i / h) sum_m a_m sin(m theta), a = 4/5, -1/5, 4/105, -1/280; 3
 *       Fourier i xi (signed wavenumber, zero at Nyquist).  2D grids only
 *       (EUNSUPPORTED in 3D).  With 1..3 the mechanics and the diffusion
 *       homogenisation run the paper's projected CG on the strain / the
 *       concentration gradient through the transform passes (FP64), and the
 *       phase field and the phase-table diffusion step their spectral form;
 *       the adjoint, the per-voxel diffusion step, the operator hooks and
 *       batches take the forward difference only (EUNSUPPORTED).  The central
 *       operators vanish at the Nyquist wavenumber of even grids, which the
 *       projections then leave out (checkerboard modes are not controlled).
 *   FGCG_OPT_STRAIN_FORM      1: the strain / gradient-form solvers of
 *       FGCG_OPT_GRADIENT with the forward difference too (2D, FP64); 0
 *       (default): the displacement-form solvers.  Setting either option away
 *       from its default allocates that solver's workspace (9 N doubles and
 *       three half spectra).
 *   FGCG_OPT_SPECTRAL_RES     1 (default): the mechanics PCG of 2D FP64
 *       contexts with the unit Green operator and the forward difference, on
 *       grids whose nx is a multiple of 64, keeps the residual as its half
 *       spectra: r_hat -= alpha FFT(K p) in the Green column pass and the
 *       solution update x += alpha p in the pass that forms the next
 *       direction, so that the stiffness stencil is applied inside a row
 *       transform: two passes per iteration (the row stage fused, see
 *       FGCG_OPT_MECH_FORM) or, where nx is a multiple of 256, three (185
 *       instead of 233 bytes per voxel).  The same alpha, beta and stop test
 *       as the projected CG of eq. solid-final (rounding aside); 0: the
 *       four-pass form everywhere.  Allocates the residual's half spectra
 *       (and the two-pass form's buffers) on the first solve that uses them.
 *       On grids of at least 2^18 voxels the autotuner (before the first
 *       mechanics solve) tunes the passes of every available form, times one
 *       whole iteration of each and keeps the fastest; smaller grids take the
 *       two-pass form.
 *   FGCG_OPT_MECH_PASSES      read only (fgcg_get_option): transform and
 *       stencil passes per mechanics CG iteration of a 2D context's current
 *       form, 2, 3 or 4 (after the first mechanics solve, which tunes it); 0
 *       in 3D.  EINVAL to set.
 *   FGCG_OPT_MECH_FORM        2D contexts where FGCG_OPT_SPECTRAL_RES applies:
 *       the form of the mechanics PCG, by its passes per iteration.  0
 *       (default): tuned as FGCG_OPT_SPECTRAL_RES says (grids below 2^18
 *       voxels take 2); 2: the residual spectra with the row stage fused (the
 *       inverse x transforms and direction update of iteration k and the
 *       stiffness stencil and forward x transforms of iteration k + 1 in one
 *       pass, beside the Green column pass; each block transforms one extra
 *       row above and below its own, the direction is double-buffered and
 *       K p gets its own half spectra: one more direction field and two more
 *       half spectra of memory); 3: the residual spectra in three passes; 4:
 *       four passes.  EUNSUPPORTED for 2 and 3 where FGCG_OPT_SPECTRAL_RES
 *       does not apply, and for 3 where nx is not a multiple of 256.  All
 *       forms give the same iterates up to rounding.
 *   FGCG_OPT_SCALAR_CG        the CG of the stencil phase-field and diffusion
 *       solves on 2D grids: 1 (default) the one-reduction form of Chronopoulos
 *       and Gear (w = A r and s = A p carried along; one pass per iteration
 *       updates p, s, x, r and applies the stencil to the new r, with both dot
 *       products of the next iteration), the alpha, beta and stop test of
 *       textbook CG in exact arithmetic; 0: textbook CG in two passes (the 3D
 *       grids' form).
 *   FGCG_OPT_ROW_SPLIT        3D grids: displacement components per block of
 *       the mechanics row passes, 1 + f + 2 i with f (forward pass with the CG
 *       update) and i (inverse pass with the direction update) 1 for one
 *       component per block (three launches' worth of blocks), 0 for all
 *       three in one block.  0 (default): autotune before the next mechanics
 *       solve on grids of at least 2^18 voxels (each pass timed both ways on
 *       the context's workspace, the faster kept), else 3 (FP64) or 2
 *       (FP32-mixed).  Changes timing only, never results.  EUNSUPPORTED in 2D.
 *   FGCG_OPT_ZTILES           3D grids: z tiles per block of the z pass, 1 or
 *       2 (the second tile's loads overlap the first's transforms).  0
 *       (default): autotune as FGCG_OPT_ROW_SPLIT (the non-default choice kept
 *       only when more than 3 % faster), else 2 (FP64) or 1 (FP32-mixed).  The
 *       block count orders the r.z partial sums, so results change by
 *       rounding.  EUNSUPPORTED in 2D.
 * Returns EINVAL for an unknown option or value. */
enum { FGCG_OPT_SCALAR_SPECTRAL = 0, FGCG_OPT_GRAPHS = 1, FGCG_OPT_CHUNK = 2,
       FGCG_OPT_ROWS = 3, FGCG_OPT_ROW_PLAN = 4, FGCG_OPT_COL_PLAN = 5, FGCG_OPT_PRECOND = 6, FGCG_OPT_GRADIENT = 7,
       FGCG_OPT_STRAIN_FORM = 8, FGCG_OPT_SPECTRAL_RES = 9, FGCG_OPT_MECH_PASSES = 10, FGCG_OPT_SCALAR_CG = 11,
       FGCG_OPT_ROW_SPLIT = 12, FGCG_OPT_ZTILES = 13, FGCG_OPT_MECH_FORM = 14 };
int fgcg_set_option(fgcg_ctx* ctx, int option, int value);
/* Reference medium of FGCG_OPT_PRECOND = 1: Lame constants (only lam0 / mu0
 * matters); (0, 0) restores the automatic choice.  EDOMAIN unless mu0 > 0 and
 * lam0 + 2 mu0 / 3 > 0. */
int fgcg_set_reference(fgcg_ctx* ctx, double lam0, double mu0);
/* Current value of an option (FGCG_OPT_ROWS, _ROW_PLAN, _COL_PLAN,
 * _ROW_SPLIT, _ZTILES: the tuned or fixed choice, 0 before the first
 * mechanics solve of an autotuned context). */
int fgcg_get_option(fgcg_ctx* ctx, int option, int* value);

/* Mechanical equilibrium with isotropic eigenstrain e(x) I (Sec. 2.3,
 * eq. solid): solves G[g C : sym(x)] = -G[g C : (eps_mac - e I)] for the
 * compatible fluctuation x (App. A projection G) by CG from x = 0, stopping
 * when ||r|| <= tol ||b|| or after maxit iterations (tol = 0 runs exactly
 * maxit iterations).  The iteration is carried on the displacement, x = grad u:
 * CG on grad^H g C grad u = -grad^H g C (eps_mac - e I) preconditioned by the
 * Fourier Green operator (grad^H grad)^-1, which has the same iterates, alpha,
 * beta and residual norms as CG on x. */
/*   d        device [N] damage or NULL (d = 0); g = (1 - d)^2 + kappa
 *   eig      device [N] scalar eigenstrain e or NULL (0)
 *   eps_mac  host [n_s] macroscopic strain (Voigt, tensor shear)
 *   strain   device [n_s][N] out: eps = eps_mac + sym(x)
 *   stress   device [n_s][N] out or NULL: sigma = g C : (eps - e I)
 *   mean_stress host [n_s] out or NULL: mean of sigma over all voxels
 *   energy   host out or NULL: W = h^dim/2 sum_x (eps - e I) : sigma
 * 3D grids: the same method with 3 displacement components and the 3D
 * transforms; fgcg_material.E_field is not supported there (EUNSUPPORTED).
 */
int fgcg_mech_solve(fgcg_ctx* ctx, const fgcg_material* mat, const double* d, double kappa,
                    const double* eig, const double* eps_mac, double tol, int maxit,
                    double* strain, double* stress, double* mean_stress, double* energy,
                    fgcg_info* info);

/* Gradient of a mechanical objective J with respect to the per-voxel Young's
 * modulus (FP64 contexts).  The forward solve of fgcg_mech_solve is recomputed
 * (no CG history is stored); with G = dJ/deps the adjoint lam solves
 * K lam = grad^H G on the same preconditioned CG engine (K symmetric), and
 *     grad_E[x] = dJ/dE_x|_eps - sym(grad lam)_x : sigma_x / E_x
 * (dC_x/dE_x = C_x / E_x; E_x is the undegraded modulus of voxel x).
 *   objective  FGCG_J_USER: dJ_dstrain (device [3][N], tensor components
 *              G11, G22, G12 with dJ = sum_x G11 de11 + G22 de22 + 2 G12 de12)
 *              required, no explicit part, *J untouched;
 *              FGCG_J_ENERGY: J = W (the energy of fgcg_mech_solve); lam = 0 by
 *              the envelope theorem, so no second solve is run;
 *              FGCG_J_C11: J = <sigma_11> / eps_mac[0] (eps_mac[0] != 0).
 *   grad_E     device [N] out, or NULL: only the forward solve and J (no
 *              adjoint solve; info_adj zeroed).   J  host out or NULL.
 *   info_fwd / info_adj  the two solves (info_adj->iters = 0 for the energy).
 * Returns EUNSUPPORTED in FP32-mixed contexts and on 3D grids, EINVAL/EDOMAIN
 * as mech_solve. */
enum { FGCG_J_USER = 0, FGCG_J_ENERGY = 1, FGCG_J_C11 = 2 };
int fgcg_mech_adjoint(fgcg_ctx* ctx, const fgcg_material* mat, const double* d, double kappa,
                      const double* eig, const double* eps_mac, const double* dJ_dstrain, int objective,
                      double tol, int maxit, double* grad_E, double* J, fgcg_info* info_fwd,
                      fgcg_info* info_adj);

/* Batched mechanics: many microstructures of uneven sizes solved together.
 * fgcg_batch_create groups the nb samples by grid size (nx[i], ny[i], each
 * 2^a 3^b in 8..2048, voxel size h for all) and allocates their workspace.
 * fgcg_mech_solve_batched solves, for every sample i, the problem of
 * fgcg_mech_solve with phase field phases[i] (device [ny_i][nx_i]), the shared
 * tables E_tab/nu_tab (host [nphase]), no damage or eigenstrain, and macro
 * strain eps_mac[3 i .. 3 i + 2] (host).  All samples iterate in one graph
 * launch per chunk (one chain of passes per size group, each pass covering
 * every sample of its group); a converged sample's blocks exit at once, so
 * samples stop independently, each on its own tolerance test.
 *   strains      host array of nb device pointers ([3][N_i] out), entries may be NULL
 *   mean_stress  host [nb][3] out or NULL;  energy host [nb] or NULL
 *   infos        host [nb] or NULL
 * Returns the worst status over the samples. */
typedef struct fgcg_batch fgcg_batch;
int fgcg_batch_create(int nb, const int* nx, const int* ny, double h, int precision, void* hip_stream,
                      fgcg_batch** out);
void fgcg_batch_destroy(fgcg_batch* batch);
int fgcg_mech_solve_batched(fgcg_batch* batch, const uint8_t* const* phases, int nphase, const double* E_tab,
                            const double* nu_tab, const double* eps_mac, double tol, int maxit,
                            double* const* strains, double* mean_stress, double* energy, fgcg_info* infos);

/* AT2 phase field (Sec. 2.4, eq. crack-fft) with the Laplacian taken as
 * -D^H D: [(Gc/(2 l0) + H) + (Gc l0 / 2) F^-1 |D|^2 F] d = H, solved by CG
 * starting from the d passed in (in: d^n, out: d^{n+1}).  H device [N]. */
int fgcg_phasefield_solve(fgcg_ctx* ctx, const double* H, double Gc, double l0, double* d,
                          double tol, int maxit, fgcg_info* info);

/* One backward-Euler step of dc/dt = div(D(x) grad c) - k(x) c with the flux
 * of Sec. 2.1 (j = -D grad c, D defined voxel by voxel through the phase
 * indicator) and a first-order sink:
 *     [(1/dt + k) - div D grad] c = c^n / dt,
 * div = -grad^H with the forward-difference gradient, applied as the 5-point
 * (7-point in 3D) flux stencil.  Voxels with dirichlet_mask != 0 hold
 * c = c_dir; CG runs on the other voxels from c^n (stop: ||r|| <= tol ||b||).
 *   c               device [N], in c^n, out c^{n+1}
 *   Dfield          device [N] diffusion coefficient per voxel (m^2/s, >= 0)
 *   krate           device [N] first-order rate per voxel (1/s, >= 0) or NULL (0)
 *   dirichlet_mask  device [N] uint8 or NULL (no Dirichlet voxels)
 * The fields are not checked on the host: a negative or non-finite value ends
 * the solve with EBREAKDOWN or EDOMAIN.  EINVAL for NULL c/Dfield or bad
 * tol/maxit, EDOMAIN for dt <= 0 or a non-finite c_dir. */
int fgcg_diffusion_step(fgcg_ctx* ctx, double* c, const double* Dfield, const double* krate,
                        const uint8_t* dirichlet_mask, double c_dir, double dt, double tol, int maxit,
                        fgcg_info* info);

/* The same step with per-phase tables (the fast path of the staggered step:
 * one byte per voxel instead of seventeen): D = D_tab[phase], k = k_tab[phase]
 * (host [nphase]), Dirichlet voxels x index < band_width with c = c_dir. */
int fgcg_diffusion_step_phases(fgcg_ctx* ctx, const uint8_t* phase, int nphase, const double* D_tab,
                               const double* k_tab, int band_width, double c_dir, double dt, double* c,
                               double tol, int maxit, fgcg_info* info);

/* Static diffusion homogenisation on the representative volume (Sec. 2.1,
 * eq. diffusion / eq. diffusion-weak-form / eq. diffusion-final; the diffusion
 * block of Alg. 1): the concentration gradient is the primary unknown,
 * grad c = grad c_mac + x with x compatible (range of the vector projection G
 * of App. A, forward-difference gradient of Sec. 2.6) and G[D grad c] = 0,
 * i.e. div j = 0 with j = -D grad c and <grad c> = grad c_mac.  Solved by CG
 * from x = 0 carried on the scalar fluctuation phi (x = grad phi), with the
 * Green operator (grad^H grad)^-1 as preconditioner: the same iterates as the
 * projected CG on x.  Stop when ||r|| <= tol ||b|| (norm of the projected
 * flux residual) or after maxit iterations.  FP64 contexts, 2D and 3D.
 *   Dfield     device [N] diffusion coefficient per voxel (> 0)
 *   grad_cmac  host [dim] macroscopic concentration gradient
 *   grad_c     device [dim][N] out or NULL: grad c = grad c_mac + grad phi
 *   phi        device [N] out or NULL: the periodic fluctuation (mean zero)
 *   mean_flux  host [dim] out or NULL: <j> = -<D grad c>
 * EUNSUPPORTED in FP32-mixed contexts; Dfield is not checked on the host (a
 * non-positive or non-finite value ends the solve with EBREAKDOWN/EDOMAIN). */
int fgcg_diffusion_homogenize(fgcg_ctx* ctx, const double* Dfield, const double* grad_cmac, double tol,
                              int maxit, double* grad_c, double* phi, double* mean_flux, fgcg_info* info);

/* Effective diffusivity of the volume (the quantity of App. B's sensitivity
 * study): <j> = -D_eff grad c_mac; column a from the homogenisation with
 * grad c_mac = e_a.  Deff: host [dim][dim] row-major out; infos: host [dim]
 * or NULL.  Returns the worst status of the dim solves. */
int fgcg_diffusivity_eff(fgcg_ctx* ctx, const double* Dfield, double tol, int maxit, double* Deff,
                         fgcg_info* infos);

/* Concentration from a concentration-gradient field (eqs. micro-gradient,
 * concentration, phi-fft, psi-two-values, concentration-correct; the
 * "periodic fluctuations" and "concentration" lines of Alg. 1):
 * phi_hat = (i xi)^-1 . (grad c)_hat with the inverse gradient of eq. g-42
 * (zero at k = 0), then c(x) = grad c_mac . x + phi(x) + beta_phase with x of
 * voxel (ix, iy, iz) = (ix, iy, iz) h, beta_pore chosen so that the pore mean
 * is c_mac / eta and beta_solid so that the solid mean is 0 (eta = pore share;
 * pores are phase 0).
 *   phase  device [N] uint8;  grad_c device [dim][N];  grad_cmac host [dim]
 *   c      device [N] out;  beta host [2] out or NULL: beta_pore, beta_solid
 * FP64 contexts. */
int fgcg_concentration(fgcg_ctx* ctx, const uint8_t* phase, const double* grad_c, const double* grad_cmac,
                       double c_mac, double* c, double* beta);

/* Staggered corrosion-fracture step (Alg. 1).  State fields are device [N]
 * (strain: [n_s][N]) owned by the caller and updated in place.  On 3D grids
 * the diffusion step and the phase field run as real-space stencil CG. */
typedef struct {
  double* c;      /* ferrous-ion concentration (normalised) */
  double* f;      /* precipitate volume fraction */
  double* e;      /* isotropic eigenstrain */
  double* H;      /* history field max psi+ */
  double* d;      /* damage */
  double* strain; /* [n_s][N] last total strain */
  int step;
} fgcg_state;

typedef struct {
  fgcg_material mat;
  const double* D_tab; /* host [nphase] diffusion coefficient per phase */
  const double* k_tab; /* host [nphase] first-order rate per phase: the sink of the
                          diffusion step and the precipitation f += dt k c in the
                          same voxels (f unchanged where k = 0) */
  int band_width;      /* Dirichlet band x < band_width, c = c_dir */
  double c_dir;
  double dt;
  double e_per_f;      /* eigenstrain e = e_per_f f per unit precipitate fraction */
  double Gc, l0, kappa;
  double eps_mac[6];   /* n_s entries used */
  double tol_diff, tol_mech, tol_pf;
  int maxit;
  int diffuse;         /* 0: skip diffusion, prescribe e = e_ramp (step+1)/n_ramp in pores */
  double e_ramp;
  int n_ramp;
} fgcg_params;

typedef struct {
  fgcg_info diff, mech, pf;
  double mean_stress[6]; /* n_s entries used */
  double energy;
  double max_d;
  double damaged_fraction;   /* share of solid voxels with d > 0.9 */
  double porosity_increase;  /* sum of d over solid voxels / N */
  double total_precipitate;  /* sum of f */
} fgcg_step_info;

int fgcg_staggered_step(fgcg_ctx* ctx, fgcg_state* state, const fgcg_params* prm,
                        fgcg_step_info* info);

/* ---- multiscale coupling (Sec. 3.2) ------------------------------------ */
/* A macroscopic bar from the steel interface Y = 0 (ion influx J_in) to
 * Y = L (no flux) whose material points carry copies of one representative
 * volume, the volume of a context.  The bar runs along the volume's y axis.
 * Its flux is the volume's upscaled flux <j> = -D_eff grad c_mac (D_eff of
 * fgcg_diffusivity_eff, computed at creation); it is advanced by finite
 * volumes (ncell cells of width L / ncell, backward Euler, face conductance
 * D_eff,yy / dY) and hands the volume of cell i its concentration c_mac and
 * gradient g (the mean of the cell's two face gradients, -J_in / D_eff,yy at
 * Y = 0).  The volume's local concentration follows eq.
 * concentration-correct, c = g u + [pore] c_mac / eta, u the concentration of
 * the unit gradient along y (fgcg_concentration of the homogenisation with
 * grad c_mac = e_y and c_mac = 0, computed at creation); ions above the
 * solubility limit S precipitate irreversibly, c_ppt = max(c_ppt, (c - S)_+)
 * in the pores; the eigenstrain is e = (c_ppt M_ppt - 1)_+ (eq.
 * eigen-simplify); then, as in Alg. 1, the mechanics with eps_mac = 0 and the
 * damage of the previous step, the history and the phase field. */
typedef struct {
  int ncell;           /* bar cells, >= 2 */
  double length;       /* bar length L (m), > 0 */
  double dt;           /* time step (s), > 0 */
  double J_in;         /* influx at Y = 0 (mol / (m^2 s)), >= 0 */
  double solubility;   /* S (mol / m^3), >= 0 */
  double molar_volume; /* M_ppt (m^3 / mol), >= 0 */
  double Gc, l0;       /* phase field, > 0 */
  double kappa;        /* residual stiffness, >= 0 */
  double tol;          /* CG tolerance of the mechanics and phase-field solves */
  double tol_homog;    /* CG tolerance of the homogenisations at creation */
  int maxit;           /* CG iteration cap of every solve, >= 1 */
} fgcg_ms_params;

typedef struct {
  double c_mac, grad_mac;  /* concentration and gradient of the volume's cell */
  double mean_cppt;        /* volume mean of c_ppt */
  double max_e, max_d;     /* maxima of the eigenstrain and of the damage */
  double mean_stress[6];   /* n_s entries used */
  double energy;
  fgcg_info mech, pf;
} fgcg_ms_info;

typedef struct fgcg_ms fgcg_ms;

/* Create the bar (c_bar = 0) and nrve volumes placed in the cells rve_cells
 * (host [nrve], 0..ncell-1; several volumes may share a cell), all of them
 * with zero precipitate, history and damage.  ctx: an FP64 context of the
 * volume's grid (2D or 3D), used by every call and to outlive the object;
 * mat: phase tables (E_field NULL; mat->phase device [N], kept by pointer,
 * pores are phase 0 and must exist); D_rve: device [N] diffusion coefficient
 * per voxel, read at creation only.  Allocates 8 N (2D) or 11 N (3D) doubles
 * per volume.  EINVAL for NULL pointers or a cell outside the bar; EDOMAIN for
 * a parameter outside its domain, a volume without pores or D_eff,yy <= 0;
 * EUNSUPPORTED for FP32-mixed or batch contexts; homogenisation errors as
 * fgcg_diffusion_homogenize. */
int fgcg_ms_create(fgcg_ctx* ctx, const fgcg_material* mat, const double* D_rve, const fgcg_ms_params* prm,
                   int nrve, const int* rve_cells, fgcg_ms** out);
/* One time step: the bar, then every volume in turn.  infos: host [nrve] or
 * NULL.  Returns FGCG_OK, the worst non-converged status of the volume solves,
 * or the first error. */
int fgcg_ms_step(fgcg_ms* ms, fgcg_ms_info* infos);
/* The bar: c_bar, grad_bar host [ncell], D_eff host [dim][dim], time host [1];
 * each may be NULL. */
int fgcg_ms_read(const fgcg_ms* ms, double* c_bar, double* grad_bar, double* D_eff, double* time);
/* Copy the state of volume rve into device buffers (each may be NULL): the
 * local concentration, c_ppt, e, H, d [N] and the strain [n_s][N] of the
 * last step. */
int fgcg_ms_volume(const fgcg_ms* ms, int rve, double* c, double* cppt, double* e, double* H, double* d,
                   double* strain);
void fgcg_ms_destroy(fgcg_ms* ms);

/* ---- no allocation --------------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * fgcg_phasefield_solve with the stencil operator (the default) in textbook CG
 * form (FGCG_OPT_SCALAR_CG = 0 on 2D grids), FP64, without
 * a context.  Every work buffer lives in a device array of the library
 * (40 MiB per device, held until the process ends); the call allocates
 * nothing.  grid->precision must be FGCG_FP64, axis lengths as fgcg_create,
 * at most 2^20 voxels (EINVAL beyond).  hip_stream: the stream the work goes
 * to (NULL: the null stream); the call returns after it has finished.  H, d
 * as fgcg_phasefield_solve (d: in d^n, out d^{n+1}).  Calls that overlap on
 * one device race on the shared array. */
int fgcg_phasefield_solve_noalloc(const fgcg_grid* grid, void* hip_stream, const double* H, double Gc,
                                  double l0, double* d, double tol, int maxit, fgcg_info* info);

/* ---- kernel-level test hooks ------------------------------------------ */
/* One application of an operator of the mechanics solver through the very
 * kernels a solve launches, in the context's precision (FP32-mixed: in is
 * rounded to FP32, out is the FP32 result widened), on 2D and 3D grids:
 *   FGCG_OP_MECH_K  out = K in, K = grad^H g C sym(grad) (Sec. 2.3 with the
 *                   forward difference of Sec. 2.6), the tiled stiffness pass;
 *   FGCG_OP_MECH_M  out = M in, M = (grad^H grad)^-1 per component (App. A's
 *                   projection factored through the displacement; zero mean),
 *                   the row / column (2D) or x / y / z (3D) transform passes
 *                   with the Green symbol, tuned radix plans.
 * in, out: device [n_u][N] displacement-like fields, n_u = 2 (2D) or 3 (3D).
 * The workspace and CG state of the context are overwritten.  EINVAL for NULL
 * pointers or an unknown op; material errors as fgcg_mech_solve. */
enum { FGCG_OP_MECH_K = 0, FGCG_OP_MECH_M = 1 };
int fgcg_debug_apply(fgcg_ctx* ctx, int op, const fgcg_material* mat, const double* d, double kappa,
                     const double* in, double* out);
/* 2D grids only (EUNSUPPORTED in 3D): the scalar operators through the
 * spectral passes. */
/* q = (Gc/(2 l0) + H) v + (Gc l0/2) F^-1 |D|^2 F v. */
int fgcg_phasefield_apply(fgcg_ctx* ctx, const double* H, double Gc, double l0, const double* v,
                          double* q);
/* q = (1/dt + k) v + sum_a F^-1 conj(D_a) F D(x) F^-1 D_a F v (no band). */
int fgcg_diffusion_apply(fgcg_ctx* ctx, const uint8_t* phase, int nphase, const double* D_tab,
                         const double* k_tab, double dt, const double* v, double* q);

/* Real-input discrete Fourier transform of one field (exp(-2 pi i k.x / n),
 * the transform of Sec. 2.1) through the transform passes of the solvers, FP64.
 *   dir > 0: in device [N] real -> out device [nz][ny][nx/2+1] complex
 *            (interleaved re, im; nz = 1 in 2D), unnormalised;
 *   dir < 0: in that half spectrum -> out [N] real, with the factor 1/N.
 * A kernel-level test hook: the forward output has the layout of the usual
 * real-input FFT routines.  Returns EINVAL for NULL pointers. */
int fgcg_debug_fft(fgcg_ctx* ctx, int dir, const double* in, double* out);

/* ---- profiling -------------------------------------------------------- */
/* Measurement hook for the HBM roofline of the 2D mechanics passes (Sec. 2.6
 * iteration): launches the pass of kind FGCG_K_MECH_ROW_FWD, _ROW_INV or
 * _COL (enum below; of the context's iteration form: in the two-pass form
 * _ROW_FWD is the fused row stage and there is no _ROW_INV, EUNSUPPORTED;
 * in the three-pass form _ROW_FWD is the stiffness + transform pass) reps
 * times back to back (after 3 untimed launches) on the
 * context's stream, between two HIP events, with the context's tuned rows per
 * block and radix plans (tuned first if not yet tuned), and stores the
 * average duration of one launch in microseconds (host double).  Unlike
 * events around every launch inside the CG graphs, back-to-back launches do
 * not add the dispatch gap of an event node to each launch.  The workspace is
 * first set to zero fields with a running CG state, so the pass does its full
 * work on data of the context's sizes; the previous solution in the workspace
 * is lost (the next solve starts over as always).  Synchronises the stream.
 * EINVAL for NULL pointers, another kind or reps outside 1..100000;
 * EUNSUPPORTED on 3D contexts. */
int fgcg_time_pass(fgcg_ctx* ctx, int kind, int reps, double* us_per_launch);

/* Kernel kinds that can be timed with HIP events around every launch. */
enum {
  FGCG_K_MECH_ROW_FWD = 0,
  FGCG_K_MECH_COL = 1,
  FGCG_K_MECH_ROW_INV = 2,
  FGCG_K_PF_ROW_FWD = 3,
  FGCG_K_PF_COL = 4,
  FGCG_K_PF_ROW_INV = 5,
  FGCG_K_DIFF_ROW_FWD = 6,
  FGCG_K_DIFF_COL_GRAD = 7,
  FGCG_K_DIFF_ROW_MID = 8,
  FGCG_K_DIFF_COL_DIV = 9,
  FGCG_K_DIFF_ROW_INV = 10,
  FGCG_K_MECH_KP = 11,
  FGCG_K_MECH_Y_FWD = 12, /* 3D: y transforms of the Green operator */
  FGCG_K_MECH_Y_INV = 13,
  FGCG_K_EVENT_GAP = 14, /* an empty one-block kernel (see below) */
  FGCG_K_NKINDS = 15
};
/* While FGCG_K_EVENT_GAP is profiled, every CG iteration of a graph chunk ends
 * with an empty one-block kernel node, timed like the others: its duration is
 * the dispatch gap that the two event-record nodes around a kernel node add to
 * that kernel's event-timed duration. */
/* On 3D grids FGCG_K_MECH_COL times the z pass (forward z transform, Green
 * symbol, inverse z transform). */
/* mask: bit k enables event timing of kind k (0 disables); resets counters. */
int fgcg_profile(fgcg_ctx* ctx, unsigned mask);
/* Accumulated device time (ms) and launch count of kind k since fgcg_profile. */
int fgcg_profile_read(fgcg_ctx* ctx, int kind, double* ms, long long* launches);
/* Kernel symbol name of kind k (for matching profiler output). */
const char* fgcg_kernel_name(fgcg_ctx* ctx, int kind);

#ifdef __cplusplus
}
#endif
#endif
