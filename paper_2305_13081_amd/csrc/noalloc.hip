// fgcg_phasefield_solve_noalloc: the AT2 phase-field solve of
// fgcg_phasefield_solve (the stencil CG, FP64) for callers that cannot
// allocate device memory.  Every work buffer (solution, residual, the two
// direction buffers, A p, the partial sums and the CG state) lives in one
// file-scope device array; the entry point calls no allocating routine and
// needs no context.
//
// Each device the library runs on holds its own copy of the array until the
// process ends.  Its device address is looked up once per device (with that
// device current) and kept; host code passes that address to the kernels,
// never the array's name.  All calls on one device share the array: calls
// that overlap on one device race.  Nothing in it has to start at zero (every
// kernel writes what the next one reads).
#include <mutex>

#include "engine.hpp"

using namespace fgcg;

namespace {

constexpr long long NOALLOC_MAX_VOXELS = 1LL << 20;    // 1024^2 or 128 x 128 x 64
constexpr int PART_A = 2048, PART_RR = 512, PART_B = 512;  // partial sums of the stencil CG
constexpr long long STATE_DOUBLES = (sizeof(CgState) + 7) / 8;
constexpr long long SCRATCH_DOUBLES = 5 * NOALLOC_MAX_VOXELS + PART_A + PART_RR + PART_B + STATE_DOUBLES;

__device__ __align__(256) double scratch[SCRATCH_DOUBLES];  // 40.0 MiB

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {nullptr};

// Device address of the array on the current device (looked up once).
int scratch_on_current(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(FGCG_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return 0;
}

__global__ void __launch_bounds__(NT) k_fill(double* v, long long n, double val) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) v[i] = val;
}

}  // namespace

extern "C" int fgcg_phasefield_solve_noalloc(const fgcg_grid* grid, void* hip_stream, const double* H, double Gc,
                                             double l0, double* d, double tol, int maxit, fgcg_info* info) {
  if (!grid || !H || !d) return fail(FGCG_EINVAL, "grid/H/d is NULL");
  int rc;
  if ((rc = check_solver_args(tol, maxit))) return rc;
  if (grid->ndim != 2 && grid->ndim != 3) return fail(FGCG_EINVAL, "ndim must be 2 or 3");
  if (grid->precision != FGCG_FP64) return fail(FGCG_EUNSUPPORTED, "the no-allocation solve is FP64");
  if (!(grid->h > 0.0) || !std::isfinite(grid->h)) return fail(FGCG_EDOMAIN, "h <= 0");
  if (!(Gc > 0.0) || !std::isfinite(Gc)) return fail(FGCG_EDOMAIN, "Gc <= 0");
  if (!(l0 > 0.0) || !std::isfinite(l0)) return fail(FGCG_EDOMAIN, "l0 <= 0");
  const int nx = grid->n[0], ny = grid->n[1], nz = grid->ndim == 3 ? grid->n[2] : 1;
  if (grid->ndim == 2 ? !(size_supported(nx) && size_supported(ny))
                      : !(size3_supported(nx) && size3_supported(ny) && size3_supported(nz)))
    return fail(FGCG_EINVAL, "axis lengths as for fgcg_create");
  const long long n = (long long)nx * ny * nz;
  if (n > NOALLOC_MAX_VOXELS) return fail(FGCG_EINVAL, "grid larger than the no-allocation limit of 2^20 voxels");
  const double t0 = now();
  double* base = nullptr;
  if ((rc = scratch_on_current(&base))) return rc;
  double* X = base;
  double* R = X + n;
  double* P0 = R + n;
  double* P1 = P0 + n;
  double* Q = P1 + n;
  double* part_a = base + 5 * NOALLOC_MAX_VOXELS;
  double* part_rr = part_a + PART_A;
  double* part_b = part_rr + PART_RR;
  CgState* st = (CgState*)(part_b + PART_B);
  hipStream_t s = (hipStream_t)hip_stream;
  // the launch shapes of the context solve, so the two give the same result
  const int sblocks = (int)std::max<long long>(8, std::min<long long>((n + NT - 1) / NT, 512) & ~7LL);
  const dim3 sgrid(sblocks);
  const int ndir = std::min(scg_chunks(nx, ny, nz), PART_A);
  const PfStencil op{H, Gc / (2.0 * l0), 0.5 * Gc * l0 / (grid->h * grid->h)};
  hipLaunchKernelGGL((k_scg_init<double, PfStencil>), sgrid, dim3(NT), 0, s, op, (const double*)d, 1.0, H, 0.0, X, R,
                     nx, ny, nz, part_b, part_rr);
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(NT), 0, s, st, (const double*)part_b, sblocks, 0, tol, maxit);
  HIPCHK(hipGetLastError());
  const CgCtl cc{st, part_a, part_rr, ndir, sblocks, 0, 0};
  CgState hs;
  long long k = 0;
  int chunk = 2, parity = 0;
  for (;;) {
    HIPCHK(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hs.done) break;
    if (k > (long long)maxit + 1) return fail(FGCG_EHIP, "CG driver overran the iteration limit");
    for (int j = 0; j < chunk; ++j, ++k) {
      double* pin = parity ? P1 : P0;
      double* pout = parity ? P0 : P1;
      parity ^= 1;
      hipLaunchKernelGGL((k_scg_dir<double, PfStencil>), dim3(ndir), dim3(NT), 0, s, op, (const double*)R,
                         (const double*)pin, pout, Q, nx, ny, nz, cc);
      hipLaunchKernelGGL((k_scg_upd<double>), sgrid, dim3(NT), 0, s, X, R, (const double*)pout, (const double*)Q, nx,
                         (int)((long long)ny * nz), cc);
    }
    HIPCHK(hipGetLastError());
    chunk = chunk < 32 ? chunk * 2 : 32;
  }
  const int nb = (int)std::min<long long>((n + NT - 1) / NT, 1024);
  if (hs.zero_rhs)
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(NT), 0, s, d, n, 0.0);
  else
    hipLaunchKernelGGL((k_convert<double, double>), dim3(nb), dim3(PT), 0, s, d, (const double*)X, n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  fill_info(info, hs, now() - t0);
  return status_of(hs);
}
