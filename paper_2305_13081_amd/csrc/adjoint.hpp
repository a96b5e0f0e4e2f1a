// Adjoint of the mechanical equilibrium with respect to the per-voxel Young's
// modulus.
//
// With sigma = C_x : (eps - e I), C_x = g(d_x) E_x C_hat(nu) (so
// dC_x/dE_x = C_x / E_x) and an objective J(eps, E) with first variation
// dJ = sum_x G_x : d eps_x (G symmetric, "dJ/deps"), the gradient is
//     dJ/dE_x = dJ/dE_x|_eps - sym(grad lam)_x : sigma_x / E_x,
// where lam solves the adjoint problem K lam = grad^H G with the forward
// operator K = grad^H g C grad (symmetric), i.e. a second preconditioned CG
// solve on the same engine; the forward strain is recomputed, no CG history
// is stored.  Built-in objectives:
//   energy W = h^2/2 sum_x (eps - eI) : sigma: G = h^2 sigma, grad^H G = 0 at
//            equilibrium, lam = 0 (envelope theorem), explicit part
//            h^2/2 (eps - eI) : sigma / E_x;
//   C11    <sigma_11> / eps11_mac: G = C_x : e_11 / (N eps11), explicit part
//            sigma_11 / (N eps11 E_x).
#pragma once
#include "mech_u.hpp"

namespace fgcg {

enum { ADJ_USER = 0, ADJ_ENERGY = 1, ADJ_C11 = 2 };

// Young's modulus from the Lame constants: E = mu (3 lambda + 2 mu) / (lambda + mu).
__device__ __forceinline__ double young(double lam, double mu) { return mu * (3.0 * lam + 2.0 * mu) / (lam + mu); }

// G field (Voigt, tensor shear) of the objective.
__global__ void __launch_bounds__(NT) k_adj_g(MechMat m, const double* __restrict__ strain,
                                              const double* __restrict__ eig, const double* __restrict__ dJ,
                                              int objective, double scale, long long n, double* __restrict__ G) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    double g0 = 0, g1 = 0, g2 = 0;
    if (objective == ADJ_USER) {
      g0 = dJ[i];
      g1 = dJ[n + i];
      g2 = dJ[2 * n + i];
    } else {
      double lam, mu;
      m.get(0, i, lam, mu);
      if (objective == ADJ_ENERGY) {
        const double e = eig ? eig[i] : 0.0;
        const double l11 = strain[i] - e, l22 = strain[n + i] - e, l12 = strain[2 * n + i];
        const double tr = l11 + l22;
        g0 = scale * (lam * tr + 2.0 * mu * l11);
        g1 = scale * (lam * tr + 2.0 * mu * l22);
        g2 = scale * (2.0 * mu * l12);
      } else {  // C11: C : e_11
        g0 = scale * (lam + 2.0 * mu);
        g1 = scale * lam;
        g2 = 0.0;
      }
    }
    G[i] = g0;
    G[n + i] = g1;
    G[2 * n + i] = g2;
  }
}

// r = grad^H G (two components), x = 0
__global__ void __launch_bounds__(NT) k_adj_rhs(const double* __restrict__ G, double* __restrict__ r,
                                                double* __restrict__ x, long long n, int nx, int ny, double ih) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const int y = (int)(i / nx), xx = (int)(i - (long long)y * nx);
    const long long ixm = (long long)y * nx + (xx == 0 ? nx - 1 : xx - 1);
    const long long iym = (long long)(y == 0 ? ny - 1 : y - 1) * nx + xx;
    const double g0[3] = {G[i], G[n + i], G[2 * n + i]};
    const double gx[3] = {G[ixm], G[n + ixm], G[2 * n + ixm]};
    const double gy[3] = {G[iym], G[n + iym], G[2 * n + iym]};
    double q[2];
    div_adj<double>(g0, gx, gy, ih, q);
    r[i] = q[0];
    r[n + i] = q[1];
    x[i] = 0.0;
    x[n + i] = 0.0;
  }
}

// grad_E = explicit part - sym(grad lam) : sigma / E_x
__global__ void __launch_bounds__(NT) k_adj_grad(MechMat m, const double* __restrict__ strain,
                                                 const double* __restrict__ eig, const double* __restrict__ lam_u,
                                                 int objective, double scale, int have_lam, long long n, int nx,
                                                 int ny, double ih, double* __restrict__ grad) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const int y = (int)(i / nx), xx = (int)(i - (long long)y * nx);
    double lam, mu, lam0, mu0;
    m.get(0, i, lam, mu);
    MechMat m0 = m;
    m0.d = nullptr;
    m0.get(0, i, lam0, mu0);
    const double E = young(lam0, mu0);  // undegraded: dC/dE = C / E
    const double e = eig ? eig[i] : 0.0;
    const double l11 = strain[i] - e, l22 = strain[n + i] - e, l12 = strain[2 * n + i];
    const double tr = l11 + l22;
    const double s11 = lam * tr + 2.0 * mu * l11, s22 = lam * tr + 2.0 * mu * l22, s12 = 2.0 * mu * l12;
    double g = 0.0;
    if (objective == ADJ_ENERGY) g = 0.5 * scale * (l11 * s11 + l22 * s22 + 2.0 * l12 * s12) / E;
    else if (objective == ADJ_C11) g = scale * s11 / E;
    if (have_lam) {
      const long long ixp = (long long)y * nx + (xx + 1 == nx ? 0 : xx + 1);
      const long long iyp = (long long)(y + 1 == ny ? 0 : y + 1) * nx + xx;
      const double a11 = (lam_u[ixp] - lam_u[i]) * ih;
      const double a12 = (lam_u[iyp] - lam_u[i]) * ih;
      const double a21 = (lam_u[n + ixp] - lam_u[n + i]) * ih;
      const double a22 = (lam_u[n + iyp] - lam_u[n + i]) * ih;
      g -= (a11 * s11 + a22 * s22 + (a12 + a21) * s12) / E;
    }
    grad[i] = g;
  }
}

}  // namespace fgcg
