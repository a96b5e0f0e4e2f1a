"""Constitutive relations (test infrastructure).

* Isotropic stiffness per phase, Sec. 2.3: C_i = lambda_i I(x)I + 2 mu_i II,
  mixed voxel by voxel through the phase indicator.
* Degradation, Sec. 2.4: ((1 - d)^2 + kappa) C.
* Tension/compression energy split, Sec. 2.4 eq. energy (2D form):
  psi+ = (lambda + mu)/2 [tr e]_+^2 + mu e_dev : e_dev, e_dev = e - tr(e)/2 I.
  The 3D form uses the bulk modulus lambda + 2 mu / 3 and e_dev = e - tr(e)/3 I,
  which keeps psi+ + psi- equal to the full energy.
* Lame constants from (E, nu): lambda = E nu / ((1 + nu)(1 - 2 nu)),
  mu = E / (2 (1 + nu)); 2D problems are plane strain.
"""
import numpy as np


def lame(E, nu):
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def degradation(d, kappa):
    return (1.0 - d) ** 2 + kappa


def sym(t):
    return 0.5 * (t + np.swapaxes(t, 0, 1))


def trace(t):
    dim = t.shape[0]
    return sum(t[i, i] for i in range(dim))


def stress(eps, lam, mu):
    """sigma = lambda tr(eps) I + 2 mu eps for a symmetric tensor field."""
    dim = eps.shape[0]
    tr = trace(eps)
    sig = 2.0 * mu * eps
    for i in range(dim):
        sig[i, i] = sig[i, i] + lam * tr
    return sig


def energy_density(eps, lam, mu):
    """psi = eps : C : eps / 2."""
    return 0.5 * np.sum(eps * stress(eps, lam, mu), axis=(0, 1))


def _split(eps, lam, mu):
    dim = eps.shape[0]
    tr = trace(eps)
    dev = np.array(eps, dtype=np.float64, copy=True)
    for i in range(dim):
        dev[i, i] = dev[i, i] - tr / dim
    bulk = lam + mu if dim == 2 else lam + 2.0 * mu / 3.0
    devdev = np.sum(dev * dev, axis=(0, 1))
    tr_pos = 0.5 * (tr + np.abs(tr))
    tr_neg = 0.5 * (tr - np.abs(tr))
    return bulk, devdev, tr_pos, tr_neg


def psi_plus(eps, lam, mu):
    bulk, devdev, tr_pos, _ = _split(eps, lam, mu)
    return 0.5 * bulk * tr_pos ** 2 + mu * devdev


def psi_minus(eps, lam, mu):
    bulk, _, _, tr_neg = _split(eps, lam, mu)
    return 0.5 * bulk * tr_neg ** 2


def voigt_pairs(dim):
    """Voigt order: 2D (11, 22, 12); 3D (11, 22, 33, 23, 13, 12)."""
    if dim == 2:
        return [(0, 0), (1, 1), (0, 1)]
    return [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def to_voigt(t):
    return np.array([t[i, j] for (i, j) in voigt_pairs(t.shape[0])])


def from_voigt(v, dim):
    grid = v.shape[1:]
    t = np.zeros((dim, dim) + grid, dtype=v.dtype)
    for c, (i, j) in enumerate(voigt_pairs(dim)):
        t[i, j] = v[c]
        t[j, i] = v[c]
    return t
