"""Multiscale coupling of the diffusion (Sec. 3.2): a macroscopic bar whose
material points each carry a representative volume (test infrastructure).

The bar runs from the steel interface Y = 0 (constant influx J_in of ferrous
ions) to Y = L (no flux).  Macroscopic diffusion, Sec. 3.2: the RVE flux
<j> = -D_eff grad c_mac is upscaled and the bar is solved by finite
differences; the macroscopic concentration c(X) is passed back to the RVE,
where the local concentration follows from eq. concentration-correct, the
precipitate from the solubility limit (Sec. 3.1: ions above S(pH)
precipitate), the eigenstrain from eq. eigen-simplify, then the stresses
(eps_mac = 0) and the phase field, every time step.

Readings (the paper gives the scheme in words only):
* the RVE problem is linear in grad c_mac, so its flux is -D_eff grad c_mac
  with D_eff from one homogenisation per axis (App. B's quantity), and its
  fluctuation for grad c_mac = g e_y is g phi_y (phi_y: unit gradient);
* the bar is along the RVE's y axis; cells of width dY, centres
  (i + 1/2) dY; backward Euler, face diffusivity the harmonic mean of the
  two cells, influx J_in through the face at Y = 0, none at Y = L;
* the gradient handed to the RVE of cell i is the mean of the gradients of
  its two faces (the boundary faces take the gradient their flux implies);
* precipitation is irreversible: c_ppt = max over time of (c(x) - S)_+ in
  the pores; the eigenstrain is e = (c_ppt M_ppt - 1)_+ in the pores
  (eq. eigen-simplify);
* history, phase field and degradation as in the staggered step (Alg. 1).
"""
from dataclasses import dataclass, field

import numpy as np

from . import homogenisation as _hm
from . import material as _mat
from . import mech as _mech
from . import phasefield as _pf


@dataclass
class BarParams:
    """SI units: m, s, mol / m^3."""
    ncell: int = 20
    length: float = 0.02        # m (20 mm)
    J_in: float = 1e-2          # mol / (m^2 s)
    dt: float = 1e4             # s
    D_eff: float = 1e-10        # m^2 / s, bar direction


def bar_step(c, prm, D_eff=None):
    """One backward-Euler step of the finite-volume bar; D_eff per cell
    (default: uniform prm.D_eff).  Returns the new c (host array)."""
    n = prm.ncell
    dY = prm.length / n
    D = np.full(n, prm.D_eff) if D_eff is None else np.asarray(D_eff, dtype=np.float64)
    Df = 2.0 * D[:-1] * D[1:] / (D[:-1] + D[1:])  # interior faces
    A = np.zeros((n, n))
    rhs = c * dY / prm.dt
    for i in range(n):
        A[i, i] = dY / prm.dt
    for f in range(n - 1):  # face between cells f and f + 1
        g = Df[f] / dY
        A[f, f] += g
        A[f, f + 1] -= g
        A[f + 1, f + 1] += g
        A[f + 1, f] -= g
    rhs = rhs.copy()
    rhs[0] += prm.J_in
    return np.linalg.solve(A, rhs)


def cell_gradients(c, prm, D_eff=None):
    """dc/dY at the cell centres: the mean of the two face gradients; the
    face at Y = 0 carries J_in = -D dc/dY, the face at Y = L none."""
    n = prm.ncell
    dY = prm.length / n
    D = np.full(n, prm.D_eff) if D_eff is None else np.asarray(D_eff, dtype=np.float64)
    faces = np.zeros(n + 1)
    faces[0] = -prm.J_in / D[0]
    faces[1:n] = (c[1:] - c[:-1]) / dY
    faces[n] = 0.0
    return 0.5 * (faces[:-1] + faces[1:])


def constant_flux_solution(Y, t, J, D):
    """Semi-infinite medium, influx J at Y = 0 from t = 0 (closed form):
    c = (2 J / D) sqrt(D t / pi) exp(-Y^2 / (4 D t)) - (J Y / D) erfc(Y / (2 sqrt(D t)))."""
    from scipy.special import erfc
    s = np.sqrt(D * t)
    return (2.0 * J / D) * s / np.sqrt(np.pi) * np.exp(-Y * Y / (4.0 * D * t)) - (J * Y / D) * erfc(Y / (2.0 * s))


@dataclass
class RveParams:
    h: float = 5e-6
    E_tab: tuple = (3e6, 30e9)
    nu_tab: tuple = (0.2, 0.2)
    D_tab: tuple = (1e-9, 1e-12)
    solubility: float = 1.0          # mol / m^3 (1e-9 mol / mm^3, Sec. 3.1)
    molar_volume: float = 2.6e-5     # m^3 / mol (Fe(OH)2, 26 cm^3 / mol; eq. eigen-simplify)
    Gc: float = 50.0
    l0: float = 1e-5
    kappa: float = 1e-6
    tol: float = 1e-12
    maxit: int = 50000


@dataclass
class RveState:
    cppt: np.ndarray
    e: np.ndarray
    H: np.ndarray
    d: np.ndarray
    strain: np.ndarray = None
    info: dict = field(default_factory=dict)


def rve_setup(phase, prm):
    """D_eff of the RVE and the unit-gradient fluctuation along y."""
    phase = np.asarray(phase)
    Df = np.asarray(prm.D_tab)[phase]
    Deff, _ = _hm.effective_diffusivity(Df, prm.h, tol=prm.tol, maxit=prm.maxit)
    unit = _hm.diffusion_homogenise(Df, _along_y(1.0, phase.ndim), prm.h, tol=prm.tol, maxit=prm.maxit)
    return Deff, unit["grad_c"]


def _along_y(g, dim):
    """The vector g e_y (components ordered x, y[, z])."""
    v = [0.0] * dim
    v[1] = g
    return tuple(v)


def rve_initial(phase):
    z = np.zeros(np.asarray(phase).shape)
    return RveState(cppt=z.copy(), e=z.copy(), H=z.copy(), d=z.copy())


def rve_step(phase, st, grad_c_unit, g, c_mac, prm):
    """One RVE update (2D or 3D) for the macroscopic gradient g (along y) and
    concentration c_mac: local concentration (eq. concentration-correct with
    grad c = g grad_c_unit), precipitation, eigenstrain (eq. eigen-simplify),
    mechanics with the previous damage, history, phase field."""
    phase = np.asarray(phase)
    dim = phase.ndim
    pore = phase == 0
    rec = _hm.concentration(phase, g * np.asarray(grad_c_unit), _along_y(g, dim), c_mac, prm.h)
    c = rec["c"]
    cppt = np.where(pore, np.maximum(st.cppt, np.maximum(c - prm.solubility, 0.0)), 0.0)
    e = np.where(pore, np.maximum(cppt * prm.molar_volume - 1.0, 0.0), 0.0)
    m = _mech.mech_solve(phase, prm.E_tab, prm.nu_tab, (0.0,) * (3 if dim == 2 else 6), prm.h, d=st.d,
                         kappa=prm.kappa, e=e, tol=prm.tol, maxit=prm.maxit)
    lam, mu = _mech.voxel_lame(phase, prm.E_tab, prm.nu_tab)
    el = _mat.from_voigt(m["strain"], dim) - _mech.eigen_tensor(e, dim, phase.shape)
    H = np.maximum(st.H, _mat.psi_plus(el, lam, mu))
    p = _pf.phasefield_solve(H, prm.Gc, prm.l0, prm.h, d0=st.d, tol=prm.tol, maxit=prm.maxit)
    info = dict(c=c, mean_stress=m["mean_stress"], mean_cppt=float(cppt.mean()), max_d=float(p["d"].max()))
    return RveState(cppt=cppt, e=e, H=H, d=p["d"], strain=m["strain"], info=info)
