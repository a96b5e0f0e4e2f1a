"""One step of the staggered corrosion-fracture scheme (test infrastructure).

Alg. 1 order, each mechanism solved in turn:

1. diffusion of ferrous ions (here the transient backward-Euler step of
   ``oracle.diffusion`` with a Dirichlet source band and a first-order sink
   k c in the pores);
2. precipitation in the pores, f <- min(1, f + dt k c), and the isotropic
   eigenstrain e = e_per_f * f in the pores (eq. eigen-simplify with a linear
   precipitate-to-strain map);
3. mechanical equilibrium with the current damage (``oracle.mech``);
4. history update H <- max(H, psi+(eps - e I)) with the undegraded Lame
   constants of the voxel's phase (Sec. 2.4, eq. energy);
5. AT2 phase field from the previous damage (``oracle.phasefield``), which
   degrades the stiffness for the next step.

When ``diffuse`` is False, steps 1-2 are replaced by a prescribed pore
eigenstrain ramp e = e_ramp * (n + 1) / n_ramp.

Phase ids: 0 = pore, 1 = solid (the indicator omega of Sec. 2.1/2.3).
"""
from dataclasses import dataclass, field

import numpy as np

from . import diffusion as _diff
from . import material as _mat
from . import mech as _mech
from . import phasefield as _pf


@dataclass
class Params:
    h: float = 5e-6
    E_tab: tuple = (3e6, 30e9)
    nu_tab: tuple = (0.2, 0.2)
    D_tab: tuple = (1e-9, 1e-12)
    k_rate: float = 1e-3
    dt: float = 40.0
    band_width: int = 16
    c_dir: float = 1.0
    e_per_f: float = 0.005
    Gc: float = 50.0
    l0: float = 1e-5
    kappa: float = 1e-6
    eps_mac: tuple = (0.0, 0.0, 0.0)
    tol_diff: float = 1e-8
    tol_mech: float = 1e-8
    tol_pf: float = 1e-8
    maxit: int = 20000
    diffuse: bool = True
    e_ramp: float = 1e-3
    n_ramp: int = 20


@dataclass
class State:
    c: np.ndarray
    f: np.ndarray
    e: np.ndarray
    H: np.ndarray
    d: np.ndarray
    strain: np.ndarray = None
    step: int = 0
    info: dict = field(default_factory=dict)


def band_mask(grid, width):
    if width <= 0:
        return None
    x = np.arange(grid[-1])
    return np.broadcast_to(x < width, grid).copy()


def initial_state(phase, prm):
    grid = phase.shape
    z = np.zeros(grid)
    c = z.copy()
    band = band_mask(grid, prm.band_width) if prm.diffuse else None
    if band is not None:
        c[band] = prm.c_dir
    return State(c=c, f=z.copy(), e=z.copy(), H=z.copy(), d=z.copy())


def step(phase, st, prm):
    phase = np.asarray(phase)
    grid = phase.shape
    dim = phase.ndim
    pore = phase == 0
    info = {}
    if prm.diffuse:
        Dfield = np.asarray(prm.D_tab)[phase]
        react = np.where(pore, prm.k_rate, 0.0)
        band = band_mask(grid, prm.band_width)
        r = _diff.diffusion_step(st.c, Dfield, react, prm.dt, prm.h, band=band,
                                 c_dir=prm.c_dir, tol=prm.tol_diff,
                                 maxit=prm.maxit)
        c = r["c"]
        info["diff_iters"] = r["iters"]
        f = np.where(pore, np.minimum(1.0, st.f + prm.dt * prm.k_rate * c), 0.0)
        e = np.where(pore, prm.e_per_f * f, 0.0)
    else:
        c = st.c
        f = st.f
        e = np.where(pore, prm.e_ramp * (st.step + 1) / prm.n_ramp, 0.0)
    m = _mech.mech_solve(phase, prm.E_tab, prm.nu_tab, prm.eps_mac, prm.h,
                         d=st.d, kappa=prm.kappa, e=e, tol=prm.tol_mech,
                         maxit=prm.maxit)
    info["mech_iters"] = m["iters"]
    info["mean_stress"] = m["mean_stress"]
    info["energy"] = m["energy"]
    lam, mu = _mech.voxel_lame(phase, prm.E_tab, prm.nu_tab)
    el = _mat.from_voigt(m["strain"], dim) - _mech.eigen_tensor(e, dim, grid)
    H = np.maximum(st.H, _mat.psi_plus(el, lam, mu))
    p = _pf.phasefield_solve(H, prm.Gc, prm.l0, prm.h, d0=st.d, tol=prm.tol_pf,
                             maxit=prm.maxit)
    d = p["d"]
    info["pf_iters"] = p["iters"]
    info["max_d"] = float(d.max())
    info["damaged_fraction"] = float(np.mean(d[~pore] > 0.9)) if (~pore).any() else 0.0
    info["total_precipitate"] = float(f.sum())
    return State(c=c, f=f, e=e, H=H, d=d, strain=m["strain"], step=st.step + 1,
                 info=info)
