"""Pins of the oracle's multiscale coupling (Sec. 3.2), CPU only.

* the finite-volume bar conserves the ions: sum c dY = J_in t;
* it converges to the closed-form constant-influx solution of a
  semi-infinite medium (first order in dt);
* the cell gradients reproduce a linear profile and the boundary fluxes;
* one RVE update equals the same update assembled from the reconstruction
  formula written out, the sparse direct solvers and eq. energy by hand; the
  eigenstrain switches on only past the threshold of eq. eigen-simplify, and
  only in the pores; the same in 3D on a sphere pore.
"""
import numpy as np
import pytest

from oracle import direct, multiscale as ms
from paper_2305_13081_amd import inputs


def test_bar_conserves_ions():
    prm = ms.BarParams(ncell=16, dt=5e3)
    c = np.zeros(prm.ncell)
    dY = prm.length / prm.ncell
    for k in range(1, 11):
        c = ms.bar_step(c, prm, D_eff=1e-10 * (1 + 0.5 * np.sin(np.arange(prm.ncell))))
        assert abs(c.sum() * dY - prm.J_in * prm.dt * k) < 1e-12 * prm.J_in * prm.dt * k


def test_bar_converges_to_constant_flux_solution():
    T, D, J = 2e5, 1e-10, 1e-2
    errs = []
    for n, steps in ((40, 10), (80, 20), (160, 40)):
        prm = ms.BarParams(ncell=n, length=0.04, dt=T / steps, D_eff=D, J_in=J)
        c = np.zeros(n)
        for _ in range(steps):
            c = ms.bar_step(c, prm)
        Y = (np.arange(n) + 0.5) * prm.length / n
        exact = ms.constant_flux_solution(Y, T, J, D)
        errs.append(np.max(np.abs(c - exact)) / np.max(exact))
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1] and errs[2] < 0.05


def test_cell_gradients():
    prm = ms.BarParams(ncell=10)
    dY = prm.length / prm.ncell
    Y = (np.arange(10) + 0.5) * dY
    g = ms.cell_gradients(3.0 * Y, prm)
    assert np.allclose(g[1:-1], 3.0, rtol=1e-12)
    assert abs(g[0] - 0.5 * (-prm.J_in / prm.D_eff + 3.0)) < 1e-9 * abs(g[0])
    assert abs(g[-1] - 0.5 * 3.0) < 1e-12


def _psi_plus_by_hand(strain, e, lam, mu):
    l11, l22, l12 = strain[0] - e, strain[1] - e, strain[2]
    tr = l11 + l22
    d11, d22 = l11 - 0.5 * tr, l22 - 0.5 * tr
    return 0.5 * (lam + mu) * np.maximum(tr, 0.0) ** 2 + mu * (d11 ** 2 + d22 ** 2 + 2 * l12 ** 2)


@pytest.mark.parametrize("c_mac,g", [(8.5e3, -1e7), (3e3, -1e7)])
def test_rve_step_matches_assembled(c_mac, g):
    phase = inputs.circle_pore(16, 4.0)
    prm = ms.RveParams(E_tab=(3e8, 30e9), Gc=10.0, tol=1e-14)
    _, gcu = ms.rve_setup(phase, prm)
    st = ms.rve_initial(phase)
    pore = phase == 0
    for step in range(2):
        cm = c_mac * (1 + 0.1 * step)
        nxt = ms.rve_step(phase, st, gcu, g, cm, prm)
        # assembled: phi_y from the sparse direct homogenisation, c from eq.
        # concentration-correct written out, precipitation, eigenstrain, direct solves
        Df = np.asarray(prm.D_tab)[phase]
        phi = direct.diffusion_static_direct(Df, (0.0, 1.0), prm.h)["phi"]
        y = prm.h * np.arange(16)[:, None] * np.ones((1, 16))
        u = y + phi  # the unit-gradient part of c
        eta = pore.mean()
        bp = cm / eta - g * u[pore].mean()
        bs = -g * u[~pore].mean()
        c = g * u + np.where(pore, bp, bs)
        cppt = np.where(pore, np.maximum(st.cppt, np.maximum(c - prm.solubility, 0.0)), 0.0)
        e = np.where(pore, np.maximum(cppt * prm.molar_volume - 1.0, 0.0), 0.0)
        m = direct.mech_direct(phase, prm.E_tab, prm.nu_tab, (0.0, 0.0, 0.0), prm.h, d=st.d, kappa=prm.kappa, e=e)
        E, nu = np.asarray(prm.E_tab)[phase], np.asarray(prm.nu_tab)[phase]
        lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
        H = np.maximum(st.H, _psi_plus_by_hand(m["strain"], e, lam, mu))
        d = direct.phasefield_direct(H, prm.Gc, prm.l0, prm.h)
        assert np.max(np.abs(nxt.info["c"] - c)) < 1e-10 * np.max(np.abs(c))
        for k, ref in (("cppt", cppt), ("e", e), ("H", H), ("d", d), ("strain", m["strain"])):
            got = getattr(nxt, k)
            scale = max(np.linalg.norm(ref), 1e-300)
            assert np.linalg.norm(got - ref) <= 1e-10 * scale, (step, k)
        assert np.all(nxt.e[~pore] == 0.0)
        st = nxt
    if c_mac > 5e3:
        assert st.e.max() > 0 and st.d.max() > 1e-2
    else:
        assert st.e.max() == 0.0  # below the threshold c_ppt M_ppt = 1: no eigenstrain


def _psi_plus_3d_by_hand(strain, e, lam, mu):
    """Amor split in 3D written out: K/2 <tr>_+^2 + mu dev:dev, K = lam + 2 mu / 3,
    strain in Voigt order 11, 22, 33, 23, 13, 12 (tensor shear components)."""
    l = [strain[0] - e, strain[1] - e, strain[2] - e]
    tr = l[0] + l[1] + l[2]
    dev = sum((li - tr / 3.0) ** 2 for li in l) + 2.0 * (strain[3] ** 2 + strain[4] ** 2 + strain[5] ** 2)
    return 0.5 * (lam + 2.0 * mu / 3.0) * np.maximum(tr, 0.0) ** 2 + mu * dev


def test_rve_step_3d_matches_assembled():
    n = 8
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    phase = np.where((x - 3.5) ** 2 + (y - 3.5) ** 2 + (z - 3.5) ** 2 <= 2.6 ** 2, 0, 1).astype(np.uint8)
    prm = ms.RveParams(E_tab=(3e8, 30e9), Gc=10.0, tol=1e-14)
    _, gcu = ms.rve_setup(phase, prm)
    assert gcu.shape == (3, n, n, n)
    st = ms.rve_initial(phase)
    pore = phase == 0
    eta = pore.mean()
    cm, g = 9e3 * eta / 0.2, -1e7
    nxt = ms.rve_step(phase, st, gcu, g, cm, prm)
    Df = np.asarray(prm.D_tab)[phase]
    phi = direct.diffusion_static_direct(Df, (0.0, 1.0, 0.0), prm.h)["phi"]
    u = prm.h * y + phi
    c = g * u + np.where(pore, cm / eta - g * u[pore].mean(), -g * u[~pore].mean())
    cppt = np.where(pore, np.maximum(c - prm.solubility, 0.0), 0.0)
    e = np.where(pore, np.maximum(cppt * prm.molar_volume - 1.0, 0.0), 0.0)
    m = direct.mech_direct(phase, prm.E_tab, prm.nu_tab, (0.0,) * 6, prm.h, kappa=prm.kappa, e=e)
    E, nu = np.asarray(prm.E_tab)[phase], np.asarray(prm.nu_tab)[phase]
    lam, mu = E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))
    H = _psi_plus_3d_by_hand(m["strain"], e, lam, mu)
    d = direct.phasefield_direct(H, prm.Gc, prm.l0, prm.h)
    assert np.max(np.abs(nxt.info["c"] - c)) < 1e-10 * np.max(np.abs(c))
    assert e.max() > 0
    for k, ref in (("cppt", cppt), ("e", e), ("H", H), ("d", d), ("strain", m["strain"])):
        got = getattr(nxt, k)
        assert np.linalg.norm(got - ref) <= 1e-10 * max(np.linalg.norm(ref), 1e-300), k
