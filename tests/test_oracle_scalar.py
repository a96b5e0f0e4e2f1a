"""Pins of the oracle's phase-field, diffusion and staggered-step code (CPU only).

Phase field (Sec. 2.4): uniform history closed form, the exact periodic 1-D
crack profile of the discrete equation, sparse direct solve, maximum principle.
Diffusion step: exact decay of a Fourier mode in one CG iteration, mass
conservation without sink or band, sparse direct solve with a Dirichlet band,
band voxels held, first-order convergence in dt to exp(-(D xi^2 + k) t).
Staggered step (Alg. 1): zero source keeps every field zero; the history field
never decreases and the damage stays in [0, 1); one and two steps equal the
same steps assembled from the sparse direct solvers in Alg. 1 order (also in
the fracture regime, d -> 1), a composition with the new damage in the
mechanics differs, and the history uses the undegraded moduli.
"""
import numpy as np
import pytest

from oracle import diffusion as df, direct, phasefield as pf, spectral as sp, staggered as stg
from paper_2305_13081_amd import inputs

GC, L0, H = 50.0, 1e-5, 5e-6


def test_pf_uniform_history():
    Hf = np.full((8, 8), 3.2e6)
    r = pf.phasefield_solve(Hf, GC, L0, H, tol=1e-14)
    assert np.allclose(r["d"], 3.2e6 / (GC / (2 * L0) + 3.2e6), rtol=1e-14)


def test_pf_one_dimensional_crack_profile():
    n = 32
    Hf = np.zeros((4, n))
    Hf[:, 0] = 1e12
    r = pf.phasefield_solve(Hf, GC, L0, H, tol=1e-15, maxit=5000)
    d = r["d"][0]
    q = 1 + H ** 2 / (2 * L0 ** 2)
    rho = q - np.sqrt(q * q - 1)
    j = np.arange(1, n)
    expect = (rho ** j + rho ** (n - j)) / (rho + rho ** (n - 1))
    assert np.allclose(d[1:] / d[1], expect, rtol=1e-10)
    assert np.allclose(r["d"], r["d"][0][None, :], atol=1e-15)


def test_pf_direct_and_maximum_principle():
    rng = np.random.default_rng(3)
    Hf = 1e7 * rng.random((8, 8)) ** 4
    r = pf.phasefield_solve(Hf, GC, L0, H, d0=0.1 * rng.random((8, 8)), tol=1e-14)
    q = direct.phasefield_direct(Hf, GC, L0, H)
    assert np.max(np.abs(r["d"] - q)) < 1e-13
    assert r["d"].min() >= 0 and r["d"].max() < 1


def test_diffusion_single_mode_one_iteration():
    n, m = 16, 3
    x = np.arange(n)
    c0 = np.broadcast_to(np.cos(2 * np.pi * m * x / n)[None, :], (n, n)).copy()
    Dv, k, dt = 1e-9, 1e-3, 40.0
    r = df.diffusion_step(c0, np.full((n, n), Dv), np.full((n, n), k), dt, H, tol=1e-10)
    lam = 4 * np.sin(np.pi * m / n) ** 2 / H ** 2
    assert r["iters"] <= 1
    assert np.allclose(r["c"], c0 / (1 + dt * k + dt * Dv * lam), rtol=0, atol=1e-14)


def test_diffusion_mass_conservation_loose_tol():
    rng = np.random.default_rng(8)
    phase = (rng.random((16, 16)) < 0.5).astype(np.uint8)
    Dfield = np.where(phase == 0, 1e-9, 1e-12)
    c0 = rng.random((16, 16))
    r = df.diffusion_step(c0, Dfield, 0.0, 40.0, H, tol=1e-6)
    assert r["iters"] > 0
    assert abs(r["c"].sum() - c0.sum()) < 1e-12 * c0.sum()


def test_diffusion_direct_with_band():
    rng = np.random.default_rng(9)
    phase = (rng.random((8, 10)) < 0.5).astype(np.uint8)
    Dfield = np.where(phase == 0, 1e-9, 1e-12)
    react = np.where(phase == 0, 1e-3, 0.0)
    band = np.zeros((8, 10), bool)
    band[:, :2] = True
    c0 = rng.random((8, 10))
    r = df.diffusion_step(c0, Dfield, react, 40.0, H, band=band, c_dir=0.7, tol=1e-14)
    q = direct.diffusion_direct(c0, Dfield, react, 40.0, H, band=band, c_dir=0.7)
    assert np.max(np.abs(r["c"] - q)) < 1e-10 * np.max(np.abs(q))
    assert np.all(r["c"][band] == 0.7)


def test_diffusion_converges_to_continuum_decay():
    n, m = 32, 1
    Lx = n * H
    xi = 2 * np.pi * m / Lx
    Dv, k, T = 1e-9, 1e-3, 200.0
    x = np.arange(n)
    c0 = np.broadcast_to(np.cos(2 * np.pi * m * x / n)[None, :], (4, n)).copy()
    errs = []
    for steps in (5, 10, 20):
        c = c0
        for _ in range(steps):
            c = df.diffusion_step(c, np.full(c.shape, Dv), np.full(c.shape, k), T / steps, H, tol=1e-13)["c"]
        errs.append(abs(c[0, 0] - np.exp(-(Dv * xi ** 2 + k) * T)))
    # first order in dt (spatial error is far smaller at this resolution)
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]


def _small_params(**kw):
    p = stg.Params(band_width=2, maxit=20000, tol_diff=1e-12, tol_mech=1e-12, tol_pf=1e-12)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_staggered_zero_source_stays_zero():
    phase, _ = inputs.box_fractal(16, 2, 2, 1.8, 0.3, np.random.default_rng(1))
    prm = _small_params(c_dir=0.0)
    st = stg.initial_state(phase, prm)
    for _ in range(2):
        st = stg.step(phase, st, prm)
    for f in (st.c, st.f, st.e, st.H, st.d, st.strain):
        assert np.max(np.abs(f)) == 0.0


def test_staggered_history_monotone_and_damage_bounded():
    phase, _ = inputs.box_fractal(16, 2, 2, 1.8, 0.3, np.random.default_rng(2))
    prm = _small_params(k_rate=5e-2, e_per_f=0.05, E_tab=(3e8, 30e9), Gc=1e-3)
    st = stg.initial_state(phase, prm)
    prev_H = st.H
    for _ in range(3):
        st = stg.step(phase, st, prm)
        assert np.all(st.H >= prev_H)
        assert st.d.min() >= 0 and st.d.max() < 1
        prev_H = st.H
    assert st.d.max() > 1e-6


# ---------------------------------------------------------------------------
# Alg. 1 composition pin: one and two oracle steps against the same step
# assembled here from the definition-level sparse solvers (no FFT, no CG).
# Order (Alg. 1): diffusion -> precipitation/eigenstrain from the NEW
# concentration -> mechanics with the PREVIOUS damage -> history from the
# elastic strain with UNDEGRADED moduli (eq. energy) -> phase field.

def _psi_plus_2d_by_hand(strain, e, lam, mu):
    """Sec. 2.4 eq. energy, 2D: (lam + mu)/2 <tr>_+^2 + mu dev:dev of the
    elastic strain eps - e I (Voigt 11, 22, 12 with tensor shear)."""
    l11, l22, l12 = strain[0] - e, strain[1] - e, strain[2]
    tr = l11 + l22
    trp = np.maximum(tr, 0.0)
    d11, d22 = l11 - 0.5 * tr, l22 - 0.5 * tr
    return 0.5 * (lam + mu) * trp ** 2 + mu * (d11 ** 2 + d22 ** 2 + 2 * l12 ** 2)


def _assembled_step(phase, st, prm, d_mech=None):
    from oracle import material as omat
    pore = phase == 0
    Dfield = np.asarray(prm.D_tab)[phase]
    react = np.where(pore, prm.k_rate, 0.0)
    band = stg.band_mask(phase.shape, prm.band_width)
    c = direct.diffusion_direct(st.c, Dfield, react, prm.dt, prm.h, band=band, c_dir=prm.c_dir)
    f = np.where(pore, np.minimum(1.0, st.f + prm.dt * prm.k_rate * c), 0.0)
    e = np.where(pore, prm.e_per_f * f, 0.0)
    dm = st.d if d_mech is None else d_mech
    m = direct.mech_direct(phase, prm.E_tab, prm.nu_tab, prm.eps_mac, prm.h, d=dm, kappa=prm.kappa, e=e)
    E = np.asarray(prm.E_tab)[phase]
    nu = np.asarray(prm.nu_tab)[phase]
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    H = np.maximum(st.H, _psi_plus_2d_by_hand(m["strain"], e, lam, mu))
    d = direct.phasefield_direct(H, prm.Gc, prm.l0, prm.h)
    return dict(c=c, f=f, e=e, H=H, d=d, strain=m["strain"])


@pytest.mark.parametrize("grid,Gc", [((8, 8), 2e-1), ((12, 8), 5e-3)])
def test_staggered_step_matches_assembled_alg1(grid, Gc):
    ny, nx = grid
    rng = np.random.default_rng(ny * 100 + nx)
    phase = (rng.random(grid) < 0.55).astype(np.uint8)
    phase[:, :2] = 0  # the source band lies in the pore space
    # pore stiffness 1/10 of the solid keeps the damaged mechanics well enough
    # conditioned for the CG solves to reach the direct solutions to 1e-10
    prm = _small_params(k_rate=5e-3, e_per_f=0.05, E_tab=(3e9, 30e9), Gc=Gc, eps_mac=(2e-4, -1e-4, 5e-5),
                        tol_diff=1e-15, tol_mech=1e-15, tol_pf=1e-15, maxit=20000)
    st = stg.initial_state(phase, prm)
    for step in range(2):
        ref = _assembled_step(phase, st, prm)
        nxt = stg.step(phase, st, prm)
        for k in ("c", "f", "e", "H", "d", "strain"):
            a, b = getattr(nxt, k), ref[k]
            err = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert err < 1e-10, (step, k, err)
        # every field moves, so a dropped coupling cannot hide
        for k in ("c", "f", "e", "H", "d"):
            assert np.linalg.norm(ref[k] - getattr(st, k)) > 1e-3 * np.linalg.norm(ref[k]), (step, k)
        if step == 1:
            # the pin can fail: mechanics with the NEW damage gives another strain
            wrong = _assembled_step(phase, st, prm, d_mech=nxt.d)
            assert np.linalg.norm(wrong["strain"] - ref["strain"]) > 1e-6 * np.linalg.norm(ref["strain"])
        st = nxt
    if Gc <= 5e-3:
        assert st.d.max() > 0.99  # the fracture regime: damage close to 1


def test_staggered_history_uses_undegraded_moduli():
    """H after a step differs from psi+ evaluated with degraded moduli once d > 0."""
    phase = np.ones((8, 8), np.uint8)
    phase[3:5, 3:5] = 0
    prm = _small_params(band_width=0, diffuse=False, e_ramp=1e-2, n_ramp=1, E_tab=(3e8, 30e9), Gc=1e-3,
                        tol_mech=1e-15, tol_pf=1e-15, maxit=50000)
    st = stg.initial_state(phase, prm)
    st = stg.step(phase, st, prm)
    st.d = np.full_like(st.d, 0.5)
    nxt = stg.step(phase, st, prm)
    E = np.asarray(prm.E_tab)[phase]
    nu = np.asarray(prm.nu_tab)[phase]
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    psi_u = _psi_plus_2d_by_hand(nxt.strain, nxt.e, lam, mu)
    g = (1 - 0.5) ** 2 + prm.kappa
    assert np.allclose(nxt.H, np.maximum(st.H, psi_u), rtol=1e-12, atol=0)
    assert not np.allclose(nxt.H, np.maximum(st.H, g * psi_u), rtol=1e-3, atol=0)
    # eigenstrain only in the pores, prescribed by the ramp
    assert np.all(nxt.e[phase != 0] == 0) and np.allclose(nxt.e[phase == 0], 1e-2 * 2)
