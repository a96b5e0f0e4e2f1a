"""Pins of the oracle's phase-field, diffusion and staggered-step code (CPU only).

Phase field (Sec. 2.4): uniform history closed form, the exact periodic 1-D
crack profile of the discrete equation, sparse direct solve, maximum principle.
Diffusion step: exact decay of a Fourier mode in one CG iteration, mass
conservation without sink or band, sparse direct solve with a Dirichlet band,
band voxels held, first-order convergence in dt to exp(-(D xi^2 + k) t).
Staggered step (Alg. 1): zero source keeps every field zero; the history field
never decreases and the damage stays in [0, 1).
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
