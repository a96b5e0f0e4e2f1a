"""GPU parity of the hand-written adjoint (dJ/dE per voxel).

* small grids: GPU gradient vs the oracle's adjoint gradient, energy and C11
  objectives, with damage (both solves at tol 1e-13, <= 1e-10 relative);
* user objective J = sum_x w_x eps_11(x): GPU gradient vs central
  differences of the oracle's forward solves;
* torch.autograd: E.grad equals the adjoint gradient;
* 1024^2 fractal (E = 30 GPa / 3 MPa, nu = 0.2, eps_11 = 1e-3): the C11
  adjoint (a second CG solve) reproduces the Hill-Mandel closed form
  eps:sigma / (N eps11^2 E) built from the forward strain, and central
  differences (relative step 1e-6, energies summed with math.fsum) at 32
  random solid voxels agree with the energy gradient to the cancellation limit.
"""
import math

import numpy as np
import pytest

from oracle import adjoint as oadj, material as omat, mech as omech
from paper_2305_13081_amd import inputs

pytestmark = pytest.mark.gpu
H = 5e-6
NU = 0.2


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _efield(ny, nx, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((ny, nx)) < 0.35, 3e8, 30e9) * (1 + 0.1 * rng.random((ny, nx)))


@pytest.mark.parametrize("objective", ["W", "C11"])
@pytest.mark.parametrize("nx,ny", [(32, 32), (48, 64)])
def test_adjoint_matches_oracle(torch_dev, objective, nx, ny):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    E = _efield(ny, nx, nx + ny)
    d = 0.3 * np.random.default_rng(5).random((ny, nx))
    em = (1e-3, 2e-4, 0.0)
    Jo, go, _ = oadj.gradient_E(E, NU, em, H, objective, d=d, kappa=1e-6, tol=1e-13)
    ctx = fgcg.Context(nx, ny, H)
    g, J, i1, i2 = ctx.mech_adjoint(torch.from_numpy(E).to(dev), NU, em,
                                    objective=fgcg.J_ENERGY if objective == "W" else fgcg.J_C11,
                                    d=torch.from_numpy(d).to(dev), kappa=1e-6, tol=1e-13)
    err = rel(g.cpu().numpy(), go)
    print(f"adjoint {objective} {nx}x{ny}: J rel err {abs(J - Jo) / abs(Jo):.2e}, grad rel err {err:.2e}, "
          f"iters fwd {i1['iters']} adj {i2['iters']}", flush=True)
    assert abs(J - Jo) < 1e-10 * abs(Jo)
    assert err < 1e-10
    # the objective alone (no adjoint solve) gives the same J
    _, J1, _, i3 = ctx.mech_adjoint(torch.from_numpy(E).to(dev), NU, em,
                                    objective=fgcg.J_ENERGY if objective == "W" else fgcg.J_C11,
                                    d=torch.from_numpy(d).to(dev), kappa=1e-6, tol=1e-13, want_grad=False)
    assert J1 == J and i3["iters"] == 0


def test_adjoint_user_objective_finite_differences(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    n = 16
    E = _efield(n, n, 11)
    w = np.random.default_rng(12).standard_normal((n, n))
    em = (1e-3, 0.0, 0.0)
    dJ = np.zeros((3, n, n))
    dJ[0] = w
    ctx = fgcg.Context(n, n, H)
    g, _, _, _ = ctx.mech_adjoint(torch.from_numpy(E).to(dev), NU, em, objective=fgcg.J_USER,
                                  dJ_dstrain=torch.from_numpy(dJ).to(dev), tol=1e-14)
    g = g.cpu().numpy()

    def J(Ef):
        r = omech.mech_solve(np.zeros((n, n), np.uint8), None, None, em, H, E_field=Ef, nu=NU, tol=1e-14,
                             maxit=20000)
        return float(np.sum(w * r["strain"][0]))

    for (iy, ix) in [(3, 4), (10, 2), (7, 13)]:
        step = 1e-4 * E[iy, ix]
        Ep, Em = E.copy(), E.copy()
        Ep[iy, ix] += step
        Em[iy, ix] -= step
        fd = (J(Ep) - J(Em)) / (2 * step)
        assert abs(fd - g[iy, ix]) < 1e-6 * np.abs(g).max(), (fd, g[iy, ix])


def test_autograd_function(torch_dev):
    from paper_2305_13081_amd import autograd, fgcg
    torch, dev = torch_dev
    n = 32
    E = torch.from_numpy(_efield(n, n, 21)).to(dev).requires_grad_(True)
    ctx = fgcg.Context(n, n, H)
    J = autograd.mech_objective(E, ctx, NU, (1e-3, 0.0, 0.0), objective="C11", tol=1e-13)
    J.backward()
    g, Jd, _, _ = ctx.mech_adjoint(E.detach(), NU, (1e-3, 0.0, 0.0), objective=fgcg.J_C11, tol=1e-13)
    assert float(J.detach()) == Jd  # the forward value is the library's J
    assert float((E.grad - g).abs().max()) <= 1e-10 * float(g.abs().max())


def test_adjoint_c4_full_size(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    phase, _ = inputs.c2_microstructure(1024)
    E = np.where(phase == 0, 3e6, 30e9)
    Eg = torch.from_numpy(E).to(dev)
    e11 = 1e-3
    em = (e11, 0.0, 0.0)
    N = E.size
    ctx = fgcg.Context(1024, 1024, H)
    gc, Jc, i1, i2 = ctx.mech_adjoint(Eg, NU, em, objective=fgcg.J_C11, tol=1e-12, maxit=200000)
    res = ctx.mech_solve(None, None, None, em, E_field=Eg, nu_field=NU, tol=1e-12, maxit=200000)
    eps = omat.from_voigt(res["strain"].cpu().numpy(), 2)
    lam, mu = omat.lame(E, NU)
    sig = omat.stress(eps, lam, mu)
    closed = np.sum(eps * sig, axis=(0, 1)) / (N * e11 ** 2 * E)
    err = rel(gc.cpu().numpy(), closed)
    print(f"C4 1024^2: C11 {Jc:.6e}, adjoint iters fwd {i1['iters']} adj {i2['iters']}, "
          f"adjoint vs Hill-Mandel closed form {err:.2e}", flush=True)
    assert err < 1e-6
    gw, Jw, _, _ = ctx.mech_adjoint(Eg, NU, em, objective=fgcg.J_ENERGY, tol=1e-13, maxit=200000)
    gw = gw.cpu().numpy()

    def W(Ef):
        r = ctx.mech_solve(None, None, None, em, E_field=torch.from_numpy(Ef).to(dev), nu_field=NU, tol=1e-13,
                           maxit=200000, want_stress=True)
        s = r["stress"].cpu().numpy()
        st = r["strain"].cpu().numpy()
        dens = st[0] * s[0] + st[1] * s[1] + 2 * st[2] * s[2]
        return 0.5 * H ** 2 * math.fsum(dens.ravel())

    rng = np.random.default_rng(4)
    solid = np.argwhere(phase == 1)
    worst = 0.0
    for j in rng.choice(len(solid), 32, replace=False):
        iy, ix = solid[j]
        step = 1e-6 * E[iy, ix]
        Ep, Em = E.copy(), E.copy()
        Ep[iy, ix] += step
        Em[iy, ix] -= step
        fd = (W(Ep) - W(Em)) / (2 * step)
        worst = max(worst, abs(fd - gw[iy, ix]) / abs(gw[iy, ix]))
    print(f"C4 1024^2: energy gradient vs central differences at 32 voxels, worst rel err {worst:.2e}", flush=True)
    assert worst < 5e-3
