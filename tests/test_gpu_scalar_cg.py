"""GPU parity of the one-reduction form of the stencil scalar CG (2D grids,
the phase field of Sec. 2.4 and the diffusion step) through the C ABI.

Its alpha, beta and stop test are textbook CG's in exact arithmetic, so:
* k fixed iterations equal the oracle's textbook CG (k = 1, 2, 5, 20) to
  1e-12, for the phase field and for the diffusion step with a Dirichlet band
  (warm start from c^n), on square, non-square and ragged grids (partial
  64 x 16 tiles);
* converged solves (tol 1e-13) equal the two-pass textbook form on the GPU to
  1e-11 with iteration counts within one, and the oracle to 1e-10;
* zero history gives d = 0 after 0 iterations.
"""
import numpy as np
import pytest

from oracle import diffusion as odf, phasefield as opf

pytestmark = pytest.mark.gpu
H, GC, L0 = 5e-6, 50.0, 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


SHAPES = [(64, 64), (96, 48), (24, 16), (384, 8), (256, 256)]


def _pf_case(ny, nx, seed):
    rng = np.random.default_rng(seed)
    return 2e6 * rng.random((ny, nx)) ** 4, 0.2 * rng.random((ny, nx))


def _diff_case(ny, nx, seed):
    rng = np.random.default_rng(seed)
    phase = (rng.random((ny, nx)) < 0.5).astype(np.uint8)
    c0 = rng.random((ny, nx))
    c0[:, :4] = 1.0
    return phase, c0


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_onered_fixed_iterations(torch_dev, nx, ny):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    ctx = fgcg.Context(nx, ny, H)
    assert ctx.get_option("scalar_cg") == 1
    Hf, d0 = _pf_case(ny, nx, nx + ny)
    phase, c0 = _diff_case(ny, nx, 2 * nx + ny)
    band = np.zeros((ny, nx), bool)
    band[:, :4] = True
    Df, kr = np.asarray((1e-9, 1e-12))[phase], np.asarray((1e-3, 0.0))[phase]
    for k in (1, 2, 5, 20):
        print(f"one-reduction CG {nx}x{ny} k={k}", flush=True)
        dg = torch.from_numpy(d0.copy()).to(dev)
        info = ctx.phasefield_solve(torch.from_numpy(Hf).to(dev), GC, L0, dg, tol=0.0, maxit=k)
        o = opf.phasefield_solve(Hf, GC, L0, H, d0=d0, fixed_iters=k)
        ep = rel(dg.cpu().numpy(), o["d"])
        cg = torch.from_numpy(c0.copy()).to(dev)
        di = ctx.diffusion_step_phases(torch.from_numpy(phase).to(dev), (1e-9, 1e-12), (1e-3, 0.0), 4, 1.0, 40.0,
                                       cg, tol=0.0, maxit=k)
        od = odf.diffusion_step(c0, Df, kr, 40.0, H, band=band, c_dir=1.0, fixed_iters=k)
        ed = rel(cg.cpu().numpy(), od["c"])
        print(f"  phase field {ep:.2e} ({info['iters']} iters), diffusion {ed:.2e} ({di['iters']} iters)", flush=True)
        assert info["iters"] == k and di["iters"] == k and ep < 1e-12 and ed < 1e-12
    ctx.close()


@pytest.mark.parametrize("nx,ny", [(256, 256), (96, 48)])
def test_onered_equals_textbook(torch_dev, nx, ny):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    Hf, d0 = _pf_case(ny, nx, 7 * nx + ny)
    phase, c0 = _diff_case(ny, nx, 5 * nx + ny)
    out = {}
    for form in (1, 0):
        ctx = fgcg.Context(nx, ny, H)
        ctx.set_option("scalar_cg", form)
        dg = torch.from_numpy(d0.copy()).to(dev)
        pi = ctx.phasefield_solve(torch.from_numpy(Hf).to(dev), GC, L0, dg, tol=1e-13)
        cg = torch.from_numpy(c0.copy()).to(dev)
        di = ctx.diffusion_step_phases(torch.from_numpy(phase).to(dev), (1e-9, 1e-12), (1e-3, 0.0), 4, 1.0, 40.0,
                                       cg, tol=1e-13)
        out[form] = (dg.cpu().numpy(), pi, cg.cpu().numpy(), di)
        ctx.close()
    a, b = out[1], out[0]
    ep, ed = rel(a[0], b[0]), rel(a[2], b[2])
    print(f"{nx}x{ny}: phase field {a[1]['iters']} / {b[1]['iters']} iters, rel {ep:.2e}; "
          f"diffusion {a[3]['iters']} / {b[3]['iters']} iters, rel {ed:.2e}", flush=True)
    assert abs(a[1]["iters"] - b[1]["iters"]) <= 1 and abs(a[3]["iters"] - b[3]["iters"]) <= 1
    assert ep < 1e-11 and ed < 1e-11
    o = opf.phasefield_solve(Hf, GC, L0, H, d0=d0, tol=1e-13)
    assert rel(a[0], o["d"]) < 1e-10


def test_onered_zero_history(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    ctx = fgcg.Context(64, 48, H)
    dg = torch.rand((48, 64), dtype=torch.float64, device=dev)
    info = ctx.phasefield_solve(torch.zeros((48, 64), dtype=torch.float64, device=dev), GC, L0, dg)
    assert info["iters"] == 0 and float(dg.abs().max()) == 0.0
    ctx.close()
