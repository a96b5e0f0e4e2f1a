"""GPU tests of the row-pass autotuner (rows per block of the 2D mechanics
passes, FGCG_OPT_ROWS).

* an autotuned context ends its first mechanics solve with one of the
  candidates (the default for nx times 1/2, 1, 2, even, 2..16, at most 4096
  voxels per block);
* every candidate gives bitwise the same solution and iteration count (the
  choice changes timing only), FP64 and FP32-mixed;
* values outside the candidate set are rejected.
"""
import numpy as np
import pytest

from paper_2305_13081_amd import inputs

pytestmark = pytest.mark.gpu
E_TAB, NU_TAB, H = (3e6, 30e9), (0.2, 0.2), 5e-6


def rows_default(nx):
    return 2 if nx >= 768 else 4 if nx >= 384 else 8 if nx >= 256 else 16


def candidates(nx):
    r0 = rows_default(nx)
    ok = lambda r: r == r0 or (2 <= r <= 16 and r % 2 == 0 and r * nx <= 4096)
    return [r for r in (r0 // 2, r0, 2 * r0) if ok(r)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda", 0)


@pytest.mark.parametrize("nx,ny,prec", [(256, 128, 0), (512, 64, 1), (1024, 48, 0), (96, 96, 0)])
def test_rows_candidates_identical(torch_dev, nx, ny, prec):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    ph, _ = inputs.box_fractal(max(nx, ny), 2, 4, 1.7, 0.3, np.random.default_rng(nx + ny))
    phase = torch.from_numpy(np.ascontiguousarray(ph[:ny, :nx])).to(dev)
    ctx = fgcg.Context(nx, ny, H, precision=prec)
    assert ctx.get_option("rows") == 0
    ref = ctx.mech_solve(phase, E_TAB, NU_TAB, (1e-3, 0.0, 2e-4), tol=1e-9, maxit=20000)
    picked = ctx.get_option("rows")
    print(f"autotune {nx}x{ny} prec={prec}: candidates {candidates(nx)}, picked {picked}", flush=True)
    assert picked in candidates(nx)
    for r in candidates(nx):
        ctx.set_option("rows", r)
        assert ctx.get_option("rows") == r
        out = ctx.mech_solve(phase, E_TAB, NU_TAB, (1e-3, 0.0, 2e-4), tol=1e-9, maxit=20000)
        assert out["info"]["iters"] == ref["info"]["iters"]
        assert torch.equal(out["strain"], ref["strain"]), r


def test_rows_option_rejects(torch_dev):
    from paper_2305_13081_amd import fgcg
    ctx = fgcg.Context(256, 64, H)
    with pytest.raises(fgcg.FgcgError):
        ctx.set_option("rows", 3)
    with pytest.raises(fgcg.FgcgError):
        ctx.set_option("rows", 64)
    ctx.set_option("rows", 0)
    assert ctx.get_option("rows") == 0
