"""GPU tests of the autotuner of the 3D mechanics passes: displacement
components per block of the two row passes (FGCG_OPT_ROW_SPLIT) and z tiles
per block of the Green z pass (FGCG_OPT_ZTILES).

* every pinned candidate (row split 1..4 x z tiles 1, 2), FP64 and
  FP32-mixed, equals the oracle's projected CG after a fixed number of
  iterations (1e-12 / 1e-5, max-norm and L2), on grids with ragged z tiles;
* the four row splits give bitwise the same solution at a fixed z-tile count
  (the split changes timing only);
* a 64^3 context (2^18 voxels) ends its first solve with tuned picks in
  range, a second context of the same shape takes the same picks from the
  per-process cache, a context with those picks pinned gives bitwise the
  same solution, and the tuned solve equals the oracle at fixed iterations;
* the options are rejected on 2D contexts and out of range.
"""
import numpy as np
import pytest

from oracle import mech as omech

pytestmark = pytest.mark.gpu
E_TAB, NU_TAB, H = (3e6, 30e9), (0.2, 0.2), 5e-6
EM = (2e-4, -1e-4, 3e-4, 1e-4, -2e-4, 5e-5)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda", 0)


def _case(shape, seed):
    rng = np.random.default_rng(seed)
    phase = (rng.random(shape) > 0.3).astype(np.uint8)
    d = 0.4 * rng.random(shape)
    e = np.where(phase == 0, 1e-3, 0.0) * (1 + rng.random(shape))
    return phase, d, e


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _solve(ctx, torch, dev, phase, d, e, k):
    T = lambda a: torch.from_numpy(a).to(dev)
    r = ctx.mech_solve(T(phase), E_TAB, NU_TAB, EM, d=T(d), kappa=1e-6, eig=T(e), tol=0.0, maxit=k)
    assert r["info"]["iters"] == k
    return r["strain"].cpu().numpy()


# (nz, ny, nx): ny = 12 leaves a ragged FP64 z tile (8 ky values per tile)
@pytest.mark.parametrize("shape", [(16, 16, 16), (8, 12, 48)])
@pytest.mark.parametrize("prec", [0, 1])
def test_pinned_candidates(torch_dev, shape, prec):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    k = 6
    phase, d, e = _case(shape, sum(shape))
    print(f"3D candidates {shape} prec={prec}: oracle", flush=True)
    o = omech.mech_solve(phase, E_TAB, NU_TAB, EM, H, d=d, kappa=1e-6, e=e, tol=0.0, maxit=k, fixed_iters=k)
    bar = 1e-12 if prec == 0 else 1e-5
    for zt in (1, 2):
        first = None
        for split in (1, 2, 3, 4):
            ctx = fgcg.Context(shape[2], shape[1], H, precision=prec, nz=shape[0])
            ctx.set_option("row_split", split)
            ctx.set_option("ztiles", zt)
            s = _solve(ctx, torch, dev, phase, d, e, k)
            assert ctx.get_option("row_split") == split and ctx.get_option("ztiles") == zt
            ctx.close()
            err, emax = rel(s, o["strain"]), maxrel(s, o["strain"])
            print(f"  ztiles {zt} split {split}: rel {err:.2e}, max rel {emax:.2e}", flush=True)
            assert err < bar and emax < bar
            if first is None:
                first = s
            else:
                assert np.array_equal(s, first), "row splits must not change results"


@pytest.mark.parametrize("prec", [0, 1])
def test_tuner_picks_cached_and_reproducible(torch_dev, prec):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    shape = (64, 64, 64)  # 2^18 voxels: the passes are timed
    k = 4
    phase, d, e = _case(shape, 5 + prec)
    ctx = fgcg.Context(64, 64, H, precision=prec, nz=64)
    assert ctx.get_option("row_split") == 0 and ctx.get_option("ztiles") == 0
    print(f"3D tuner 64^3 prec={prec}", flush=True)
    s = _solve(ctx, torch, dev, phase, d, e, k)
    picks = (ctx.get_option("row_split"), ctx.get_option("ztiles"))
    print(f"  picks row_split={picks[0]} ztiles={picks[1]}", flush=True)
    assert 1 <= picks[0] <= 4 and picks[1] in (1, 2)
    ctx.close()
    ctx2 = fgcg.Context(64, 64, H, precision=prec, nz=64)
    s2 = _solve(ctx2, torch, dev, phase, d, e, k)
    assert (ctx2.get_option("row_split"), ctx2.get_option("ztiles")) == picks
    ctx2.close()
    assert np.array_equal(s, s2)
    ctx3 = fgcg.Context(64, 64, H, precision=prec, nz=64)
    ctx3.set_option("row_split", picks[0])
    ctx3.set_option("ztiles", picks[1])
    s3 = _solve(ctx3, torch, dev, phase, d, e, k)
    ctx3.close()
    assert np.array_equal(s, s3)
    print("  oracle", flush=True)
    o = omech.mech_solve(phase, E_TAB, NU_TAB, EM, H, d=d, kappa=1e-6, e=e, tol=0.0, maxit=k, fixed_iters=k)
    err, emax = rel(s, o["strain"]), maxrel(s, o["strain"])
    print(f"  tuned solve vs oracle after {k} iterations: rel {err:.2e}, max rel {emax:.2e}", flush=True)
    bar = 1e-12 if prec == 0 else 1e-5
    assert err < bar and emax < bar


def test_options_rejected(torch_dev):
    from paper_2305_13081_amd import fgcg
    ctx2 = fgcg.Context(64, 64, H)
    for name in ("row_split", "ztiles"):
        with pytest.raises(fgcg.FgcgError) as ei:
            ctx2.set_option(name, 1)
        assert ei.value.status == fgcg.FGCG_EUNSUPPORTED
    ctx2.close()
    ctx3 = fgcg.Context(16, 16, H, nz=16)
    for name, bad in (("row_split", 5), ("row_split", -1), ("ztiles", 3)):
        with pytest.raises(fgcg.FgcgError) as ei:
            ctx3.set_option(name, bad)
        assert ei.value.status == fgcg.FGCG_EINVAL
    ctx3.close()
