"""The no-allocation phase-field entry point against the context entry point
(the same textbook stencil CG kernels and launch shapes): two calls in a row,
the second on a smaller grid, each equal bitwise to fgcg_phasefield_solve in
textbook form (FGCG_OPT_SCALAR_CG = 0 on 2D grids, the only form in 3D), to
the default one-reduction form within 1e-11 and to the FP64 oracle within
1e-10; 2D and 3D; sizes beyond the limit rejected."""
import ctypes

import numpy as np
import pytest

from oracle import phasefield as opf

pytestmark = pytest.mark.gpu
GC, L0, H = 50.0, 1e-5, 5e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda", 0)


def _case(shape, seed):
    rng = np.random.default_rng(seed)
    return 2e6 * rng.random(shape) ** 4, 0.2 * rng.random(shape)


@pytest.mark.parametrize("shapes", [[(48, 64), (24, 32)], [(16, 24, 32), (8, 16, 16)]])
def test_noalloc_matches_context_solve(torch_dev, shapes):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    for i, shape in enumerate(shapes):  # the second call has a smaller input
        Hf, d0 = _case(shape, 10 + i)
        Ht = torch.from_numpy(Hf).to(dev)
        a = torch.from_numpy(d0.copy()).to(dev)
        info = fgcg.phasefield_solve_noalloc(Ht, GC, L0, a, H, tol=1e-13)
        ctx = fgcg.Context(shape[-1], shape[-2], H, nz=shape[0] if len(shape) == 3 else None)
        bd = torch.from_numpy(d0.copy()).to(dev)
        ctx.phasefield_solve(Ht, GC, L0, bd, tol=1e-13)  # the default form
        ctx.set_option("scalar_cg", 0)
        b = torch.from_numpy(d0.copy()).to(dev)
        ref = ctx.phasefield_solve(Ht, GC, L0, b, tol=1e-13)
        ed = float(torch.linalg.norm(a - bd) / torch.linalg.norm(bd))
        o = opf.phasefield_solve(Hf, GC, L0, H, d0=d0, tol=1e-13)
        err = float(np.linalg.norm(a.cpu().numpy() - o["d"]) / np.linalg.norm(o["d"]))
        print(f"no-alloc {shape}: iters {info['iters']} (context {ref['iters']}, oracle {o['iters']}), "
              f"bitwise equal {bool(torch.equal(a, b))}, oracle rel err {err:.2e}", flush=True)
        assert info["status"] == 0 and info["iters"] == ref["iters"]
        assert torch.equal(a, b)
        assert err < 1e-10 and ed < 1e-11
        ctx.close()


def test_noalloc_rejects(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    lib = fgcg.load_library()
    big = fgcg.Grid(2, (ctypes.c_int * 3)(2048, 1024, 1), H, 0)  # 2^21 voxels: beyond the limit
    info = fgcg.Info()
    assert lib.fgcg_phasefield_solve_noalloc(ctypes.byref(big), None, None, GC, L0, None, 1e-8, 10,
                                             ctypes.byref(info)) == -1
    x = torch.zeros((2048, 1024), dtype=torch.float64, device=dev)
    assert lib.fgcg_phasefield_solve_noalloc(ctypes.byref(big), None, ctypes.c_void_p(x.data_ptr()), GC, L0,
                                             ctypes.c_void_p(x.data_ptr()), 1e-8, 10, ctypes.byref(info)) == -1
    f32 = fgcg.Grid(2, (ctypes.c_int * 3)(64, 64, 1), H, 1)
    y = torch.zeros((64, 64), dtype=torch.float64, device=dev)
    assert lib.fgcg_phasefield_solve_noalloc(ctypes.byref(f32), None, ctypes.c_void_p(y.data_ptr()), GC, L0,
                                             ctypes.c_void_p(y.data_ptr()), 1e-8, 10, ctypes.byref(info)) == -6
    # zero history: d = 0 after 0 iterations, through the fill kernel
    z = torch.zeros((64, 64), dtype=torch.float64, device=dev)
    d = torch.rand((64, 64), dtype=torch.float64, device=dev)
    r = fgcg.phasefield_solve_noalloc(z, GC, L0, d, H)
    assert r["iters"] == 0 and float(d.abs().max()) == 0.0
