"""GPU tests of the autotuner of the 2D mechanics passes: rows per block of
the row passes (FGCG_OPT_ROWS) and the radix plans of the LDS transforms in
the row passes and the Green column pass (FGCG_OPT_ROW_PLAN / _COL_PLAN).

* an autotuned context ends its first mechanics solve with one of the rows
  candidates (the default for nx times 1/2, 1, 2, even, 2..16, at most 4096
  voxels per block) and a plan in {1, 2} (1 where radix 16 does not fit);
* every rows candidate gives bitwise the same solution and iteration count
  (the choice changes timing only), FP64 and FP32-mixed;
* every plan combination (radix 8 or radix 16 in the row and column
  transforms) matches the FP64 oracle at fixed iterations (<= 1e-10) and the
  FP32-mixed path with radix 16 matches the FP64 solve (<= 1e-5);
* values outside the candidate sets, and plans on 3D contexts, are rejected;
* the pass-timing hook (fgcg_time_pass) returns a positive duration for each
  2D mechanics pass and rejects other kinds, bad repetition counts and 3D.
"""
import numpy as np
import pytest

from oracle import mech as omech
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


def plan_differs(n):
    """Radix 16 gives a different schedule from radix 8 for length n."""
    a = 0
    while n % 3 ** (a + 1) == 0:
        a += 1
    b = int(np.log2(n // 3 ** a))
    return b >= 4 and b % 4 != 1 or b >= 9


@pytest.mark.parametrize("nx,ny", [(64, 48), (256, 128), (48, 512), (96, 32), (24, 1024), (16, 2048), (64, 256)])
def test_plans_fixed_iteration_parity(torch_dev, nx, ny):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    ph, _ = inputs.box_fractal(max(nx, ny), 2, 4, 1.7, 0.3, np.random.default_rng(3 * nx + ny))
    ph = np.ascontiguousarray(ph[:ny, :nx])
    if ph.min() == ph.max():  # a thin crop can miss the pores: random phases then
        ph = (np.random.default_rng(nx + ny).random((ny, nx)) < 0.7).astype(np.uint8)
    e = np.where(ph == 0, 1e-3, 0.0)
    phase, eg = torch.from_numpy(ph).to(dev), torch.from_numpy(e).to(dev)
    k = 12
    o = omech.mech_solve(ph, E_TAB, NU_TAB, (2e-4, 0.0, 1e-4), H, e=e, fixed_iters=k)
    for pr in (1, 2):
        for pc in (1, 2, 3):  # 3: one wavefront per column (lengths 256..2048; plan 1 otherwise)
            ctx = fgcg.Context(nx, ny, H)
            ctx.set_option("row_plan", pr)
            ctx.set_option("col_plan", pc)
            r = ctx.mech_solve(phase, E_TAB, NU_TAB, (2e-4, 0.0, 1e-4), eig=eg, tol=0.0, maxit=k)
            assert ctx.get_option("row_plan") == pr and ctx.get_option("col_plan") == pc
            err = float(np.linalg.norm(r["strain"].cpu().numpy() - o["strain"]) / np.linalg.norm(o["strain"]))
            print(f"plans {nx}x{ny} row {pr} col {pc}: fixed k={k} strain rel err {err:.2e}", flush=True)
            assert r["info"]["iters"] == k and err < 1e-10


def test_plans_tuned_and_fp32(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    nx, ny = 512, 96
    ph, _ = inputs.box_fractal(512, 2, 5, 1.8, 0.3, np.random.default_rng(11))
    phase = torch.from_numpy(np.ascontiguousarray(ph[:ny, :nx])).to(dev)
    ref_ctx = fgcg.Context(nx, ny, H)
    ref_ctx.set_option("row_plan", 1)
    ref_ctx.set_option("col_plan", 1)
    ref = ref_ctx.mech_solve(phase, E_TAB, NU_TAB, (1e-3, 0.0, 0.0), tol=1e-12, maxit=50000)
    # autotuned FP64: a plan in {1, 2} for both passes, same solution to rounding
    ctx = fgcg.Context(nx, ny, H)
    assert ctx.get_option("row_plan") == 0 and ctx.get_option("col_plan") == 0
    out = ctx.mech_solve(phase, E_TAB, NU_TAB, (1e-3, 0.0, 0.0), tol=1e-12, maxit=50000)
    pr, pc = ctx.get_option("row_plan"), ctx.get_option("col_plan")
    print(f"tuned {nx}x{ny}: rows {ctx.get_option('rows')} row plan {pr} col plan {pc}", flush=True)
    assert pr in ((1, 2) if plan_differs(nx) else (1,))
    assert pc in ((1, 2) if plan_differs(ny) else (1,)) + ((3,) if ny in (256, 512, 1024, 2048) else ())
    err = float((out["strain"] - ref["strain"]).norm() / ref["strain"].norm())
    assert err < 1e-10, err
    # FP32-mixed with radix 16 in both passes against the FP64 solve
    c32 = fgcg.Context(nx, ny, H, precision=fgcg.FP32_MIXED)
    c32.set_option("row_plan", 2)
    c32.set_option("col_plan", 2)
    o32 = c32.mech_solve(phase, E_TAB, NU_TAB, (1e-3, 0.0, 0.0), tol=1e-10, maxit=50000)
    err = float((o32["strain"] - ref["strain"]).norm() / ref["strain"].norm())
    print(f"FP32-mixed radix-16 plans vs FP64: strain rel diff {err:.2e}", flush=True)
    assert o32["info"]["status"] == 0 and err < 1e-5


def test_plan_option_rejects(torch_dev):
    from paper_2305_13081_amd import fgcg
    ctx = fgcg.Context(256, 64, H)
    for name, top in (("row_plan", 2), ("col_plan", 3)):
        for bad in (top + 1, -1):
            with pytest.raises(fgcg.FgcgError):
                ctx.set_option(name, bad)
        ctx.set_option(name, 2)
        assert ctx.get_option(name) == 2
        ctx.set_option(name, 0)
        assert ctx.get_option(name) == 0
    c3 = fgcg.Context(16, 16, H, nz=16)
    with pytest.raises(fgcg.FgcgError):
        c3.set_option("row_plan", 1)


def test_time_pass(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    for form in (3, 2):
        ctx = fgcg.Context(256, 128, H)
        ctx.set_option("mech_form", form)
        times = {k: ctx.time_pass(k, 20) for k in ("mech_row_fwd", "mech_col")}
        if form == 3:
            times["mech_row_inv"] = ctx.time_pass("mech_row_inv", 20)
        else:  # the two-pass form has no inverse row pass
            with pytest.raises(fgcg.FgcgError) as ei:
                ctx.time_pass("mech_row_inv", 20)
            assert ei.value.status == fgcg.FGCG_EUNSUPPORTED
        print(f"time_pass 256x128 form {form}: {times}", flush=True)
        assert all(0.0 < t < 1e4 for t in times.values())
        assert ctx.get_option("rows") != 0  # tuned on the way
    for kind, reps in (("mech_kp", 10), ("mech_row_fwd", 0), ("mech_row_fwd", 100001)):
        with pytest.raises(fgcg.FgcgError):
            ctx.time_pass(kind, reps)
    # the context still solves afterwards
    ph, _ = inputs.box_fractal(256, 2, 4, 1.7, 0.3, np.random.default_rng(9))
    out = ctx.mech_solve(torch.from_numpy(np.ascontiguousarray(ph[:128, :256])).to(dev), E_TAB, NU_TAB,
                         (1e-3, 0.0, 0.0), tol=1e-10, maxit=20000)
    assert out["info"]["status"] == 0
    c3 = fgcg.Context(16, 16, H, nz=16)
    with pytest.raises(fgcg.FgcgError):
        c3.time_pass("mech_row_fwd", 10)


def test_tuned_picks_cached(torch_dev):
    """A second context of the same shape and settings takes the first one's
    tuned picks (no timing), and its solves equal the first context's bitwise;
    another preconditioner or iteration form is tuned on its own."""
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    nx, ny = 512, 256
    ph, _ = inputs.box_fractal(512, 2, 5, 1.7, 0.3, np.random.default_rng(4))
    phase = torch.from_numpy(np.ascontiguousarray(ph[:ny, :nx])).to(dev)
    picks, outs = [], []
    for _ in range(2):
        ctx = fgcg.Context(nx, ny, H)
        outs.append(ctx.mech_solve(phase, E_TAB, NU_TAB, (1e-3, 0.0, 0.0), tol=1e-10, maxit=20000))
        picks.append(tuple(ctx.get_option(o) for o in ("rows", "row_plan", "col_plan", "mech_form")))
        ctx.close()
    print(f"cached picks {picks}", flush=True)
    assert picks[0] == picks[1] and all(v != 0 for v in picks[0])
    assert torch.equal(outs[0]["strain"], outs[1]["strain"])
    ctx = fgcg.Context(nx, ny, H)
    ctx.set_option("spectral_residual", 0)
    out = ctx.mech_solve(phase, E_TAB, NU_TAB, (1e-3, 0.0, 0.0), tol=1e-10, maxit=20000)
    assert out["info"]["status"] == 0 and all(ctx.get_option(o) != 0 for o in ("rows", "row_plan", "col_plan"))
    ctx.close()
