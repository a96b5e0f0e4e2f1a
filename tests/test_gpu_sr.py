"""GPU parity of the residual-spectrum mechanics PCG through the C ABI.

2D FP64 contexts with nx a multiple of 64 keep the CG residual as its half
spectra (the stiffness stencil fused into the forward row transform, the
solution update in the pass that forms the next direction), in three passes
per iteration (form 3) or two (form 2: the inverse row stage of one
iteration and the stiffness + forward row stage of the next in one pass;
the only residual-spectrum form where nx is not a multiple of 256).  Both
forms are tested.  The iterates are those of the projected CG of
Sec. 2.3 / App. A:
* fixed-iteration parity with the oracle's projected CG (k = 1, 2, 7, 20;
  the solve ends by the iteration limit, so the last solution update is the
  deferred one), <= 1e-12, on square, non-square and ragged grids (ny not a
  multiple of the rows per block, fewer rows than a block holds);
* converged solves equal the four-pass form (option off) to 1e-10 with the
  same iteration count, and the oracle to 1e-10;
* the stiffness of each form's own kernel (the fused row stage, the stiffness
  + transform pass, the stencil pass), brought back to real space, equals the
  sparse stencil matrix element-wise (<= 1e-12);
* zero right-hand side, and a solve that converges at the first test;
* the fracture regime: a band with d up to 0.999 (g(d) down to about kappa),
  fixed-iteration parity.
"""
import numpy as np
import pytest

from oracle import mech as omech

pytestmark = pytest.mark.gpu
E_TAB, NU_TAB, H = (3e6, 30e9), (0.2, 0.2), 5e-6
E_MILD = (3e9, 30e9)  # converged comparisons with the oracle: fewer CPU iterations


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def maxrel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


def _case(ny, nx, seed):
    rng = np.random.default_rng(seed)
    phase = (rng.random((ny, nx)) < 0.6).astype(np.uint8)
    d = 0.3 * rng.random((ny, nx))
    e = np.where(phase == 0, 1e-3, 0.0)
    return phase, d, e


# (nx, ny): square, non-square, ny not a multiple of the rows per block of
# the three-pass form, fewer rows than a block (every supported length is even,
# so the two rows of a two-pass block are always both in the grid)
SHAPES = [(256, 256), (512, 96), (768, 48), (1024, 8), (256, 12), (512, 24), (2048, 16)]
FORMS = [2, 3]
# rows that are a multiple of 64 but not of 256: the two-pass form only (one
# wavefront or 128 threads per block)
SHAPES_64 = [(64, 64), (128, 48), (192, 24), (384, 32)]


@pytest.mark.parametrize("nx,ny,form", [s + (f,) for f in FORMS for s in SHAPES] + [s + (2,) for s in SHAPES_64])
def test_sr_fixed_iterations(torch_dev, nx, ny, form):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    phase, d, e = _case(ny, nx, nx + ny)
    T = lambda a: torch.from_numpy(a).to(dev)
    ctx = fgcg.Context(nx, ny, H)
    assert ctx.get_option("spectral_residual") == 1
    ctx.set_option("mech_form", form)
    em = (1e-3, -2e-4, 3e-4)
    for k in (1, 2, 7, 20):
        print(f"SR fixed {nx}x{ny} form {form} k={k}", flush=True)
        r = ctx.mech_solve(T(phase), E_TAB, NU_TAB, em, d=T(d), kappa=1e-6, eig=T(e), tol=0.0, maxit=k)
        o = omech.mech_solve(phase, E_TAB, NU_TAB, em, H, d=d, kappa=1e-6, e=e, fixed_iters=k)
        err = rel(r["strain"].cpu().numpy(), o["strain"])
        print(f"  iters {r['info']['iters']} strain rel {err:.2e}", flush=True)
        assert r["info"]["iters"] == k and r["info"]["status"] == 1 and err < 1e-12
    assert ctx.get_option("mech_passes") == form
    ctx.close()


@pytest.mark.parametrize("form", FORMS)
def test_sr_fracture_regime(torch_dev, form):
    """A cracked band (d up to 0.999: g(d) down to about kappa) across the
    grid, fixed-iteration parity with the oracle's projected CG."""
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    nx, ny = 512, 64
    phase, d, e = _case(ny, nx, 31)
    yy = np.arange(ny)[:, None] * np.ones((1, nx))
    d = np.where(np.abs(yy - ny / 2) < 3, 0.9 + 0.099 * np.random.default_rng(32).random((ny, nx)), d)
    T = lambda a: torch.from_numpy(a).to(dev)
    ctx = fgcg.Context(nx, ny, H)
    ctx.set_option("mech_form", form)
    em = (1e-3, 2e-4, -3e-4)
    for k in (1, 5, 20):
        print(f"SR fracture form {form} k={k}", flush=True)
        r = ctx.mech_solve(T(phase), E_TAB, NU_TAB, em, d=T(d), kappa=1e-6, eig=T(e), tol=0.0, maxit=k)
        o = omech.mech_solve(phase, E_TAB, NU_TAB, em, H, d=d, kappa=1e-6, e=e, fixed_iters=k)
        err = rel(r["strain"].cpu().numpy(), o["strain"])
        emax = maxrel(r["strain"].cpu().numpy(), o["strain"])
        print(f"  strain rel {err:.2e}, max rel {emax:.2e}", flush=True)
        assert r["info"]["iters"] == k and err < 1e-12 and emax < 1e-12
    ctx.close()


@pytest.mark.parametrize("nx,ny,with_oracle,form", [(256, 256, False, 2), (1024, 96, False, 2), (256, 8, True, 2),
                                                     (256, 256, False, 3), (1024, 96, False, 3), (256, 8, True, 3),
                                                     (64, 64, True, 2), (384, 32, False, 2)])
def test_sr_equals_four_pass_form(torch_dev, nx, ny, with_oracle, form):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    phase, d, e = _case(ny, nx, 3 * nx + ny)
    T = lambda a: torch.from_numpy(a).to(dev)
    et = E_MILD if with_oracle else E_TAB
    args = (T(phase), et, NU_TAB, (1e-3, 0.0, 0.0))
    kw = dict(d=T(d), kappa=1e-6, eig=T(e), tol=1e-13, maxit=50000)
    out = {}
    for sr in (1, 0):
        ctx = fgcg.Context(nx, ny, H)
        ctx.set_option("spectral_residual", sr)
        if sr:
            ctx.set_option("mech_form", form)
        out[sr] = ctx.mech_solve(*args, **kw)
        assert ctx.get_option("mech_passes") == (form if sr else 4)
        ctx.close()
    a, b = out[1], out[0]
    errs = dict(strain=rel(a["strain"].cpu().numpy(), b["strain"].cpu().numpy()),
                stress=rel(a["stress"].cpu().numpy(), b["stress"].cpu().numpy()),
                energy=abs(a["energy"] - b["energy"]) / abs(b["energy"]))
    print(f"SR form {form} vs four-pass {nx}x{ny}: iters {a['info']['iters']} / {b['info']['iters']}, {errs}", flush=True)
    if with_oracle:
        o = omech.mech_solve(phase, et, NU_TAB, (1e-3, 0.0, 0.0), H, d=d, kappa=1e-6, e=e, tol=1e-13,
                             maxit=50000)
        errs["oracle"] = rel(a["strain"].cpu().numpy(), o["strain"])
        print(f"  oracle: iters {o['iters']}, strain rel {errs['oracle']:.2e}", flush=True)
    assert a["info"]["status"] == 0 and b["info"]["status"] == 0
    assert abs(a["info"]["iters"] - b["info"]["iters"]) <= 1
    assert max(errs.values()) < 1e-10


def test_sr_stiffness_hook(torch_dev):
    from oracle import direct as odir
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    nx, ny = 512, 48
    phase, d, _ = _case(ny, nx, 11)
    u = np.random.default_rng(12).standard_normal((2, ny, nx))
    q_ref = odir.mech_stiffness_apply(phase, E_TAB, NU_TAB, u, H, d=d, kappa=1e-6)
    T = lambda a: torch.from_numpy(a).to(dev)
    for form in (2, 3, 4):  # the fused row stage, the stiffness + transform pass, the stencil pass
        ctx = fgcg.Context(nx, ny, H)
        ctx.set_option("mech_form", form)
        q = ctx.debug_apply(fgcg.OP_MECH_K, T(phase), E_TAB, NU_TAB, T(u), d=T(d), kappa=1e-6).cpu().numpy()
        err = maxrel(q, q_ref)
        print(f"K hook form {form}: max rel {err:.2e}", flush=True)
        assert err < 1e-12
        ctx.close()


@pytest.mark.parametrize("form", FORMS)
def test_sr_edge_cases(torch_dev, form):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    nx, ny = 256, 8
    phase, d, e = _case(ny, nx, 21)
    T = lambda a: torch.from_numpy(a).to(dev)
    ctx = fgcg.Context(nx, ny, H)
    ctx.set_option("mech_form", form)
    # zero right-hand side: x = 0 after 0 iterations
    r = ctx.mech_solve(T(phase), E_TAB, NU_TAB, (0.0, 0.0, 0.0), tol=1e-10)
    assert r["info"]["iters"] == 0 and float(r["strain"].abs().max()) == 0.0
    # a loose tolerance met after few iterations, then a tight one on the same context
    r1 = ctx.mech_solve(T(phase), E_TAB, NU_TAB, (1e-3, 0, 0), d=T(d), kappa=1e-6, eig=T(e), tol=1e-2)
    r2 = ctx.mech_solve(T(phase), E_MILD, NU_TAB, (1e-3, 0, 0), d=T(d), kappa=1e-6, eig=T(e), tol=1e-13,
                        maxit=50000)
    print(f"edge cases: loose solve {r1['info']['iters']} iters, tight {r2['info']['iters']}", flush=True)
    o = omech.mech_solve(phase, E_TAB, NU_TAB, (1e-3, 0, 0), H, d=d, kappa=1e-6, e=e, fixed_iters=r1["info"]["iters"])
    assert rel(r1["strain"].cpu().numpy(), o["strain"]) < 1e-12
    o2 = omech.mech_solve(phase, E_MILD, NU_TAB, (1e-3, 0, 0), H, d=d, kappa=1e-6, e=e, tol=1e-13, maxit=50000)
    assert rel(r2["strain"].cpu().numpy(), o2["strain"]) < 1e-10
    ctx.close()


def test_form_option(torch_dev):
    """Forms 2 and 3 need the residual-spectrum conditions; 4 is always
    accepted; out-of-range values are rejected."""
    from paper_2305_13081_amd import fgcg
    ctx = fgcg.Context(256, 64, H)
    assert ctx.get_option("mech_form") == 0
    for f in (2, 3, 4, 0):
        ctx.set_option("mech_form", f)
        assert ctx.get_option("mech_form") == f
    for bad in (1, 5, -1):
        with pytest.raises(fgcg.FgcgError) as ei:
            ctx.set_option("mech_form", bad)
        assert ei.value.status == fgcg.FGCG_EINVAL
    ctx.close()
    ctx = fgcg.Context(96, 64, H)  # nx not a multiple of 64
    with pytest.raises(fgcg.FgcgError) as ei:
        ctx.set_option("mech_form", 2)
    assert ei.value.status == fgcg.FGCG_EUNSUPPORTED
    ctx.set_option("mech_form", 4)
    ctx.close()
    ctx = fgcg.Context(128, 64, H)  # a multiple of 64, not of 256: no three-pass form
    ctx.set_option("mech_form", 2)
    with pytest.raises(fgcg.FgcgError) as ei:
        ctx.set_option("mech_form", 3)
    assert ei.value.status == fgcg.FGCG_EUNSUPPORTED
    ctx.close()


def test_two_pass_graph_chunks(torch_dev):
    """The two-pass form keeps p double-buffered by iteration parity, baked
    into the launches of each graph chunk: solves replayed as graphs of 2, 6
    and 16 iterations and solves launched plainly are bitwise equal."""
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    nx, ny = 256, 64
    phase, d, e = _case(ny, nx, 41)
    T = lambda a: torch.from_numpy(a).to(dev)
    outs = []
    for graphs, chunk in ((1, 16), (1, 2), (1, 6), (0, 16)):
        ctx = fgcg.Context(nx, ny, H)
        ctx.set_option("mech_form", 2)
        ctx.set_option("graphs", graphs)
        ctx.set_option("chunk", chunk)
        r = ctx.mech_solve(T(phase), E_TAB, NU_TAB, (1e-3, 0.0, 2e-4), d=T(d), kappa=1e-6, eig=T(e), tol=1e-10,
                           maxit=20000)
        print(f"two-pass graphs {graphs} chunk {chunk}: iters {r['info']['iters']}", flush=True)
        assert r["info"]["status"] == 0
        outs.append((r["info"]["iters"], r["strain"].cpu().numpy()))
        ctx.close()
    for it, st in outs[1:]:
        assert it == outs[0][0] and np.array_equal(st, outs[0][1])


@pytest.mark.parametrize("form", FORMS)
def test_sr_three_phases(torch_dev, form):
    """Three phases (the general per-phase table lookup of the stiffness
    stencil, not the two-phase selection), fixed-iteration parity."""
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    nx, ny = 256, 32
    rng = np.random.default_rng(51)
    phase = rng.integers(0, 3, (ny, nx)).astype(np.uint8)
    d = 0.3 * rng.random((ny, nx))
    e = np.where(phase == 0, 1e-3, 0.0)
    E3, NU3 = (3e6, 30e9, 5e9), (0.2, 0.2, 0.3)
    T = lambda a: torch.from_numpy(a).to(dev)
    ctx = fgcg.Context(nx, ny, H)
    ctx.set_option("mech_form", form)
    for k in (3, 12):
        r = ctx.mech_solve(T(phase), E3, NU3, (1e-3, -2e-4, 1e-4), d=T(d), kappa=1e-6, eig=T(e), tol=0.0, maxit=k)
        o = omech.mech_solve(phase, E3, NU3, (1e-3, -2e-4, 1e-4), H, d=d, kappa=1e-6, e=e, fixed_iters=k)
        err = maxrel(r["strain"].cpu().numpy(), o["strain"])
        print(f"SR three phases form {form} k={k}: max rel {err:.2e}", flush=True)
        assert r["info"]["iters"] == k and err < 1e-12
    ctx.close()
