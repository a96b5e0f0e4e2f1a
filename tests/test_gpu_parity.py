"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Operator level (one application): the mechanics solver's own K (stiffness
pass) and M (Green transform passes) element-wise against the sparse stencil
matrix and the oracle transforms (max |a - b| / max |b| <= 1e-12 FP64,
1e-5 FP32-mixed), also at 1024^2; phase field and diffusion through the
spectral passes (relative error <= 1e-12); square, non-square, radix-3 and
ragged shapes (ny not a multiple of the rows per block).
Solve level: fixed-iteration parity (same k CG iterations from the same
start, <= 1e-10) and converged parity (both to tol 1e-12/1e-13, <= 1e-10 on
strain, stress, mean stress and energy), staggered steps, edge cases (zero
right-hand side, iteration limit, non-finite input), and the 1024^2 fractal
of the benchmark (fixed-iteration parity plus size-independent properties).
"""
import numpy as np
import pytest

from oracle import diffusion as odf, material as omat, mech as omech, phasefield as opf
from oracle import spectral as osp, staggered as ostg
from paper_2305_13081_amd import inputs

pytestmark = pytest.mark.gpu

E_TAB = (3e6, 30e9)
NU_TAB = (0.2, 0.2)
H = 5e-6
GC, L0 = 50.0, 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda", 0)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ctx_for(nx, ny):
    from paper_2305_13081_amd import fgcg
    return fgcg.Context(nx, ny, H)


def rand_phase(ny, nx, seed, frac=0.4):
    rng = np.random.default_rng(seed)
    return (rng.random((ny, nx)) >= frac).astype(np.uint8)


SHAPES = [(8, 8), (24, 16), (16, 12), (64, 64), (48, 96), (384, 8), (96, 384), (256, 256)]


def maxrel(a, b):
    """Element-wise: max |a - b| / max |b| (a single bad voxel cannot hide)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _k_m_refs(phase, d, u, kappa=1e-6):
    from oracle import direct as odir, precond as opc
    q_ref = odir.mech_stiffness_apply(phase, E_TAB, NU_TAB, u, H, d=d, kappa=kappa)
    z_ref = opc.apply_green(u, osp.grad_symbols(phase.shape, H))
    return q_ref, z_ref


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_solver_operators_parity(torch_dev, nx, ny):
    """K (k_mech_kp) and M (Green passes) of the solver, element-wise against
    the sparse stencil matrix and the oracle transforms, FP64 and FP32."""
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    print(f"solver operators {nx}x{ny}", flush=True)
    rng = np.random.default_rng(nx * 1000 + ny)
    phase = rand_phase(ny, nx, 1)
    d = 0.5 * rng.random((ny, nx))
    u = rng.standard_normal((2, ny, nx))
    q_ref, z_ref = _k_m_refs(phase, d, u)
    for prec, bar in ((fgcg.FP64, 1e-12), (fgcg.FP32_MIXED, 1e-5)):
        ctx = fgcg.Context(nx, ny, H, precision=prec)
        args = (torch.from_numpy(phase).to(dev), E_TAB, NU_TAB, torch.from_numpy(u).to(dev))
        q = ctx.debug_apply(fgcg.OP_MECH_K, *args, d=torch.from_numpy(d).to(dev), kappa=1e-6).cpu().numpy()
        z = ctx.debug_apply(fgcg.OP_MECH_M, *args).cpu().numpy()
        eq, ez = maxrel(q, q_ref), maxrel(z, z_ref)
        print(f"  prec {prec}: K max rel {eq:.2e}, M max rel {ez:.2e}", flush=True)
        assert eq < bar and ez < bar
        ctx.close()


def test_solver_operators_full_size(torch_dev):
    """The 1024^2 instantiations of the staggered workload (tuned plans): in
    FP64 each mechanics form's own kernels (mech_form 2: the fused row stage,
    whose init mode applies M's last step and whose stiffness gives K; 3: the
    stiffness + transform pass and the inverse pass; 4: the stencil pass and
    the four-pass transforms), and the form the tuner keeps."""
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    n = 1024
    phase, _ = inputs.c2_microstructure(n)
    rng = np.random.default_rng(5)
    d = 0.5 * rng.random((n, n))
    u = rng.standard_normal((2, n, n))
    q_ref, z_ref = _k_m_refs(phase, d, u)
    cases = [(fgcg.FP64, 1e-12, f) for f in (0, 2, 3, 4)] + [(fgcg.FP32_MIXED, 1e-5, 0)]
    for prec, bar, form in cases:
        ctx = fgcg.Context(n, n, H, precision=prec)
        if form:
            ctx.set_option("mech_form", form)
        args = (torch.from_numpy(phase).to(dev), E_TAB, NU_TAB, torch.from_numpy(u).to(dev))
        z = ctx.debug_apply(fgcg.OP_MECH_M, *args).cpu().numpy()  # (tunes the passes and the form)
        q = ctx.debug_apply(fgcg.OP_MECH_K, *args, d=torch.from_numpy(d).to(dev), kappa=1e-6).cpu().numpy()
        eq, ez = maxrel(q, q_ref), maxrel(z, z_ref)
        print(f"1024^2 prec {prec} form {ctx.get_option('mech_passes')} plans {ctx.get_option('row_plan')}/"
              f"{ctx.get_option('col_plan')}: K max rel {eq:.2e}, M max rel {ez:.2e}", flush=True)
        assert eq < bar and ez < bar
        if form:
            assert ctx.get_option("mech_passes") == form
        ctx.close()


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_phasefield_apply_parity(torch_dev, nx, ny):
    torch, dev = torch_dev
    rng = np.random.default_rng(7 + nx + ny)
    Hf = 1e6 * rng.random((ny, nx))
    v = rng.standard_normal((ny, nx))
    ctx = ctx_for(nx, ny)
    q = ctx.phasefield_apply(torch.from_numpy(Hf).to(dev), GC, L0, torch.from_numpy(v).to(dev)).cpu().numpy()
    n2 = osp.norm2(osp.grad_symbols((ny, nx), H))
    ref = opf.pf_operator(v, Hf, GC, L0, n2)
    assert rel(q, ref) < 1e-12


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_diffusion_apply_parity(torch_dev, nx, ny):
    torch, dev = torch_dev
    rng = np.random.default_rng(11 + nx + ny)
    phase = rand_phase(ny, nx, 3)
    v = rng.standard_normal((ny, nx))
    Dt, kt, dt = (1e-9, 1e-12), (1e-3, 0.0), 40.0
    ctx = ctx_for(nx, ny)
    q = ctx.diffusion_apply(torch.from_numpy(phase).to(dev), Dt, kt, dt, torch.from_numpy(v).to(dev)).cpu().numpy()
    D = osp.grad_symbols((ny, nx), H)
    ref = odf.diffusion_operator(v, np.asarray(Dt)[phase], np.asarray(kt)[phase], dt, D)
    assert rel(q, ref) < 1e-12


def _c1():
    phase = inputs.circle_pore(64, 10.0)
    return phase, np.where(phase == 0, 1e-3, 0.0)


def test_mech_fixed_iteration_parity_c1(torch_dev):
    torch, dev = torch_dev
    phase, e = _c1()
    ctx = ctx_for(64, 64)
    for k in (1, 5, 40):
        r = ctx.mech_solve(torch.from_numpy(phase).to(dev), E_TAB, NU_TAB, (0, 0, 0),
                           eig=torch.from_numpy(e).to(dev), tol=0.0, maxit=k)
        o = omech.mech_solve(phase, E_TAB, NU_TAB, (0, 0, 0), H, e=e, fixed_iters=k)
        assert r["info"]["iters"] == k and r["info"]["status"] == 1
        err = rel(r["strain"].cpu().numpy(), o["strain"])
        print(f"C1 fixed k={k}: strain rel err {err:.2e}", flush=True)
        assert err < 1e-10


def test_mech_converged_parity_c1(torch_dev):
    torch, dev = torch_dev
    phase, e = _c1()
    ctx = ctx_for(64, 64)
    r = ctx.mech_solve(torch.from_numpy(phase).to(dev), E_TAB, NU_TAB, (0, 0, 0), eig=torch.from_numpy(e).to(dev),
                       tol=1e-13, maxit=50000)
    o = omech.mech_solve(phase, E_TAB, NU_TAB, (0, 0, 0), H, e=e, tol=1e-13, maxit=50000)
    es = rel(r["strain"].cpu().numpy(), o["strain"])
    ss = rel(r["stress"].cpu().numpy(), o["stress"])
    ee = abs(r["energy"] - o["energy"]) / abs(o["energy"])
    ms = rel(r["mean_stress"], o["mean_stress"]) if np.linalg.norm(o["mean_stress"]) > 0 else 0
    print(f"C1 converged: iters gpu {r['info']['iters']} oracle {o['iters']}; rel err strain {es:.2e} "
          f"stress {ss:.2e} energy {ee:.2e} mean-stress {ms:.2e}", flush=True)
    assert r["info"]["status"] == 0
    assert es < 1e-10 and ss < 1e-10 and ee < 1e-10
    # mean stress is ~0 here (zero macro strain), compare against the stress scale
    assert np.max(np.abs(r["mean_stress"] - o["mean_stress"])) < 1e-10 * np.max(np.abs(o["stress"]))


def test_mech_macro_strain_damage_parity(torch_dev):
    torch, dev = torch_dev
    nx, ny = 48, 32
    phase, _ = inputs.box_fractal(48, 2, 3, 1.8, 0.3, np.random.default_rng(5))
    phase = phase[:ny, :]
    rng = np.random.default_rng(9)
    d = 0.6 * rng.random((ny, nx))
    e = 1e-3 * rng.random((ny, nx)) * (phase == 0)
    em = (1e-3, -3e-4, 2e-4)
    ctx = ctx_for(nx, ny)
    r = ctx.mech_solve(torch.from_numpy(phase).to(dev), E_TAB, NU_TAB, em, d=torch.from_numpy(d).to(dev),
                       kappa=1e-6, eig=torch.from_numpy(e).to(dev), tol=1e-13, maxit=50000)
    o = omech.mech_solve(phase, E_TAB, NU_TAB, em, H, d=d, kappa=1e-6, e=e, tol=1e-13, maxit=50000)
    assert rel(r["strain"].cpu().numpy(), o["strain"]) < 1e-10
    assert rel(r["mean_stress"], o["mean_stress"]) < 1e-10
    assert abs(r["energy"] - o["energy"]) < 1e-10 * abs(o["energy"])


def test_mech_edge_cases(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    phase, e = _c1()
    ctx = ctx_for(64, 64)
    ph = torch.from_numpy(phase).to(dev)
    # zero right-hand side: zero iterations, strain = 0
    r = ctx.mech_solve(ph, E_TAB, NU_TAB, (0, 0, 0), tol=1e-10)
    assert r["info"]["iters"] == 0 and r["info"]["status"] == 0
    assert float(r["strain"].abs().max()) == 0.0
    # iteration limit
    r = ctx.mech_solve(ph, E_TAB, NU_TAB, (0, 0, 0), eig=torch.from_numpy(e).to(dev), tol=1e-10, maxit=1)
    assert r["info"]["status"] == fgcg.FGCG_NOT_CONVERGED and r["info"]["iters"] == 1
    # non-finite input is reported, not propagated silently
    bad = e.copy()
    bad[3, 3] = np.nan
    with pytest.raises(fgcg.FgcgError) as ei:
        ctx.mech_solve(ph, E_TAB, NU_TAB, (0, 0, 0), eig=torch.from_numpy(bad).to(dev), tol=1e-10)
    assert ei.value.status == -2
    # domain errors on the host
    with pytest.raises(fgcg.FgcgError):
        ctx.mech_solve(ph, (-1.0, 30e9), NU_TAB, (0, 0, 0))
    with pytest.raises(fgcg.FgcgError):
        ctx.mech_solve(ph, E_TAB, (0.2, 0.5), (0, 0, 0))
    # repeated solves are bitwise identical (deterministic reductions)
    a = ctx.mech_solve(ph, E_TAB, NU_TAB, (1e-3, 0, 0), eig=torch.from_numpy(e).to(dev), tol=1e-10)
    b = ctx.mech_solve(ph, E_TAB, NU_TAB, (1e-3, 0, 0), eig=torch.from_numpy(e).to(dev), tol=1e-10)
    assert torch.equal(a["strain"], b["strain"]) and a["energy"] == b["energy"]


@pytest.mark.parametrize("spectral", [0, 1])
def test_phasefield_solve_parity(torch_dev, spectral):
    torch, dev = torch_dev
    nx, ny = 64, 48
    rng = np.random.default_rng(21)
    Hf = 2e6 * rng.random((ny, nx)) ** 4
    d0 = 0.2 * rng.random((ny, nx))
    ctx = ctx_for(nx, ny)
    ctx.set_option("scalar_spectral", spectral)
    dg = torch.from_numpy(d0.copy()).to(dev)
    info = ctx.phasefield_solve(torch.from_numpy(Hf).to(dev), GC, L0, dg, tol=1e-13)
    o = opf.phasefield_solve(Hf, GC, L0, H, d0=d0, tol=1e-13)
    err = rel(dg.cpu().numpy(), o["d"])
    print(f"pf: iters gpu {info['iters']} oracle {o['iters']} rel err {err:.2e}", flush=True)
    assert info["status"] == 0 and err < 1e-10
    # fixed iterations
    dg = torch.from_numpy(d0.copy()).to(dev)
    print(f"pf spectral={spectral} ok", flush=True)
    ctx.phasefield_solve(torch.from_numpy(Hf).to(dev), GC, L0, dg, tol=0.0, maxit=3)
    o = opf.phasefield_solve(Hf, GC, L0, H, d0=d0, fixed_iters=3)
    assert rel(dg.cpu().numpy(), o["d"]) < 1e-12
    # zero history: d = 0
    dg = torch.from_numpy(d0.copy()).to(dev)
    info = ctx.phasefield_solve(torch.zeros((ny, nx), dtype=torch.float64, device=dev), GC, L0, dg)
    assert info["iters"] == 0 and float(dg.abs().max()) == 0.0


@pytest.mark.parametrize("spectral", [0, 1])
@pytest.mark.parametrize("band", [0, 4])
def test_diffusion_step_parity(torch_dev, band, spectral):
    torch, dev = torch_dev
    nx, ny = 64, 64
    phase, _ = inputs.box_fractal(64, 2, 4, 1.8, 0.3, np.random.default_rng(2))
    rng = np.random.default_rng(4)
    c0 = rng.random((ny, nx))
    if band:
        c0[:, :band] = 1.0
    Dt, kt, dt = (1e-9, 1e-12), (1e-3, 0.0), 40.0
    ctx = ctx_for(nx, ny)
    ctx.set_option("scalar_spectral", spectral)
    cg = torch.from_numpy(c0.copy()).to(dev)
    info = ctx.diffusion_step_phases(torch.from_numpy(phase).to(dev), Dt, kt, band, 1.0, dt, cg, tol=1e-13)
    o = odf.diffusion_step(c0, np.asarray(Dt)[phase], np.asarray(kt)[phase], dt, H,
                           band=ostg.band_mask((ny, nx), band), c_dir=1.0, tol=1e-13)
    err = rel(cg.cpu().numpy(), o["c"])
    print(f"diffusion band={band} spectral={spectral}: iters gpu {info['iters']} oracle {o['iters']} rel err {err:.2e}", flush=True)
    assert info["status"] == 0 and err < 1e-10
    if band:
        assert float((cg[:, :band] - 1.0).abs().max()) == 0.0


@pytest.mark.parametrize("spectral", [0, 1])
def test_diffusion_mass_conservation(torch_dev, spectral):
    torch, dev = torch_dev
    nx = ny = 64
    phase = rand_phase(ny, nx, 8, 0.5)
    c0 = np.random.default_rng(8).random((ny, nx))
    ctx = ctx_for(nx, ny)
    ctx.set_option("scalar_spectral", spectral)
    cg = torch.from_numpy(c0.copy()).to(dev)
    ctx.diffusion_step_phases(torch.from_numpy(phase).to(dev), (1e-9, 1e-12), (0.0, 0.0), 0, 1.0, 40.0, cg, tol=1e-6)
    assert abs(float(cg.sum()) - c0.sum()) < 1e-12 * c0.sum()


def test_staggered_parity(torch_dev):
    torch, dev = torch_dev
    n = 32
    phase, _ = inputs.box_fractal(n, 2, 3, 1.8, 0.3, np.random.default_rng(3))
    # Gc chosen so the damage stays moderate (max d ~ 0.13): near d = 1 the
    # stiffness contrast reaches 1/kappa and two correct solves differ by ~kappa^-1 tol
    prm = ostg.Params(band_width=4, k_rate=5e-2, e_per_f=0.05, E_tab=(3e8, 30e9), Gc=1.0, maxit=50000,
                      tol_diff=1e-13, tol_mech=1e-13, tol_pf=1e-13)
    st = ostg.initial_state(phase, prm)
    ctx = ctx_for(n, n)
    gs = ctx.new_state(band_width=4, c_dir=1.0)
    gp = dict(E_tab=prm.E_tab, nu_tab=prm.nu_tab, D_tab=prm.D_tab, k_tab=(prm.k_rate, 0.0),
              band_width=prm.band_width, c_dir=prm.c_dir, dt=prm.dt, e_per_f=prm.e_per_f, Gc=prm.Gc, l0=prm.l0,
              kappa=prm.kappa, eps_mac=prm.eps_mac, tol_diff=prm.tol_diff, tol_mech=prm.tol_mech,
              tol_pf=prm.tol_pf, maxit=prm.maxit, diffuse=1)
    ph = torch.from_numpy(phase).to(dev)
    for step in range(3):
        st = ostg.step(phase, st, prm)
        info = ctx.staggered_step(gs, ph, gp)
        errs = {k: rel(gs[k].cpu().numpy(), getattr(st, k)) for k in ("c", "f", "e", "H", "d", "strain")}
        print(f"staggered step {step}: {errs} max_d {info['max_d']:.3e}", flush=True)
        for k, v in errs.items():
            assert v < 1e-10, (k, v)
        assert abs(info["energy"] - st.info["energy"]) < 1e-10 * abs(st.info["energy"])
    assert st.d.max() > 1e-2


def _gpu_params(prm):
    return dict(E_tab=prm.E_tab, nu_tab=prm.nu_tab, D_tab=prm.D_tab, k_tab=(prm.k_rate, 0.0),
                band_width=prm.band_width, c_dir=prm.c_dir, dt=prm.dt, e_per_f=prm.e_per_f, Gc=prm.Gc, l0=prm.l0,
                kappa=prm.kappa, eps_mac=prm.eps_mac, tol_diff=prm.tol_diff, tol_mech=prm.tol_mech,
                tol_pf=prm.tol_pf, maxit=prm.maxit, diffuse=1)


def test_staggered_parity_c2_parameters(torch_dev):
    """Two steps with the parameters of the 1024^2 staggered workload as
    configured (3 MPa / 30 GPa, D 1e-9 / 1e-12, k 1e-3, e_per_f 0.005, Gc 50,
    l0 10 um, kappa 1e-6, band 16 px) on a 64^2 fractal of the same generator,
    both sides converged to 1e-13."""
    torch, dev = torch_dev
    n = 64
    phase, _ = inputs.c2_microstructure(n)
    prm = ostg.Params(tol_diff=1e-13, tol_mech=1e-13, tol_pf=1e-13, maxit=100000)
    assert (prm.E_tab, prm.D_tab, prm.k_rate, prm.e_per_f, prm.Gc, prm.l0, prm.kappa, prm.band_width) == \
        ((3e6, 30e9), (1e-9, 1e-12), 1e-3, 0.005, 50.0, 1e-5, 1e-6, 16)
    st = ostg.initial_state(phase, prm)
    ctx = ctx_for(n, n)
    gs = ctx.new_state(band_width=prm.band_width, c_dir=prm.c_dir)
    ph = torch.from_numpy(phase).to(dev)
    for step in range(2):
        st = ostg.step(phase, st, prm)
        info = ctx.staggered_step(gs, ph, _gpu_params(prm))
        errs = {k: rel(gs[k].cpu().numpy(), getattr(st, k)) for k in ("c", "f", "e", "H", "d", "strain")}
        print(f"C2 parameters step {step}: {errs} iters {info['diff']['iters']}/{info['mech']['iters']}/"
              f"{info['pf']['iters']} max_d {info['max_d']:.2e}", flush=True)
        for k, v in errs.items():
            assert v < 1e-10, (k, v)
        assert abs(info["energy"] - st.info["energy"]) < 1e-10 * abs(st.info["energy"])


def _stencil_diffusion_cg(c_n, Dfield, react, dt, band, c_dir, k):
    """k CG iterations of the masked diffusion step with the operator as the
    sparse stencil matrix of oracle.direct (no transforms), from c^n."""
    import scipy.sparse as sps
    from oracle import cg as ocg, direct as odir
    grid = c_n.shape
    A = sps.diags((1.0 / dt + react).ravel())
    for a in range(len(grid)):
        B = odir.fwd_diff_matrix(grid, a, H)
        A = A + B.T @ sps.diags(Dfield.ravel()) @ B
    A = A.tocsr()
    M = (~band).ravel().astype(np.float64)
    cB = np.where(band, c_dir, 0.0).ravel()
    b = M * (c_n.ravel() / dt - A @ cB)
    x, _, _, _ = ocg.cg(lambda v: M * (A @ (M * v)), b, x0=M * c_n.ravel(), fixed_iters=k)
    return (M * x + cB).reshape(grid)


def test_staggered_fracture_regime_fixed_iterations(torch_dev):
    """d -> 1: both sides start each sub-solve from the same oracle state and
    run k fixed CG iterations (near d = 1 the stiffness contrast reaches
    1/kappa, so converged solves differ by up to the condition number times
    the tolerance; fixed iterations compare the kernels).  Mechanics and phase
    field against the oracle at 1e-10.  The diffusion step starts from c^n,
    which already nearly solves the step (|r0| / |b| ~ 4e-4), so rounding in
    the first residual decides the last digits of every iterate: two FP64
    oracles of the same iteration (the operator by transforms, and as the
    sparse stencil matrix) differ by ~4e-10 after 5 iterations.  The GPU
    iterate must lie within twice that spread of both (and within 1e-10
    where the spread is smaller)."""
    torch, dev = torch_dev
    n = 32
    phase, _ = inputs.box_fractal(n, 2, 3, 1.8, 0.3, np.random.default_rng(3))
    prm = ostg.Params(band_width=4, k_rate=5e-2, e_per_f=0.05, E_tab=(3e8, 30e9), Gc=1e-3, maxit=50000,
                      tol_diff=1e-12, tol_mech=1e-12, tol_pf=1e-12)
    st = ostg.initial_state(phase, prm)
    for _ in range(2):
        st = ostg.step(phase, st, prm)
    assert st.d.max() > 0.99
    ctx = ctx_for(n, n)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ph = T(phase)
    pore = phase == 0
    for k in (5, 20):
        # mechanics with the damaged stiffness
        r = ctx.mech_solve(ph, prm.E_tab, prm.nu_tab, prm.eps_mac, d=T(st.d), kappa=prm.kappa, eig=T(st.e),
                           tol=0.0, maxit=k)
        o = omech.mech_solve(phase, prm.E_tab, prm.nu_tab, prm.eps_mac, H, d=st.d, kappa=prm.kappa, e=st.e,
                             fixed_iters=k)
        em = rel(r["strain"].cpu().numpy(), o["strain"])
        # phase field from the current damage and history
        dg = T(st.d.copy())
        ctx.phasefield_solve(T(st.H), prm.Gc, prm.l0, dg, tol=0.0, maxit=k)
        op = opf.phasefield_solve(st.H, prm.Gc, prm.l0, H, d0=st.d, fixed_iters=k)
        ep = rel(dg.cpu().numpy(), op["d"])
        # diffusion from the current concentration
        cg = T(st.c.copy())
        ctx.diffusion_step_phases(ph, prm.D_tab, (prm.k_rate, 0.0), prm.band_width, prm.c_dir, prm.dt, cg,
                                  tol=0.0, maxit=k)
        Dfield, react = np.asarray(prm.D_tab)[phase], np.where(pore, prm.k_rate, 0.0)
        band = ostg.band_mask((n, n), prm.band_width)
        od = odf.diffusion_step(st.c, Dfield, react, prm.dt, H, band=band, c_dir=prm.c_dir, fixed_iters=k)
        # the same k iterations with the operator as the sparse stencil matrix
        # of the definition level: the warm start c^n leaves |r0| / |b| ~ 4e-4,
        # so two FP64 evaluations of the same operator (transforms, stencil)
        # already differ by a few 1e-10 after k iterations
        oc = _stencil_diffusion_cg(st.c, Dfield, react, prm.dt, band, prm.c_dir, k)
        floor = rel(oc, od["c"])
        ed = rel(cg.cpu().numpy(), oc)
        ed_fft = rel(cg.cpu().numpy(), od["c"])
        print(f"  diffusion: vs stencil-form oracle CG {ed:.2e}, vs transform-form oracle {ed_fft:.2e} "
              f"(the two oracle forms differ by {floor:.2e})", flush=True)
        bar_d = max(1e-10, 2.0 * floor)  # the spread of two FP64 evaluations of the same iteration
        assert ed < bar_d and ed_fft < bar_d
        print(f"fracture regime k={k}: mech {em:.2e} pf {ep:.2e} diff {ed:.2e}", flush=True)
        assert em < 1e-10 and ep < 1e-10


def test_c2_full_size(torch_dev):
    """1024^2 box-removal fractal, the benchmark workload."""
    torch, dev = torch_dev
    phase, _ = inputs.c2_microstructure(1024)
    rng = np.random.default_rng(77)
    e = np.where(phase == 0, 1e-3 * rng.random(phase.shape), 0.0)
    ctx = ctx_for(1024, 1024)
    ph = torch.from_numpy(phase).to(dev)
    eg = torch.from_numpy(e).to(dev)
    k = 2
    r = ctx.mech_solve(ph, E_TAB, NU_TAB, (1e-4, 0, 0), eig=eg, tol=0.0, maxit=k)
    o = omech.mech_solve(phase, E_TAB, NU_TAB, (1e-4, 0, 0), H, e=e, fixed_iters=k)
    err = rel(r["strain"].cpu().numpy(), o["strain"])
    print(f"1024^2 fixed k={k}: strain rel err {err:.2e}", flush=True)
    assert err < 1e-10
    r = ctx.mech_solve(ph, E_TAB, NU_TAB, (1e-4, 0, 0), eig=eg, tol=1e-8, maxit=100000)
    s = r["strain"].cpu().numpy()
    print(f"1024^2 converged: iters {r['info']['iters']} rel_res {r['info']['rel_res']:.2e}", flush=True)
    assert r["info"]["status"] == 0
    assert abs(s[0].mean() - 1e-4) < 1e-15 and abs(s[1].mean()) < 1e-15 and abs(s[2].mean()) < 1e-15
    res = omech.mech_residual(s, phase, E_TAB, NU_TAB, H, e=e)
    print(f"1024^2 oracle residual of the GPU strain: {res:.2e}", flush=True)
    assert res < 1e-7


@pytest.mark.parametrize("nx,ny", [(24, 12), (384, 8), (256, 96)])
def test_scalar_stencil_fixed_iterations_ragged(torch_dev, nx, ny):
    """Stencil CG on shapes whose rows do not fill the reduction grid evenly."""
    torch, dev = torch_dev
    rng = np.random.default_rng(nx + 7 * ny)
    phase = rand_phase(ny, nx, 5, 0.5)
    c0 = rng.random((ny, nx))
    c0[:, :2] = 1.0
    Dt, kt, dt = (1e-9, 1e-12), (1e-3, 0.0), 40.0
    ctx = ctx_for(nx, ny)
    for k in (1, 7):
        cg = torch.from_numpy(c0.copy()).to(dev)
        info = ctx.diffusion_step_phases(torch.from_numpy(phase).to(dev), Dt, kt, 2, 1.0, dt, cg, tol=0.0, maxit=k)
        o = odf.diffusion_step(c0, np.asarray(Dt)[phase], np.asarray(kt)[phase], dt, H,
                               band=ostg.band_mask((ny, nx), 2), c_dir=1.0, fixed_iters=k)
        assert info["iters"] == k
        assert rel(cg.cpu().numpy(), o["c"]) < 1e-12
    Hf = 1e6 * rng.random((ny, nx))
    d0 = 0.1 * rng.random((ny, nx))
    dg = torch.from_numpy(d0.copy()).to(dev)
    ctx.phasefield_solve(torch.from_numpy(Hf).to(dev), GC, L0, dg, tol=0.0, maxit=5)
    o = opf.phasefield_solve(Hf, GC, L0, H, d0=d0, fixed_iters=5)
    assert rel(dg.cpu().numpy(), o["d"]) < 1e-12


def _ctx_prec(nx, ny, prec):
    from paper_2305_13081_amd import fgcg
    return fgcg.Context(nx, ny, H, precision=prec)


def test_fp32_mixed_c1_against_fp64_oracle(torch_dev):
    """FP32 transforms and constitutive passes, FP64 reductions and true
    residual every 10 iterations: converges to tol 1e-10 and stays within
    1e-5 of the FP64 oracle."""
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    phase, e = _c1()
    ctx = _ctx_prec(64, 64, fgcg.FP32_MIXED)
    r = ctx.mech_solve(torch.from_numpy(phase).to(dev), E_TAB, NU_TAB, (0, 0, 0), eig=torch.from_numpy(e).to(dev),
                       tol=1e-10, maxit=20000)
    o = omech.mech_solve(phase, E_TAB, NU_TAB, (0, 0, 0), H, e=e, tol=1e-12, maxit=50000)
    es = rel(r["strain"].cpu().numpy(), o["strain"])
    ee = abs(r["energy"] - o["energy"]) / abs(o["energy"])
    print(f"C1 FP32-mixed: iters {r['info']['iters']} (FP64 oracle {o['iters']}), strain rel err {es:.2e}, "
          f"energy rel err {ee:.2e}", flush=True)
    assert r["info"]["status"] == 0
    assert es < 1e-5 and ee < 1e-5


def test_fp32_mixed_fractal_macro_strain(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    n = 128
    phase, _ = inputs.box_fractal(n, 2, 5, 1.7, 0.25, np.random.default_rng(31))
    em = (1e-3, 0.0, 0.0)
    ctx = _ctx_prec(n, n, fgcg.FP32_MIXED)
    r = ctx.mech_solve(torch.from_numpy(phase).to(dev), E_TAB, NU_TAB, em, tol=1e-8, maxit=50000)
    o = omech.mech_solve(phase, E_TAB, NU_TAB, em, H, tol=1e-12, maxit=50000)
    es = rel(r["strain"].cpu().numpy(), o["strain"])
    ms = abs(r["mean_stress"][0] - o["mean_stress"][0]) / abs(o["mean_stress"][0])
    print(f"128^2 fractal FP32-mixed: iters {r['info']['iters']} (oracle {o['iters']}), strain rel err {es:.2e}, "
          f"C11 rel err {ms:.2e}", flush=True)
    assert r["info"]["status"] == 0
    assert es < 1e-5 and ms < 1e-5


def test_fp32_mixed_full_size(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    phase, _ = inputs.c2_microstructure(1024)
    rng = np.random.default_rng(77)
    e = np.where(phase == 0, 1e-3 * rng.random(phase.shape), 0.0)
    ph = torch.from_numpy(phase).to(dev)
    eg = torch.from_numpy(e).to(dev)
    r32 = _ctx_prec(1024, 1024, fgcg.FP32_MIXED).mech_solve(ph, E_TAB, NU_TAB, (1e-4, 0, 0), eig=eg, tol=1e-8,
                                                           maxit=100000)
    r64 = _ctx_prec(1024, 1024, fgcg.FP64).mech_solve(ph, E_TAB, NU_TAB, (1e-4, 0, 0), eig=eg, tol=1e-8,
                                                     maxit=100000)
    s32 = r32["strain"].cpu().numpy()
    d = rel(s32, r64["strain"].cpu().numpy())
    res = omech.mech_residual(s32, phase, E_TAB, NU_TAB, H, e=e)
    print(f"1024^2 FP32-mixed: iters {r32['info']['iters']} (FP64 {r64['info']['iters']}), vs FP64 GPU {d:.2e}, "
          f"oracle residual {res:.2e}", flush=True)
    assert r32["info"]["status"] == 0
    assert d < 1e-5 and res < 1e-7



@pytest.mark.parametrize("nx,ny,masked,sink", [(64, 48, True, True), (24, 16, True, False), (96, 64, False, True)])
def test_diffusion_field_form(torch_dev, nx, ny, masked, sink):
    """Per-voxel D (not a phase table), per-voxel rate and an arbitrary
    Dirichlet mask (the form Sec. 2.1 states D in)."""
    torch, dev = torch_dev
    rng = np.random.default_rng(nx + 7 * ny)
    Df = 10.0 ** rng.uniform(-12.0, -9.0, (ny, nx))
    kr = 1e-3 * rng.random((ny, nx)) if sink else None
    mask = (rng.random((ny, nx)) < 0.1).astype(np.uint8) if masked else None
    c0 = rng.random((ny, nx))
    dt, c_dir = 40.0, 0.7
    T = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = ctx_for(nx, ny)
    cg = T(c0.copy())
    info = ctx.diffusion_step(cg, T(Df), dt, krate=T(kr), mask=T(mask), c_dir=c_dir, tol=1e-13)
    o = odf.diffusion_step(c0, Df, 0.0 if kr is None else kr, dt, H, band=None if mask is None else mask.astype(bool),
                           c_dir=c_dir, tol=1e-13)
    c = cg.cpu().numpy()
    err, emax = rel(c, o["c"]), maxrel(c, o["c"])
    print(f"diffusion field form {nx}x{ny} mask={masked} sink={sink}: iters {info['iters']} / {o['iters']}, "
          f"rel {err:.2e} max rel {emax:.2e}", flush=True)
    assert info["status"] == 0 and err < 1e-10 and emax < 1e-10
    if masked:
        assert np.all(c[mask != 0] == c_dir)
    # fixed iterations
    cg = T(c0.copy())
    ctx.diffusion_step(cg, T(Df), dt, krate=T(kr), mask=T(mask), c_dir=c_dir, tol=0.0, maxit=4)
    o = odf.diffusion_step(c0, Df, 0.0 if kr is None else kr, dt, H, band=None if mask is None else mask.astype(bool),
                           c_dir=c_dir, fixed_iters=4)
    assert maxrel(cg.cpu().numpy(), o["c"]) < 1e-12
    if not masked and not sink:
        assert abs(float(cg.sum()) - c0.sum()) < 1e-12 * c0.sum()


def test_diffusion_field_matches_phase_tables(torch_dev):
    """The field form given D and k from the phase tables and the band as a
    mask reproduces the phase-table fast path."""
    torch, dev = torch_dev
    n = 64
    phase, _ = inputs.box_fractal(n, 2, 4, 1.8, 0.3, np.random.default_rng(2))
    c0 = np.random.default_rng(4).random((n, n))
    Dt, kt, dt, band = (1e-9, 1e-12), (1e-3, 0.0), 40.0, 4
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = ctx_for(n, n)
    a = T(c0.copy())
    ctx.diffusion_step_phases(T(phase), Dt, kt, band, 1.0, dt, a, tol=1e-12)
    b = T(c0.copy())
    mask = np.zeros((n, n), np.uint8)
    mask[:, :band] = 1
    ctx.diffusion_step(b, T(np.asarray(Dt)[phase]), dt, krate=T(np.asarray(kt)[phase]), mask=T(mask), c_dir=1.0,
                       tol=1e-12)
    assert torch.equal(a, b)
