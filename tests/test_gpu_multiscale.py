"""GPU parity of the multiscale coupling (Sec. 3.2) through the C ABI.

The oracle drives the same scheme step by step (oracle.multiscale: bar_step,
cell_gradients, rve_step with the volume's own D_eff and unit-gradient
fluctuation); the GPU object (fgcg_ms_*) must give the same D_eff (1e-10),
bar concentrations and gradients (1e-10) and, for every volume, the same local
concentration, precipitate, eigenstrain, history, damage and strain (1e-10
relative in the 2-norm), over steps that take the first cell past the
eigenstrain threshold while the others stay below it.  Also: a 3D volume, and
the errors the host checks report.
"""
import numpy as np
import pytest

from oracle import multiscale as oms
from paper_2305_13081_amd import inputs

pytestmark = pytest.mark.gpu
BAR = dict(ncell=8, length=2e-3, J_in=4e-5, dt=2e4)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda", 0)


def rel(a, b):
    b = np.asarray(b)
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def _prm(rp, tol_homog):
    return dict(BAR, solubility=rp.solubility, molar_volume=rp.molar_volume, Gc=rp.Gc, l0=rp.l0, kappa=rp.kappa,
                tol=rp.tol, tol_homog=tol_homog, maxit=rp.maxit)


def _run(torch, dev, phase, rp, cells, steps, fields=True):
    from paper_2305_13081_amd import fgcg
    shape = phase.shape
    ctx = fgcg.Context(shape[-1], shape[-2], rp.h, nz=shape[0] if phase.ndim == 3 else None)
    ph = torch.from_numpy(phase).to(dev)
    Dg = torch.from_numpy(np.asarray(rp.D_tab)[phase]).to(dev)
    ms = fgcg.Multiscale(ctx, ph, rp.E_tab, rp.nu_tab, Dg, _prm(rp, rp.tol), cells)
    # oracle, the same scheme
    Deff, gcu = oms.rve_setup(phase, rp)
    bp = oms.BarParams(ncell=BAR["ncell"], length=BAR["length"], J_in=BAR["J_in"], dt=BAR["dt"], D_eff=Deff[1, 1])
    cbar = np.zeros(bp.ncell)
    sts = [oms.rve_initial(phase) for _ in cells]
    out = []
    for step in range(steps):
        infos = ms.step()
        cbar = oms.bar_step(cbar, bp)
        g = oms.cell_gradients(cbar, bp)
        sts = [oms.rve_step(phase, st, gcu, g[k], cbar[k], rp) for st, k in zip(sts, cells)]
        b = ms.bar()
        errs = dict(D_eff=rel(b["D_eff"], Deff), c_bar=rel(b["c"], cbar), grad_bar=rel(b["grad"], g))
        for r, (st, k) in enumerate(zip(sts, cells)):
            assert infos[r]["c_mac"] == b["c"][k] and infos[r]["grad_mac"] == b["grad"][k]
            if fields:
                v = {n: t.cpu().numpy() for n, t in ms.volume(r).items()}
                for n, ref in (("c", st.info["c"]), ("cppt", st.cppt), ("e", st.e), ("H", st.H), ("d", st.d),
                               ("strain", st.strain)):
                    errs[f"{n}[{r}]"] = rel(v[n], ref) if np.any(ref) else float(np.max(np.abs(v[n])))
            assert abs(infos[r]["max_e"] - st.e.max()) <= 1e-10 * max(st.e.max(), 1e-300)
            assert abs(infos[r]["mean_cppt"] - st.cppt.mean()) <= 1e-10 * max(st.cppt.mean(), 1e-300)
            assert abs(infos[r]["max_d"] - st.d.max()) <= 1e-9 * max(st.d.max(), 1e-12)
        worst = max(errs.values())
        print(f"step {step}: c_bar[0] {cbar[0]:.4e}, max e {[round(float(s.e.max()), 6) for s in sts]}, "
              f"max d {[round(float(s.d.max()), 6) for s in sts]}, worst rel {worst:.2e} "
              f"({max(errs, key=errs.get)}); iters mech {[i['mech']['iters'] for i in infos]} "
              f"pf {[i['pf']['iters'] for i in infos]}", flush=True)
        assert worst < 1e-10, errs
        out.append((infos, sts))
    ms.close()
    ctx.close()
    return out


def test_multiscale_2d_matches_oracle(torch_dev):
    torch, dev = torch_dev
    phase = inputs.circle_pore(32, 8.0)
    rp = oms.RveParams(E_tab=(3e8, 30e9), Gc=10.0, tol=1e-13)
    out = _run(torch, dev, phase, rp, cells=[0, 0, 2], steps=5)
    infos, sts = out[-1]
    # the first cell is past the eigenstrain threshold, the third is not; two
    # volumes in one cell evolve alike
    assert sts[0].e.max() > 0 and sts[2].e.max() == 0.0 and infos[2]["max_e"] == 0.0
    assert infos[0]["max_e"] == infos[1]["max_e"] and infos[0]["max_d"] == infos[1]["max_d"]


def test_multiscale_3d_matches_oracle(torch_dev):
    torch, dev = torch_dev
    n = 16
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    phase = np.where((x - 7.5) ** 2 + (y - 7.5) ** 2 + (z - 7.5) ** 2 <= 5.0 ** 2, 0, 1).astype(np.uint8)
    rp = oms.RveParams(E_tab=(3e8, 30e9), Gc=10.0, tol=1e-13)
    _run(torch, dev, phase, rp, cells=[0, 3], steps=3)


def test_multiscale_errors(torch_dev):
    from paper_2305_13081_amd import fgcg
    torch, dev = torch_dev
    phase = inputs.circle_pore(32, 8.0)
    rp = oms.RveParams()
    ctx = fgcg.Context(32, 32, rp.h)
    ph = torch.from_numpy(phase).to(dev)
    Dg = torch.from_numpy(np.asarray(rp.D_tab)[phase]).to(dev)
    ok = _prm(rp, 1e-12)
    for bad, status in ((dict(ok, ncell=1), fgcg.FGCG_EDOMAIN), (dict(ok, dt=0.0), fgcg.FGCG_EDOMAIN),
                        (dict(ok, J_in=-1.0), fgcg.FGCG_EDOMAIN), (dict(ok, maxit=0), fgcg.FGCG_EDOMAIN)):
        with pytest.raises(fgcg.FgcgError) as ei:
            fgcg.Multiscale(ctx, ph, rp.E_tab, rp.nu_tab, Dg, bad, [0])
        assert ei.value.status == status
    with pytest.raises(fgcg.FgcgError) as ei:
        fgcg.Multiscale(ctx, ph, rp.E_tab, rp.nu_tab, Dg, ok, [8])
    assert ei.value.status == fgcg.FGCG_EINVAL
    solid = torch.ones_like(ph)
    with pytest.raises(fgcg.FgcgError) as ei:
        fgcg.Multiscale(ctx, solid, rp.E_tab, rp.nu_tab, Dg, ok, [0])
    assert ei.value.status == fgcg.FGCG_EDOMAIN
    c32 = fgcg.Context(32, 32, rp.h, precision=fgcg.FP32_MIXED)
    with pytest.raises(fgcg.FgcgError) as ei:
        fgcg.Multiscale(c32, ph, rp.E_tab, rp.nu_tab, Dg, ok, [0])
    assert ei.value.status == fgcg.FGCG_EUNSUPPORTED
    # no volumes: the bar alone
    ms = fgcg.Multiscale(ctx, ph, rp.E_tab, rp.nu_tab, Dg, ok, [])
    assert ms.step() == []
    b = ms.bar()
    dY = BAR["length"] / BAR["ncell"]
    assert abs(b["c"].sum() * dY - BAR["J_in"] * BAR["dt"]) < 1e-12 * BAR["J_in"] * BAR["dt"]
    ms.close()
    c32.close()
    ctx.close()
