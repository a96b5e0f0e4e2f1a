"""Benchmark: FP64 staggered corrosion-fracture steps on a 1024^2 fractal.

Workload (one "step" = one pass of the whole hot path): a 2D 1024 x 1024
periodic grid, h = 5 um, with a seeded box-removal fractal pore mask (8
levels, number-size exponent 1.8, porosity 0.3); one staggered step =
transient ferrous-ion diffusion (D = 1e-9 / 1e-12 m^2/s in pores / solid,
Dirichlet band x < 16 px, sink k = 1e-3 /s in pores, dt = 40 s) ->
precipitation and pore eigenstrain (0.5 % per unit precipitate) ->
projected-CG mechanics (E = 30 GPa / 3 MPa, nu = 0.2, degraded by the
damage) -> history update -> AT2 phase field (Gc = 50 J/m^2, l0 = 2 px), all
CG tolerances 1e-8, FP64.  Synthetic inputs, resident in HBM before timing.

value = total voxel-CG-iterations (all three solvers) / wall time of the
timed steps; mech_voxel_cg_iters_per_s is the mechanics solves alone.  The
roofline block reports the dominant kernel (largest summed device time of the
four mechanics passes in the last warm-up step): its algorithmic bytes per
voxel (ALGO_BYTES) over the average duration of 200 back-to-back launches
between HIP events on the library's stream; the same passes on a 2048^2
workspace (larger than the Infinity Cache) are reported beside it.  traffic
is the counter-measured HBM bytes per launch recorded under profiles/,
reported only while the kernel sources are the ones it was measured on.  The
CPU baseline times the FP64 oracle before any GPU work: the median of five
mechanics CG iterations at 1024^2 after a warm-up, the full single-pore solve
and a sample of the batched workload on one core and on a process pool.

The "variants" block reports the other workloads of the method on the same
GPU: 64^2 single-pore latency, the 1024^2 adjoint against the forward solve,
256 batched uneven-size samples (FP64 and FP32-mixed) against the same solves
one at a time, the 256^3 3D staggered loop in FP32-mixed against plain FP64,
the static diffusion homogenisation of the 1024^2 fractal, and the mechanics
with the reference-medium preconditioner against the unit Green operator,
each with its accuracy.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-variants]
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_SIDE = 1024
H = 5e-6
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per voxel per launch of the FP64 mechanics CG passes
# (displacement form: 2 components; 16-byte complex half spectrum of
# 513 x 1024 modes = 8.0156 B per voxel per component):
#   kp     : read p (16) + phase (1) + damage (8), write q (16); stencil
#            neighbours of p and the material counted once
#   row_fwd: read x, r, p, q (64), write x, r (32), write 2 spectra (16.03)
#   col    : read 2 spectra (16.03), write 2 spectra (16.03)
#   row_inv: read 2 spectra (16.03), read p (16), write p (16)
SPEC_B = 16.0 * (N_SIDE // 2 + 1) / N_SIDE
ALGO_BYTES = {
    "mech_kp": 16 + 1 + 8 + 16,
    "mech_row_fwd": 64 + 32 + 2 * SPEC_B,
    "mech_col": 2 * SPEC_B + 2 * SPEC_B,
    "mech_row_inv": 2 * SPEC_B + 16 + 16,
}


# The residual-spectrum PCG (FP64 2D contexts with nx a multiple of 256, the
# library's default there), bytes per voxel (sp: one component's half
# spectrum per voxel):
# three passes per iteration,
#   row_fwd (k_kp_fwd2): read p (16), phase (1), damage (8); write 2 spectra
#   col    : read 2 spectra of q and 2 of r, write 2 of r and 2 of z
#   row_inv: read 2 spectra, p and x (32); write p and x (32)
# two passes per iteration (the row stage fused: k_sr_row),
#   row_fwd: read 2 spectra of z, p, x, phase and damage; write x, p and 2
#            spectra of q (the halo rows it also transforms are re-reads of
#            lines its neighbours own: not algorithmic bytes)
#   col    : as above
# (the timing hooks use phase and damage fields too)
def algo_bytes_sr(n, timing=False, passes=3):
    sp = 16.0 * (n // 2 + 1) / n
    if passes == 2:
        return {"mech_row_fwd": 2 * sp + 16 + 32 + 16 + 9 + 2 * sp, "mech_col": 8 * sp}
    return {"mech_row_fwd": 16 + 9 + 2 * sp, "mech_col": 8 * sp, "mech_row_inv": 2 * sp + 64}


ITERATION_FORM = {2: "two passes, residual spectrum, row stage fused", 3: "three passes, residual spectrum",
                  4: "four passes"}


def kinds_of(passes):
    """The timed mechanics kinds of an iteration form."""
    return {2: ["mech_row_fwd", "mech_col"], 3: ["mech_row_fwd", "mech_col", "mech_row_inv"],
            4: ["mech_kp", "mech_row_fwd", "mech_col", "mech_row_inv"]}[passes]


# 3D (256^3) mechanics passes, bytes per voxel with w-byte words (3
# displacement components; half spectrum 129/256 of a word per component and
# direction of storage, complex = 2 words): kp reads p, phase, damage and
# writes q; row_fwd reads x, r, p, q, writes x, r and 3 spectra; the y and z
# passes read and write 3 spectra; row_inv reads 3 spectra and p, writes p.
def algo_bytes_3d(w, n=256):
    sp = 3 * 2 * w * (n // 2 + 1) / n
    return {"mech_kp": 6 * w + 1 + 8, "mech_row_fwd": 18 * w + sp, "mech_y_fwd": 2 * sp, "mech_col": 2 * sp,
            "mech_y_inv": 2 * sp, "mech_row_inv": sp + 6 * w}


KINDS_3D = ["mech_kp", "mech_row_fwd", "mech_y_fwd", "mech_col", "mech_y_inv", "mech_row_inv"]

# HBM traffic per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# recorded under profiles/ (scaled by the copy probe), valid only for the
# kernel sources they were taken with: the key is the SHA-256 of csrc/.
MEASURED_TRAFFIC = {
    # hash of the 2D pass sources -> {kernel kind: HBM bytes per launch}
    # (profiles/mech_passes_1024_fp64_hbm_traffic.md); the two-pass
    # residual-spectrum form: mech_row_fwd is the fused row stage
    "656aa0d4b0023065ef3a7d5530a041da0f584925a16c0e199e4142353b5cd033": {
        "mech_row_fwd": 110683231, "mech_col": 65986538},
}


def csrc_hash():
    """SHA-256 over the translation unit of the 2D passes: fgcg.hip and every
    header it includes (transitively), so that a change to another source
    keeps the measured traffic valid and a change to these voids it."""
    import hashlib
    d = os.path.join(ROOT, "paper_2305_13081_amd", "csrc")
    seen, todo = set(), ["fgcg.hip"]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(os.path.join(d, f)):
            continue
        seen.add(f)
        with open(os.path.join(d, f)) as fh:
            todo += [m for m in re.findall(r'^#include "([^"]+)"', fh.read(), re.M)]
    h = hashlib.sha256()
    for f in sorted(seen):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def c2_params():
    return dict(E_tab=(3e6, 30e9), nu_tab=(0.2, 0.2), D_tab=(1e-9, 1e-12), k_tab=(1e-3, 0.0), band_width=16,
                c_dir=1.0, dt=40.0, e_per_f=0.005, Gc=50.0, l0=2 * H, kappa=1e-6, eps_mac=(0.0, 0.0, 0.0),
                tol_diff=1e-8, tol_mech=1e-8, tol_pf=1e-8, maxit=200000, diffuse=1)


def _oracle_mech_problem(phase, e_val=1e-3, eps_mac=(0.0, 0.0, 0.0)):
    from oracle import mech as omech, spectral as osp
    e = np.where(phase == 0, e_val, 0.0)
    lam, mu = omech.voxel_lame(phase, (3e6, 30e9), (0.2, 0.2))
    D = osp.grad_symbols(phase.shape, H)
    E0 = omech.macro_tensor(eps_mac, 2, phase.shape) - omech.eigen_tensor(e, 2, phase.shape)
    b = -omech.mech_operator(E0, lam, mu, D, "full")
    return b, (lambda p: omech.mech_operator(p, lam, mu, D, "full"))


def _oracle_iteration_seconds(phase, iters, eps_mac=(0.0, 0.0, 0.0), e_val=1e-3):
    """Durations of `iters` oracle CG iterations (the interval between the
    operator applications that start them; the last ends with the solve)."""
    from oracle import cg as ocg
    b, A = _oracle_mech_problem(phase, e_val, eps_mac)
    stamps = []

    def A_timed(p):
        stamps.append(time.perf_counter())
        return A(p)

    ocg.cg(A_timed, b, fixed_iters=iters)
    stamps.append(time.perf_counter())
    return [stamps[i + 1] - stamps[i] for i in range(iters)]


def _c3_oracle_sample(args):
    """One batched-workload sample: seconds of `iters` oracle CG iterations
    (pool worker; no GPU)."""
    phase, iters = args
    t0 = time.perf_counter()
    _oracle_iteration_seconds(phase, iters, eps_mac=(1e-3, 0.0, 0.0), e_val=0.0)
    return time.perf_counter() - t0


def cpu_baseline(phase, pool_cap=16):
    """The FP64 oracle on the machine's host cores, before any GPU work:
    * the median of 5 mechanics CG iterations at 1024^2 after one warm-up
      iteration (the headline workload's mechanics operator);
    * the full single-pore 64^2 solve to tol 1e-10;
    * a sample of the batched workload (its first 8 microstructures, 3 CG
      iterations each) on one core, and the same samples over a process pool
      on all host cores (joined before the function returns)."""
    import multiprocessing as mp
    from oracle import mech as omech
    from paper_2305_13081_amd import inputs

    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    print("cpu baseline: 6 oracle iterations at 1024^2 ...", file=sys.stderr, flush=True)
    secs = _oracle_iteration_seconds(phase, 6)
    med = float(np.median(secs[1:]))
    print(f"cpu baseline: median {med:.2f} s per iteration; single pore 64^2 solve ...", file=sys.stderr, flush=True)
    c1 = inputs.circle_pore(64)
    t0 = time.perf_counter()
    o = omech.mech_solve(c1, (3e6, 30e9), (0.2, 0.2), (0.0, 0.0, 0.0), H, e=np.where(c1 == 0, 1e-3, 0.0),
                         tol=1e-10, maxit=20000)
    t_c1 = time.perf_counter() - t0
    samples = [p for p, _ in inputs.c3_samples(8)]
    iters = 3
    work = float(sum(p.size for p in samples) * iters)
    print(f"cpu baseline: single pore {t_c1:.2f} s ({o['iters']} iterations); batched sample on 1 core ...",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for p in samples:
        _c3_oracle_sample((p, iters))
    t_one = time.perf_counter() - t0
    ncore = max(1, min(pool_cap, avail))
    print(f"cpu baseline: batched sample on {ncore} processes ...", file=sys.stderr, flush=True)
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(processes=min(ncore, len(samples))) as pool:
        pool.map(_c3_oracle_sample, [(p, iters) for p in samples])
        pool.close()
        pool.join()
    t_all = time.perf_counter() - t0
    return {"value": phase.size / med, "unit": "voxel-CG-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"median of 5 FP64 mechanics CG iterations of the oracle (naive recursive DFT, strain form) "
                      f"at 1024^2 after one warm-up iteration: {med:.2f} s per iteration, single thread "
                      f"(host: {avail} cores available)",
            "iteration_seconds": secs,
            "single_pore_64": {"seconds": t_c1, "iters": o["iters"], "us_per_iter": t_c1 / o["iters"] * 1e6,
                               "cores": 1},
            "batched_sample": {"samples": len(samples), "voxels": int(sum(p.size for p in samples)),
                               "iters_each": iters,
                               "one_core_voxel_cg_iters_per_s": work / t_one,
                               "pool_voxel_cg_iters_per_s": work / t_all, "pool_processes": min(ncore, len(samples)),
                               "note": "the first 8 microstructures of the batched workload, 3 oracle CG "
                                       "iterations each"}}


def c5_variant(torch, fgcg, inputs, dev, steps=2):
    """256^3 Menger-type fractal, mechanics + AT2 phase field with the pore
    eigenstrain ramp, FP32-mixed against plain FP64 (same GPU, same steps)."""
    n = 256
    phase_np, info = inputs.c5_microstructure(n)
    phase = torch.from_numpy(phase_np).to(dev)
    prm = dict(E_tab=(3e6, 30e9), nu_tab=(0.2, 0.2), D_tab=(1e-9, 1e-12), k_tab=(1e-3, 0.0), band_width=0,
               c_dir=1.0, dt=40.0, e_per_f=0.005, Gc=50.0, l0=2 * H, kappa=1e-6, eps_mac=(0.0,) * 6,
               tol_diff=1e-8, tol_mech=1e-8, tol_pf=1e-8, maxit=200000, diffuse=0, e_ramp=1e-3, n_ramp=20)
    out, fields = {}, {}
    for prec, name in ((fgcg.FP32_MIXED, "fp32_mixed"), (fgcg.FP64, "fp64")):
        ctx = fgcg.Context(n, n, H, precision=prec, nz=n)
        st = ctx.new_state()
        ctx.profile(KINDS_3D)
        ctx.staggered_step(st, phase, prm)  # warm-up step (graphs built), all passes timed
        prof = {k: ctx.profile_read(k) for k in KINDS_3D}
        ctx.profile([])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [ctx.staggered_step(st, phase, prm) for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        it = {s: sum(i[s]["iters"] for i in infos) for s in ("mech", "pf")}
        secs = {s: sum(i[s]["seconds"] for i in infos) for s in ("mech", "pf")}
        ab = algo_bytes_3d(8 if prec == fgcg.FP64 else 4, n)
        kern = {}
        for k in KINDS_3D:
            ms, nl, kn = prof[k]
            us = ms * 1e3 / max(nl, 1)
            kern[k] = {"avg_us": us, "launches": nl, "algo_bytes_per_voxel": round(ab[k], 3),
                       "achieved_GBs": ab[k] * n ** 3 / (us * 1e-6) / 1e9 if us > 0 else None, "kernel": kn}
        out[name] = {"voxel_cg_iters_per_s": n ** 3 * sum(it.values()) / el, "steps": steps, "seconds": el,
                     "iters": it, "mech_voxel_cg_iters_per_s": n ** 3 * it["mech"] / secs["mech"],
                     "pf_voxel_cg_iters_per_s": n ** 3 * it["pf"] / secs["pf"],
                     "kernels_warmup_step": kern, "max_d": infos[-1]["max_d"],
                     "tuned": {"row_split": ctx.get_option("row_split"), "ztiles": ctx.get_option("ztiles")}}
        fields[name] = (st["strain"].cpu().numpy(), st["d"].cpu().numpy())
        del ctx, st
        torch.cuda.empty_cache()
    a, b = fields["fp32_mixed"], fields["fp64"]
    out["fp32_vs_fp64_rel_diff"] = {
        "strain": float(np.linalg.norm(a[0] - b[0]) / np.linalg.norm(b[0])),
        "d": float(np.linalg.norm(a[1] - b[1]) / np.linalg.norm(b[1])) if np.linalg.norm(b[1]) > 0 else 0.0}
    out["speedup_fp32_mixed_vs_fp64"] = (out["fp32_mixed"]["voxel_cg_iters_per_s"] /
                                         out["fp64"]["voxel_cg_iters_per_s"])
    out["workload"] = (f"3D {n}^3 Menger-type fractal (b 3, 4 levels, D 2.7, porosity {info['porosity']:.4f}), "
                       f"{steps} timed staggered steps (mechanics + AT2 phase field, pore eigenstrain ramp "
                       f"1e-3 over 20 steps) after 1 warm-up step, CG tol 1e-8")
    return out


def c3_variant(torch, fgcg, inputs, dev, count=256):
    """256 fractal samples of uneven sizes: one batched solve vs the same
    solves one sample at a time (plain FP64 contexts), FP64 and FP32-mixed."""
    samples = inputs.c3_samples(count)
    sizes = [(p.shape[1], p.shape[0]) for p, _ in samples]
    phases = [torch.from_numpy(p).to(dev) for p, _ in samples]
    E_tab, nu_tab, em = (3e6, 30e9), (0.2, 0.2), (1e-3, 0.0, 0.0)
    nvox = np.array([nx * ny for nx, ny in sizes], dtype=np.float64)
    out, strains = {}, {}
    for prec, name in ((fgcg.FP64, "batched_fp64"), (fgcg.FP32_MIXED, "batched_fp32_mixed")):
        b = fgcg.Batch(sizes, H, precision=prec)
        b.mech_solve(phases, E_tab, nu_tab, [em] * count, tol=1e-8, maxit=100000, want_strain=False)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = b.mech_solve(phases, E_tab, nu_tab, [em] * count, tol=1e-8, maxit=100000)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        its = np.array([i["iters"] for i in r["infos"]], dtype=np.float64)
        out[name] = {"voxel_cg_iters_per_s": float((nvox * its).sum() / el), "seconds": el,
                     "iters_min": int(its.min()), "iters_max": int(its.max())}
        strains[name] = [s.cpu().numpy() for s in r["strains"]]
        b.close()
        del b, r
    ctxs = {}
    t_el, work = 0.0, 0.0
    plain = []
    for i, (nx, ny) in enumerate(sizes):
        if (nx, ny) not in ctxs:
            ctxs[(nx, ny)] = fgcg.Context(nx, ny, H)
            ctxs[(nx, ny)].mech_solve(phases[i], E_tab, nu_tab, em, tol=1e-8, maxit=100000, want_stress=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (nx, ny) in enumerate(sizes):
        r = ctxs[(nx, ny)].mech_solve(phases[i], E_tab, nu_tab, em, tol=1e-8, maxit=100000, want_stress=False)
        work += nvox[i] * r["info"]["iters"]
        plain.append(r["strain"].cpu().numpy() if i < 16 else None)
    torch.cuda.synchronize()
    t_el = time.perf_counter() - t0
    out["plain_fp64_one_at_a_time"] = {"voxel_cg_iters_per_s": work / t_el, "seconds": t_el}
    out["batched_vs_plain_fp64"] = out["batched_fp64"]["voxel_cg_iters_per_s"] / (work / t_el)
    out["batched_fp64_vs_plain_max_rel_diff_first16"] = max(
        float(np.linalg.norm(strains["batched_fp64"][i] - plain[i]) / np.linalg.norm(plain[i])) for i in range(16))
    out["fp32_mixed_vs_fp64_max_rel_diff"] = max(
        float(np.linalg.norm(a - b) / np.linalg.norm(b))
        for a, b in zip(strains["batched_fp32_mixed"], strains["batched_fp64"]))
    out["workload"] = (f"{count} 2D box-removal fractals, n in {{128, 256, 384, 512}}, "
                       f"{int(nvox.sum())} voxels, eps11 = 1e-3, CG tol 1e-8")
    return out


def c4_variant(torch, fgcg, inputs, dev):
    """1024^2 fractal, E field 30 GPa / 3 MPa: forward solve vs adjoint
    gradient of C11 (forward + adjoint solve) and of the energy (lam = 0)."""
    phase_np, _ = inputs.c2_microstructure(N_SIDE)
    E = torch.from_numpy(np.where(phase_np == 0, 3e6, 30e9)).to(dev)
    em = (1e-3, 0.0, 0.0)
    ctx = fgcg.Context(N_SIDE, N_SIDE, H)
    ctx.mech_solve(None, None, None, em, E_field=E, nu_field=0.2, tol=1e-8, maxit=200000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fw = ctx.mech_solve(None, None, None, em, E_field=E, nu_field=0.2, tol=1e-8, maxit=200000)
    torch.cuda.synchronize()
    t_fw = time.perf_counter() - t0
    ctx.mech_adjoint(E, 0.2, em, objective=fgcg.J_C11, tol=1e-8, maxit=200000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, J, i1, i2 = ctx.mech_adjoint(E, 0.2, em, objective=fgcg.J_C11, tol=1e-8, maxit=200000)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    # Hill-Mandel closed form of dC11/dE from the forward strain (GPU, FP64)
    s = fw["strain"]
    sg = fw["stress"]
    dens = s[0] * sg[0] + s[1] * sg[1] + 2 * s[2] * sg[2]
    closed = dens / (N_SIDE * N_SIDE * em[0] ** 2 * E)
    err = float((g - closed).norm() / closed.norm())
    nv = N_SIDE * N_SIDE
    return {"forward": {"seconds": t_fw, "iters": fw["info"]["iters"],
                        "voxel_cg_iters_per_s": nv * fw["info"]["iters"] / t_fw},
            "adjoint_C11": {"seconds": t_adj, "iters_fwd": i1["iters"], "iters_adj": i2["iters"],
                            "voxel_cg_iters_per_s": nv * (i1["iters"] + i2["iters"]) / t_adj},
            "adjoint_over_forward_time": t_adj / t_fw,
            "grad_C11_vs_hill_mandel_closed_form_rel_err": err, "C11": J,
            "workload": "2D 1024^2 box-removal fractal, E 30 GPa / 3 MPa per voxel, nu 0.2, eps11 1e-3, "
                        "CG tol 1e-8, FP64"}


def c1_variant(torch, fgcg, inputs, dev, reps=20):
    """64^2 single circular pore, FP64, tol 1e-10: latency per solve."""
    phase_np = inputs.circle_pore(64)
    phase = torch.from_numpy(phase_np).to(dev)
    e = torch.from_numpy(np.where(phase_np == 0, 1e-3, 0.0)).to(dev)
    ctx = fgcg.Context(64, 64, H)
    r = ctx.mech_solve(phase, (3e6, 30e9), (0.2, 0.2), (0.0, 0.0, 0.0), eig=e, tol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = ctx.mech_solve(phase, (3e6, 30e9), (0.2, 0.2), (0.0, 0.0, 0.0), eig=e, tol=1e-10)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    return {"us_per_solve": el * 1e6, "iters": r["info"]["iters"], "us_per_iter": el * 1e6 / r["info"]["iters"],
            "workload": "2D 64^2 plane strain, one circular pore (316 voxels, E 3 MPa, eigenstrain 1e-3), "
                        "matrix 30 GPa, FP64, tol 1e-10"}


def hbm_resident_passes(torch, fgcg, dev, n=2048, reps=100):
    """The 2D FP64 mechanics passes on a 2048^2 workspace (about 330 MB, more
    than the 256 MB Infinity Cache, so the traffic comes from HBM): average
    duration of back-to-back launches between HIP events (fgcg_time_pass)."""
    ctx = fgcg.Context(n, n, H)
    spec_b = 16.0 * (n // 2 + 1) / n
    ab = {"mech_row_fwd": 64 + 32 + 2 * spec_b, "mech_col": 4 * spec_b, "mech_row_inv": 2 * spec_b + 32}
    first = ctx.time_pass("mech_col", 3)  # tunes the passes and the iteration form first
    passes = ctx.get_option("mech_passes")
    if passes < 4:
        ab = algo_bytes_sr(n, timing=True, passes=passes)
    out = {"iteration": ITERATION_FORM[passes] + " (the tuned form on this grid)"}
    del first
    for k in [k for k in kinds_of(passes) if k != "mech_kp"]:
        us = ctx.time_pass(k, reps)
        gbs = ab[k] * n * n / (us * 1e-6) / 1e9
        out[k] = {"avg_launch_us": us, "algo_bytes_per_voxel": round(ab[k], 3), "achieved_GBs": gbs,
                  "frac": gbs / HBM_PEAK_GBS}
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    out["note"] = (f"{n}^2 FP64 workspace, {reps} back-to-back launches per pass after 3 untimed, tuned plans; "
                   f"the working set exceeds the Infinity Cache")
    return out


def homogenisation_variant(torch, fgcg, inputs, dev):
    """Static diffusion homogenisation (Sec. 2.1) on the 1024^2 fractal with
    D = 1e-9 / 1e-12 m^2/s: the effective diffusivity (two solves, tol 1e-8)
    and the concentration reconstruction."""
    phase_np, _ = inputs.c2_microstructure(N_SIDE)
    Df = torch.from_numpy(np.where(phase_np == 0, 1e-9, 1e-12)).to(dev)
    ph = torch.from_numpy(phase_np).to(dev)
    ctx = fgcg.Context(N_SIDE, N_SIDE, H)
    ctx.diffusivity_eff(Df, tol=1e-8, maxit=200000)  # warm-up (graphs built)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Deff, infos = ctx.diffusivity_eff(Df, tol=1e-8, maxit=200000)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    iters = sum(i["iters"] for i in infos)
    r = ctx.diffusion_homogenize(Df, (1.0, 0.0), tol=1e-8, maxit=200000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, bp, bs = ctx.concentration(ph, r["grad_c"], (1.0, 0.0), 1.0)
    torch.cuda.synchronize()
    t_c = time.perf_counter() - t0
    return {"D_eff": Deff.tolist(), "D_eff_over_D_pore": (Deff / 1e-9).tolist(), "iters": [i["iters"] for i in infos],
            "seconds": el, "voxel_cg_iters_per_s": N_SIDE * N_SIDE * iters / el,
            "reconstruction_seconds": t_c, "beta_pore": bp, "beta_solid": bs,
            "workload": "2D 1024^2 box-removal fractal, D 1e-9 (pores) / 1e-12 (solid) m^2/s, effective "
                        "diffusivity (grad c_mac = e_x, e_y), CG tol 1e-8, FP64"}


def precond_variant(torch, fgcg, inputs, dev):
    """Mechanics of the staggered workload (1024^2 fractal, pore eigenstrain
    1e-3, tol 1e-8): unit Green operator against the isotropic reference
    medium, FP64 and FP32-mixed; accuracy against a reference solve at tol
    1e-13."""
    phase_np, _ = inputs.c2_microstructure(N_SIDE)
    ph = torch.from_numpy(phase_np).to(dev)
    e = torch.from_numpy(np.where(phase_np == 0, 1e-3, 0.0)).to(dev)
    em = (0.0, 0.0, 0.0)
    ctx = fgcg.Context(N_SIDE, N_SIDE, H)
    ctx.set_option("precond", 1)
    ref = ctx.mech_solve(ph, (3e6, 30e9), (0.2, 0.2), em, eig=e, tol=1e-13, maxit=200000)["strain"].cpu().numpy()
    ctx.close()
    out = {}
    for prec, pname in ((fgcg.FP64, "fp64"), (fgcg.FP32_MIXED, "fp32_mixed")):
        for pc, name in ((0, "unit"), (1, "reference")):
            c = fgcg.Context(N_SIDE, N_SIDE, H, precision=prec)
            c.set_option("precond", pc)
            c.mech_solve(ph, (3e6, 30e9), (0.2, 0.2), em, eig=e, tol=1e-8, maxit=200000)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = c.mech_solve(ph, (3e6, 30e9), (0.2, 0.2), em, eig=e, tol=1e-8, maxit=200000)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            s = r["strain"].cpu().numpy()
            out[f"{pname}_{name}"] = {"iters": r["info"]["iters"], "seconds": el,
                                      "us_per_iter": el / r["info"]["iters"] * 1e6,
                                      "voxel_cg_iters_per_s": N_SIDE * N_SIDE * r["info"]["iters"] / el,
                                      "strain_rel_err_vs_tight": float(np.linalg.norm(s - ref) / np.linalg.norm(ref))}
            c.close()
            del c
    out["time_to_solution_speedup_fp64"] = out["fp64_unit"]["seconds"] / out["fp64_reference"]["seconds"]
    out["workload"] = ("2D 1024^2 box-removal fractal, E 30 GPa / 3 MPa, nu 0.2, pore eigenstrain 1e-3, CG tol 1e-8; "
                       "unit Green operator (the projected CG) vs isotropic reference medium (nu 0.2)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variant", default=None,
                    help="run only this variant (c1_latency_64, c4_adjoint_1024, c3_batched_256, c5_3d_256, "
                         "homogenisation_1024, precond_1024) and print its JSON")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-MiB FP64 buffer 5 times with an elementwise kernel (reads "
                         "and writes MIB MiB each): the reference for scaling HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the library has no "
              f"multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    from paper_2305_13081_amd import inputs

    phase_np, finfo = inputs.c2_microstructure(N_SIDE)
    # the oracle runs first, on the host cores, before anything touches the GPU
    base = cpu_baseline(phase_np) if not (args.no_cpu_baseline or args.variant) else None

    import torch

    from paper_2305_13081_amd import fgcg

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.variant:
        fn = VARIANTS[args.variant]
        print(json.dumps({args.variant: fn(torch, fgcg, inputs, dev)}), flush=True)
        copy_probe(torch, dev, args.copy_probe)
        return
    phase = torch.from_numpy(phase_np).to(dev)
    ctx = fgcg.Context(N_SIDE, N_SIDE, H)
    prm = c2_params()
    state = ctx.new_state(band_width=prm["band_width"], c_dir=prm["c_dir"])
    mech_kinds = ["mech_kp", "mech_row_fwd", "mech_col", "mech_row_inv"]
    for w in range(args.warmup):
        if w == args.warmup - 1:
            ctx.profile(mech_kinds)  # last warm-up step: find the dominant pass
        info = ctx.staggered_step(state, phase, prm)
        print(f"warmup step {w}: iters diff {info['diff']['iters']} mech {info['mech']['iters']} "
              f"pf {info['pf']['iters']}", file=sys.stderr, flush=True)
    # the iteration form the tuner kept (two or three passes: no separate
    # stiffness pass; two: no inverse row pass either)
    passes = ctx.get_option("mech_passes")
    sr = passes < 4
    mech_kinds = kinds_of(passes)
    algo = algo_bytes_sr(N_SIDE, passes=passes) if sr else ALGO_BYTES
    algo_timing = algo_bytes_sr(N_SIDE, timing=True, passes=passes) if sr else ALGO_BYTES
    warm = {k: ctx.profile_read(k) for k in mech_kinds}
    dom = max(mech_kinds, key=lambda k: warm[k][0]) if args.warmup > 0 else "mech_row_fwd"
    # time only the dominant pass during the timed steps: every event-record
    # node adds idle time, so the other passes are reported from the warm-up
    ctx.profile([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        infos.append(ctx.staggered_step(state, phase, prm))
        i = infos[-1]
        print(f"step {k}: iters diff {i['diff']['iters']} mech {i['mech']['iters']} pf {i['pf']['iters']} "
              f"({i['diff']['seconds']:.3f}/{i['mech']['seconds']:.3f}/{i['pf']['seconds']:.3f} s) "
              f"max d {i['max_d']:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    nvox = N_SIDE * N_SIDE
    it = {s: sum(i[s]["iters"] for i in infos) for s in ("diff", "mech", "pf")}
    secs = {s: sum(i[s]["seconds"] for i in infos) for s in ("diff", "mech", "pf")}
    total_iters = sum(it.values())
    value = nvox * total_iters / elapsed
    prof = {k: (ctx.profile_read(k) if k == dom else warm[k]) for k in mech_kinds}
    ms, launches, kname = prof[dom]
    in_graph_s = ms / 1e3 / max(launches, 1)
    # the same kernel (tuned configuration, workspace of this grid) launched
    # back to back between two events right after the timed steps: no event
    # node between launches, so no dispatch gap is added to each launch
    avg_s = in_graph_s
    by_hook = dom in ("mech_row_fwd", "mech_row_inv", "mech_col")
    if by_hook:
        avg_s = ctx.time_pass(dom, 200) * 1e-6
    # (the timing hook's stiffness pass reads a per-voxel E field: its bytes)
    dom_bytes = (algo_timing if by_hook else algo)[dom]
    achieved = dom_bytes * nvox / avg_s / 1e9
    tr = MEASURED_TRAFFIC.get(csrc_hash(), {}).get(dom)
    per_kernel = {k: {"avg_us": prof[k][0] * 1e3 / max(prof[k][1], 1), "launches": prof[k][1],
                      "timed_in": "timed steps" if k == dom else "last warm-up step",
                      "algo_bytes_per_voxel": round(algo[k], 3),
                      "achieved_GBs": algo[k] * nvox / (prof[k][0] / 1e3 / prof[k][1]) / 1e9 if prof[k][1] else None,
                      "kernel": prof[k][2]} for k in mech_kinds}
    out = {
        "metric": "voxel-CG-iters/s",
        "value": value,
        "unit": "voxel-CG-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D 1024x1024 box-removal fractal (8 levels, D 1.8, porosity 0.3), FP64 "
                               "staggered step: diffusion + mechanics + AT2 phase field, CG tol 1e-8",
                   "grid": [N_SIDE, N_SIDE], "h": H, "porosity": finfo["porosity"],
                   "parallelism": "single GPU"},
        "breakdown": {
            "iters": it, "seconds": secs,
            "voxel_cg_iters_per_s": {s: (nvox * it[s] / secs[s] if secs[s] > 0 else None) for s in it},
            "mech_kernels": per_kernel,
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": tr, "kernel": kname,
                     "algo_bytes_per_launch": dom_bytes * nvox, "avg_launch_us": avg_s * 1e6,
                     "iteration": ITERATION_FORM[passes],
                     "in_graph_event_us": in_graph_s * 1e6,
                     "timing": "avg_launch_us: HIP events on the library stream around 200 back-to-back "
                               "launches of the kernel (the tuned configuration, on the workspace of this "
                               "grid) right after the timed steps (fgcg_time_pass); in_graph_event_us: HIP "
                               "events around every launch of the kernel inside the CG graphs during the "
                               "timed steps, which adds the dispatch gap of the event nodes to each launch"},
    }
    out["mech_voxel_cg_iters_per_s"] = out["breakdown"]["voxel_cg_iters_per_s"]["mech"]
    del ctx, state
    torch.cuda.empty_cache()
    out["roofline"]["hbm_resident_2048"] = hbm_resident_passes(torch, fgcg, dev)
    if not args.no_variants:
        variants = {}
        for name, fn in VARIANTS.items():
            print(f"variant {name} ...", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            variants[name] = fn(torch, fgcg, inputs, dev)
            print(f"variant {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        out["variants"] = variants
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)
    copy_probe(torch, dev, args.copy_probe)


VARIANTS = {"c1_latency_64": c1_variant, "c4_adjoint_1024": c4_variant, "c3_batched_256": c3_variant,
            "c5_3d_256": c5_variant, "homogenisation_1024": homogenisation_variant, "precond_1024": precond_variant}


def copy_probe(torch, dev, mib):
    if mib <= 0:
        return
    x = torch.rand(mib * 2 ** 20 // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(f"copy probe: 5 x {mib} MiB read + {mib} MiB written", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
