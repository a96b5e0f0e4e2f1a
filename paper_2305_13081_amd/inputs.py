"""Seeded synthetic microstructures and fields.

The paper's inputs are a FIB-SEM scan of cement paste (Sec. 3) that is not
available; these generators stand in for it.  They hold none of the solver
arithmetic and are shared by the tests, the benchmark and the oracle checks.

Phase ids: 0 = pore, 1 = solid (the indicator omega of Sec. 2.1 and 2.3).

* ``circle_pore``: one circular pore of radius r centred at ((n-1)/2, (n-1)/2),
  strict inequality, in an n x n solid.
* ``box_fractal``: recursive box removal.  At level l = 1..L every box that is
  still fully solid splits into b^dim children (box edges at floor(i n / b^l));
  m_l = round(p_l * eligible_l) children are removed, chosen uniformly without
  replacement, with p_l = a * b^(-l (dim - D)).  The prefactor a is solved so
  that 1 - prod_l (1 - p_l) equals the target porosity; m_l is chosen so the
  removed volume tracks 1 - prod_{j<=l} (1 - p_j) level by level, and the
  finest level absorbs the remainder so the voxel porosity is exact to one
  finest box.
  The removed-box counts then scale as (box size)^(-D): D is the number-size
  exponent.  2D uses b = 2, 3D (Menger-type) b = 3.
"""
import numpy as np
from scipy.optimize import brentq

SEED_BASE = 230513081


def seed_for(config, sample=0):
    return SEED_BASE + 1000 * config + sample


def circle_pore(n=64, radius=10.0):
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n]
    pore = (x - c) ** 2 + (y - c) ** 2 < radius ** 2
    return np.where(pore, 0, 1).astype(np.uint8)


def _edges(n, nb):
    return (np.arange(nb + 1) * n) // nb


def box_fractal(n, dim, levels, D, porosity, rng, b=None):
    """Returns (phase u8 array of shape (n,)*dim, info dict)."""
    if b is None:
        b = 2 if dim == 2 else 3
    rho = float(b) ** (-(dim - D))
    a_max = 1.0 / rho * 0.999999

    def poro(a):
        keep = 1.0
        for l in range(1, levels + 1):
            keep *= 1.0 - min(1.0, a * rho ** l)
        return 1.0 - keep

    if poro(a_max) < porosity:
        a = a_max
    else:
        a = brentq(lambda t: poro(t) - porosity, 0.0, a_max, xtol=1e-14)
    ntot = n ** dim
    target_removed = int(round(porosity * ntot))
    solid = np.ones((1,) * dim, dtype=bool)
    removed_at = []
    removed_vox = 0
    counts = []
    for l in range(1, levels + 1):
        nb = b ** l
        eligible = solid
        for ax in range(dim):
            eligible = np.repeat(eligible, b, axis=ax)
        idx = np.flatnonzero(eligible.ravel())
        e = _edges(n, nb)
        widths = np.diff(e)
        if l < levels:
            # track the cumulative porosity of the continuous model so that
            # rounding at coarse levels does not pile up at the finest one
            keep = 1.0
            for j in range(1, l + 1):
                keep *= 1.0 - min(1.0, a * rho ** j)
            goal = (1.0 - keep) * ntot - removed_vox
            m = int(round(goal / (ntot / nb ** dim)))
            m = max(0, min(m, idx.size))
            choice = rng.choice(idx, size=m, replace=False)
        else:
            # finest level absorbs the remainder, box by box
            perm = rng.permutation(idx)
            vols = np.ones(perm.size, dtype=np.int64)
            multi = np.unravel_index(perm, (nb,) * dim)
            for ax in range(dim):
                vols = vols * widths[multi[ax]]
            need = target_removed - removed_vox
            csum = np.cumsum(vols)
            m = int(np.searchsorted(csum, need, side="left"))
            if m < perm.size and m > 0 and abs(csum[m] - need) < abs(csum[m - 1] - need):
                m += 1
            elif m == 0 and need > 0 and abs(csum[0] - need) < need:
                m = 1
            m = max(0, min(m, perm.size))
            choice = perm[:m]
        mask = np.zeros(nb ** dim, dtype=bool)
        mask[choice] = True
        mask = mask.reshape((nb,) * dim)
        multi = np.nonzero(mask)
        vols = np.ones(len(multi[0]), dtype=np.int64)
        for ax in range(dim):
            vols = vols * widths[multi[ax]]
        removed_vox += int(vols.sum())
        counts.append(int(m))
        removed_at.append(mask)
        solid = eligible & ~mask
    # render: a finest box is pore if it or an ancestor was removed
    nbL = b ** levels
    # boxes never eligible at the finest level were removed at a coarser one
    pore_box = ~solid
    owner = np.searchsorted(_edges(n, nbL), np.arange(n), side="right") - 1
    grids = np.meshgrid(*([owner] * dim), indexing="ij")
    phase = np.where(pore_box[tuple(grids)], 0, 1).astype(np.uint8)
    sizes = [n / b ** l for l in range(1, levels + 1)]
    ok = [i for i, c in enumerate(counts) if c >= 8]
    slope = float("nan")
    if len(ok) >= 2:
        slope = float(np.polyfit(np.log([1.0 / sizes[i] for i in ok]),
                                 np.log([counts[i] for i in ok]), 1)[0])
    info = dict(a=a, counts=counts, porosity=float(np.mean(phase == 0)),
                fitted_dimension=slope, levels=levels, b=b)
    return phase, info


def c2_microstructure(n=1024, seed=None):
    """2D box-removal fractal: 8 levels, D = 1.8, porosity 0.3."""
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    levels = max(1, int(round(np.log2(n / 4))))
    return box_fractal(n, 2, levels, 1.8, 0.3, rng)


def c5_microstructure(n=256, seed=None):
    """3D Menger-type fractal: b = 3, 4 levels, D = 2.7, porosity 0.25."""
    rng = np.random.default_rng(seed_for(5) if seed is None else seed)
    return box_fractal(n, 3, 4, 2.7, 0.25, rng)


def c3_samples(count=256, seed=None):
    """Batched set: n ~ U{128, 256, 384, 512}, porosity ~ U(0.15, 0.4),
    D ~ U(1.6, 1.9); levels = floor(log2(n / 3)) so the finest box is 3-4 px."""
    rng = np.random.default_rng(seed_for(3) if seed is None else seed)
    out = []
    for s in range(count):
        n = int(rng.choice([128, 256, 384, 512]))
        eta = float(rng.uniform(0.15, 0.4))
        D = float(rng.uniform(1.6, 1.9))
        levels = int(np.floor(np.log2(n / 3.0)))
        sub = np.random.default_rng(seed_for(3, s + 1) if seed is None else seed + s + 1)
        phase, info = box_fractal(n, 2, levels, D, eta, sub)
        out.append((phase, info))
    return out


def random_fields(grid, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * rng.random(grid)
