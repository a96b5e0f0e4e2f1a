"""Definition-level solves: real-space stencils and a sparse direct solver.

No Fourier transform appears here.  The forward-difference gradient of
Sec. 2.6 is the periodic stencil (f(x + h e_a) - f(x)) / h, assembled as a
sparse matrix B_a; its transpose is the (negative) divergence.  Each discrete
problem of the path is written as the stationarity condition it encodes and
solved with ``scipy.sparse.linalg.spsolve``:

* mechanics (Sec. 2.3): minimise sum_x (E0 + sym grad u) : gC : (E0 + sym grad u)
  over periodic u, E0 = eps_mac - e I; the range of the projection of App. A is
  exactly {grad u}, so this is the solution the projected CG reaches;
* phase field (Sec. 2.4): [diag(Gc/(2 l0) + H) + (Gc l0/2) sum_a B_a^T B_a] d = H;
* diffusion step: [diag(1/dt + k_r) + sum_a B_a^T diag(D) B_a] c = c^n/dt on the
  free voxels, with c = c_dir held on the Dirichlet band.
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from . import material as _mat
from . import mech as _mech


def fwd_diff_matrix(grid, alpha, h):
    grid = tuple(grid)
    dim = len(grid)
    N = int(np.prod(grid))
    idx = np.arange(N).reshape(grid)
    nbr = np.roll(idx, -1, axis=dim - 1 - alpha)
    S = sps.csr_matrix((np.ones(N), (idx.ravel(), nbr.ravel())), shape=(N, N))
    return ((S - sps.identity(N, format="csr")) / h).tocsr()


def _stiffness_matrix(glam, gmu):
    """Sparse map eps -> sigma on tensor fields stored [i][j][x]."""
    dim = glam.ndim
    N = glam.size
    Lam = sps.diags(glam.ravel())
    Mu2 = sps.diags(2.0 * gmu.ravel())
    blocks = [[None] * (dim * dim) for _ in range(dim * dim)]
    Z = sps.csr_matrix((N, N))
    for i in range(dim):
        for j in range(dim):
            for k in range(dim):
                for l in range(dim):
                    m = Z
                    if i == j and k == l:
                        m = m + Lam
                    if i == k and j == l:
                        m = m + Mu2
                    blocks[i * dim + j][k * dim + l] = m
    return sps.bmat(blocks, format="csr")


def _symgrad_matrix(grid, h):
    """Sparse map u (stored [i][x]) -> sym(grad u) (stored [i][j][x])."""
    dim = len(grid)
    N = int(np.prod(grid))
    B = [fwd_diff_matrix(grid, a, h) for a in range(dim)]
    Z = sps.csr_matrix((N, N))
    rows = []
    for i in range(dim):
        for j in range(dim):
            row = [Z] * dim
            row[i] = row[i] + 0.5 * B[j]
            row[j] = row[j] + 0.5 * B[i]
            rows.append(row)
    return sps.bmat(rows, format="csr")


def mech_direct(phase, E_tab, nu_tab, eps_mac, h, d=None, kappa=0.0, e=None,
                E_field=None, nu=None):
    phase = np.asarray(phase)
    grid = phase.shape
    dim = phase.ndim
    N = phase.size
    lam, mu = _mech.voxel_lame(phase, E_tab, nu_tab, E_field, nu)
    g = np.ones(grid) if d is None else _mat.degradation(np.asarray(d), kappa)
    C = _stiffness_matrix(g * lam, g * mu)
    L = _symgrad_matrix(grid, h)
    E0 = _mech.macro_tensor(eps_mac, dim, grid) - _mech.eigen_tensor(e, dim, grid)
    K = (L.T @ C @ L).tocsc()
    f = -(L.T @ (C @ E0.reshape(-1)))
    # rigid translations: pin u_i at voxel 0
    keep = np.ones(dim * N, dtype=bool)
    keep[[i * N for i in range(dim)]] = False
    u = np.zeros(dim * N)
    u[keep] = spla.spsolve(K[keep][:, keep], f[keep])
    eps = _mech.macro_tensor(eps_mac, dim, grid) + (L @ u).reshape((dim, dim) + grid)
    el = eps - _mech.eigen_tensor(e, dim, grid)
    sig = _mat.stress(el, g * lam, g * mu)
    return dict(strain=_mat.to_voigt(eps), stress=_mat.to_voigt(sig),
                mean_stress=np.array([np.mean(s) for s in _mat.to_voigt(sig)]),
                energy=0.5 * h ** dim * float(np.sum(el * sig)))


def phasefield_direct(H, Gc, l0, h):
    H = np.asarray(H, dtype=np.float64)
    grid = H.shape
    B = [fwd_diff_matrix(grid, a, h) for a in range(H.ndim)]
    A = sps.diags((Gc / (2.0 * l0) + H).ravel())
    for Ba in B:
        A = A + 0.5 * Gc * l0 * (Ba.T @ Ba)
    return spla.spsolve(A.tocsc(), H.ravel()).reshape(grid)


def diffusion_direct(c_n, Dfield, react, dt, h, band=None, c_dir=1.0):
    c_n = np.asarray(c_n, dtype=np.float64)
    grid = c_n.shape
    B = [fwd_diff_matrix(grid, a, h) for a in range(c_n.ndim)]
    Dd = sps.diags(np.broadcast_to(Dfield, grid).ravel())
    A = sps.diags((1.0 / dt + np.broadcast_to(react, grid)).ravel())
    for Ba in B:
        A = A + Ba.T @ Dd @ Ba
    A = A.tocsr()
    rhs = c_n.ravel() / dt
    if band is None:
        return spla.spsolve(A.tocsc(), rhs).reshape(grid)
    band = np.asarray(band, dtype=bool).ravel()
    free = ~band
    cB = np.where(band, c_dir, 0.0)
    rhsF = rhs[free] - A[free][:, band] @ cB[band]
    c = cB.copy()
    c[free] = spla.spsolve(A[free][:, free].tocsc(), rhsF)
    return c.reshape(grid)


def diffusion_static_direct(Dfield, grad_cmac, h):
    """Static homogenisation (Sec. 2.1) at definition level: minimise
    sum_x (grad c_mac + B phi) . D (grad c_mac + B phi) over periodic phi, i.e.
    sum_a B_a^T D B_a phi = -sum_a B_a^T D grad_a c_mac, with phi pinned at voxel
    0 and then shifted to mean zero.  Returns grad c = grad c_mac + B phi
    (components first) and phi."""
    Dfield = np.asarray(Dfield, dtype=np.float64)
    grid = Dfield.shape
    dim = Dfield.ndim
    N = Dfield.size
    B = [fwd_diff_matrix(grid, a, h) for a in range(dim)]
    Dd = sps.diags(Dfield.ravel())
    K = sps.csr_matrix((N, N))
    f = np.zeros(N)
    for a in range(dim):
        K = K + B[a].T @ Dd @ B[a]
        f = f - B[a].T @ (Dfield.ravel() * grad_cmac[a])
    keep = np.ones(N, dtype=bool)
    keep[0] = False
    phi = np.zeros(N)
    K = K.tocsr()
    phi[keep] = spla.spsolve(K[keep][:, keep].tocsc(), f[keep])
    phi -= phi.mean()
    grad_c = np.array([grad_cmac[a] + (B[a] @ phi).reshape(grid) for a in range(dim)])
    return dict(grad_c=grad_c, phi=phi.reshape(grid))


def mech_stiffness_apply(phase, E_tab, nu_tab, u, h, d=None, kappa=0.0, E_field=None, nu=None):
    """q = L^T C L u: the displacement-form stiffness grad^H g C : sym(grad u)
    as the sparse stencil matrix (no FFT).  u and q are (dim, *grid)."""
    phase = np.asarray(phase)
    grid = phase.shape
    dim = phase.ndim
    lam, mu = _mech.voxel_lame(phase, E_tab, nu_tab, E_field, nu)
    g = np.ones(grid) if d is None else _mat.degradation(np.asarray(d), kappa)
    C = _stiffness_matrix(g * lam, g * mu)
    L = _symgrad_matrix(grid, h)
    return (L.T @ (C @ (L @ np.asarray(u, dtype=np.float64).reshape(-1)))).reshape((dim,) + grid)


def diff_matrix(grid, alpha, h, op="forward"):
    """Real-space matrix of the gradient along axis alpha for the operators of
    Sec. 2.6: forward (f(x+h) - f(x))/h, central (f(x+h) - f(x-h))/(2h),
    central8 (sum_m a_m (f(x+mh) - f(x-mh))/h, a = 4/5, -1/5, 4/105, -1/280)
    and fourier (the periodic spectral differentiation matrix: entries
    (pi / L) (-1)^(j-k) csc(pi (j-k) / n) for odd n, cot for even n, with the
    Nyquist mode differentiated to zero; L = n h).  Built from shifts and
    closed forms, no transform."""
    if op == "forward":
        return fwd_diff_matrix(grid, alpha, h)
    grid = tuple(grid)
    dim = len(grid)
    N = int(np.prod(grid))
    axis = dim - 1 - alpha
    idx = np.arange(N).reshape(grid)

    def shift(m):  # (S_m f)(x) = f(x + m e_alpha)
        nbr = np.roll(idx, -m, axis=axis)
        return sps.csr_matrix((np.ones(N), (idx.ravel(), nbr.ravel())), shape=(N, N))

    if op == "central":
        return ((shift(1) - shift(-1)) / (2.0 * h)).tocsr()
    if op == "central8":
        coef = (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0)
        M = sps.csr_matrix((N, N))
        for m, a in enumerate(coef, start=1):
            M = M + a * (shift(m) - shift(-m))
        return (M / h).tocsr()
    if op == "fourier":
        n = grid[axis]
        j = np.arange(n)
        dj = (j[:, None] - j[None, :]) % n
        with np.errstate(divide="ignore"):
            ang = np.pi * dj / n
            core = 1.0 / np.tan(ang) if n % 2 == 0 else 1.0 / np.sin(ang)
        D1 = np.where(dj == 0, 0.0, (np.pi / (n * h)) * (-1.0) ** dj * core)
        # D1 acts along `axis`: Kronecker product with identities on the other axes
        mats = [np.eye(g) for g in grid]
        mats[axis] = D1
        M = mats[0]
        for m in mats[1:]:
            M = np.kron(M, m)
        return sps.csr_matrix(M)
    raise ValueError(op)


def mech_direct_op(phase, E_tab, nu_tab, eps_mac, h, op, d=None, kappa=0.0, e=None):
    """mech_direct with the gradient operator `op`: the strain is unique even
    where the operator has more null modes than the translations (least
    squares on the normal equations)."""
    phase = np.asarray(phase)
    grid = phase.shape
    dim = phase.ndim
    N = phase.size
    lam, mu = _mech.voxel_lame(phase, E_tab, nu_tab)
    g = np.ones(grid) if d is None else _mat.degradation(np.asarray(d), kappa)
    C = _stiffness_matrix(g * lam, g * mu)
    B = [diff_matrix(grid, a, h, op) for a in range(dim)]
    Z = sps.csr_matrix((N, N))
    rows = []
    for i in range(dim):
        for j in range(dim):
            row = [Z] * dim
            row[i] = row[i] + 0.5 * B[j]
            row[j] = row[j] + 0.5 * B[i]
            rows.append(row)
    L = sps.bmat(rows, format="csr")
    E0 = _mech.macro_tensor(eps_mac, dim, grid) - _mech.eigen_tensor(e, dim, grid)
    K = (L.T @ C @ L).toarray()
    f = -(L.T @ (C @ E0.reshape(-1)))
    u = np.linalg.lstsq(K, f, rcond=1e-13)[0]
    eps = _mech.macro_tensor(eps_mac, dim, grid) + (L @ u).reshape((dim, dim) + grid)
    return dict(strain=_mat.to_voigt(eps))


def diffusion_static_direct_op(Dfield, grad_cmac, h, op):
    """diffusion_static_direct with the gradient operator `op` (least squares,
    so extra null modes of the operator do not matter)."""
    Dfield = np.asarray(Dfield, dtype=np.float64)
    grid = Dfield.shape
    dim = Dfield.ndim
    B = [diff_matrix(grid, a, h, op) for a in range(dim)]
    Dd = sps.diags(Dfield.ravel())
    K = sum((B[a].T @ Dd @ B[a]) for a in range(dim)).toarray()
    f = -sum(B[a].T @ (Dfield.ravel() * grad_cmac[a]) for a in range(dim))
    phi = np.linalg.lstsq(K, f, rcond=1e-13)[0]
    return np.array([grad_cmac[a] + (B[a] @ phi).reshape(grid) for a in range(dim)])
