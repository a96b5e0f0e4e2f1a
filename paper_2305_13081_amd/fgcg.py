"""Thin Python binding of the fgcg C ABI (include/fgcg.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libfgcg.so``.  PyTorch provides device memory and the current stream.  The
binding checks shapes, dtypes, devices and contiguity of every tensor before
handing raw pointers to the library, and raises ``FgcgError`` for any status
other than OK (NOT_CONVERGED is reported in the returned info instead).  If
the library is missing, every call raises: there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfgcg.so")

FGCG_OK, FGCG_NOT_CONVERGED = 0, 1
FGCG_EINVAL, FGCG_EDOMAIN, FGCG_EBREAKDOWN, FGCG_ENOMEM, FGCG_EHIP, FGCG_EUNSUPPORTED = -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED = 0, 1
J_USER, J_ENERGY, J_C11 = 0, 1, 2
OP_MECH_K, OP_MECH_M = 0, 1
MAX_PHASES = 8
KINDS = {
    "mech_row_fwd": 0, "mech_col": 1, "mech_row_inv": 2,
    "pf_row_fwd": 3, "pf_col": 4, "pf_row_inv": 5,
    "diff_row_fwd": 6, "diff_col_grad": 7, "diff_row_mid": 8, "diff_col_div": 9, "diff_row_inv": 10,
    "mech_kp": 11, "mech_y_fwd": 12, "mech_y_inv": 13, "event_gap": 14,
}


class FgcgError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("precision", ctypes.c_int)]


class Material(ctypes.Structure):
    _fields_ = [("phase", ctypes.c_void_p), ("nphase", ctypes.c_int), ("E_tab", ctypes.POINTER(ctypes.c_double)),
                ("nu_tab", ctypes.POINTER(ctypes.c_double)), ("E_field", ctypes.c_void_p),
                ("nu_field", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return dict(iters=self.iters, status=self.status, rel_res=self.rel_res, bnorm=self.bnorm,
                    seconds=self.seconds)


class State(ctypes.Structure):
    _fields_ = [("c", ctypes.c_void_p), ("f", ctypes.c_void_p), ("e", ctypes.c_void_p), ("H", ctypes.c_void_p),
                ("d", ctypes.c_void_p), ("strain", ctypes.c_void_p), ("step", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("mat", Material), ("D_tab", ctypes.POINTER(ctypes.c_double)),
                ("k_tab", ctypes.POINTER(ctypes.c_double)), ("band_width", ctypes.c_int), ("c_dir", ctypes.c_double),
                ("dt", ctypes.c_double), ("e_per_f", ctypes.c_double), ("Gc", ctypes.c_double),
                ("l0", ctypes.c_double), ("kappa", ctypes.c_double), ("eps_mac", ctypes.c_double * 6),
                ("tol_diff", ctypes.c_double), ("tol_mech", ctypes.c_double), ("tol_pf", ctypes.c_double),
                ("maxit", ctypes.c_int), ("diffuse", ctypes.c_int), ("e_ramp", ctypes.c_double),
                ("n_ramp", ctypes.c_int)]


class StepInfo(ctypes.Structure):
    _fields_ = [("diff", Info), ("mech", Info), ("pf", Info), ("mean_stress", ctypes.c_double * 6),
                ("energy", ctypes.c_double), ("max_d", ctypes.c_double), ("damaged_fraction", ctypes.c_double),
                ("porosity_increase", ctypes.c_double), ("total_precipitate", ctypes.c_double)]

    def as_dict(self):
        return dict(diff=self.diff.as_dict(), mech=self.mech.as_dict(), pf=self.pf.as_dict(),
                    mean_stress=list(self.mean_stress), energy=self.energy, max_d=self.max_d,
                    damaged_fraction=self.damaged_fraction, porosity_increase=self.porosity_increase,
                    total_precipitate=self.total_precipitate)


class MsParams(ctypes.Structure):
    _fields_ = [("ncell", ctypes.c_int), ("length", ctypes.c_double), ("dt", ctypes.c_double),
                ("J_in", ctypes.c_double), ("solubility", ctypes.c_double), ("molar_volume", ctypes.c_double),
                ("Gc", ctypes.c_double), ("l0", ctypes.c_double), ("kappa", ctypes.c_double), ("tol", ctypes.c_double),
                ("tol_homog", ctypes.c_double), ("maxit", ctypes.c_int)]


class MsInfo(ctypes.Structure):
    _fields_ = [("c_mac", ctypes.c_double), ("grad_mac", ctypes.c_double), ("mean_cppt", ctypes.c_double),
                ("max_e", ctypes.c_double), ("max_d", ctypes.c_double), ("mean_stress", ctypes.c_double * 6),
                ("energy", ctypes.c_double), ("mech", Info), ("pf", Info)]

    def as_dict(self, ns):
        return dict(c_mac=self.c_mac, grad_mac=self.grad_mac, mean_cppt=self.mean_cppt, max_e=self.max_e,
                    max_d=self.max_d, mean_stress=list(self.mean_stress)[:ns], energy=self.energy,
                    mech=self.mech.as_dict(), pf=self.pf.as_dict())


_lib = None
_vp, _dp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
_SIGS = {
    "fgcg_create": (_ip, [ctypes.POINTER(Grid), _vp, ctypes.POINTER(_vp)]),
    "fgcg_destroy": (None, [_vp]),
    "fgcg_set_stream": (_ip, [_vp, _vp]),
    "fgcg_strerror": (ctypes.c_char_p, [_ip]),
    "fgcg_last_error": (ctypes.c_char_p, []),
    "fgcg_set_option": (_ip, [_vp, _ip, _ip]),
    "fgcg_get_option": (_ip, [_vp, _ip, ctypes.POINTER(ctypes.c_int)]),
    "fgcg_set_reference": (_ip, [_vp, ctypes.c_double, ctypes.c_double]),
    "fgcg_mech_solve": (_ip, [_vp, ctypes.POINTER(Material), _vp, ctypes.c_double, _vp, _dp, ctypes.c_double, _ip,
                              _vp, _vp, _dp, _dp, ctypes.POINTER(Info)]),
    "fgcg_mech_adjoint": (_ip, [_vp, ctypes.POINTER(Material), _vp, ctypes.c_double, _vp, _dp, _vp, _ip,
                                ctypes.c_double, _ip, _vp, _dp, ctypes.POINTER(Info), ctypes.POINTER(Info)]),
    "fgcg_batch_create": (_ip, [_ip, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.c_double, _ip,
                                _vp, ctypes.POINTER(_vp)]),
    "fgcg_batch_destroy": (None, [_vp]),
    "fgcg_mech_solve_batched": (_ip, [_vp, ctypes.POINTER(_vp), _ip, _dp, _dp, _dp, ctypes.c_double, _ip,
                                      ctypes.POINTER(_vp), _dp, _dp, ctypes.POINTER(Info)]),
    "fgcg_phasefield_solve": (_ip, [_vp, _vp, ctypes.c_double, ctypes.c_double, _vp, ctypes.c_double, _ip,
                                    ctypes.POINTER(Info)]),
    "fgcg_diffusion_step": (_ip, [_vp, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _ip,
                                  ctypes.POINTER(Info)]),
    "fgcg_diffusion_step_phases": (_ip, [_vp, _vp, _ip, _dp, _dp, _ip, ctypes.c_double, ctypes.c_double, _vp,
                                         ctypes.c_double, _ip, ctypes.POINTER(Info)]),
    "fgcg_diffusion_homogenize": (_ip, [_vp, _vp, _dp, ctypes.c_double, _ip, _vp, _vp, _dp, ctypes.POINTER(Info)]),
    "fgcg_diffusivity_eff": (_ip, [_vp, _vp, ctypes.c_double, _ip, _dp, ctypes.POINTER(Info)]),
    "fgcg_concentration": (_ip, [_vp, _vp, _vp, _dp, ctypes.c_double, _vp, _dp]),
    "fgcg_staggered_step": (_ip, [_vp, ctypes.POINTER(State), ctypes.POINTER(Params), ctypes.POINTER(StepInfo)]),
    "fgcg_debug_apply": (_ip, [_vp, _ip, ctypes.POINTER(Material), _vp, ctypes.c_double, _vp, _vp]),
    "fgcg_phasefield_apply": (_ip, [_vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "fgcg_diffusion_apply": (_ip, [_vp, _vp, _ip, _dp, _dp, ctypes.c_double, _vp, _vp]),
    "fgcg_phasefield_solve_noalloc": (_ip, [ctypes.POINTER(Grid), _vp, _vp, ctypes.c_double, ctypes.c_double, _vp,
                                            ctypes.c_double, _ip, ctypes.POINTER(Info)]),
    "fgcg_debug_fft": (_ip, [_vp, _ip, _vp, _vp]),
    "fgcg_time_pass": (_ip, [_vp, _ip, _ip, _dp]),
    "fgcg_profile": (_ip, [_vp, ctypes.c_uint]),
    "fgcg_profile_read": (_ip, [_vp, _ip, _dp, ctypes.POINTER(ctypes.c_longlong)]),
    "fgcg_kernel_name": (ctypes.c_char_p, [_vp, _ip]),
    "fgcg_ms_create": (_ip, [_vp, ctypes.POINTER(Material), _vp, ctypes.POINTER(MsParams), _ip,
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_vp)]),
    "fgcg_ms_step": (_ip, [_vp, ctypes.POINTER(MsInfo)]),
    "fgcg_ms_read": (_ip, [_vp, _dp, _dp, _dp, _dp]),
    "fgcg_ms_volume": (_ip, [_vp, _ip, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fgcg_ms_destroy": (None, [_vp]),
}
EXPORTS = tuple(_SIGS)


def load_library(path=LIB_PATH):
    """Load libfgcg.so and declare every exported signature (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FgcgError(-5, "load", f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, where, allow_nc=False):
    if status == FGCG_OK or (allow_nc and status == FGCG_NOT_CONVERGED):
        return status
    lib = load_library()
    raise FgcgError(status, where, lib.fgcg_strerror(status).decode() + ": " + lib.fgcg_last_error().decode())


def _dvec(vals):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


def _torch():
    import torch
    return torch


class Context:
    """One fgcg context (workspace for one grid).  Fields are torch CUDA
    tensors shaped (ny, nx) or (nz, ny, nx) (scalars), or with a leading
    component axis.  nz given: a 3D grid (strain/stress with 6 components)."""

    def __init__(self, nx, ny, h, precision=FP64, device=None, nz=None):
        torch = _torch()
        self.lib = load_library()
        self.nx, self.ny, self.h = int(nx), int(ny), float(h)
        self.nz = None if nz is None else int(nz)
        self.ndim = 2 if nz is None else 3
        self.shape = (self.ny, self.nx) if nz is None else (self.nz, self.ny, self.nx)
        self.ns = 3 if nz is None else 6
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        g = Grid(self.ndim, (ctypes.c_int * 3)(self.nx, self.ny, 1 if nz is None else self.nz), self.h,
                 int(precision))
        out = _vp()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
        _check(self.lib.fgcg_create(ctypes.byref(g), _vp(stream), ctypes.byref(out)), "fgcg_create")
        self.ptr = out

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.fgcg_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    OPTIONS = {"scalar_spectral": 0, "graphs": 1, "chunk": 2, "rows": 3, "row_plan": 4, "col_plan": 5, "precond": 6,
               "gradient": 7, "strain_form": 8, "spectral_residual": 9, "mech_passes": 10, "scalar_cg": 11,
               "row_split": 12, "ztiles": 13, "mech_form": 14}
    GRADIENTS = {"forward": 0, "central": 1, "central8": 2, "fourier": 3}

    def set_option(self, name, value):
        _check(self.lib.fgcg_set_option(self.ptr, self.OPTIONS[name], int(value)), "fgcg_set_option")

    def set_reference(self, lam0=0.0, mu0=0.0):
        """Reference medium of the "precond" = 1 option ((0, 0): automatic)."""
        _check(self.lib.fgcg_set_reference(self.ptr, float(lam0), float(mu0)), "fgcg_set_reference")

    def get_option(self, name):
        v = ctypes.c_int()
        _check(self.lib.fgcg_get_option(self.ptr, self.OPTIONS[name], ctypes.byref(v)), "fgcg_get_option")
        return v.value

    # ----------------------------------------------------------- helpers
    def _sync_stream(self):
        torch = _torch()
        _check(self.lib.fgcg_set_stream(self.ptr, _vp(torch.cuda.current_stream(self.device).cuda_stream)),
               "fgcg_set_stream")

    def _t(self, t, name, dtype, comps=None, allow_none=False):
        torch = _torch()
        if t is None:
            if allow_none:
                return None
            raise FgcgError(-1, name, "required tensor is None")
        shape = self.shape if comps is None else (comps,) + self.shape
        if not isinstance(t, torch.Tensor):
            raise FgcgError(-1, name, "expected a torch tensor")
        if t.device != self.device:
            raise FgcgError(-1, name, f"tensor on {t.device}, context on {self.device}")
        if t.dtype != dtype:
            raise FgcgError(-1, name, f"dtype {t.dtype}, expected {dtype}")
        if tuple(t.shape) != shape:
            raise FgcgError(-1, name, f"shape {tuple(t.shape)}, expected {shape}")
        if not t.is_contiguous():
            raise FgcgError(-1, name, "tensor must be contiguous")
        return t

    def _ptr(self, t):
        return None if t is None else _vp(t.data_ptr())

    def _material(self, phase, E_tab, nu_tab, E_field=None, nu_field=0.2):
        torch = _torch()
        keep = []
        if E_field is not None:
            self._t(E_field, "E_field", torch.float64)
            m = Material(None, 0, None, None, _vp(E_field.data_ptr()), float(nu_field))
        else:
            self._t(phase, "phase", torch.uint8)
            E_tab = list(E_tab)
            nu_tab = list(nu_tab)
            if not (1 <= len(E_tab) <= MAX_PHASES and len(E_tab) == len(nu_tab)):
                raise FgcgError(-1, "material", "E_tab/nu_tab must have equal length 1..8")
            Ea, na = _dvec(E_tab), _dvec(nu_tab)
            keep = [Ea, na]
            m = Material(_vp(phase.data_ptr()), len(E_tab), Ea, na, None, 0.0)
        return m, keep

    # ---------------------------------------------------------- entries
    def mech_solve(self, phase, E_tab, nu_tab, eps_mac, d=None, kappa=0.0, eig=None, tol=1e-10, maxit=20000,
                   want_stress=True, E_field=None, nu_field=0.2, strain=None, stress=None):
        torch = _torch()
        m, keep = self._material(phase, E_tab, nu_tab, E_field, nu_field)
        self._t(d, "d", torch.float64, allow_none=True)
        self._t(eig, "eig", torch.float64, allow_none=True)
        ns = self.ns
        if len(eps_mac) != ns:
            raise FgcgError(-1, "mech_solve", f"eps_mac needs {ns} Voigt components")
        if strain is None:
            strain = torch.empty((ns,) + self.shape, dtype=torch.float64, device=self.device)
        self._t(strain, "strain", torch.float64, comps=ns)
        if want_stress and stress is None:
            stress = torch.empty((ns,) + self.shape, dtype=torch.float64, device=self.device)
        self._t(stress, "stress", torch.float64, comps=ns, allow_none=True)
        em = _dvec(eps_mac)
        mean = (ctypes.c_double * ns)()
        energy = ctypes.c_double()
        info = Info()
        self._sync_stream()
        st = self.lib.fgcg_mech_solve(self.ptr, ctypes.byref(m), self._ptr(d), float(kappa), self._ptr(eig), em,
                                      float(tol), int(maxit), self._ptr(strain), self._ptr(stress), mean,
                                      ctypes.byref(energy), ctypes.byref(info))
        _check(st, "fgcg_mech_solve", allow_nc=True)
        del keep
        return dict(strain=strain, stress=stress, mean_stress=np.array(list(mean)), energy=energy.value,
                    info=info.as_dict())

    def mech_adjoint(self, E_field, nu, eps_mac, objective=J_ENERGY, dJ_dstrain=None, d=None, kappa=0.0,
                     eig=None, tol=1e-12, maxit=50000, phase=None, E_tab=None, nu_tab=None, want_grad=True):
        """dJ/dE per voxel.  With E_field given the material is (E_field, nu);
        otherwise (phase, E_tab, nu_tab).  Returns (grad_E, J, info_fwd,
        info_adj); want_grad=False runs the forward solve only (grad_E None)."""
        torch = _torch()
        m, keep = self._material(phase, E_tab, nu_tab, E_field, nu)
        self._t(d, "d", torch.float64, allow_none=True)
        self._t(eig, "eig", torch.float64, allow_none=True)
        self._t(dJ_dstrain, "dJ_dstrain", torch.float64, comps=3, allow_none=True)
        grad = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) if want_grad else None
        J = ctypes.c_double(0.0)
        i1, i2 = Info(), Info()
        self._sync_stream()
        st = self.lib.fgcg_mech_adjoint(self.ptr, ctypes.byref(m), self._ptr(d), float(kappa), self._ptr(eig),
                                        _dvec(eps_mac), self._ptr(dJ_dstrain), int(objective), float(tol),
                                        int(maxit), self._ptr(grad), ctypes.byref(J), ctypes.byref(i1),
                                        ctypes.byref(i2))
        _check(st, "fgcg_mech_adjoint", allow_nc=True)
        del keep
        return grad, J.value, i1.as_dict(), i2.as_dict()

    def phasefield_solve(self, H, Gc, l0, d, tol=1e-10, maxit=20000):
        torch = _torch()
        self._t(H, "H", torch.float64)
        self._t(d, "d", torch.float64)
        info = Info()
        self._sync_stream()
        st = self.lib.fgcg_phasefield_solve(self.ptr, self._ptr(H), float(Gc), float(l0), self._ptr(d), float(tol),
                                            int(maxit), ctypes.byref(info))
        _check(st, "fgcg_phasefield_solve", allow_nc=True)
        return info.as_dict()

    def diffusion_step(self, c, Dfield, dt, krate=None, mask=None, c_dir=0.0, tol=1e-10, maxit=20000):
        """One implicit step with per-voxel D (float64), optional rate field
        (float64) and Dirichlet mask (uint8, nonzero = fixed at c_dir)."""
        torch = _torch()
        self._t(c, "c", torch.float64)
        self._t(Dfield, "Dfield", torch.float64)
        self._t(krate, "krate", torch.float64, allow_none=True)
        self._t(mask, "mask", torch.uint8, allow_none=True)
        info = Info()
        self._sync_stream()
        st = self.lib.fgcg_diffusion_step(self.ptr, self._ptr(c), self._ptr(Dfield), self._ptr(krate), self._ptr(mask),
                                          float(c_dir), float(dt), float(tol), int(maxit), ctypes.byref(info))
        _check(st, "fgcg_diffusion_step", allow_nc=True)
        return info.as_dict()

    def diffusion_step_phases(self, phase, D_tab, k_tab, band_width, c_dir, dt, c, tol=1e-10, maxit=20000):
        torch = _torch()
        self._t(phase, "phase", torch.uint8)
        self._t(c, "c", torch.float64)
        if len(D_tab) != len(k_tab) or not 1 <= len(D_tab) <= MAX_PHASES:
            raise FgcgError(-1, "diffusion_step_phases", "D_tab/k_tab must have equal length 1..8")
        info = Info()
        self._sync_stream()
        st = self.lib.fgcg_diffusion_step_phases(self.ptr, self._ptr(phase), len(D_tab), _dvec(D_tab), _dvec(k_tab),
                                                 int(band_width), float(c_dir), float(dt), self._ptr(c), float(tol),
                                                 int(maxit), ctypes.byref(info))
        _check(st, "fgcg_diffusion_step_phases", allow_nc=True)
        return info.as_dict()

    def diffusion_homogenize(self, Dfield, grad_cmac, tol=1e-10, maxit=20000, want_fields=True):
        """Static homogenisation: returns grad_c (dim, *grid), phi, the mean
        flux and the CG info."""
        torch = _torch()
        self._t(Dfield, "Dfield", torch.float64)
        dim = self.ndim
        if len(grad_cmac) != dim:
            raise FgcgError(-1, "diffusion_homogenize", f"grad_cmac needs {dim} components")
        gc = torch.empty((dim,) + self.shape, dtype=torch.float64, device=self.device) if want_fields else None
        phi = torch.empty(self.shape, dtype=torch.float64, device=self.device) if want_fields else None
        mf = (ctypes.c_double * dim)()
        info = Info()
        self._sync_stream()
        st = self.lib.fgcg_diffusion_homogenize(self.ptr, self._ptr(Dfield), _dvec(grad_cmac), float(tol), int(maxit),
                                                self._ptr(gc), self._ptr(phi), mf, ctypes.byref(info))
        _check(st, "fgcg_diffusion_homogenize", allow_nc=True)
        return dict(grad_c=gc, phi=phi, mean_flux=np.array(list(mf)), info=info.as_dict())

    def diffusivity_eff(self, Dfield, tol=1e-10, maxit=20000):
        torch = _torch()
        self._t(Dfield, "Dfield", torch.float64)
        dim = self.ndim
        D = (ctypes.c_double * (dim * dim))()
        infos = (Info * dim)()
        self._sync_stream()
        st = self.lib.fgcg_diffusivity_eff(self.ptr, self._ptr(Dfield), float(tol), int(maxit), D, infos)
        _check(st, "fgcg_diffusivity_eff", allow_nc=True)
        return np.array(list(D)).reshape(dim, dim), [i.as_dict() for i in infos]

    def concentration(self, phase, grad_c, grad_cmac, c_mac):
        """c(x) from a concentration-gradient field (eq. concentration-correct);
        returns (c, beta_pore, beta_solid)."""
        torch = _torch()
        self._t(phase, "phase", torch.uint8)
        self._t(grad_c, "grad_c", torch.float64, comps=self.ndim)
        c = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        beta = (ctypes.c_double * 2)()
        self._sync_stream()
        _check(self.lib.fgcg_concentration(self.ptr, self._ptr(phase), self._ptr(grad_c), _dvec(grad_cmac),
                                           float(c_mac), self._ptr(c), beta), "fgcg_concentration")
        return c, beta[0], beta[1]

    def new_state(self, band_width=0, c_dir=1.0):
        torch = _torch()
        z = lambda *s: torch.zeros(s, dtype=torch.float64, device=self.device)
        st = dict(c=z(*self.shape), f=z(*self.shape), e=z(*self.shape), H=z(*self.shape), d=z(*self.shape),
                  strain=z(self.ns, *self.shape), step=0)
        if band_width > 0:
            st["c"][..., :band_width] = c_dir
        return st

    def staggered_step(self, state, phase, prm):
        """prm: dict with the fields of fgcg_params (see oracle.staggered.Params)."""
        torch = _torch()
        for k in ("c", "f", "e", "H", "d"):
            self._t(state[k], k, torch.float64)
        self._t(state["strain"], "strain", torch.float64, comps=self.ns)
        m, keep = self._material(phase, prm["E_tab"], prm["nu_tab"])
        Dt, kt = _dvec(prm["D_tab"]), _dvec(prm["k_tab"])
        if len(prm["D_tab"]) != m.nphase or len(prm["k_tab"]) != m.nphase:
            raise FgcgError(-1, "staggered_step", "D_tab/k_tab length must equal nphase")
        p = Params(m, Dt, kt, int(prm["band_width"]), float(prm["c_dir"]), float(prm["dt"]), float(prm["e_per_f"]),
                   float(prm["Gc"]), float(prm["l0"]), float(prm["kappa"]),
                   (ctypes.c_double * 6)(*(list(prm["eps_mac"]) + [0.0] * (6 - len(prm["eps_mac"])))),
                   float(prm["tol_diff"]), float(prm["tol_mech"]), float(prm["tol_pf"]), int(prm["maxit"]),
                   int(prm["diffuse"]), float(prm.get("e_ramp", 0.0)), int(prm.get("n_ramp", 0)))
        s = State(*[_vp(state[k].data_ptr()) for k in ("c", "f", "e", "H", "d", "strain")], int(state["step"]))
        info = StepInfo()
        self._sync_stream()
        st = self.lib.fgcg_staggered_step(self.ptr, ctypes.byref(s), ctypes.byref(p), ctypes.byref(info))
        _check(st, "fgcg_staggered_step", allow_nc=True)
        state["step"] = s.step
        del keep
        out = info.as_dict()
        out["mean_stress"] = out["mean_stress"][:self.ns]
        return out

    # ------------------------------------------------------- test hooks
    def debug_fft(self, x, inverse=False):
        """Real-input transform of one field through the solver passes:
        forward (nz, ny, nx) float64 -> (nz, ny, nx//2+1) complex128 half
        spectrum (no nz axis in 2D); inverse maps it back with 1/N."""
        torch = _torch()
        half = self.shape[:-1] + (self.nx // 2 + 1,)
        if not inverse:
            self._t(x, "x", torch.float64)
            out = torch.empty(half, dtype=torch.complex128, device=self.device)
        else:
            if not (isinstance(x, torch.Tensor) and x.dtype == torch.complex128 and tuple(x.shape) == half
                    and x.device == self.device and x.is_contiguous()):
                raise FgcgError(-1, "debug_fft", f"expected a contiguous complex128 tensor of shape {half}")
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._sync_stream()
        _check(self.lib.fgcg_debug_fft(self.ptr, -1 if inverse else 1, self._ptr(x), self._ptr(out)),
               "fgcg_debug_fft")
        return out
    def debug_apply(self, op, phase, E_tab, nu_tab, v, d=None, kappa=0.0, E_field=None, nu_field=0.2):
        """One application of the solver's K (op OP_MECH_K) or M (OP_MECH_M)
        to a displacement-like float64 field v of shape (n_u, *grid)."""
        torch = _torch()
        m, keep = self._material(phase, E_tab, nu_tab, E_field, nu_field)
        nu = self.ndim
        self._t(v, "v", torch.float64, comps=nu)
        self._t(d, "d", torch.float64, allow_none=True)
        q = torch.empty_like(v)
        self._sync_stream()
        _check(self.lib.fgcg_debug_apply(self.ptr, int(op), ctypes.byref(m), self._ptr(d), float(kappa), self._ptr(v),
                                         self._ptr(q)), "fgcg_debug_apply")
        del keep
        return q

    def phasefield_apply(self, H, Gc, l0, v):
        torch = _torch()
        self._t(H, "H", torch.float64)
        self._t(v, "v", torch.float64)
        q = torch.empty_like(v)
        self._sync_stream()
        _check(self.lib.fgcg_phasefield_apply(self.ptr, self._ptr(H), float(Gc), float(l0), self._ptr(v),
                                              self._ptr(q)), "fgcg_phasefield_apply")
        return q

    def diffusion_apply(self, phase, D_tab, k_tab, dt, v):
        torch = _torch()
        self._t(phase, "phase", torch.uint8)
        self._t(v, "v", torch.float64)
        q = torch.empty_like(v)
        self._sync_stream()
        _check(self.lib.fgcg_diffusion_apply(self.ptr, self._ptr(phase), len(D_tab), _dvec(D_tab), _dvec(k_tab),
                                             float(dt), self._ptr(v), self._ptr(q)), "fgcg_diffusion_apply")
        return q

    # --------------------------------------------------------- profiling
    def profile(self, kinds):
        mask = 0
        for k in kinds:
            mask |= 1 << KINDS[k]
        _check(self.lib.fgcg_profile(self.ptr, mask), "fgcg_profile")

    def time_pass(self, kind, reps=200):
        """Average microseconds of one back-to-back launch of a 2D mechanics
        pass ("mech_row_fwd", "mech_row_inv", "mech_col"); clears the
        workspace (fgcg_time_pass)."""
        us = ctypes.c_double()
        self._sync_stream()
        _check(self.lib.fgcg_time_pass(self.ptr, KINDS[kind], int(reps), ctypes.byref(us)), "fgcg_time_pass")
        return us.value

    def profile_read(self, kind):
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        _check(self.lib.fgcg_profile_read(self.ptr, KINDS[kind], ctypes.byref(ms), ctypes.byref(n)),
               "fgcg_profile_read")
        name = self.lib.fgcg_kernel_name(self.ptr, KINDS[kind]).decode()
        return ms.value, n.value, name


def phasefield_solve_noalloc(H, Gc, l0, d, h, tol=1e-10, maxit=20000):
    """fgcg_phasefield_solve_noalloc: the phase-field solve without a context
    or any allocation; H and d are float64 CUDA tensors of the grid's shape
    ((ny, nx) or (nz, ny, nx)), d is updated in place."""
    torch = _torch()
    lib = load_library()
    for t, name in ((H, "H"), (d, "d")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise FgcgError(-1, name, "expected a contiguous float64 CUDA tensor")
    if tuple(H.shape) != tuple(d.shape) or H.device != d.device or H.dim() not in (2, 3):
        raise FgcgError(-1, "phasefield_solve_noalloc", "H and d need the same 2D or 3D shape and device")
    sh = tuple(d.shape)
    n = (sh[-1], sh[-2], sh[0] if len(sh) == 3 else 1)
    g = Grid(len(sh), (ctypes.c_int * 3)(*n), float(h), FP64)
    info = Info()
    with torch.cuda.device(d.device):
        stream = torch.cuda.current_stream().cuda_stream
        st = lib.fgcg_phasefield_solve_noalloc(ctypes.byref(g), _vp(stream), _vp(H.data_ptr()), float(Gc), float(l0),
                                               _vp(d.data_ptr()), float(tol), int(maxit), ctypes.byref(info))
    _check(st, "fgcg_phasefield_solve_noalloc", allow_nc=True)
    return info.as_dict()


class Batch:
    """Many 2D microstructures of uneven sizes solved together
    (fgcg_batch_create / fgcg_mech_solve_batched)."""

    def __init__(self, sizes, h, precision=FP64, device=None):
        torch = _torch()
        self.lib = load_library()
        self.sizes = [(int(nx), int(ny)) for nx, ny in sizes]
        self.nb = len(self.sizes)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        nx = (ctypes.c_int * self.nb)(*[s[0] for s in self.sizes])
        ny = (ctypes.c_int * self.nb)(*[s[1] for s in self.sizes])
        out = _vp()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
        _check(self.lib.fgcg_batch_create(self.nb, nx, ny, float(h), int(precision), _vp(stream), ctypes.byref(out)),
               "fgcg_batch_create")
        self.ptr = out

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.fgcg_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mech_solve(self, phases, E_tab, nu_tab, eps_mac, tol=1e-10, maxit=50000, want_strain=True):
        torch = _torch()
        if len(phases) != self.nb or len(eps_mac) != self.nb:
            raise FgcgError(-1, "Batch.mech_solve", "need one phase field and one macro strain per sample")
        for (nx, ny), ph in zip(self.sizes, phases):
            if not (isinstance(ph, torch.Tensor) and ph.dtype == torch.uint8 and ph.device == self.device
                    and tuple(ph.shape) == (ny, nx) and ph.is_contiguous()):
                raise FgcgError(-1, "Batch.mech_solve", f"phase must be a contiguous uint8 ({ny}, {nx}) tensor")
        # one table for every sample, or one row per sample
        per = isinstance(E_tab[0], (list, tuple, np.ndarray))
        Et = [list(r) for r in E_tab] if per else [list(E_tab)] * self.nb
        Nt = [list(r) for r in nu_tab] if per else [list(nu_tab)] * self.nb
        if len(Et) != self.nb or len(Nt) != self.nb:
            raise FgcgError(-1, "Batch.mech_solve", "per-sample tables need one row per sample")
        nph = len(Et[0])
        if not (1 <= nph <= MAX_PHASES and all(len(r) == nph for r in Et + Nt)):
            raise FgcgError(-1, "Batch.mech_solve", "E_tab/nu_tab rows must have equal length 1..8")
        strains = [torch.empty((3, ny, nx), dtype=torch.float64, device=self.device) for nx, ny in self.sizes] \
            if want_strain else None
        ph = (_vp * self.nb)(*[p.data_ptr() for p in phases])
        sp = (_vp * self.nb)(*[t.data_ptr() for t in strains]) if strains else None
        em = _dvec([v for e in eps_mac for v in e])
        mean = (ctypes.c_double * (3 * self.nb))()
        en = (ctypes.c_double * self.nb)()
        infos = (Info * self.nb)()
        st = self.lib.fgcg_mech_solve_batched(self.ptr, ph, nph, _dvec([v for r in Et for v in r]),
                                              _dvec([v for r in Nt for v in r]), em, float(tol), int(maxit), sp, mean,
                                              en, infos)
        _check(st, "fgcg_mech_solve_batched", allow_nc=True)
        return dict(strains=strains, mean_stress=np.array(list(mean)).reshape(self.nb, 3),
                    energy=np.array(list(en)), infos=[i.as_dict() for i in infos])


class Multiscale:
    """The multiscale coupling of Sec. 3.2 (fgcg_ms_*): a bar of prm["ncell"]
    cells carrying copies of the context's volume in the cells `cells`.
    prm: the fields of fgcg_ms_params (oracle.multiscale's BarParams and
    RveParams hold the same names).  The context must outlive the object."""

    FIELDS = ("c", "cppt", "e", "H", "d", "strain")

    def __init__(self, ctx, phase, E_tab, nu_tab, D_field, prm, cells):
        torch = _torch()
        self.ctx, self.lib = ctx, ctx.lib
        ctx._t(D_field, "D_field", torch.float64)
        m, keep = ctx._material(phase, E_tab, nu_tab)
        self._phase = phase  # the library keeps the phase by pointer
        self.ncell, self.nrve = int(prm["ncell"]), len(cells)
        p = MsParams(self.ncell, float(prm["length"]), float(prm["dt"]), float(prm["J_in"]),
                     float(prm["solubility"]), float(prm["molar_volume"]), float(prm["Gc"]), float(prm["l0"]),
                     float(prm.get("kappa", 0.0)), float(prm.get("tol", 1e-10)), float(prm.get("tol_homog", 1e-12)),
                     int(prm.get("maxit", 20000)))
        cl = (ctypes.c_int * max(1, self.nrve))(*[int(c) for c in cells])
        out = _vp()
        ctx._sync_stream()
        _check(self.lib.fgcg_ms_create(ctx.ptr, ctypes.byref(m), ctx._ptr(D_field), ctypes.byref(p), self.nrve, cl,
                                       ctypes.byref(out)), "fgcg_ms_create")
        self.ptr = out

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.fgcg_ms_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        infos = (MsInfo * max(1, self.nrve))()
        self.ctx._sync_stream()
        _check(self.lib.fgcg_ms_step(self.ptr, infos), "fgcg_ms_step", allow_nc=True)
        return [infos[i].as_dict(self.ctx.ns) for i in range(self.nrve)]

    def bar(self):
        dim = self.ctx.ndim
        c = (ctypes.c_double * self.ncell)()
        g = (ctypes.c_double * self.ncell)()
        D = (ctypes.c_double * (dim * dim))()
        t = ctypes.c_double()
        _check(self.lib.fgcg_ms_read(self.ptr, c, g, D, ctypes.byref(t)), "fgcg_ms_read")
        return dict(c=np.array(list(c)), grad=np.array(list(g)), D_eff=np.array(list(D)).reshape(dim, dim),
                    time=t.value)

    def volume(self, rve):
        """The state of volume rve after the last step: a dict of float64
        CUDA tensors (strain with a leading component axis)."""
        torch = _torch()
        ctx = self.ctx
        f = {k: torch.empty(((ctx.ns,) if k == "strain" else ()) + ctx.shape, dtype=torch.float64,
                            device=ctx.device) for k in self.FIELDS}
        ctx._sync_stream()
        _check(self.lib.fgcg_ms_volume(self.ptr, int(rve), *[ctx._ptr(f[k]) for k in self.FIELDS]),
               "fgcg_ms_volume")
        return f
