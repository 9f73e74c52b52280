"""ctypes binding of the C ABI in ``include/pisoc.h`` (``libpisoc.so``).

Argument marshalling only: every step of the solver runs in the HIP kernels of
the library.  PyTorch provides device memory (the workspace and the field
buffers) and the HIP stream.  There is no CPU fallback: if the library is not
built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpisoc.so")

MAX_CLASSES = 8
MAX_CORR = 4

OK, WARN_NOT_CONVERGED, WARN_GUESS_FALLBACK, WARN_DUST = 0, 1, 2, 3
ERR_INVALID, ERR_HIP, ERR_DIVERGED, ERR_WORKSPACE = -1, -2, -3, -4
FP64, FP32_REFINED = 0, 1
GUESS_ZERO, GUESS_LEARNED, GUESS_PREVIOUS = 0, 1, 2
FLAG_PCG_MAXIT, FLAG_NONFINITE, FLAG_RHO_NONPOS, FLAG_GUESS_FALLBACK, FLAG_BAD_DT = 1, 2, 4, 8, 16
FLAG_GUESS_SKIPPED = 32
FLAG_DUST_NEG, FLAG_DUST_NONFINITE, FLAG_DUST_DIAG, FLAG_DUST_COURANT = 64, 128, 256, 512
FLAG_MOM_MAXIT = 1024

FIELD_RHO, FIELD_U, FIELD_PHI, FIELD_RHO_P, FIELD_P = 1, 2, 4, 8, 16
FIELD_PSOLVE_B, FIELD_PSOLVE_X, FIELD_P_PREV, FIELD_PSOLVE_DIAG = 32, 64, 128, 256
FIELD_USTAR, FIELD_GUESS, FIELD_GUESS_X0, FIELD_PSOLVE_W = 512, 1024, 2048, 4096
FIELD_PSOLVE_PSIDT, FIELD_T = 8192, 16384
BAROTROPIC, FOURIER = 0, 1
BDF1, BDF2 = 0, 1

EXPORTED = [
    "pisoc_workspace_bytes", "pisoc_init", "pisoc_step", "pisoc_fields", "pisoc_get_stats",
    "pisoc_time", "pisoc_steps_done", "pisoc_destroy", "pisoc_last_error", "pisoc_status_string",
    "pisoc_helm_apply", "pisoc_helm_workspace_bytes", "pisoc_helm_solve",
    "pisoc_helm_solve_precond", "pisoc_set_temperature",
    "pisoc_helm_solve_noalloc",
    "pisoc_profile", "pisoc_profile_read",
    "pisoc_net_workspace_bytes", "pisoc_net_forward", "pisoc_net_grad", "pisoc_net_adam",
    "pisoc_net_grad_residual",
    "pisoc_net_inputs",
    "pisoc_ens_workspace_bytes", "pisoc_ens_init", "pisoc_ens_step", "pisoc_ens_fields",
    "pisoc_ens_get_stats", "pisoc_ens_time", "pisoc_ens_steps_done", "pisoc_ens_num_classes",
    "pisoc_ens_class_info", "pisoc_ens_autotune", "pisoc_ens_destroy", "pisoc_ens_last_error",
    "pisoc_diag_spectrum_bins", "pisoc_diag_workspace_bytes", "pisoc_diag_spectrum",
    "pisoc_diag_qcrit", "pisoc_diag_sgs", "pisoc_stream_probe",
]
ENS_EAGER, ENS_GRAPH, ENS_GRAPH_ONE = 0, 1, 2
NET_NWEIGHTS = 15120
NET_CH = (2, 16, 16, 16, 1)

MAX_KSTATS = 24


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("n_classes", C.c_int32),
        ("gamma", C.c_double), ("C", C.c_double), ("mu", C.c_double),
        ("tau_p", C.c_double * MAX_CLASSES),
        ("cfl", C.c_double), ("dt_growth", C.c_double), ("dt_fixed", C.c_double),
        ("dt_max", C.c_double),
        ("n_corr", C.c_int32), ("n_mom_sweeps", C.c_int32), ("n_dust_sweeps", C.c_int32),
        ("p_tol", C.c_double), ("p_maxit", C.c_int32),
        ("precision", C.c_int32), ("guess", C.c_int32),
        ("d_guess_weights", C.c_void_p),
        ("inner_tol", C.c_double), ("max_refine", C.c_int32),
        ("capture", C.c_int32), ("guess_audit", C.c_int32),
        ("two_way", C.c_int32), ("gravity", C.c_double * 3),
        ("closure", C.c_int32), ("R_gas", C.c_double), ("cv", C.c_double),
        ("kappa", C.c_double), ("T0", C.c_double), ("time_scheme", C.c_int32),
        ("mom_tol", C.c_double), ("mom_maxit", C.c_int32),
    ]


class StepInfo(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("dt", C.c_double), ("courant", C.c_double),
        ("pcg_iters", C.c_int32 * MAX_CORR), ("pcg_relres", C.c_double * MAX_CORR),
        ("refinements", C.c_int32 * MAX_CORR),
        ("flags", C.c_int32), ("mass_gas", C.c_double),
        ("mass_p", C.c_double * MAX_CLASSES), ("courant_dust", C.c_double),
        ("mom_iters", C.c_int32), ("mom_relres", C.c_double),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("ke", C.c_double), ("enstrophy", C.c_double), ("rho_rms", C.c_double),
        ("mach_rms", C.c_double), ("mass_gas", C.c_double),
        ("conc_var", C.c_double * MAX_CLASSES), ("mass_p", C.c_double * MAX_CLASSES),
    ]


class EnsClass(C.Structure):
    _fields_ = [("n", C.c_int32), ("members", C.c_int32), ("block_x", C.c_int32),
                ("block_y", C.c_int32), ("cells_z", C.c_int32), ("blocks", C.c_int32),
                ("caps", C.c_int32 * MAX_CORR), ("cap_later", C.c_int32), ("rounds", C.c_int32),
                ("guess_mask", C.c_int32), ("cg_cells_z", C.c_int32), ("tiled_cells_z", C.c_int32)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double)]


_lib = None


def lib():
    """Load ``libpisoc.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1404_0959_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, f64, sz = C.c_void_p, C.c_int32, C.c_double, C.c_size_t
    L.pisoc_workspace_bytes.argtypes = [C.POINTER(Params)]
    L.pisoc_workspace_bytes.restype = sz
    L.pisoc_init.argtypes = [C.POINTER(Params), vp, sz, vp, vp, vp, vp, C.POINTER(vp)]
    L.pisoc_init.restype = C.c_int
    L.pisoc_step.argtypes = [vp, i32, C.POINTER(StepInfo)]
    L.pisoc_step.restype = C.c_int
    L.pisoc_fields.argtypes = [vp, C.c_uint32, C.POINTER(vp)]
    L.pisoc_fields.restype = C.c_int
    L.pisoc_get_stats.argtypes = [vp, C.POINTER(Stats)]
    L.pisoc_get_stats.restype = C.c_int
    L.pisoc_time.argtypes = [vp]
    L.pisoc_time.restype = f64
    L.pisoc_steps_done.argtypes = [vp]
    L.pisoc_steps_done.restype = C.c_int64
    L.pisoc_destroy.argtypes = [vp]
    L.pisoc_destroy.restype = None
    L.pisoc_last_error.argtypes = [vp]
    L.pisoc_last_error.restype = C.c_char_p
    L.pisoc_status_string.argtypes = [C.c_int]
    L.pisoc_status_string.restype = C.c_char_p
    L.pisoc_helm_apply.argtypes = [i32, vp, vp, vp, vp, vp]
    L.pisoc_helm_apply.restype = C.c_int
    L.pisoc_helm_workspace_bytes.argtypes = [i32]
    L.pisoc_helm_workspace_bytes.restype = sz
    L.pisoc_helm_solve.argtypes = [i32, vp, vp, vp, vp, f64, i32, vp, sz, vp,
                                   C.POINTER(i32), C.POINTER(f64)]
    L.pisoc_helm_solve.restype = C.c_int
    L.pisoc_helm_solve_precond.argtypes = [i32, vp, vp, vp, vp, f64, i32, i32, vp, sz, vp,
                                           C.POINTER(i32), C.POINTER(f64)]
    L.pisoc_helm_solve_precond.restype = C.c_int
    L.pisoc_set_temperature.argtypes = [vp, vp]
    L.pisoc_set_temperature.restype = C.c_int
    L.pisoc_helm_solve_noalloc.argtypes = [i32, vp, vp, vp, vp, f64, i32, vp,
                                           C.POINTER(i32), C.POINTER(f64)]
    L.pisoc_helm_solve_noalloc.restype = C.c_int
    L.pisoc_profile.argtypes = [vp, i32]
    L.pisoc_profile.restype = C.c_int
    L.pisoc_profile_read.argtypes = [vp, C.POINTER(KernelStat), i32]
    L.pisoc_profile_read.restype = i32
    fp = C.c_void_p
    L.pisoc_net_workspace_bytes.argtypes = [i32, i32]
    L.pisoc_net_workspace_bytes.restype = sz
    L.pisoc_net_forward.argtypes = [i32, i32, fp, fp, fp, vp, sz, vp]
    L.pisoc_net_forward.restype = C.c_int
    L.pisoc_net_grad.argtypes = [i32, i32, fp, fp, fp, fp, C.POINTER(f64), vp, sz, vp]
    L.pisoc_net_grad.restype = C.c_int
    L.pisoc_net_grad_residual.argtypes = [i32, i32, fp, fp, vp, vp, vp, fp, C.POINTER(f64), vp, sz,
                                          vp]
    L.pisoc_net_grad_residual.restype = C.c_int
    L.pisoc_net_adam.argtypes = [i32, fp, fp, fp, fp, i32, C.c_float, C.c_float, C.c_float,
                                 C.c_float, vp]
    L.pisoc_net_adam.restype = C.c_int
    L.pisoc_net_inputs.argtypes = [i32, vp, vp, vp, vp, fp, fp, C.POINTER(f64), vp, sz, vp]
    L.pisoc_net_inputs.restype = C.c_int
    pp = C.POINTER(vp)
    L.pisoc_ens_workspace_bytes.argtypes = [C.POINTER(Params), i32]
    L.pisoc_ens_workspace_bytes.restype = sz
    L.pisoc_ens_init.argtypes = [C.POINTER(Params), i32, vp, sz, pp, pp, pp, vp, C.POINTER(vp)]
    L.pisoc_ens_init.restype = C.c_int
    L.pisoc_ens_step.argtypes = [vp, i32, i32, C.POINTER(StepInfo)]
    L.pisoc_ens_step.restype = C.c_int
    L.pisoc_ens_fields.argtypes = [vp, i32, C.c_uint32, pp]
    L.pisoc_ens_fields.restype = C.c_int
    L.pisoc_ens_get_stats.argtypes = [vp, C.POINTER(Stats)]
    L.pisoc_ens_get_stats.restype = C.c_int
    L.pisoc_ens_time.argtypes = [vp, C.POINTER(f64)]
    L.pisoc_ens_time.restype = C.c_int
    L.pisoc_ens_steps_done.argtypes = [vp]
    L.pisoc_ens_steps_done.restype = C.c_int64
    L.pisoc_ens_num_classes.argtypes = [vp]
    L.pisoc_ens_num_classes.restype = i32
    L.pisoc_ens_class_info.argtypes = [vp, i32, C.POINTER(EnsClass)]
    L.pisoc_ens_class_info.restype = C.c_int
    L.pisoc_ens_autotune.argtypes = [vp, C.c_char_p, i32]
    L.pisoc_ens_autotune.restype = C.c_int
    L.pisoc_ens_destroy.argtypes = [vp]
    L.pisoc_ens_destroy.restype = None
    L.pisoc_ens_last_error.argtypes = [vp]
    L.pisoc_ens_last_error.restype = C.c_char_p
    L.pisoc_diag_spectrum_bins.argtypes = [i32]
    L.pisoc_diag_spectrum_bins.restype = i32
    L.pisoc_diag_workspace_bytes.argtypes = [i32]
    L.pisoc_diag_workspace_bytes.restype = sz
    L.pisoc_diag_spectrum.argtypes = [i32, vp, C.POINTER(f64), i32, C.POINTER(f64),
                                      C.POINTER(f64), vp, sz, vp]
    L.pisoc_diag_spectrum.restype = C.c_int
    L.pisoc_diag_qcrit.argtypes = [i32, vp, vp, C.POINTER(f64), vp, sz, vp]
    L.pisoc_diag_qcrit.restype = C.c_int
    L.pisoc_diag_sgs.argtypes = [i32, vp, C.POINTER(f64), vp, sz, vp]
    L.pisoc_diag_sgs.restype = C.c_int
    L.pisoc_stream_probe.argtypes = [i32, i32, C.c_int64, C.POINTER(vp), C.POINTER(vp), i32, vp]
    L.pisoc_stream_probe.restype = C.c_int
    _lib = L
    return L


class PisocError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"pisoc status {status}: {msg}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("pisoc needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream_ptr(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def make_params(n, *, gamma, C_, mu, tau_p=(), cfl=0.5, dt_growth=1.2, dt_fixed=0.0, dt_max=0.0,
                n_corr=2, n_mom_sweeps=4, n_dust_sweeps=4, p_tol=1e-8, p_maxit=500,
                precision=FP64, guess=GUESS_ZERO, guess_weights=None, inner_tol=1e-7,
                max_refine=20, capture=False, guess_audit=0, two_way=False,
                gravity=(0.0, 0.0, 0.0), fourier=None, bdf2=False, mom_tol=0.0,
                mom_maxit=200) -> Params:
    """fourier: None (barotropic) or dict(R=, cv=, kappa=, T0=) for the ideal gas
    with the energy equation; bdf2: the variable-step BDF2 time scheme."""
    p = Params()
    p.n = n
    p.n_classes = len(tau_p)
    p.gamma, p.C, p.mu = gamma, C_, mu
    for i, t in enumerate(tau_p):
        p.tau_p[i] = t
    p.cfl, p.dt_growth, p.dt_fixed, p.dt_max = cfl, dt_growth, dt_fixed, dt_max
    p.n_corr, p.n_mom_sweeps, p.n_dust_sweeps = n_corr, n_mom_sweeps, n_dust_sweeps
    p.p_tol, p.p_maxit = p_tol, p_maxit
    p.precision, p.guess = precision, guess
    p.d_guess_weights = guess_weights
    p.inner_tol, p.max_refine = inner_tol, max_refine
    p.capture = 1 if capture else 0
    p.guess_audit = guess_audit
    p.two_way = 1 if two_way else 0
    for d in range(3):
        p.gravity[d] = gravity[d]
    if fourier is not None:
        p.closure = FOURIER
        p.R_gas, p.cv, p.kappa, p.T0 = fourier["R"], fourier["cv"], fourier["kappa"], fourier["T0"]
    p.time_scheme = BDF2 if bdf2 else BDF1
    p.mom_tol, p.mom_maxit = mom_tol, mom_maxit
    return p


class Solver:
    """One simulation on one GPU, bound to a workspace tensor and a stream."""

    def __init__(self, n, rho, u, rho_p=None, *, device="cuda:0", stream=None, T=None, **kw):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.n = n
        self.prm = make_params(n, **kw)
        self.K = self.prm.n_classes
        L = lib()
        nbytes = L.pisoc_workspace_bytes(C.byref(self.prm))
        if nbytes == 0:
            raise PisocError(ERR_INVALID, "invalid parameters")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream
        dev = self.device
        rho_d = torch.as_tensor(rho, dtype=torch.float64, device=dev).contiguous()
        u_d = torch.as_tensor(u, dtype=torch.float64, device=dev).contiguous()
        if self.K:
            rp_d = torch.as_tensor(rho_p, dtype=torch.float64, device=dev).contiguous()
            rp_ptr = rp_d.data_ptr()
        else:
            rp_ptr = None
        N = n ** 3
        assert rho_d.numel() == N and u_d.numel() == 3 * N
        h = C.c_void_p()
        st = L.pisoc_init(C.byref(self.prm), self.ws.data_ptr(), nbytes, rho_d.data_ptr(),
                          u_d.data_ptr(), rp_ptr, _stream_ptr(torch, stream), C.byref(h))
        if st != OK:
            raise PisocError(st, "pisoc_init failed")
        self._h = h
        if T is not None:
            t_d = torch.as_tensor(T, dtype=torch.float64, device=dev).contiguous()
            st = L.pisoc_set_temperature(h, t_d.data_ptr())
            if st != OK:
                raise PisocError(st, self.last_error())

    @classmethod
    def from_case(cls, case, **kw):
        return cls(case.n, case.rho, case.u, case.rho_p, gamma=case.gamma, C_=case.C, mu=case.mu,
                   tau_p=case.tau_p, **kw)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.pisoc_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def last_error(self) -> str:
        return lib().pisoc_last_error(self._h).decode()

    def step(self, n_steps=1, raise_on_error=True):
        infos = (StepInfo * max(n_steps, 1))()
        before = lib().pisoc_steps_done(self._h)
        st = lib().pisoc_step(self._h, n_steps, infos)
        if st < 0 and raise_on_error:
            raise PisocError(st, self.last_error())
        nc = self.prm.n_corr
        done = n_steps if st >= 0 else lib().pisoc_steps_done(self._h) - before
        return st, [_info_dict(infos[i], nc, self.K) for i in range(done)]

    def fields(self, which):
        """Return {bit: float64 tensor} for the requested field bits."""
        torch = self.torch
        n = self.n
        shapes = {FIELD_RHO: (n, n, n), FIELD_U: (3, n, n, n), FIELD_PHI: (3, n, n, n),
                  FIELD_RHO_P: (max(self.K, 1), n, n, n), FIELD_P: (n, n, n),
                  FIELD_PSOLVE_B: (n, n, n), FIELD_PSOLVE_X: (n, n, n),
                  FIELD_P_PREV: (n, n, n), FIELD_PSOLVE_DIAG: (n, n, n),
                  FIELD_USTAR: (3, n, n, n), FIELD_GUESS: (n, n, n), FIELD_GUESS_X0: (n, n, n),
                  FIELD_PSOLVE_W: (n, n, n), FIELD_PSOLVE_PSIDT: (n, n, n),
                  FIELD_T: (n, n, n)}
        bits = [b for b in sorted(shapes) if which & b]
        outs = [torch.empty(shapes[b], dtype=torch.float64, device=self.device) for b in bits]
        arr = (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        st = lib().pisoc_fields(self._h, which, arr)
        if st != OK:
            raise PisocError(st, self.last_error())
        torch.cuda.current_stream().synchronize() if self.stream is None else self.stream.synchronize()
        res = dict(zip(bits, outs))
        if FIELD_RHO_P in res:
            res[FIELD_RHO_P] = res[FIELD_RHO_P][: self.K]
        return res

    def get(self, bit):
        return self.fields(bit)[bit]

    def stats(self):
        s = Stats()
        st = lib().pisoc_get_stats(self._h, C.byref(s))
        if st != OK:
            raise PisocError(st, self.last_error())
        K = self.K
        return dict(ke=s.ke, enstrophy=s.enstrophy, rho_rms=s.rho_rms, mach_rms=s.mach_rms,
                    mass_gas=s.mass_gas, conc_var=list(s.conc_var[:K]), mass_p=list(s.mass_p[:K]))

    @property
    def t(self):
        return lib().pisoc_time(self._h)

    def profile(self, enable=True):
        """Enable (and reset) or disable per-kernel event timing."""
        st = lib().pisoc_profile(self._h, 1 if enable else 0)
        if st != OK:
            raise PisocError(st, self.last_error())

    def profile_read(self):
        """{kernel name: dict(launches, ms, bytes)} of the counted launches."""
        arr = (KernelStat * MAX_KSTATS)()
        n = lib().pisoc_profile_read(self._h, arr, MAX_KSTATS)
        return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].ms,
                                           bytes=arr[i].bytes) for i in range(n)}


def _info_dict(r, nc, K):
    return dict(t=r.t, dt=r.dt, courant=r.courant, pcg_iters=list(r.pcg_iters[:nc]),
                pcg_relres=list(r.pcg_relres[:nc]), refinements=list(r.refinements[:nc]),
                flags=r.flags, mass_gas=r.mass_gas, mass_p=list(r.mass_p[:K]),
                courant_dust=r.courant_dust, mom_iters=r.mom_iters, mom_relres=r.mom_relres)


class Ensemble:
    """Independent members (mixed grid sizes) stepped together on one GPU.

    ``cases``: objects with n, rho, u, rho_p, gamma, C, mu, tau_p (as made by
    ``inputs.make_hit_case``); ``kw``: the parameters every member shares."""

    def __init__(self, cases, *, device="cuda:0", **kw):
        torch = _torch()
        self.torch, self.device = torch, torch.device(device)
        self.count = len(cases)
        prms = (Params * self.count)()
        keep = []
        for m, c in enumerate(cases):
            prms[m] = make_params(c.n, gamma=c.gamma, C_=c.C, mu=c.mu, tau_p=c.tau_p, **kw)
        self.prms = prms
        self.ns = [c.n for c in cases]
        self.K = prms[0].n_classes
        L = lib()
        nbytes = L.pisoc_ens_workspace_bytes(prms, self.count)
        if nbytes == 0:
            raise PisocError(ERR_INVALID, "invalid ensemble parameters")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        arrs = [[], [], []]
        for c in cases:
            r = torch.as_tensor(c.rho, dtype=torch.float64, device=self.device).contiguous()
            u = torch.as_tensor(c.u, dtype=torch.float64, device=self.device).contiguous()
            keep += [r, u]
            arrs[0].append(r.data_ptr())
            arrs[1].append(u.data_ptr())
            if self.K:
                rp = torch.as_tensor(c.rho_p, dtype=torch.float64, device=self.device).contiguous()
                keep.append(rp)
                arrs[2].append(rp.data_ptr())
            else:
                arrs[2].append(None)
        ptrs = [(C.c_void_p * self.count)(*a) for a in arrs]
        h = C.c_void_p()
        st = L.pisoc_ens_init(prms, self.count, self.ws.data_ptr(), nbytes, ptrs[0], ptrs[1],
                              ptrs[2] if self.K else None,
                              _stream_ptr(torch, None), C.byref(h))
        if st != OK:
            raise PisocError(st, "pisoc_ens_init failed")
        self._h = h
        del keep

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.pisoc_ens_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def last_error(self) -> str:
        return lib().pisoc_ens_last_error(self._h).decode()

    def step(self, n_steps=1, mode=ENS_GRAPH, raise_on_error=True):
        """Advance every member; returns (status, [last-step record per member])."""
        infos = (StepInfo * self.count)()
        st = lib().pisoc_ens_step(self._h, n_steps, mode, infos)
        if st < 0 and raise_on_error:
            raise PisocError(st, self.last_error())
        nc = self.prms[0].n_corr
        return st, [_info_dict(infos[m], nc, self.K) for m in range(self.count)]

    def autotune(self, cache_path=None, force=False):
        st = lib().pisoc_ens_autotune(self._h, cache_path.encode() if cache_path else None,
                                      1 if force else 0)
        if st != OK:
            raise PisocError(st, self.last_error())

    def classes(self):
        out = []
        for c in range(lib().pisoc_ens_num_classes(self._h)):
            e = EnsClass()
            st = lib().pisoc_ens_class_info(self._h, c, C.byref(e))
            if st != OK:
                raise PisocError(st, self.last_error())
            out.append(dict(n=e.n, members=e.members, block=(e.block_x, e.block_y),
                            cells_z=e.cells_z, blocks=e.blocks, caps=list(e.caps),
                            cap_later=e.cap_later, rounds=e.rounds, guess_mask=e.guess_mask,
                            cg_cells_z=e.cg_cells_z, tiled_cells_z=e.tiled_cells_z))
        return out

    def fields(self, m, which):
        torch = self.torch
        n = self.ns[m]
        shapes = {FIELD_RHO: (n, n, n), FIELD_U: (3, n, n, n), FIELD_PHI: (3, n, n, n),
                  FIELD_RHO_P: (max(self.K, 1), n, n, n), FIELD_P: (n, n, n),
                  FIELD_PSOLVE_B: (n, n, n), FIELD_PSOLVE_X: (n, n, n),
                  FIELD_P_PREV: (n, n, n), FIELD_PSOLVE_DIAG: (n, n, n),
                  FIELD_USTAR: (3, n, n, n), FIELD_GUESS: (n, n, n), FIELD_GUESS_X0: (n, n, n),
                  FIELD_PSOLVE_W: (n, n, n), FIELD_PSOLVE_PSIDT: (n, n, n),
                  FIELD_T: (n, n, n)}
        bits = [b for b in sorted(shapes) if which & b]
        outs = [torch.empty(shapes[b], dtype=torch.float64, device=self.device) for b in bits]
        arr = (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        st = lib().pisoc_ens_fields(self._h, m, which, arr)
        if st != OK:
            raise PisocError(st, self.last_error())
        torch.cuda.synchronize(self.device)
        res = dict(zip(bits, outs))
        if FIELD_RHO_P in res:
            res[FIELD_RHO_P] = res[FIELD_RHO_P][: self.K]
        return res

    def get(self, m, bit):
        return self.fields(m, bit)[bit]

    def stats(self):
        arr = (Stats * self.count)()
        st = lib().pisoc_ens_get_stats(self._h, arr)
        if st != OK:
            raise PisocError(st, self.last_error())
        K = self.K
        return [dict(ke=s.ke, enstrophy=s.enstrophy, rho_rms=s.rho_rms, mach_rms=s.mach_rms,
                     mass_gas=s.mass_gas, conc_var=list(s.conc_var[:K]), mass_p=list(s.mass_p[:K]))
                for s in arr]

    def times(self):
        arr = (C.c_double * self.count)()
        st = lib().pisoc_ens_time(self._h, arr)
        if st != OK:
            raise PisocError(st, self.last_error())
        return list(arr)

    @property
    def steps_done(self):
        return lib().pisoc_ens_steps_done(self._h)


class Net:
    """Workspace-bound access to the network kernels for grids of n^3, batch b."""

    def __init__(self, n, batch, device="cuda:0", stream=None):
        torch = _torch()
        self.torch, self.n, self.batch, self.stream = torch, n, batch, stream
        nbytes = lib().pisoc_net_workspace_bytes(n, batch)
        if nbytes == 0:
            raise PisocError(ERR_INVALID, "network needs n % 16 == 0")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes

    def forward(self, w, x):
        """x: FP32 [batch, n^3, 2] (device); returns FP32 [batch, n^3]."""
        torch = self.torch
        y = torch.empty(x.shape[0], self.n ** 3, dtype=torch.float32, device=x.device)
        st = lib().pisoc_net_forward(self.n, x.shape[0], w.data_ptr(), x.data_ptr(), y.data_ptr(),
                                     self.ws.data_ptr(), self.nbytes, _stream_ptr(torch, self.stream))
        if st != OK:
            raise PisocError(st, "pisoc_net_forward")
        return y

    def grad(self, w, x, t, out=None):
        """(loss, FP32 gradient) of the mean squared error."""
        torch = self.torch
        g = out if out is not None else torch.empty_like(w)
        loss = C.c_double(0.0)
        st = lib().pisoc_net_grad(self.n, x.shape[0], w.data_ptr(), x.data_ptr(), t.data_ptr(),
                                  g.data_ptr(), C.byref(loss), self.ws.data_ptr(), self.nbytes,
                                  _stream_ptr(torch, self.stream))
        if st != OK:
            raise PisocError(st, "pisoc_net_grad")
        return loss.value, g

    def grad_residual(self, w, x, b, diag, wk, out=None):
        """(loss, FP32 gradient) of the relative residual |b - alpha M g|^2/|b|^2
        the solve would start from (b, diag, wk: FP64 [batch, n^3] systems)."""
        torch = self.torch
        g = out if out is not None else torch.empty_like(w)
        loss = C.c_double(0.0)
        st = lib().pisoc_net_grad_residual(self.n, x.shape[0], w.data_ptr(), x.data_ptr(),
                                           b.data_ptr(), diag.data_ptr(), wk.data_ptr(),
                                           g.data_ptr(), C.byref(loss), self.ws.data_ptr(),
                                           self.nbytes, _stream_ptr(torch, self.stream))
        if st != OK:
            raise PisocError(st, "pisoc_net_grad_residual")
        return loss.value, g

    def adam(self, w, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        st = lib().pisoc_net_adam(w.numel(), w.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(),
                                  step, lr, beta1, beta2, eps, _stream_ptr(self.torch, self.stream))
        if st != OK:
            raise PisocError(st, "pisoc_net_adam")


def net_inputs(b, diag, p0, psol=None, stream=None):
    """Network inputs (FP32 [n^3, 2]), optional target (FP32 [n^3]) and (s1, s2)
    from one captured pressure system (FP64 device arrays)."""
    torch = _torch()
    n = b.shape[-1]
    x = torch.empty(n ** 3, 2, dtype=torch.float32, device=b.device)
    t = torch.empty(n ** 3, dtype=torch.float32, device=b.device) if psol is not None else None
    nbytes = lib().pisoc_helm_workspace_bytes(n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    sc = (C.c_double * 2)()
    st = lib().pisoc_net_inputs(n, b.data_ptr(), diag.data_ptr(), p0.data_ptr(),
                                psol.data_ptr() if psol is not None else None, x.data_ptr(),
                                t.data_ptr() if t is not None else None, sc, ws.data_ptr(), nbytes,
                                _stream_ptr(torch, stream))
    if st != OK:
        raise PisocError(st, "pisoc_net_inputs")
    return x, t, (sc[0], sc[1])


def helm_apply(psidt, w, x, stream=None):
    """y = M x with M the pressure operator (see pisoc.h).  Device FP64 tensors."""
    torch = _torch()
    n = x.shape[-1]
    y = torch.empty_like(x)
    st = lib().pisoc_helm_apply(n, psidt.data_ptr(), w.data_ptr(), x.data_ptr(), y.data_ptr(),
                                _stream_ptr(torch, stream))
    if st != OK:
        raise PisocError(st, "pisoc_helm_apply")
    return y


def helm_solve(psidt, w, b, x0=None, tol=1e-10, maxit=1000, stream=None, precond=None):
    """Preconditioned CG on M x = b (Jacobi, or PRECOND_CHEB); returns
    (x, iterations, relres, status)."""
    torch = _torch()
    n = b.shape[-1]
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    nbytes = lib().pisoc_helm_workspace_bytes(n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    it = C.c_int32(0)
    rel = C.c_double(0.0)
    if precond is None:
        st = lib().pisoc_helm_solve(n, psidt.data_ptr(), w.data_ptr(), b.data_ptr(), x.data_ptr(),
                                    tol, maxit, ws.data_ptr(), nbytes, _stream_ptr(torch, stream),
                                    C.byref(it), C.byref(rel))
    else:
        st = lib().pisoc_helm_solve_precond(n, psidt.data_ptr(), w.data_ptr(), b.data_ptr(),
                                            x.data_ptr(), tol, maxit, precond, ws.data_ptr(),
                                            nbytes, _stream_ptr(torch, stream), C.byref(it),
                                            C.byref(rel))
    if st < 0:
        raise PisocError(st, "pisoc_helm_solve")
    return x, it.value, rel.value, st


PRECOND_JACOBI, PRECOND_CHEB = 0, 1
HELM_NOALLOC_MAX_N = 64


def helm_solve_noalloc(psidt, w, b, x0=None, tol=1e-10, maxit=1000, stream=None):
    """As helm_solve, through the entry point that allocates nothing (its scratch
    is the library's own device array; grids up to HELM_NOALLOC_MAX_N).  The
    output x is allocated here by torch, as every output of this binding is;
    the library call itself allocates nothing."""
    torch = _torch()
    n = b.shape[-1]
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    it = C.c_int32(0)
    rel = C.c_double(0.0)
    st = lib().pisoc_helm_solve_noalloc(n, psidt.data_ptr(), w.data_ptr(), b.data_ptr(),
                                        x.data_ptr(), tol, maxit, _stream_ptr(torch, stream),
                                        C.byref(it), C.byref(rel))
    if st < 0:
        raise PisocError(st, "pisoc_helm_solve_noalloc")
    return x, it.value, rel.value, st


def spectrum(u, stream=None):
    """Energy spectrum of a velocity field u (FP64 device tensor [3, n, n, n]):
    (E per shell as a numpy array, Taylor micro-scale, D = sum |k|^2 |u_hat|^2 / 2)."""
    import numpy as np
    torch = _torch()
    n = u.shape[-1]
    bins = lib().pisoc_diag_spectrum_bins(n)
    if bins == 0:
        raise PisocError(ERR_INVALID, "spectrum needs n a power of two in 8..1024")
    nbytes = lib().pisoc_diag_workspace_bytes(n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=u.device)
    E = (C.c_double * bins)()
    lam, D = C.c_double(0.0), C.c_double(0.0)
    st = lib().pisoc_diag_spectrum(n, u.data_ptr(), E, bins, C.byref(lam), C.byref(D),
                                   ws.data_ptr(), nbytes, _stream_ptr(torch, stream))
    if st != OK:
        raise PisocError(st, "pisoc_diag_spectrum")
    return np.array(E[:]), lam.value, D.value


def qcriterion(u, stream=None):
    """Q of a velocity field u (FP64 device tensor [3, n, n, n]): (Q tensor, <Q>, <(div u)^2>)."""
    torch = _torch()
    n = u.shape[-1]
    nbytes = lib().pisoc_diag_workspace_bytes(n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=u.device)
    q = torch.empty(u.shape[1:], dtype=torch.float64, device=u.device)
    means = (C.c_double * 2)()
    st = lib().pisoc_diag_qcrit(n, u.data_ptr(), q.data_ptr(), means, ws.data_ptr(), nbytes,
                                _stream_ptr(torch, stream))
    if st != OK:
        raise PisocError(st, "pisoc_diag_qcrit")
    return q, means[0], means[1]


def sgs_stats(u, stream=None):
    """Filtered statistics of a velocity field u (FP64 device tensor [3, n, n, n]):
    (<|u_bar|^2>/2, <k_sgs>, <Pi>, fraction of cells with Pi < 0)."""
    torch = _torch()
    n = u.shape[-1]
    nbytes = lib().pisoc_diag_workspace_bytes(n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=u.device)
    out = (C.c_double * 4)()
    st = lib().pisoc_diag_sgs(n, u.data_ptr(), out, ws.data_ptr(), nbytes,
                              _stream_ptr(torch, stream))
    if st != OK:
        raise PisocError(st, "pisoc_diag_sgs")
    return tuple(out)


def stream_probe(ins, outs, blocks=0, stream=None):
    """One launch of the streaming probe: outs[w] = (w + 1) * sum(ins) over
    FP32 device tensors of one size (the HBM ceiling of that read/write mix)."""
    torch = _torch()
    count = ins[0].numel()
    if any(t.dtype != torch.float32 or t.numel() != count or not t.is_contiguous()
           for t in list(ins) + list(outs)):
        raise PisocError(ERR_INVALID, "stream_probe: contiguous FP32 tensors of one size")
    pin = (C.c_void_p * len(ins))(*[t.data_ptr() for t in ins])
    pout = (C.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    st = lib().pisoc_stream_probe(len(ins), len(outs), count, pin, pout, blocks,
                                  _stream_ptr(torch, stream))
    if st != OK:
        raise PisocError(st, "pisoc_stream_probe")
