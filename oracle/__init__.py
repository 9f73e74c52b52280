"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The oracle (``oracle.c``) is a plain, slow FP64 implementation of
one barotropic PISO step with Equilibrium-Eulerian dust, written from the
method's equations; it shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "conv.c"),
           os.path.join(HERE, "guess.c")]

MAX_CLASSES = 8
MAX_CORR = 8

OK, WARN_NOT_CONVERGED, WARN_DUST, ERR_INVALID, ERR_DIVERGED = 0, 1, 3, -1, -3
FLAG_PCG_MAXIT, FLAG_NONFINITE, FLAG_RHO_NONPOS, FLAG_KFACE_NONPOS = 1, 2, 4, 8
FLAG_DUST_NEG, FLAG_DUST_NONFINITE, FLAG_DUST_DIAG, FLAG_DUST_COURANT = 64, 128, 256, 512
DUST_COURANT_MAX = 0.638
FLAG_MOM_MAXIT = 1024

RHO, U, PHI, RHO_P, P, T = 0, 1, 2, 3, 4, 5
BAROTROPIC, FOURIER = 0, 1
SYS_B, SYS_W, SYS_PSIDT, SYS_K, SYS_X, SYS_P0, SYS_DIAG, SYS_USTAR = 10, 11, 12, 13, 14, 15, 16, 17

STAT_KE, STAT_ENSTROPHY, STAT_RHO_RMS, STAT_MACH_RMS, STAT_MASS_GAS = 0, 1, 2, 3, 4
STAT_CONC_VAR = 5
STAT_MASS_P = 5 + MAX_CLASSES
N_STATS = 5 + 2 * MAX_CLASSES


class OraParams(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("n_classes", C.c_int32),
        ("gamma", C.c_double), ("C", C.c_double), ("mu", C.c_double),
        ("tau_p", C.c_double * MAX_CLASSES),
        ("cfl", C.c_double), ("dt_growth", C.c_double), ("dt_fixed", C.c_double),
        ("dt_max", C.c_double),
        ("n_corr", C.c_int32), ("n_mom_sweeps", C.c_int32), ("n_dust_sweeps", C.c_int32),
        ("p_tol", C.c_double), ("p_maxit", C.c_int32),
        ("two_way", C.c_int32), ("gravity", C.c_double * 3),
        ("closure", C.c_int32), ("R_gas", C.c_double), ("cv", C.c_double),
        ("kappa", C.c_double), ("T0", C.c_double), ("time_scheme", C.c_int32),
        ("mom_tol", C.c_double), ("mom_maxit", C.c_int32),
    ]


class OraInfo(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("dt", C.c_double), ("courant", C.c_double),
        ("pcg_iters", C.c_int32 * MAX_CORR), ("pcg_relres", C.c_double * MAX_CORR),
        ("flags", C.c_int32), ("mass_gas", C.c_double),
        ("mass_p", C.c_double * MAX_CLASSES), ("courant_dust", C.c_double),
        ("mom_iters", C.c_int32), ("mom_relres", C.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP) into ``liboracle.so``."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    srcs = [s for s in SOURCES if os.path.exists(s)]
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.ora_create.argtypes = [C.POINTER(OraParams), dp, dp, dp, C.POINTER(C.c_void_p)]
        L.ora_create.restype = C.c_int
        L.ora_step.argtypes = [C.c_void_p, C.c_int32, C.POINTER(OraInfo)]
        L.ora_step.restype = C.c_int
        L.ora_get.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp]
        L.ora_get.restype = C.c_int
        L.ora_stats.argtypes = [C.c_void_p, dp]
        L.ora_stats.restype = C.c_int
        L.ora_time.argtypes = [C.c_void_p]
        L.ora_time.restype = C.c_double
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_destroy.restype = None
        L.ora_set_capture.argtypes = [C.c_void_p, C.c_int32]
        L.ora_set_capture.restype = None
        L.ora_set_temperature.argtypes = [C.c_void_p, dp]
        L.ora_set_temperature.restype = C.c_int
        L.ora_num_threads.argtypes = []
        L.ora_num_threads.restype = C.c_int
        L.ora_i4.argtypes = [C.c_int32, C.c_int32, dp, dp]
        L.ora_sngrad.argtypes = [C.c_int32, C.c_int32, dp, dp]
        L.ora_div_flux.argtypes = [C.c_int32, dp, dp, dp, dp]
        L.ora_grad.argtypes = [C.c_int32, dp, dp, dp, dp]
        L.ora_div_vel.argtypes = [C.c_int32, dp, dp, dp, dp]
        L.ora_lap.argtypes = [C.c_int32, dp, dp]
        L.ora_kfaces.argtypes = [C.c_int32, dp, dp, dp, dp]
        L.ora_helm_apply.argtypes = [C.c_int32, dp, dp, dp, dp, dp, dp]
        L.ora_pcg.argtypes = [C.c_int32, dp, dp, dp, dp, dp, dp, C.c_double, C.c_int32, dp]
        L.ora_pcg.restype = C.c_int32
        L.ora_pcg_cheb.argtypes = [C.c_int32, dp, dp, dp, dp, dp, dp, C.c_double, C.c_int32, dp]
        L.ora_pcg_cheb.restype = C.c_int32
        L.ora_cheb_coef.argtypes = [C.c_int32, dp, dp, dp, dp, dp]
        L.ora_cheb_coef.restype = None
        L.ora_cheb_apply.argtypes = [C.c_int32, dp, dp, dp, dp, dp, dp]
        L.ora_cheb_apply.restype = None
        if hasattr(L, "ora_conv_forward"):
            _bind_conv(L)
        L.ora_net_inputs.argtypes = [C.c_int32, dp, dp, dp, dp, dp]
        L.ora_net_inputs.restype = C.c_int
        L.ora_guess_start.argtypes = [C.c_int32, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.ora_guess_start.restype = C.c_int
        _lib = L
    return _lib


def _bind_conv(L):
    dp = C.POINTER(C.c_double)
    L.ora_conv_forward.argtypes = [C.c_int32, C.c_int32, dp, dp, dp]
    L.ora_conv_forward.restype = C.c_int
    L.ora_conv_backward.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, dp]
    L.ora_conv_backward.restype = C.c_int
    L.ora_conv_backward_dy.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp]
    L.ora_conv_backward_dy.restype = C.c_int
    L.ora_conv_nweights.argtypes = []
    L.ora_conv_nweights.restype = C.c_int32


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().ora_num_threads())


# ---------------------------------------------------------------- operators
def i4(q, d):
    q = _f64(q); out = np.empty_like(q)
    lib().ora_i4(q.shape[0], d, _p(q), _p(out)); return out


def sngrad(q, d):
    q = _f64(q); out = np.empty_like(q)
    lib().ora_sngrad(q.shape[0], d, _p(q), _p(out)); return out


def div_flux(f):
    f = [_f64(x) for x in f]; out = np.empty_like(f[0])
    lib().ora_div_flux(f[0].shape[0], _p(f[0]), _p(f[1]), _p(f[2]), _p(out)); return out


def grad(q):
    q = _f64(q); g = [np.empty_like(q) for _ in range(3)]
    lib().ora_grad(q.shape[0], _p(q), _p(g[0]), _p(g[1]), _p(g[2])); return g


def div_vel(u):
    u = [_f64(x) for x in u]; out = np.empty_like(u[0])
    lib().ora_div_vel(u[0].shape[0], _p(u[0]), _p(u[1]), _p(u[2]), _p(out)); return out


def lap(q):
    q = _f64(q); out = np.empty_like(q)
    lib().ora_lap(q.shape[0], _p(q), _p(out)); return out


def kfaces(w):
    w = _f64(w); k = [np.empty_like(w) for _ in range(3)]
    lib().ora_kfaces(w.shape[0], _p(w), _p(k[0]), _p(k[1]), _p(k[2])); return k


def helm_apply(psidt, K, x):
    psidt = _f64(psidt); K = [_f64(k) for k in K]; x = _f64(x); y = np.empty_like(x)
    lib().ora_helm_apply(x.shape[0], _p(psidt), _p(K[0]), _p(K[1]), _p(K[2]), _p(x), _p(y))
    return y


def pcg(psidt, K, b, x0=None, tol=1e-10, maxit=1000):
    """Jacobi-PCG; returns (x, iterations, relres); iterations < 0 means not converged."""
    psidt = _f64(psidt); K = [_f64(k) for k in K]; b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    rel = C.c_double(0.0)
    it = lib().ora_pcg(b.shape[0], _p(psidt), _p(K[0]), _p(K[1]), _p(K[2]), _p(b), _p(x),
                       tol, maxit, C.byref(rel))
    return x, int(it), rel.value


def pcg_cheb(psidt, K, b, x0=None, tol=1e-10, maxit=1000):
    """CG preconditioned by the degree-1 Chebyshev polynomial of the
    Jacobi-scaled operator; returns (x, iterations, relres) as pcg."""
    psidt = _f64(psidt); K = [_f64(k) for k in K]; b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    rel = C.c_double(0.0)
    it = lib().ora_pcg_cheb(b.shape[0], _p(psidt), _p(K[0]), _p(K[1]), _p(K[2]), _p(b), _p(x),
                            tol, maxit, C.byref(rel))
    return x, int(it), rel.value


def cheb_coef(psidt, K):
    """(c0, c1, a) of the Chebyshev preconditioner p(lambda) = c0 + c1 lambda on
    [a, 2 - a]."""
    psidt = _f64(psidt); K = [_f64(k) for k in K]
    c = np.empty(3)
    lib().ora_cheb_coef(psidt.shape[0], _p(psidt), _p(K[0]), _p(K[1]), _p(K[2]), _p(c))
    return float(c[0]), float(c[1]), float(c[2])


def cheb_apply(psidt, K, r):
    """z = p(D^-1 M) D^-1 r."""
    psidt = _f64(psidt); K = [_f64(k) for k in K]; r = _f64(r)
    z = np.empty_like(r)
    lib().ora_cheb_apply(r.shape[0], _p(psidt), _p(K[0]), _p(K[1]), _p(K[2]), _p(r), _p(z))
    return z


# ---------------------------------------------------------------- learned guess
def net_inputs(b, diag, p0):
    """Network inputs [n^3][2] ((b/diag)/s1, (p0 - <p0>)/s2) and (s1, s2)."""
    b = _f64(b); diag = _f64(diag); p0 = _f64(p0)
    n = b.shape[0]
    x = np.empty((n ** 3, 2))
    sc = np.empty(2)
    st = lib().ora_net_inputs(n, _p(b), _p(diag), _p(p0), _p(x), _p(sc))
    if st != OK:
        raise ValueError(f"ora_net_inputs failed with status {st}")
    return x, (float(sc[0]), float(sc[1]))


def guess_start(psidt, K, b, g):
    """Solve start from the guess g: (x0, alpha, ||b - alpha M g|| / ||b||, fell_back)."""
    psidt = _f64(psidt); K = [_f64(k) for k in K]; b = _f64(b); g = _f64(g)
    x0 = np.empty_like(b)
    a = C.c_double(0.0)
    rr = C.c_double(0.0)
    st = lib().ora_guess_start(b.shape[0], _p(psidt), _p(K[0]), _p(K[1]), _p(K[2]), _p(b), _p(g),
                               _p(x0), C.byref(a), C.byref(rr))
    if st < 0:
        raise ValueError(f"ora_guess_start failed with status {st}")
    return x0, a.value, rr.value, bool(st)


# ---------------------------------------------------------------- diagnostics
# The paper's validation quantities of the flow (Results section: the energy
# spectrum, the enstrophy and kinetic energy, the Taylor micro-scale; third
# figure: iso-surfaces of the second invariant Q).  Their discrete readings:
#  * spectrum: u_hat(k) = DFT(u)(k) / n^3 over integer wavevectors k with
#    components in [-n/2, n/2); shell s holds the k with s - 1/2 <= |k| < s + 1/2;
#    E(s) = sum over the shell of |u_hat(k)|^2 / 2, so that sum_s E(s) = <|u|^2>/2
#    (Parseval);
#  * Taylor micro-scale: lambda = sqrt(5 sum_k |u_hat|^2/2 / sum_k |k|^2 |u_hat|^2/2)
#    (the isotropic relation lambda^2 = 15 nu u'^2 / eps with u'^2 = (2/3) int E
#    and eps = 2 nu int k^2 E), with |k|^2 of each wavevector, not of its shell;
#  * Q = (|Omega|^2 - |S|^2)/2 = -(1/2) sum_ij (d_j u_i)(d_i u_j) per cell, with
#    the Gauss-I4 cell derivatives of the enstrophy statistic;
#  * filtered (a-priori sub-grid) statistics, the DNS data base's second use
#    named in the Results section: the separable top-hat of width 2h with
#    weights (1/4, 1/2, 1/4), the sub-grid stress tau_ij = bar(u_i u_j) -
#    u_bar_i u_bar_j, its energy k_sgs = tau_ii/2 and the energy flux
#    Pi = -tau_ij S_bar_ij to the sub-grid scales.


def spectrum_bins(n):
    """Number of shells of an n^3 grid: shell(3 (n/2)^2) + 1."""
    return shell_index(3 * (n // 2) ** 2) + 1


def shell_index(k2):
    """s with s - 1/2 <= sqrt(k2) < s + 1/2 for an integer k2 >= 0 (integer arithmetic)."""
    k2 = np.asarray(k2, dtype=np.int64)
    s = np.floor(np.sqrt(k2.astype(np.float64))).astype(np.int64)
    s = np.where(s * s > k2, s - 1, s)
    s = np.where((s + 1) * (s + 1) <= k2, s + 1, s)
    return s + (k2 >= s * s + s + 1)


def spectrum(u):
    """(E[shell], lambda, D) of a velocity field u [3][n][n][n]; D = sum_k |k|^2 |u_hat|^2 / 2."""
    u = _f64(u)
    n = u.shape[-1]
    N = n ** 3
    k1 = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    e = np.zeros((n, n, n))
    for d in range(3):
        uh = np.fft.fftn(u[d]) / N
        e += 0.5 * (uh.real ** 2 + uh.imag ** 2)
    sh = shell_index(k2)
    E = np.bincount(sh.ravel(), weights=e.ravel(), minlength=spectrum_bins(n))
    D = float(np.sum(k2 * e))
    tot = float(np.sum(e))
    lam = math.sqrt(5.0 * tot / D) if D > 0 else 0.0
    return E, lam, D


def qcriterion(u):
    """Q [n][n][n] of a velocity field u [3][n][n][n] (Gauss-I4 derivatives)."""
    u = _f64(u)
    G = [grad(u[i]) for i in range(3)]          # G[i][j] = d_j u_i
    Q = np.zeros_like(u[0])
    for i in range(3):
        for j in range(3):
            Q -= 0.5 * G[i][j] * G[j][i]
    return Q


def box_filter(q):
    """Separable discrete top-hat of width 2h: weights (1/4, 1/2, 1/4) along each
    axis (transfer function prod_d (1 + cos k_d h) / 2), periodic."""
    q = _f64(q)
    out = q
    for ax in (0, 1, 2):
        out = 0.25 * np.roll(out, 1, axis=ax) + 0.5 * out + 0.25 * np.roll(out, -1, axis=ax)
    return out


def sgs_stats(u):
    """A-priori statistics of the filter box_filter applied to u [3][n][n][n]:
    (<|u_bar|^2>/2, <k_sgs>, <Pi>, fraction of cells with Pi < 0), where
    tau_ij = bar(u_i u_j) - u_bar_i u_bar_j, k_sgs = tau_ii / 2,
    S_bar_ij = (d_j u_bar_i + d_i u_bar_j) / 2 (Gauss-I4) and Pi = -tau_ij S_bar_ij.
    Also returns the per-cell k_sgs and Pi fields."""
    u = _f64(u)
    ub = [box_filter(u[i]) for i in range(3)]
    G = [grad(ub[i]) for i in range(3)]          # G[i][j] = d_j ubar_i
    ksgs = np.zeros_like(u[0])
    Pi = np.zeros_like(u[0])
    for i in range(3):
        for j in range(3):
            tau = box_filter(u[i] * u[j]) - ub[i] * ub[j]
            if i == j:
                ksgs += 0.5 * tau
            Pi -= tau * 0.5 * (G[i][j] + G[j][i])
    res = float(np.mean(0.5 * (ub[0] ** 2 + ub[1] ** 2 + ub[2] ** 2)))
    return (res, float(np.mean(ksgs)), float(np.mean(Pi)), float(np.mean(Pi < 0.0))), ksgs, Pi


# ---------------------------------------------------------------- conv net
NET_CH = (2, 16, 16, 16, 1)


def conv_nweights():
    return int(lib().ora_conv_nweights())


def conv_layer_slices():
    """Slices of each layer's [co][ci][27] block in the flat weight vector."""
    out, off = [], 0
    for l in range(4):
        m = NET_CH[l] * NET_CH[l + 1] * 27
        out.append(slice(off, off + m))
        off += m
    return out


def conv_forward(w, x):
    """x: [batch][n^3][2] (or [batch,n,n,n,2]); returns y [batch][n,n,n]."""
    w = _f64(w); x = _f64(x)
    batch = x.shape[0]
    n = round((x.size // (2 * batch)) ** (1 / 3))
    y = np.empty((batch, n, n, n))
    lib().ora_conv_forward(n, batch, _p(w), _p(x), _p(y))
    return y


def conv_backward(w, x, t):
    """Loss (mean squared error) and its gradient with respect to the weights."""
    w = _f64(w); x = _f64(x); t = _f64(t)
    batch = x.shape[0]
    n = round((x.size // (2 * batch)) ** (1 / 3))
    g = np.empty_like(w)
    loss = C.c_double(0.0)
    lib().ora_conv_backward(n, batch, _p(w), _p(x), _p(t), _p(g), C.byref(loss))
    return loss.value, g


def conv_backward_dy(w, x, dy):
    """Weight gradient of sum dy * net(x) (dy: [batch][n^3] output gradient)."""
    w = _f64(w); x = _f64(x); dy = _f64(dy)
    batch = x.shape[0]
    n = round((x.size // (2 * batch)) ** (1 / 3))
    g = np.empty_like(w)
    lib().ora_conv_backward_dy(n, batch, _p(w), _p(x), _p(dy), _p(g))
    return g


def residual_loss(psidt, K, b, g):
    """The relative residual a solve started from the guess g begins with, and
    its gradient with respect to g: u = M g, alpha = g.b / g.u (the start
    rescale of the learned guess), r = b - alpha u, L = |r|^2 / |b|^2.
    Differentiating alpha (d alpha = (b - 2 alpha u).dg / g.u, M symmetric):
    dL/dg = -(2/|b|^2) [ (u.r / g.u) (b - 2 alpha u) + alpha M r ]."""
    b = _f64(b); g = _f64(g)
    u = helm_apply(psidt, K, g)
    gu = float(np.sum(g * u))
    alpha = float(np.sum(g * b)) / gu
    r = b - alpha * u
    bb = float(np.sum(b * b))
    loss = float(np.sum(r * r)) / bb
    grad = -(2.0 / bb) * (float(np.sum(u * r)) / gu * (b - 2.0 * alpha * u)
                          + alpha * helm_apply(psidt, K, r))
    return loss, grad


# ---------------------------------------------------------------- whole step
class Oracle:
    """One oracle simulation state (host memory, FP64)."""

    def __init__(self, n, rho, u, rho_p=None, *, gamma=1.4, C_=None, mu=1e-3, tau_p=(),
                 cfl=0.5, dt_growth=1.2, dt_fixed=0.0, dt_max=0.0, n_corr=2, n_mom_sweeps=4,
                 n_dust_sweeps=4, p_tol=1e-8, p_maxit=500, capture=False, two_way=False,
                 gravity=(0.0, 0.0, 0.0), fourier=None, T=None, bdf2=False, mom_tol=0.0,
                 mom_maxit=200):
        """fourier: None (barotropic) or dict(R=, cv=, kappa=, T0=) for the ideal
        gas with the energy equation; T: its initial temperature field."""
        if C_ is None:
            raise ValueError("closure constant C_ is required")
        tau_p = tuple(tau_p)
        prm = OraParams()
        prm.n = n
        prm.n_classes = len(tau_p)
        prm.gamma, prm.C, prm.mu = gamma, C_, mu
        for i, t in enumerate(tau_p):
            prm.tau_p[i] = t
        prm.cfl, prm.dt_growth, prm.dt_fixed, prm.dt_max = cfl, dt_growth, dt_fixed, dt_max
        prm.n_corr, prm.n_mom_sweeps, prm.n_dust_sweeps = n_corr, n_mom_sweeps, n_dust_sweeps
        prm.p_tol, prm.p_maxit = p_tol, p_maxit
        prm.two_way = 1 if two_way else 0
        for d in range(3):
            prm.gravity[d] = gravity[d]
        prm.time_scheme = 1 if bdf2 else 0
        prm.mom_tol, prm.mom_maxit = mom_tol, mom_maxit
        if fourier is not None:
            prm.closure = FOURIER
            prm.R_gas, prm.cv, prm.kappa, prm.T0 = (fourier["R"], fourier["cv"], fourier["kappa"],
                                                     fourier["T0"])
        self.prm = prm
        self.n = n
        self.K = len(tau_p)
        rho = _f64(rho).reshape(n, n, n)
        u = _f64(u).reshape(3, n, n, n)
        rp = _f64(rho_p).reshape(self.K, n, n, n) if self.K else np.zeros(1)
        h = C.c_void_p()
        st = lib().ora_create(C.byref(prm), _p(rho), _p(u), _p(rp), C.byref(h))
        if st != OK:
            raise ValueError(f"ora_create failed with status {st}")
        self._h = h
        if capture:
            lib().ora_set_capture(h, 1)
        if T is not None:
            if lib().ora_set_temperature(h, _p(_f64(T).reshape(n, n, n))) != OK:
                raise ValueError("ora_set_temperature needs the Fourier closure")

    @classmethod
    def from_case(cls, case, **kw):
        return cls(case.n, case.rho, case.u, case.rho_p, gamma=case.gamma, C_=case.C, mu=case.mu,
                   tau_p=case.tau_p, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ora_destroy(h)
            self._h = None

    def step(self, n_steps=1):
        """Advance n_steps; returns (status, list of info dicts)."""
        infos = (OraInfo * max(n_steps, 1))()
        st = lib().ora_step(self._h, n_steps, infos)
        out = []
        for i in range(n_steps):
            r = infos[i]
            out.append(dict(t=r.t, dt=r.dt, courant=r.courant,
                            pcg_iters=list(r.pcg_iters[: self.prm.n_corr]),
                            pcg_relres=list(r.pcg_relres[: self.prm.n_corr]),
                            flags=r.flags, mass_gas=r.mass_gas,
                            mass_p=list(r.mass_p[: self.K]), courant_dust=r.courant_dust,
                            mom_iters=r.mom_iters, mom_relres=r.mom_relres))
        return st, out

    def get(self, which, corr=0):
        n = self.n
        count = {RHO: 1, U: 3, PHI: 3, RHO_P: max(self.K, 1), P: 1, SYS_K: 3,
                 SYS_USTAR: 3}.get(which, 1)
        out = np.empty((count, n, n, n))
        st = lib().ora_get(self._h, which, corr, _p(out))
        if st != OK:
            raise ValueError(f"ora_get({which}) failed with status {st}")
        if which == RHO_P:
            return out[: self.K]
        return out[0] if count == 1 else out

    def stats(self):
        out = np.zeros(N_STATS)
        lib().ora_stats(self._h, _p(out))
        K = self.K
        return dict(ke=out[STAT_KE], enstrophy=out[STAT_ENSTROPHY], rho_rms=out[STAT_RHO_RMS],
                    mach_rms=out[STAT_MACH_RMS], mass_gas=out[STAT_MASS_GAS],
                    conc_var=list(out[STAT_CONC_VAR:STAT_CONC_VAR + K]),
                    mass_p=list(out[STAT_MASS_P:STAT_MASS_P + K]))

    @property
    def t(self):
        return lib().ora_time(self._h)
