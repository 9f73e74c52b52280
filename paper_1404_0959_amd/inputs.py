"""Seeded synthetic inputs for the decaying homogeneous isotropic turbulence runs.

The paper simulates freely decaying, subsonic homogeneous isotropic turbulence
(r.m.s. Mach 0.2 or 0.5) of a gas carrying dust (Introduction; Fig. 1 caption).
It does not print its initial condition, so the fields here are a seeded
stand-in with the structure of such a workload: a solenoidal random-phase
velocity with a prescribed energy spectrum, uniform density and a uniform dust
mass fraction per particle class.

This module is shared input plumbing.  It holds none of the solver's
arithmetic (no finite-volume operator, no time step, no pressure solve) and
imports neither the solver library nor the oracle.

Layout of every returned field: a C-ordered ``(n, n, n)`` float64 array indexed
``[k, j, i]`` (x fastest), i.e. cell ``(i, j, k)`` sits at linear offset
``i + n*(j + n*k)``.  The domain is the periodic cube ``[0, 2*pi)^3``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def spectrum_k4(k: np.ndarray, k0: float = 4.0) -> np.ndarray:
    """Energy spectrum E(k) = k^4 exp(-2 (k/k0)^2) (unnormalised)."""
    return k ** 4 * np.exp(-2.0 * (k / k0) ** 2)


def _wavenumbers(n: int):
    """Integer wavevector components on the rfftn layout of an (n,n,n) array."""
    kf = np.fft.fftfreq(n, d=1.0 / n)           # axes 0 (z) and 1 (y)
    kh = np.fft.rfftfreq(n, d=1.0 / n)          # axis 2 (x), half space
    kz = kf[:, None, None]
    ky = kf[None, :, None]
    kx = kh[None, None, :]
    return kx, ky, kz


def solenoidal_velocity(n: int, seed: int, k0: float = 4.0, u_prime: float = 1.0):
    """Random-phase solenoidal velocity with E(k) ~ k^4 exp(-2 (k/k0)^2).

    Recipe: a complex Gaussian 3-vector per wavevector of the rfftn half space,
    projected orthogonal to k, rescaled to |u_hat| = sqrt(E(|k|) / (4 pi |k|^2)),
    the mean and every Nyquist mode zeroed, inverse-transformed, then scaled so
    that the per-component r.m.s. velocity sqrt(<|u|^2>/3) equals ``u_prime``.

    Returns ``(ux, uy, uz)``, each ``(n, n, n)`` float64.
    """
    rng = np.random.default_rng(seed)
    kx, ky, kz = _wavenumbers(n)
    shape = (n, n, n // 2 + 1)
    kx = np.broadcast_to(kx, shape)
    ky = np.broadcast_to(ky, shape)
    kz = np.broadcast_to(kz, shape)
    k2 = kx * kx + ky * ky + kz * kz
    kmag = np.sqrt(k2)

    v = rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)
    safe_k2 = np.where(k2 > 0, k2, 1.0)
    kdotv = (kx * v[0] + ky * v[1] + kz * v[2]) / safe_k2
    v[0] -= kx * kdotv
    v[1] -= ky * kdotv
    v[2] -= kz * kdotv
    vnorm = np.sqrt(np.sum(np.abs(v) ** 2, axis=0))
    amp = np.sqrt(spectrum_k4(kmag, k0) / (4.0 * math.pi * safe_k2))
    scale = np.where(vnorm > 0, amp / np.where(vnorm > 0, vnorm, 1.0), 0.0)
    v *= scale
    nyq = n // 2
    kill = (k2 == 0)
    if n % 2 == 0:
        kill |= (np.abs(kx) == nyq) | (np.abs(ky) == nyq) | (np.abs(kz) == nyq)
    v[:, kill] = 0.0
    u = [np.fft.irfftn(v[c], s=(n, n, n), axes=(0, 1, 2)) for c in range(3)]
    rms = math.sqrt(sum(float(np.mean(c * c)) for c in u) / 3.0)
    if rms == 0.0:
        raise ValueError("velocity field vanished; grid too coarse for the spectrum")
    s = u_prime / rms
    return tuple(np.ascontiguousarray(c * s) for c in u)


def spectral_dissipation(u, nu: float) -> float:
    """eps0 = 2 nu <S:S> of a periodic field with exact (Fourier) derivatives,
    summed in spectral space (Parseval) over the rfftn half space."""
    n = u[0].shape[0]
    kx, ky, kz = _wavenumbers(n)
    kvec = (kx, ky, kz)
    uh = [np.fft.rfftn(c, axes=(0, 1, 2)) for c in u]
    # half-space weights: interior kx planes stand for +kx and -kx
    wgt = np.full(n // 2 + 1, 2.0)
    wgt[0] = 1.0
    if n % 2 == 0:
        wgt[-1] = 1.0
    wgt = wgt[None, None, :]
    ss = 0.0
    for a in range(3):
        for b in range(3):
            s_ab = 0.5j * (kvec[b] * uh[a] + kvec[a] * uh[b])
            ss += float(np.sum(wgt * np.abs(s_ab) ** 2))
    return 2.0 * nu * ss / float(n) ** 6


@dataclasses.dataclass
class HITCase:
    """One seeded decaying-HIT case: gas state, dust and the physical constants."""
    n: int
    seed: int
    mach: float
    stokes: tuple
    gamma: float
    nu: float
    rho0: float
    C: float            # p = C rho^gamma
    c0: float           # initial sound speed
    mu: float           # dynamic viscosity rho0*nu
    tau_p: tuple        # particle response times
    tau_eta: float      # Kolmogorov time of the initial field
    rho: np.ndarray     # (n,n,n)
    u: np.ndarray       # (3,n,n,n) SoA, x-component first
    rho_p: np.ndarray   # (K,n,n,n) particle bulk densities

    @property
    def name(self) -> str:
        return run_name(self.n, self.mach, self.stokes, self.seed)


def make_hit_case(n: int, seed: int, mach: float = 0.2, stokes=(0.1,), gamma: float = 1.4,
                  nu: float = 1e-3, mass_fraction: float = 1e-3, k0: float = 4.0,
                  rho0: float = 1.0) -> HITCase:
    """Build the seeded decaying-HIT initial state used by every run.

    * velocity: :func:`solenoidal_velocity` with u' = 1;
    * density uniform ``rho0``; sound speed c0 = sqrt(3) u' / mach so that
      sqrt(<|u|^2>)/c0 = mach; closure constant C = c0^2 rho0^(1-gamma) / gamma;
    * every particle class j carries a uniform mass fraction ``mass_fraction``
      of the gas-plus-class mixture: rho_j = Y0 rho / (1 - Y0);
    * tau_p = St * tau_eta with tau_eta = sqrt(nu / eps0), eps0 from the
      initial field (Stokes number based on the Kolmogorov time).
    """
    stokes = tuple(float(s) for s in stokes)
    ux, uy, uz = solenoidal_velocity(n, seed, k0=k0)
    u = np.stack([ux, uy, uz])
    c0 = math.sqrt(3.0) / mach
    C = c0 * c0 * rho0 ** (1.0 - gamma) / gamma
    eps0 = spectral_dissipation((ux, uy, uz), nu)
    tau_eta = math.sqrt(nu / eps0)
    tau_p = tuple(st * tau_eta for st in stokes)
    rho = np.full((n, n, n), rho0)
    ratio = mass_fraction / (1.0 - mass_fraction)
    rho_p = np.stack([ratio * rho for _ in stokes]) if stokes else np.zeros((0, n, n, n))
    return HITCase(n=n, seed=seed, mach=mach, stokes=stokes, gamma=gamma, nu=nu, rho0=rho0,
                   C=C, c0=c0, mu=rho0 * nu, tau_p=tau_p, tau_eta=tau_eta,
                   rho=rho, u=np.ascontiguousarray(u), rho_p=np.ascontiguousarray(rho_p))


def ensemble_cases(count: int = 64, seed: int = 0, sizes=(32, 32, 48, 64),
                   machs=(0.2, 0.5), stokes_range=(0.05, 0.5)):
    """Members of a mixed-size ensemble of decaying-HIT realisations.

    Member m has grid size ``sizes[m % len(sizes)]`` (the default gives 32^3,
    48^3 and 64^3 in the ratio 2:1:1), flow seed ``seed + m``, an r.m.s. Mach
    number drawn from ``machs`` and one particle class whose Stokes number is
    drawn uniformly from ``stokes_range``; both draws come from a generator
    seeded with ``seed``."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(count):
        mach = float(machs[int(rng.integers(len(machs)))])
        st = float(rng.uniform(*stokes_range))
        out.append(make_hit_case(sizes[m % len(sizes)], seed + m, mach=mach, stokes=(st,)))
    return out


def run_name(n: int, mach: float, stokes, seed: int, scheme: str = "PISO", sgs: str = "noM") -> str:
    """Run name in the paper's scheme.subgrid-model.<...>.cells-per-side pattern,
    extended with Mach, Stokes numbers and seed, e.g. ``PISO.noM.32.Ma02.St0.1.s0``."""
    ma = f"Ma{int(round(mach * 10)):02d}"
    st = "St" + "-".join(f"{s:g}" for s in stokes) if stokes else "St-"
    return f"{scheme}.{sgs}.{n}.{ma}.{st}.s{seed}"


def taylor_green_case(n: int = 32, mach: float = 0.05, nu: float = 0.01, gamma: float = 1.4,
                      rho0: float = 1.0):
    """2D Taylor-Green vortex embedded in 3D (a closed-form viscous decay case).

    u = (sin x cos y, -cos x sin y, 0), p = p0 + (rho0/4)(cos 2x + cos 2y),
    rho = (p/C)^(1/gamma), evaluated at cell centres ((i+1/2) Delta).
    The velocity amplitude of the incompressible solution decays as exp(-2 nu t).
    Returns a dict with rho (n,n,n), u (3,n,n,n), C, mu, gamma.
    """
    h = TWO_PI / n
    xc = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    ux = np.sin(x) * np.cos(y)
    uy = -np.cos(x) * np.sin(y)
    uz = np.zeros_like(ux)
    umax = 1.0
    c0 = umax / mach
    C = c0 * c0 * rho0 ** (1.0 - gamma) / gamma
    p0 = C * rho0 ** gamma
    p = p0 + 0.25 * rho0 * (np.cos(2 * x) + np.cos(2 * y))
    rho = (p / C) ** (1.0 / gamma)
    return dict(rho=np.ascontiguousarray(rho), u=np.ascontiguousarray(np.stack([ux, uy, uz])),
                C=C, mu=rho0 * nu, gamma=gamma, nu=nu)
