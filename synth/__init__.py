"""Seeded synthetic inputs for the StePS direct-summation path.

This module only builds inputs.  It is shared by the tests, the benchmark and
the smoke check, and it holds none of the arithmetic of the path itself (no
pair sum, kick, drift or time-step mapping); the oracle and the GPU library
each have their own.

Recipe (one particle set, seeded numpy PCG64):

1. g ~ N(0, I_4); u = g / |g| = (w, x, y, z) is uniform on the unit 3-sphere.
2. Stereographic projection X = D (x, y, z) / (1 - w), so |X| = D tan(omega/2)
   with omega the compact radial angle (Racz et al. 2018, Sec. 3.1 Eq. 15).
   Uniform points on S^3 have real-space number density proportional to
   (1 + r^2/D^2)^-3: this is the continuum limit of the paper's
   "constant compact-space volume" shells (Sec. 3.1 Eq. 18).
3. Redraw until exactly N points have |X| <= r_max (first N accepted, in draw
   order).
4. m_i proportional to (1 + r_i^2/D^2)^3, so the mass density is uniform,
   normalised so that sum m = Omega_m rho_crit (4 pi / 3) r_max^3
   (Sec. 3.2 Eq. 25 with R_sim = r_max, rho_crit = 3 H0^2 / (8 pi G)).
5. Local spacing s_i = (m_i / rho_bar)^(1/3) with rho_bar = Omega_m rho_crit,
   softening h_i = 0.05 s_i (the law of Sec. 2.2 Eq. 7 with
   h_min = 0.05 (m_min / rho_bar)^(1/3)).
6. Displacement Psi_i = sigma s_i N(0, I_3); x_i <- x_i + Psi_i (a white
   Gaussian stand-in for the LPT field of Sec. 3.2, which needs a power
   spectrum that is not part of this work).
7. Velocities zero, or the Zel'dovich ones v_i = f(a0) H(a0) Psi_i
   (Sec. 3.2 Eq. 24: dx/dt = (dD/dt) / D * Psi, with f = dlnD/dlna from the
   linear growth integral, Eq. 19).

Units: Mpc, Gyr, Msun; positions and velocities are SoA arrays (3, N).
Seeds: seed = 1000 * config + member.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# IAU-derived unit constants for building inputs (the oracle and the library
# derive their own).
_MPC_M = 149597870700.0 * 648000.0 / math.pi * 1.0e6
_GYR_S = 365.25 * 86400.0 * 1.0e9
KMS_TO_MPC_PER_GYR = 1.0e3 * _GYR_S / _MPC_M
G_MPC3_MSUN_GYR2 = 1.32712440018e20 * _GYR_S ** 2 / _MPC_M ** 3


@dataclass
class Cosmo:
    H0: float = 70.0          # km/s/Mpc
    omega_m: float = 0.3
    omega_l: float = 0.7
    omega_r: float = 0.0

    @property
    def omega_k(self) -> float:
        return 1.0 - self.omega_m - self.omega_l - self.omega_r

    def as_dict(self):
        return {"H0": self.H0, "omega_m": self.omega_m,
                "omega_l": self.omega_l, "omega_r": self.omega_r,
                "omega_k": self.omega_k}


@dataclass
class ParticleSet:
    pos: np.ndarray           # (3, N) float64, Mpc
    vel: np.ndarray           # (3, N) float64, Mpc/Gyr
    mass: np.ndarray          # (N,) float64, Msun
    soft: np.ndarray          # (N,) float64, Mpc
    cosmo: Cosmo
    a0: float
    a1: float
    nsteps: int
    seed: int
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])

    def a_grid(self) -> np.ndarray:
        """Log-uniform scale-factor grid a0 .. a1 with nsteps intervals."""
        k = np.arange(self.nsteps + 1, dtype=np.float64)
        g = self.a0 * (self.a1 / self.a0) ** (k / self.nsteps)
        g[0], g[-1] = self.a0, self.a1
        return g


def _e2(a, c: Cosmo):
    return (c.omega_m / a ** 3 + c.omega_r / a ** 4 + c.omega_l +
            c.omega_k / a ** 2)


def _hubble_gyr(a, c: Cosmo):
    return c.H0 * KMS_TO_MPC_PER_GYR * math.sqrt(_e2(a, c))


def growth_rate(a: float, c: Cosmo) -> float:
    """f = dlnD/dlna for D(a) proportional to E(a) int_0^a da'/(a'E)^3
    (matter + curvature + Lambda; the integral form of Sec. 3.2 Eq. 19)."""
    from scipy.integrate import quad

    def integrand(x):
        return 1.0 / (x * math.sqrt(_e2(x, c))) ** 3

    I, _ = quad(integrand, 0.0, a, epsabs=0.0, epsrel=1e-13, limit=200)
    e2 = _e2(a, c)
    dlne_dlna = (-3.0 * c.omega_m / a ** 3 - 4.0 * c.omega_r / a ** 4 -
                 2.0 * c.omega_k / a ** 2) / (2.0 * e2)
    return dlne_dlna + 1.0 / (a * a * e2 ** 1.5 * I)


def stereographic_points(rng: np.random.Generator, n: int, D: float,
                         r_max: float) -> np.ndarray:
    """n points, uniform on S^3, projected to R^3 and truncated at r_max.
    Returns (3, n)."""
    out = np.empty((3, 0), dtype=np.float64)
    while out.shape[1] < n:
        need = n - out.shape[1]
        batch = int(need * 1.02) + 64
        g = rng.standard_normal((4, batch))
        u = g / np.linalg.norm(g, axis=0)
        X = D * u[1:] / (1.0 - u[0])
        r = np.linalg.norm(X, axis=0)
        out = np.concatenate([out, X[:, r <= r_max]], axis=1)
    return np.ascontiguousarray(out[:, :n])


def make_set(n: int, D: float, r_max: float, cosmo: Cosmo, sigma: float,
             seed: int, a0: float, a1: float, nsteps: int,
             zeldovich: bool) -> ParticleSet:
    """One particle set by the recipe in the module docstring."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = stereographic_points(rng, n, D, r_max)
    r2 = np.sum(X * X, axis=0)
    w = (1.0 + r2 / (D * D)) ** 3
    h0 = cosmo.H0 * KMS_TO_MPC_PER_GYR
    rho_crit = 3.0 * h0 * h0 / (8.0 * math.pi * G_MPC3_MSUN_GYR2)
    rho_bar = cosmo.omega_m * rho_crit
    m_tot = rho_bar * 4.0 * math.pi / 3.0 * r_max ** 3
    mass = w * (m_tot / np.sum(w))
    spacing = np.cbrt(mass / rho_bar)
    soft = 0.05 * spacing
    psi = sigma * spacing * rng.standard_normal((3, n))
    pos = np.ascontiguousarray(X + psi)
    if zeldovich:
        vfac = growth_rate(a0, cosmo) * _hubble_gyr(a0, cosmo)
        vel = np.ascontiguousarray(vfac * psi)
    else:
        vel = np.zeros((3, n), dtype=np.float64)
    return ParticleSet(pos=pos, vel=vel, mass=mass, soft=soft, cosmo=cosmo,
                       a0=a0, a1=a1, nsteps=nsteps, seed=seed,
                       params={"D": D, "r_max": r_max, "sigma": sigma,
                               "zeldovich": zeldovich})


LCDM = Cosmo(H0=67.74, omega_m=0.3089, omega_l=0.6911)


def config(k: int, n: int | None = None, member: int = 0) -> ParticleSet:
    """Workloads 1, 2, 3 and 5 (workload 4 is :func:`ensemble`).

    1: N=4096, D=100, r_max=1000, flat Omega_m=0.3, H0=70, sigma=0.5%, v=0,
       a 0.02 -> 0.05 in 100 log steps.
    2: N=2^18, D=200, r_max=2000, LCDM (0.3089/0.6911/67.74), sigma=1%,
       Zel'dovich v, a 0.02 -> 1.0 in 200 log steps.
    3: N=2^21, D=300, r_max=3000, LCDM as 2, sigma=1%, Zel'dovich v at
       a=0.02 (one force evaluation per precision mode).
    5: N=2^22, D=500, r_max=4000, LCDM as 2, sigma=1%, Zel'dovich v,
       a 0.1 -> 1.0 in 50 log steps.

    n overrides N (same recipe, e.g. the 4096-particle member of config 2).
    """
    seed = 1000 * k + member
    if k == 1:
        return make_set(n or 4096, 100.0, 1000.0,
                        Cosmo(H0=70.0, omega_m=0.3, omega_l=0.7), 0.005,
                        seed, 0.02, 0.05, 100, zeldovich=False)
    if k == 2:
        return make_set(n or 262144, 200.0, 2000.0, LCDM, 0.01, seed,
                        0.02, 1.0, 200, zeldovich=True)
    if k == 3:
        return make_set(n or 2097152, 300.0, 3000.0, LCDM, 0.01, seed,
                        0.02, 0.02, 1, zeldovich=True)
    if k == 5:
        return make_set(n or 4194304, 500.0, 4000.0, LCDM, 0.01, seed,
                        0.1, 1.0, 50, zeldovich=True)
    raise ValueError("no single-set workload %r" % (k,))


def poisson_ball(n: int, radius: float, cosmo: Cosmo, seed: int,
                 a0: float = 0.01, a1: float = 1.0, nsteps: int = 150,
                 soft_frac: float = 0.05) -> ParticleSet:
    """Equal-mass Poisson points in a ball of the given comoving radius at
    the mean matter density (the starting load of a glass relaxation), at
    rest; softening soft_frac times the mean spacing."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((3, n))
    g /= np.linalg.norm(g, axis=0)
    pos = np.ascontiguousarray(g * radius * rng.uniform(size=n) ** (1.0 / 3.0))
    h0 = cosmo.H0 * KMS_TO_MPC_PER_GYR
    rho_bar = cosmo.omega_m * 3.0 * h0 * h0 / (8.0 * math.pi * G_MPC3_MSUN_GYR2)
    m = rho_bar * 4.0 * math.pi / 3.0 * radius ** 3 / n
    spacing = (m / rho_bar) ** (1.0 / 3.0)
    return ParticleSet(pos=pos, vel=np.zeros_like(pos), mass=np.full(n, m),
                       soft=np.full(n, soft_frac * spacing), cosmo=cosmo,
                       a0=a0, a1=a1, nsteps=nsteps, seed=seed,
                       params={"radius": radius, "spacing": spacing})


def ensemble_params(members: int = 64, seed: int = 4999):
    """Per-member parameters of workload 4: N ~ U{8192..131072},
    Omega_m ~ U[0.25, 0.35] (flat, H0=70), sigma ~ U[0.5%, 2%]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(8192, 131072, size=members, endpoint=True)
    om = rng.uniform(0.25, 0.35, size=members)
    sg = rng.uniform(0.005, 0.02, size=members)
    return [(int(a), float(b), float(c)) for a, b, c in zip(ns, om, sg)]


def ensemble(members: int = 64, n_scale: float = 1.0,
             nsteps: int = 100) -> list[ParticleSet]:
    """Workload 4: independent members with D=100, r_max=1000, Zel'dovich
    velocities, a 0.02 -> 1.0 in nsteps log steps; member b uses seed
    4000 + b.  n_scale shrinks every N (for small test ensembles)."""
    out = []
    for b, (n, om, sg) in enumerate(ensemble_params(members)):
        nb = max(1, int(round(n * n_scale)))
        out.append(make_set(nb, 100.0, 1000.0,
                            Cosmo(H0=70.0, omega_m=om, omega_l=1.0 - om),
                            sg, 4000 + b, 0.02, 1.0, nsteps, zeldovich=True))
    return out
