"""Independent test-side references: nothing here calls the oracle or the GPU
library.  Used to pin the oracle to mathematics it does not itself contain."""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
from scipy.integrate import quad

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def m4_density(r: float, h: float) -> float:
    """Normalised cubic-spline (M4) density of unit mass with support h
    (Monaghan & Lattanzio 1985; GADGET-2 normalisation)."""
    u = r / h
    c = 8.0 / (math.pi * h ** 3)
    if u < 0.5:
        return c * (1.0 - 6.0 * u * u + 6.0 * u ** 3)
    if u < 1.0:
        return c * 2.0 * (1.0 - u) ** 3
    return 0.0


def m4_enclosed_mass(r: float, h: float) -> float:
    """M(<r) = int_0^r 4 pi s^2 W(s) ds by adaptive quadrature."""
    if r <= 0.0:
        return 0.0
    if r >= h:
        return 1.0
    brk = [0.5 * h] if r > 0.5 * h else None
    val, _ = quad(lambda s: 4.0 * math.pi * s * s * m4_density(s, h), 0.0, r,
                  points=brk, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def m4_force(r: float, h: float) -> float:
    """Softened force magnitude per unit source mass, M(<r)/r^2 (G-free)."""
    if h <= 0.0 or r >= h:
        return 1.0 / (r * r)
    return m4_enclosed_mass(r, h) / (r * r)


def m4_potential(r: float, h: float) -> float:
    """phi(r) = -int_r^inf F(s) ds with F from the quadrature above."""
    if h <= 0.0 or r >= h:
        return -1.0 / r
    pts = [0.5 * h] if r < 0.5 * h else None
    inner, _ = quad(lambda s: m4_force(s, h) if s > 0 else 0.0, r, h,
                    points=pts, epsabs=0.0, epsrel=1e-13, limit=200)
    return -(inner + 1.0 / h)


def load_m4_golden():
    """Rows (u, h^2 F, h phi or None) from tests/golden/m4_kernel_points.txt."""
    rows = []
    with open(os.path.join(GOLDEN, "m4_kernel_points.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t = line.split()
            u = Fraction(int(t[0]), int(t[1]))
            f2 = Fraction(int(t[2]), int(t[3]))
            ph = None if t[4] == "-" else Fraction(int(t[4]), int(t[5]))
            rows.append((u, f2, ph))
    return rows


def brute_pair_sum(pos, mass, soft, i):
    """S_i by a plain Python loop with the quadrature-based kernel and exact
    (fsum) accumulation; pos is (3, n)."""
    n = len(mass)
    terms = [[], [], []]
    for j in range(n):
        if j == i:
            continue
        d = [float(pos[k][j]) - float(pos[k][i]) for k in range(3)]
        r = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
        if r == 0.0:
            continue
        f = float(mass[j]) * m4_force(r, float(soft[i]) + float(soft[j])) / r
        for k in range(3):
            terms[k].append(f * d[k])
    return np.array([math.fsum(t) for t in terms])


def fibonacci_sphere(m: int, radius: float) -> np.ndarray:
    """m nearly uniform points on a sphere (golden-angle spiral), (3, m)."""
    k = np.arange(m, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / m
    rho = np.sqrt(1.0 - z * z)
    phi = math.pi * (3.0 - math.sqrt(5.0)) * k
    return radius * np.stack([rho * np.cos(phi), rho * np.sin(phi), z])


def lattice_ball(radius_cells: float, spacing: float = 1.0) -> np.ndarray:
    """Simple-cubic lattice points within a ball, (3, n)."""
    r = int(math.ceil(radius_cells))
    g = np.arange(-r, r + 1, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    keep = np.sum(pts * pts, axis=0) <= radius_cells ** 2
    return np.ascontiguousarray(pts[:, keep] * spacing)


def kepler_position(t: float, a_semi: float, ecc: float, mu: float):
    """Relative position at time t (from pericentre at t=0) of a Kepler orbit
    in the x-y plane, by Newton iteration on Kepler's equation."""
    n = math.sqrt(mu / a_semi ** 3)
    M = n * t
    E = M if ecc < 0.8 else math.pi
    for _ in range(100):
        dE = (E - ecc * math.sin(E) - M) / (1.0 - ecc * math.cos(E))
        E -= dE
        if abs(dE) < 1e-16:
            break
    x = a_semi * (math.cos(E) - ecc)
    y = a_semi * math.sqrt(1.0 - ecc * ecc) * math.sin(E)
    return np.array([x, y, 0.0])
