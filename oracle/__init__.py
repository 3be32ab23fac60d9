"""CPU FP64 oracle for the StePS direct-summation path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything here, and this package imports nothing from it.

``oracle.c`` holds the arithmetic (plain C, FP64, Neumaier sums, OpenMP over
i); this module compiles it with gcc on first use (or when the source is newer
than the library) and wraps it with ctypes.  Every function states the passage
of Racz et al. (2018) it follows:

* :func:`kernel_F`, :func:`kernel_phi` -- spline-softened force kernel,
  Sec. 2.2 Eq. 4; its potential (derived: the paper gives only the force).
* :func:`forces` -- G-free pair sum S_i of Sec. 2.2 Eq. 8 with Eq. 3.
* :func:`potential` -- G-free softened potential (diagnostic).
* :func:`hubble`, :func:`dt` -- Sec. 2.2 Eq. 1; exact dt for a step in a
  (Sec. 2.3, the interval Eq. 13 approximates to first order).
* :func:`kdk_step` -- Sec. 2.3 Eqs. 9-11 with the acceleration of Eq. 8.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc; returns its path."""
    stale = (not os.path.exists(_LIB) or
             os.path.getmtime(_LIB) < os.path.getmtime(_SRC))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        vp = ctypes.c_void_p
        lib.oracle_kernel_F.argtypes = [d, d]
        lib.oracle_kernel_F.restype = d
        lib.oracle_kernel_phi.argtypes = [d, d]
        lib.oracle_kernel_phi.restype = d
        lib.oracle_forces.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, i32]
        lib.oracle_forces.restype = i32
        lib.oracle_potential.argtypes = [i64, vp, vp, vp, i64, vp, vp, i32]
        lib.oracle_potential.restype = i32
        lib.oracle_hubble.argtypes = [d, ctypes.POINTER(_Cosmo)]
        lib.oracle_hubble.restype = d
        lib.oracle_dt.argtypes = [d, d, ctypes.POINTER(_Cosmo)]
        lib.oracle_dt.restype = d
        lib.oracle_kdk_step.argtypes = [i64, vp, vp, vp, vp, vp, d, d,
                                        ctypes.POINTER(_Cosmo), i32]
        lib.oracle_kdk_step.restype = i32
        lib.oracle_energy.argtypes = [i64, vp, vp, vp, vp, d,
                                      ctypes.POINTER(_Cosmo), vp, i32]
        lib.oracle_energy.restype = i32
        lib.oracle_adaptive_dt.argtypes = [i64, vp, vp, vp, vp, d,
                                           ctypes.POINTER(_Cosmo), d, d,
                                           ctypes.POINTER(d), ctypes.POINTER(d)]
        lib.oracle_adaptive_dt.restype = i32
        lib.oracle_forces_periodic.argtypes = [i64, vp, vp, vp, d, i32, i64,
                                               vp, vp, i32]
        lib.oracle_forces_periodic.restype = i32
        lib.oracle_G.argtypes = []
        lib.oracle_G.restype = d
        lib.oracle_kms_to_mpc_per_gyr.argtypes = []
        lib.oracle_kms_to_mpc_per_gyr.restype = d
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = i32
        _lib = lib
    return _lib


class _Cosmo(ctypes.Structure):
    _fields_ = [("H0", ctypes.c_double), ("omega_m", ctypes.c_double),
                ("omega_l", ctypes.c_double), ("omega_r", ctypes.c_double),
                ("omega_k", ctypes.c_double), ("G", ctypes.c_double),
                ("newtonian_test", ctypes.c_int), ("reversed_gravity", ctypes.c_int),
                ("images", ctypes.c_int), ("box_L", ctypes.c_double)]


@dataclass
class Cosmology:
    """Background parameters (Sec. 2.2 Eq. 1).  H0 in km/s/Mpc; omega_k None
    means 1 - omega_m - omega_l - omega_r; G None means the oracle's value
    in Mpc^3 / (Msun Gyr^2)."""
    H0: float = 70.0
    omega_m: float = 0.3
    omega_l: float = 0.7
    omega_r: float = 0.0
    omega_k: float | None = None
    G: float | None = None
    newtonian_test: bool = False
    reversed_gravity: bool = False   # G -> -G (glass relaxation, Sec. 3)
    images: int = 0      # 0 open sphere; 1 nearest image, 2 all within 2.6 L
    box_L: float = 0.0   # periodic box side (Eq. 2), used when images > 0

    def _c(self) -> _Cosmo:
        ok = self.omega_k
        if ok is None or (isinstance(ok, float) and math.isnan(ok)):
            ok = 1.0 - self.omega_m - self.omega_l - self.omega_r
        g = G() if self.G is None else self.G
        return _Cosmo(self.H0, self.omega_m, self.omega_l, self.omega_r, ok,
                      g, 1 if self.newtonian_test else 0,
                      1 if self.reversed_gravity else 0, int(self.images),
                      float(self.box_L))


def G() -> float:
    """Newton's constant in Mpc^3 / (Msun Gyr^2)."""
    return _load().oracle_G()


def kms_to_mpc_per_gyr() -> float:
    return _load().oracle_kms_to_mpc_per_gyr()


def num_threads() -> int:
    return _load().oracle_num_threads()


def kernel_F(r: float, h: float) -> float:
    """F(r, h) of Eq. 4 (G-free force magnitude per unit source mass)."""
    return _load().oracle_kernel_F(float(r), float(h))


def kernel_phi(r: float, h: float) -> float:
    """Potential whose radial derivative is F(r, h); -1/r beyond h."""
    return _load().oracle_kernel_phi(float(r), float(h))


def _soa(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape == (n, 3) and n != 3:
        a = np.ascontiguousarray(a.T)
    if a.shape != (3, n):
        raise ValueError("expected a (3, n) or (n, 3) array, got %r" % (a.shape,))
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def forces(pos, mass, soft, idx=None, want_kappa=False, nthreads=0):
    """G-free pair sum S (Eq. 8) for all i, or for the rows listed in idx.

    pos: (3, n) SoA (an (n, 3) array is transposed).  Returns S as (3, ni),
    plus kappa (ni,) when want_kappa.
    """
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    pos = _soa(pos, n)
    soft = np.ascontiguousarray(soft, dtype=np.float64)
    if soft.shape != (n,):
        raise ValueError("soft must have shape (n,)")
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= n):
            raise ValueError("idx out of range")
        ni = idx.shape[0]
    else:
        ni = n
    acc = np.zeros((3, ni), dtype=np.float64)
    kap = np.zeros(ni, dtype=np.float64) if want_kappa else None
    rc = _load().oracle_forces(n, _ptr(pos), _ptr(mass), _ptr(soft), ni,
                               _ptr(idx), _ptr(acc), _ptr(kap), int(nthreads))
    if rc:
        raise ValueError("oracle_forces: bad argument")
    return (acc, kap) if want_kappa else acc


def potential(pos, mass, soft, idx=None, nthreads=0):
    """G-free softened potential Phi_i = sum_j m_j phi(r_ij, h_i + h_j)."""
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    pos = _soa(pos, n)
    soft = np.ascontiguousarray(soft, dtype=np.float64)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        ni = idx.shape[0]
    else:
        ni = n
    phi = np.zeros(ni, dtype=np.float64)
    rc = _load().oracle_potential(n, _ptr(pos), _ptr(mass), _ptr(soft), ni,
                                  _ptr(idx), _ptr(phi), int(nthreads))
    if rc:
        raise ValueError("oracle_potential: bad argument")
    return phi


def hubble(a: float, cosmo: Cosmology) -> float:
    """H(a) in 1/Gyr (Eq. 1)."""
    c = cosmo._c()
    return _load().oracle_hubble(float(a), ctypes.byref(c))


def dt(a: float, da: float, cosmo: Cosmology) -> float:
    """Cosmic time (Gyr) for the scale factor to go from a to a + da."""
    c = cosmo._c()
    return _load().oracle_dt(float(a), float(da), ctypes.byref(c))


def kdk_step(pos, vel, mass, soft, S, a, da, cosmo: Cosmology, nthreads=0):
    """One KDK step (Eq. 11) in place on SoA float64 arrays pos, vel, S."""
    n = mass.shape[0]
    for arr in (pos, vel, S):
        if arr.shape != (3, n) or arr.dtype != np.float64 or \
                not arr.flags.c_contiguous:
            raise ValueError("pos, vel, S must be C-contiguous float64 (3, n)")
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    soft = np.ascontiguousarray(soft, dtype=np.float64)
    c = cosmo._c()
    rc = _load().oracle_kdk_step(n, _ptr(pos), _ptr(vel), _ptr(mass),
                                 _ptr(soft), _ptr(S), float(a), float(da),
                                 ctypes.byref(c), int(nthreads))
    if rc:
        raise ValueError("oracle_kdk_step: bad argument")


def energy(pos, vel, mass, soft, a, cosmo: Cosmology, nthreads=0):
    """Comoving energies (derived from Eq. 8; see oracle.c): dict with K, W,
    U_pair, U_radial and P (peculiar momentum sum m a^2 v)."""
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    pos, vel = _soa(pos, n), _soa(vel, n)
    soft = np.ascontiguousarray(soft, dtype=np.float64)
    out = np.zeros(7)
    c = cosmo._c()
    rc = _load().oracle_energy(n, _ptr(pos), _ptr(vel), _ptr(mass), _ptr(soft),
                               float(a), ctypes.byref(c), _ptr(out),
                               int(nthreads))
    if rc:
        raise ValueError("oracle_energy: bad argument")
    return {"K": out[0], "W": out[1], "U_pair": out[2], "U_radial": out[3],
            "P": out[4:7].copy()}


def layzer_irvine(energies, a_grid, cosmo: Cosmology):
    """Residual R_n = (K+W)_n - (K+W)_0 + int_0^t H (2K + W) dt' of the
    cosmic energy equation, the integral by the trapezoid rule over the
    steps of a_grid (energies[k] at a_grid[k])."""
    out = [0.0]
    acc = 0.0
    e0 = energies[0]["K"] + energies[0]["W"]
    for k in range(1, len(energies)):
        t = dt(a_grid[k - 1], a_grid[k] - a_grid[k - 1], cosmo)
        f0 = hubble(a_grid[k - 1], cosmo) * (2 * energies[k - 1]["K"] + energies[k - 1]["W"])
        f1 = hubble(a_grid[k], cosmo) * (2 * energies[k]["K"] + energies[k]["W"])
        acc += 0.5 * (f0 + f1) * t
        out.append(energies[k]["K"] + energies[k]["W"] - e0 + acc)
    return np.array(out)


def _initial_S(pos, mass, soft, cosmo: Cosmology, nthreads=0):
    if cosmo.images:
        return forces_periodic(pos, mass, soft, cosmo.box_L, cosmo.images,
                               nthreads=nthreads)
    return forces(pos, mass, soft, nthreads=nthreads)


def forces_periodic(pos, mass, soft, L, images, idx=None, nthreads=0):
    """G-free periodic pair sum (Eqs. 2 and 5; see oracle.c): images 1 keeps
    the nearest image, 2 every image within 2.6 L.  (3, ni) array."""
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    pos = _soa(pos, n)
    soft = np.ascontiguousarray(soft, dtype=np.float64)
    if idx is None:
        ni, ip = n, None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        ni, ip = idx.shape[0], _ptr(idx)
    acc = np.zeros((3, ni), dtype=np.float64)
    rc = _load().oracle_forces_periodic(n, _ptr(pos), _ptr(mass), _ptr(soft),
                                        float(L), int(images), ni, ip,
                                        _ptr(acc), int(nthreads))
    if rc:
        raise ValueError("oracle_forces_periodic: bad argument")
    return acc


def adaptive_dt(pos, vel, soft, S, a, cosmo: Cosmology, eps, dt_max):
    """Global step of Eq. 12 at the current state (see oracle.c): returns
    (dt, da), da being the scale-factor step whose cosmic time is dt."""
    soft = np.ascontiguousarray(soft, dtype=np.float64)
    n = soft.shape[0]
    pos, vel, S = _soa(pos, n), _soa(vel, n), _soa(S, n)
    c = cosmo._c()
    dt, da = ctypes.c_double(), ctypes.c_double()
    rc = _load().oracle_adaptive_dt(n, _ptr(pos), _ptr(vel), _ptr(soft),
                                    _ptr(S), float(a), ctypes.byref(c),
                                    float(eps), float(dt_max),
                                    ctypes.byref(dt), ctypes.byref(da))
    if rc:
        raise ValueError("oracle_adaptive_dt: bad argument")
    return dt.value, da.value


def run_adaptive(pos, vel, mass, soft, a0, a1, cosmo: Cosmology, eps, dt_max,
                 max_steps=100000, nthreads=0):
    """Integrate from a0 to a1 with the step of Eq. 12 chosen before each
    KDK step, the last one shortened to end exactly at a1 (a is the time
    in the Newtonian test mode).  Copies its inputs; returns
    (pos, vel, S, list of the scale factors reached)."""
    n = mass.shape[0]
    pos = _soa(pos, n).copy()
    vel = _soa(vel, n).copy()
    S = _initial_S(pos, mass, soft, cosmo, nthreads)
    a, grid = float(a0), [float(a0)]
    for _ in range(max_steps):
        if a >= a1:
            break
        _, da = adaptive_dt(pos, vel, soft, S, a, cosmo, eps, dt_max)
        last = a + da >= a1
        if last:
            da = a1 - a
        kdk_step(pos, vel, mass, soft, S, a, da, cosmo, nthreads)
        a = a1 if last else a + da
        grid.append(a)
    return pos, vel, S, grid


def run(pos, vel, mass, soft, a_grid, cosmo: Cosmology, nthreads=0):
    """Integrate over the scale-factor grid a_grid (KDK per interval).

    Copies its inputs; returns (pos, vel, S) at a_grid[-1].
    """
    n = mass.shape[0]
    pos = _soa(pos, n).copy()
    vel = _soa(vel, n).copy()
    S = _initial_S(pos, mass, soft, cosmo, nthreads)
    for k in range(len(a_grid) - 1):
        kdk_step(pos, vel, mass, soft, S, a_grid[k],
                 a_grid[k + 1] - a_grid[k], cosmo, nthreads)
    return pos, vel, S
