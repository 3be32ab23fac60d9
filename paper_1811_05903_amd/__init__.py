"""Python binding of libsteps (include/steps.h): an MI355X (gfx950) HIP
implementation of the StePS direct-summation hot path (Racz et al. 2018):
the spline-softened O(N^2) pair sum (Sec. 2.2 Eqs. 3, 4, 8) and the
comoving KDK leapfrog around it (Sec. 2.3 Eqs. 9-11).

This module only marshals arguments: every step of the computation runs in
the HIP kernels of ``libsteps.so``.  PyTorch supplies device memory and
streams.  Arrays are torch CUDA float64 tensors in SoA layout: positions,
velocities and accelerations (3, n), masses and softenings (n,).

The functions carry the C names.  Without an explicit :class:`Context` they
run on a per-device context owned by this module whose stream follows
``torch.cuda.current_stream()``.

Importing works without a GPU; the first call loads ``libsteps.so`` and
raises if it has not been built (``python -m paper_1811_05903_amd.build``).
There is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsteps.so")

STEPS_OK = 0
STEPS_E_INVAL = -1
STEPS_E_NOMEM = -2
STEPS_E_HIP = -3
STEPS_E_NONFINITE = -4
STEPS_E_UNSUPPORTED = -5

STEPS_FP64 = 0
STEPS_MIXED_F64ACC = 1
STEPS_MIXED_KAHAN = 2
PRECISIONS = {"fp64": STEPS_FP64, "mixed": STEPS_MIXED_F64ACC,
              "mixed_f64acc": STEPS_MIXED_F64ACC, "kahan": STEPS_MIXED_KAHAN,
              "mixed_kahan": STEPS_MIXED_KAHAN}

STEPS_CHECK_FINITE = 1
STEPS_PROFILE = 2

STEPS_COMOVING_SPHERICAL = 0
STEPS_NEWTONIAN_TEST = 1
STEPS_REVERSED_GRAVITY = 1
STEPS_COMOVING_PERIODIC = 2
STEPS_IMAGES_NONE, STEPS_IMAGES_NEAREST, STEPS_IMAGES_ALL = 0, 1, 2

# every symbol include/steps.h declares
EXPORTS = (
    "steps_version", "steps_last_error", "steps_ctx_create",
    "steps_ctx_destroy", "steps_ctx_set_stream", "steps_ctx_set_precision",
    "steps_ctx_set_flags", "steps_ctx_set_tile", "steps_ctx_set_tuned",
    "steps_ctx_set_periodic",
    "steps_ctx_get_tile",
    "steps_sync", "steps_ctx_force_timing", "steps_autotune", "steps_forces_ctx",
    "steps_forces", "steps_forces_noalloc", "steps_potential_ctx",
    "steps_potential",
    "steps_step_ctx", "steps_step", "steps_energy_ctx", "steps_energy",
    "steps_kinetic_ctx", "steps_kinetic", "steps_adaptive_dt_ctx",
    "steps_adaptive_dt", "steps_run_adaptive_ctx",
    "steps_batch_run", "steps_batch_tile",
    "steps_hubble", "steps_dt", "steps_G", "steps_kms_to_mpc_per_gyr",
)

STEPS_BATCH_GRAPH = 1
STEPS_BATCH_AUTOTUNE = 2


class StepsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libsteps error %d: %s" % (code, msg))
        self.code = code


class steps_cosmology(ctypes.Structure):
    _fields_ = [("H0", ctypes.c_double), ("omega_m", ctypes.c_double),
                ("omega_l", ctypes.c_double), ("omega_r", ctypes.c_double),
                ("omega_k", ctypes.c_double), ("G", ctypes.c_double),
                ("mode", ctypes.c_int32), ("flags", ctypes.c_int32)]


class steps_batch(ctypes.Structure):
    _fields_ = [("members", ctypes.c_int32), ("nsteps", ctypes.c_int32),
                ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("pos", ctypes.c_void_p), ("vel", ctypes.c_void_p),
                ("mass", ctypes.c_void_p), ("soft", ctypes.c_void_p),
                ("acc", ctypes.c_void_p),
                ("cosmo", ctypes.POINTER(steps_cosmology)),
                ("a0", ctypes.POINTER(ctypes.c_double)),
                ("a1", ctypes.POINTER(ctypes.c_double)),
                ("flags", ctypes.c_uint32), ("resort_every", ctypes.c_int32)]


class steps_tile(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("tj", ctypes.c_int32),
                ("jsplit", ctypes.c_int32), ("variant", ctypes.c_int32)]


@dataclass
class Cosmology:
    """steps_cosmology: H0 in km/s/Mpc; omega_k None = 1 - the others;
    G 0 = the library's value (Mpc^3 / (Msun Gyr^2))."""
    H0: float = 70.0
    omega_m: float = 0.3
    omega_l: float = 0.7
    omega_r: float = 0.0
    omega_k: float | None = None
    G: float = 0.0
    newtonian_test: bool = False
    reversed_gravity: bool = False
    periodic: bool = False      # Eq. 2 (needs a periodic context)

    def to_c(self) -> steps_cosmology:
        ok = math.nan if self.omega_k is None else float(self.omega_k)
        mode = (STEPS_NEWTONIAN_TEST if self.newtonian_test else
                STEPS_COMOVING_PERIODIC if self.periodic else
                STEPS_COMOVING_SPHERICAL)
        flags = STEPS_REVERSED_GRAVITY if self.reversed_gravity else 0
        return steps_cosmology(float(self.H0), float(self.omega_m),
                               float(self.omega_l), float(self.omega_r), ok,
                               float(self.G), mode, flags)


_lib = None
_lib_lock = threading.Lock()


def load():
    """Load libsteps.so (raises if it is missing)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        # torch first: libsteps then binds to the HIP runtime torch loaded
        # (same soname), so the process holds one runtime.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libsteps.so is not built (expected at %s); run "
                "`python -m paper_1811_05903_amd.build`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        u32 = ctypes.c_uint32
        pc = ctypes.POINTER(steps_cosmology)
        pt = ctypes.POINTER(steps_tile)
        sig = {
            "steps_version": ([], ctypes.c_char_p),
            "steps_last_error": ([], ctypes.c_char_p),
            "steps_ctx_create": ([i32, ctypes.POINTER(vp)], i32),
            "steps_ctx_destroy": ([vp], i32),
            "steps_ctx_set_stream": ([vp, vp], i32),
            "steps_ctx_set_precision": ([vp, i32], i32),
            "steps_ctx_set_flags": ([vp, u32], i32),
            "steps_ctx_set_tile": ([vp, pt], i32),
            "steps_ctx_get_tile": ([vp, i64, pt], i32),
            "steps_ctx_set_tuned": ([vp, i64, pt], i32),
            "steps_ctx_set_periodic": ([vp, d, i32], i32),
            "steps_sync": ([vp], i32),
            "steps_ctx_force_timing": ([vp, ctypes.POINTER(d),
                                        ctypes.POINTER(i64), i32], i32),
            "steps_autotune": ([vp, vp, vp, vp, i64, vp, pt], i32),
            "steps_forces_ctx": ([vp, vp, vp, vp, i64, vp], i32),
            "steps_forces": ([vp, vp, vp, i64, vp], i32),
            "steps_forces_noalloc": ([vp, vp, vp, i64, vp, vp], i32),
            "steps_potential_ctx": ([vp, vp, vp, vp, i64, vp], i32),
            "steps_potential": ([vp, vp, vp, i64, vp], i32),
            "steps_step_ctx": ([vp, vp, vp, vp, vp, i64, vp, d, d, pc], i32),
            "steps_step": ([vp, vp, vp, vp, i64, vp, d, d, pc], i32),
            "steps_energy_ctx": ([vp, vp, vp, vp, vp, i64, d, pc,
                                  ctypes.POINTER(d)], i32),
            "steps_energy": ([vp, vp, vp, vp, i64, d, pc, ctypes.POINTER(d)],
                             i32),
            "steps_kinetic_ctx": ([vp, vp, vp, i64, d, ctypes.POINTER(d)], i32),
            "steps_adaptive_dt_ctx": ([vp, vp, vp, vp, vp, i64, d, pc, d, d,
                                       ctypes.POINTER(d), ctypes.POINTER(d)], i32),
            "steps_adaptive_dt": ([vp, vp, vp, vp, i64, d, pc, d, d,
                                   ctypes.POINTER(d), ctypes.POINTER(d)], i32),
            "steps_run_adaptive_ctx": ([vp, vp, vp, vp, vp, i64, vp, d, d, pc,
                                        d, d, i64, ctypes.POINTER(i64),
                                        ctypes.POINTER(d)], i32),
            "steps_kinetic": ([vp, vp, i64, d, ctypes.POINTER(d)], i32),
            "steps_batch_run": ([vp, ctypes.POINTER(steps_batch),
                                 ctypes.POINTER(ctypes.c_int32)], i32),
            "steps_batch_tile": ([vp, pt], i32),
            "steps_hubble": ([pc, d, ctypes.POINTER(d)], i32),
            "steps_dt": ([pc, d, d, ctypes.POINTER(d)], i32),
            "steps_G": ([], d),
            "steps_kms_to_mpc_per_gyr": ([], d),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
        return lib


def _check(rc: int):
    if rc != STEPS_OK:
        msg = load().steps_last_error().decode(errors="replace")
        raise StepsError(rc, msg)


def steps_version() -> str:
    return load().steps_version().decode()


def steps_G() -> float:
    return load().steps_G()


def steps_kms_to_mpc_per_gyr() -> float:
    return load().steps_kms_to_mpc_per_gyr()


def steps_hubble(cosmo: Cosmology, a: float) -> float:
    out = ctypes.c_double()
    c = cosmo.to_c()
    _check(load().steps_hubble(ctypes.byref(c), float(a), ctypes.byref(out)))
    return out.value


def steps_dt(cosmo: Cosmology, a: float, da: float) -> float:
    out = ctypes.c_double()
    c = cosmo.to_c()
    _check(load().steps_dt(ctypes.byref(c), float(a), float(da),
                           ctypes.byref(out)))
    return out.value


class Context:
    """A libsteps context (steps_ctx) on one device.

    stream None: each call runs on torch.cuda.current_stream() of the
    context's device at call time."""

    def __init__(self, device: int = 0, precision="fp64", flags: int = 0,
                 stream=None):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.steps_ctx_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = int(device)
        self._stream = stream
        self.set_precision(precision)
        if flags:
            self.set_flags(flags)

    def close(self):
        if self.handle:
            _check(self._lib.steps_ctx_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self._lib.steps_ctx_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_precision(self, precision):
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(self._lib.steps_ctx_set_precision(self.handle, p))
        self.precision = p

    def set_flags(self, flags: int):
        _check(self._lib.steps_ctx_set_flags(self.handle, int(flags)))

    def set_tile(self, r=None, tj=None, jsplit=None, variant=0):
        if r is None:
            _check(self._lib.steps_ctx_set_tile(self.handle, None))
            return
        t = steps_tile(int(r), int(tj), int(jsplit), int(variant))
        _check(self._lib.steps_ctx_set_tile(self.handle, ctypes.byref(t)))

    def set_periodic(self, L=0.0, images=STEPS_IMAGES_NONE):
        """Periodic box of side L for this context's pair sums (images: 1
        nearest image, 2 every image within 2.6 L, 0 open sphere)."""
        _check(self._lib.steps_ctx_set_periodic(self.handle, float(L), int(images)))

    def set_tuned(self, n: int, r, tj, jsplit, variant=0):
        """Record a tuned shape for n in this precision (steps_ctx_set_tuned)."""
        t = steps_tile(int(r), int(tj), int(jsplit), int(variant))
        _check(self._lib.steps_ctx_set_tuned(self.handle, int(n), ctypes.byref(t)))

    def get_tile(self, n: int):
        t = steps_tile()
        _check(self._lib.steps_ctx_get_tile(self.handle, int(n), ctypes.byref(t)))
        return {"r": t.r, "tj": t.tj, "jsplit": t.jsplit, "variant": t.variant}

    def bind_stream(self):
        """Point the context at its stream (or torch's current stream)."""
        import torch
        s = self._stream if self._stream is not None else \
            torch.cuda.current_stream(self.device)
        _check(self._lib.steps_ctx_set_stream(self.handle,
                                              ctypes.c_void_p(s.cuda_stream)))

    def sync(self):
        _check(self._lib.steps_sync(self.handle))

    def force_timing(self, reset: bool = False):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(self._lib.steps_ctx_force_timing(self.handle, ctypes.byref(ms),
                                                ctypes.byref(cnt), int(reset)))
        return ms.value, cnt.value


_default_ctx: dict[int, Context] = {}


def default_context(device: int) -> Context:
    ctx = _default_ctx.get(device)
    if ctx is None:
        ctx = Context(device)
        _default_ctx[device] = ctx
    return ctx


def _dev(t, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous (SoA)" % name)
    if shape is not None and tuple(t.shape) != shape:
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), shape))
    return ctypes.c_void_p(t.data_ptr())


def _n_of(mass):
    return int(mass.shape[0])


def steps_forces(pos, mass, soft, acc=None, ctx: Context | None = None):
    """acc <- S(pos): the G-free pair sum of Eq. 8 (see steps.h).  Returns acc."""
    import torch
    n = _n_of(mass)
    if acc is None:
        acc = torch.empty((3, n), dtype=torch.float64, device=pos.device)
    c = ctx or default_context(pos.device.index or 0)
    args = (_dev(pos, "pos", (3, n)), _dev(mass, "mass", (n,)),
            _dev(soft, "soft", (n,)), n, _dev(acc, "acc", (3, n)))
    c.bind_stream()
    _check(c._lib.steps_forces_ctx(c.handle, *args))
    return acc


def steps_forces_noalloc(pos, mass, soft, acc, stream=None):
    """acc <- S(pos) through the allocation-free entry point (FP64, fixed
    device scratch, n <= 262144; see steps.h), enqueued on `stream` (a torch
    stream; default: the current one).  acc must be allocated by the caller.
    Returns acc."""
    import torch
    n = _n_of(mass)
    s = stream if stream is not None else torch.cuda.current_stream(pos.device)
    args = (_dev(pos, "pos", (3, n)), _dev(mass, "mass", (n,)),
            _dev(soft, "soft", (n,)), n, _dev(acc, "acc", (3, n)),
            ctypes.c_void_p(s.cuda_stream))
    _check(load().steps_forces_noalloc(*args))
    return acc


def _cache_key(ctx: Context, n: int) -> str:
    import torch
    name = torch.cuda.get_device_properties(ctx.device).name
    return "%s|%s|%d|%d" % (name, steps_version(), ctx.precision, n)


def steps_autotune(pos, mass, soft, ctx: Context, acc=None, cache=None):
    """Time the compiled force kernels on these arrays and keep the fastest
    for this n in ctx (see steps.h).  Returns the chosen tile.

    cache: optional path of a JSON file keyed by (device name, library
    version, precision, n).  A hit is recorded in ctx with
    steps_ctx_set_tuned and nothing is timed; a miss is tuned and written
    back."""
    import json
    import os
    import torch
    n = _n_of(mass)
    table = {}
    if cache is not None and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        hit = table.get(_cache_key(ctx, n))
        if hit is not None:
            ctx.set_tuned(n, hit["r"], hit["tj"], hit["jsplit"], hit["variant"])
            return dict(hit)
    if acc is None:
        acc = torch.empty((3, n), dtype=torch.float64, device=pos.device)
    t = steps_tile()
    args = (_dev(pos, "pos", (3, n)), _dev(mass, "mass", (n,)),
            _dev(soft, "soft", (n,)), n, _dev(acc, "acc", (3, n)))
    ctx.bind_stream()
    _check(ctx._lib.steps_autotune(ctx.handle, *args, ctypes.byref(t)))
    out = {"r": t.r, "tj": t.tj, "jsplit": t.jsplit, "variant": t.variant}
    if cache is not None:
        table[_cache_key(ctx, n)] = out
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return out


def steps_potential(pos, mass, soft, phi=None, ctx: Context | None = None):
    """phi <- G-free softened potential (FP64)."""
    import torch
    n = _n_of(mass)
    if phi is None:
        phi = torch.empty((n,), dtype=torch.float64, device=pos.device)
    c = ctx or default_context(pos.device.index or 0)
    args = (_dev(pos, "pos", (3, n)), _dev(mass, "mass", (n,)),
            _dev(soft, "soft", (n,)), n, _dev(phi, "phi", (n,)))
    c.bind_stream()
    _check(c._lib.steps_potential_ctx(c.handle, *args))
    return phi


def steps_step(pos, vel, mass, soft, acc, a, da, cosmo: Cosmology,
               ctx: Context | None = None):
    """One KDK step from a to a + da, in place on pos, vel, acc."""
    n = _n_of(mass)
    c = ctx or default_context(pos.device.index or 0)
    k = cosmo.to_c()
    args = (_dev(pos, "pos", (3, n)), _dev(vel, "vel", (3, n)),
            _dev(mass, "mass", (n,)), _dev(soft, "soft", (n,)), n,
            _dev(acc, "acc", (3, n)), float(a), float(da), ctypes.byref(k))
    c.bind_stream()
    _check(c._lib.steps_step_ctx(c.handle, *args))


def steps_energy(pos, vel, mass, soft, a, cosmo: Cosmology,
                 ctx: Context | None = None):
    """Comoving energies (see steps.h): dict K, W, U_pair, U_radial, P."""
    n = _n_of(mass)
    c = ctx or default_context(pos.device.index or 0)
    out = (ctypes.c_double * 7)()
    k = cosmo.to_c()
    args = (_dev(pos, "pos", (3, n)), _dev(vel, "vel", (3, n)),
            _dev(mass, "mass", (n,)), _dev(soft, "soft", (n,)), n, float(a),
            ctypes.byref(k), out)
    c.bind_stream()
    _check(c._lib.steps_energy_ctx(c.handle, *args))
    return {"K": out[0], "W": out[1], "U_pair": out[2], "U_radial": out[3],
            "P": [out[4], out[5], out[6]]}


def steps_kinetic(vel, mass, a, ctx: Context | None = None):
    """Kinetic energy and peculiar momentum alone, O(N): dict K, P."""
    n = _n_of(mass)
    c = ctx or default_context(vel.device.index or 0)
    out = (ctypes.c_double * 4)()
    c.bind_stream()
    _check(c._lib.steps_kinetic_ctx(c.handle, _dev(vel, "vel", (3, n)),
                                    _dev(mass, "mass", (n,)), n, float(a), out))
    return {"K": out[0], "P": [out[1], out[2], out[3]]}


def steps_adaptive_dt(pos, vel, soft, acc, a, cosmo: Cosmology, eps, dt_max,
                      ctx: Context | None = None):
    """Step of Eq. 12 at the current state (acc = S(pos)): (dt, da)."""
    n = _n_of(soft)
    c = ctx or default_context(pos.device.index or 0)
    k = cosmo.to_c()
    dt, da = ctypes.c_double(), ctypes.c_double()
    c.bind_stream()
    _check(c._lib.steps_adaptive_dt_ctx(
        c.handle, _dev(pos, "pos", (3, n)), _dev(vel, "vel", (3, n)),
        _dev(soft, "soft", (n,)), _dev(acc, "acc", (3, n)), n, float(a),
        ctypes.byref(k), float(eps), float(dt_max), ctypes.byref(dt),
        ctypes.byref(da)))
    return dt.value, da.value


def steps_run_adaptive(pos, vel, mass, soft, a0, a1, cosmo: Cosmology, eps,
                       dt_max, max_steps=1 << 40, acc=None,
                       ctx: Context | None = None):
    """Integrate in place from a0 to a1 with the step of Eq. 12; returns
    (acc, steps taken, a reached)."""
    import torch
    n = _n_of(mass)
    if acc is None:
        acc = torch.empty((3, n), dtype=torch.float64, device=pos.device)
    c = ctx or default_context(pos.device.index or 0)
    k = cosmo.to_c()
    steps, reached = ctypes.c_int64(), ctypes.c_double()
    c.bind_stream()
    _check(c._lib.steps_run_adaptive_ctx(
        c.handle, _dev(pos, "pos", (3, n)), _dev(vel, "vel", (3, n)),
        _dev(mass, "mass", (n,)), _dev(soft, "soft", (n,)), n,
        _dev(acc, "acc", (3, n)), float(a0), float(a1), ctypes.byref(k),
        float(eps), float(dt_max), int(max_steps), ctypes.byref(steps),
        ctypes.byref(reached)))
    return acc, steps.value, reached.value


def run(pos, vel, mass, soft, a_grid, cosmo: Cosmology, ctx=None, acc=None):
    """Integrate in place over the scale-factor grid a_grid; returns acc."""
    acc = steps_forces(pos, mass, soft, acc=acc, ctx=ctx)
    for k in range(len(a_grid) - 1):
        steps_step(pos, vel, mass, soft, acc, a_grid[k],
                   a_grid[k + 1] - a_grid[k], cosmo, ctx=ctx)
    return acc


def steps_batch_run(pos, vel, mass, soft, acc, offsets, cosmos, a0, a1,
                    nsteps, flags=0, resort_every=0, ctx: Context | None = None):
    """Run an ensemble (see steps.h): arena tensors pos/vel/acc (3, N),
    mass/soft (N,), member b = columns offsets[b]:offsets[b+1].  cosmos, a0,
    a1 are per-member Python sequences.  Returns the per-member status
    codes (0 = ran).  Synchronous."""
    B = len(cosmos)
    if len(offsets) != B + 1 or len(a0) != B or len(a1) != B:
        raise ValueError("offsets must have members + 1 entries, a0/a1 members")
    n = int(offsets[-1])
    c = ctx or default_context(pos.device.index or 0)
    offs = (ctypes.c_int64 * (B + 1))(*[int(x) for x in offsets])
    cs = (steps_cosmology * B)(*[k.to_c() for k in cosmos])
    a0s = (ctypes.c_double * B)(*[float(x) for x in a0])
    a1s = (ctypes.c_double * B)(*[float(x) for x in a1])
    b = steps_batch(B, int(nsteps), offs, _dev(pos, "pos", (3, n)),
                    _dev(vel, "vel", (3, n)), _dev(mass, "mass", (n,)),
                    _dev(soft, "soft", (n,)), _dev(acc, "acc", (3, n)), cs,
                    a0s, a1s, int(flags), int(resort_every))
    status = (ctypes.c_int32 * B)()
    c.bind_stream()
    _check(c._lib.steps_batch_run(c.handle, ctypes.byref(b), status))
    return list(status)


def steps_batch_tile(ctx: Context):
    t = steps_tile()
    _check(ctx._lib.steps_batch_tile(ctx.handle, ctypes.byref(t)))
    return {"r": t.r, "tj": t.tj, "jsplit": t.jsplit, "variant": t.variant}
