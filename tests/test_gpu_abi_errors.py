"""Argument errors through the C ABI on a GPU host.  Every bad call must be
rejected on the host, before any kernel is enqueued, and write nothing.
Each case leaves a NULL pointer later in the argument list as a backstop,
so a validation bug shows up as the wrong message, never as a launch."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu

VP = ctypes.c_void_p


@pytest.fixture(scope="module")
def st():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1811_05903_amd as m
    m.load()
    return m


def _p(t):
    return VP(t.data_ptr())


def _msg(lib):
    return lib.steps_last_error().decode()


def test_negative_and_huge_n(st):
    lib = st.load()
    assert lib.steps_forces(None, None, None, -1, None) == st.STEPS_E_INVAL
    assert lib.steps_forces(None, None, None, (1 << 30) + 1, None) == st.STEPS_E_INVAL
    assert "2^30" in _msg(lib)


def test_host_pointer_rejected(st):
    lib = st.load()
    host_arr = np.zeros(3 * 64)
    rc = lib.steps_forces(VP(host_arr.ctypes.data), None, None, 64, None)
    assert rc == st.STEPS_E_INVAL
    assert "pos" in _msg(lib)


def test_undersized_allocation_rejected(st):
    # a raw hipMalloc of 4096 bytes claimed to hold 3*200 doubles
    import torch  # noqa: F401  (initialises HIP)
    hip = ctypes.CDLL("libamdhip64.so")
    ptr = VP()
    assert hip.hipMalloc(ctypes.byref(ptr), ctypes.c_size_t(4096)) == 0
    try:
        lib = st.load()
        rc = lib.steps_forces(ptr, None, None, 200, None)
        assert rc == st.STEPS_E_INVAL
        assert "pos needs" in _msg(lib), _msg(lib)
    finally:
        hip.hipFree(ptr)


def test_aliasing_rejected_and_nothing_written(st):
    ps = synth.config(1, n=300)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    lib = st.load()
    rc = lib.steps_forces(_p(p), _p(m), _p(h), 300, _p(p))
    assert rc == st.STEPS_E_INVAL and "overlap" in _msg(lib)
    assert np.array_equal(host(p), ps.pos)


def test_nonfinite_with_flag(st):
    import torch
    ps = synth.config(1, n=300)
    pos = ps.pos.copy()
    pos[1, 17] = math.nan
    ctx = st.Context(0, flags=st.STEPS_CHECK_FINITE)
    acc = torch.full((3, 300), 5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(st.StepsError) as ei:
        st.steps_forces(dev(pos), dev(ps.mass), dev(ps.soft), acc=acc, ctx=ctx)
    assert ei.value.code == st.STEPS_E_NONFINITE
    assert np.all(host(acc) == 5.0)
    ctx.close()


def test_step_bad_cosmology_writes_nothing(st):
    ps = synth.config(1, n=256)
    p, v, m, h = dev(ps.pos), dev(ps.vel), dev(ps.mass), dev(ps.soft)
    acc = st.steps_forces(p, m, h)
    before = host(acc)
    for bad in (dict(H0=-70.0), dict(G=-1.0)):
        kw = dict(H0=70.0, omega_m=0.3, omega_l=0.7)
        kw.update(bad)
        with pytest.raises(st.StepsError) as ei:
            st.steps_step(p, v, m, h, acc, 0.02, 0.001, st.Cosmology(**kw))
        assert ei.value.code == st.STEPS_E_INVAL
    with pytest.raises(st.StepsError):
        st.steps_step(p, v, m, h, acc, 0.02, -0.05, st.Cosmology())  # a+da<0
    with pytest.raises(st.StepsError):
        st.steps_step(p, v, m, h, acc, float("nan"), 0.01, st.Cosmology())
    assert np.array_equal(host(p), ps.pos)
    assert np.array_equal(host(v), ps.vel)
    assert np.array_equal(host(acc), before)


def test_step_overlapping_state_rejected(st):
    ps = synth.config(1, n=128)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    acc = st.steps_forces(p, m, h)
    with pytest.raises(st.StepsError) as ei:
        st.steps_step(p, p, m, h, acc, 0.02, 0.001, st.Cosmology())
    assert ei.value.code == st.STEPS_E_INVAL
    assert np.array_equal(host(p), ps.pos)


def test_bad_tile_rejected(st):
    ctx = st.Context(0)
    for args in ((3, 128, 1, 0), (4, 64, 1, 0), (4, 128, -1, 0),
                 (4, 128, 1025, 0), (4, 128, 1, 5), (1, 128, 1, 14)):
        with pytest.raises(st.StepsError):
            ctx.set_tile(*args)
    # jsplit 0: the forced kernel with the built-in split for each n
    ctx.set_tile(1, 256, 0, 14)
    t = ctx.get_tile(262144)
    assert t["variant"] == 14 and t["jsplit"] > 1
    ctx.set_precision("mixed")
    with pytest.raises(st.StepsError):
        ctx.set_tile(4, 128, 1, 1)   # FP64-only variant
    ctx.set_tile(4, 256, 0, 10)      # the symmetric mixed kernel
    ctx.set_precision("kahan")       # same class: the shape stays valid
    assert ctx.get_tile(262144)["variant"] == 10
    with pytest.raises(st.StepsError):
        ctx.set_tile(1, 256, 0, 14)  # FP64-only variant
    ctx.close()


def test_profile_timing_counts_launches(st):
    ps = synth.config(1, n=1024)
    ctx = st.Context(0, flags=st.STEPS_PROFILE)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    for _ in range(3):
        st.steps_forces(p, m, h, ctx=ctx)
    ms, cnt = ctx.force_timing(reset=True)
    assert cnt == 3 and ms > 0
    assert ctx.force_timing() == (0.0, 0)
    ctx.close()


def test_newer_entry_points_validate_pointers_and_values(st):
    import torch
    lib = st.load()
    ps = synth.config(1, n=200)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    v = torch.zeros_like(p)
    acc = st.steps_forces(p, m, h)
    torch.cuda.synchronize()
    ctx = st.Context(0)
    k = st.Cosmology().to_c()
    d, da = ctypes.c_double(), ctypes.c_double()
    out = (ctypes.c_double * 4)()
    host_arr = np.zeros(3 * 200)
    # kinetic: host velocity, negative n, a <= 0
    assert lib.steps_kinetic_ctx(ctx.handle, VP(host_arr.ctypes.data), _p(m), 200, 1.0, out) \
        == st.STEPS_E_INVAL and "vel" in _msg(lib)
    assert lib.steps_kinetic_ctx(ctx.handle, _p(v), _p(m), -1, 1.0, out) == st.STEPS_E_INVAL
    assert lib.steps_kinetic_ctx(ctx.handle, _p(v), _p(m), 200, 0.0, out) == st.STEPS_E_INVAL
    # adaptive step: host acc, eps <= 0, NULL outputs
    rc = lib.steps_adaptive_dt_ctx(ctx.handle, _p(p), _p(v), _p(h), VP(host_arr.ctypes.data),
                                   200, 0.5, ctypes.byref(k), 1e-2, 1.0,
                                   ctypes.byref(d), ctypes.byref(da))
    assert rc == st.STEPS_E_INVAL and "acc" in _msg(lib)
    rc = lib.steps_adaptive_dt_ctx(ctx.handle, _p(p), _p(v), _p(h), _p(acc), 200, 0.5,
                                   ctypes.byref(k), 0.0, 1.0, ctypes.byref(d), ctypes.byref(da))
    assert rc == st.STEPS_E_INVAL and "eps" in _msg(lib)
    rc = lib.steps_adaptive_dt_ctx(ctx.handle, _p(p), _p(v), _p(h), _p(acc), 200, 0.5,
                                   ctypes.byref(k), 1e-2, 1.0, None, ctypes.byref(da))
    assert rc == st.STEPS_E_INVAL
    # periodic: bad box, unknown rule
    assert lib.steps_ctx_set_periodic(ctx.handle, -5.0, 1) == st.STEPS_E_INVAL
    assert lib.steps_ctx_set_periodic(ctx.handle, 5.0, 7) == st.STEPS_E_INVAL
    # tuned shape that names no kernel
    bad = st.steps_tile(3, 128, 1, 0)
    assert lib.steps_ctx_set_tuned(ctx.handle, 200, ctypes.byref(bad)) == st.STEPS_E_INVAL
    ctx.close()
    assert np.array_equal(host(v), np.zeros_like(ps.pos))


def test_impossible_scratch_allocation_is_reported(st):
    # 2^25 particles with 1024 forced j-splits need 1024 x 3 x 2^25 x 8 B
    # (~825 GB) of partials: hipMalloc fails, STEPS_E_NOMEM is returned
    # before any launch, and the context stays usable
    import torch
    n = 1 << 25
    g = torch.Generator(device="cuda").manual_seed(3)
    p = torch.rand((3, n), dtype=torch.float64, device="cuda", generator=g)
    m = torch.ones(n, dtype=torch.float64, device="cuda")
    h = torch.full((n,), 1e-3, dtype=torch.float64, device="cuda")
    acc = torch.zeros_like(p)
    ctx = st.Context(0, precision="fp64")
    ctx.set_tile(4, 128, 1024, 0)
    with pytest.raises(st.StepsError) as ei:
        st.steps_forces(p, m, h, acc=acc, ctx=ctx)
    assert ei.value.code == st.STEPS_E_NOMEM
    assert "partial-sum" in str(ei.value)
    assert bool((acc == 0).all())
    # a step in that shape fails the same way before its first kick is
    # enqueued: positions, velocities and acc stay as they were
    v = torch.rand((3, n), dtype=torch.float64, device="cuda", generator=g)
    p0, v0 = p.clone(), v.clone()
    acc.fill_(1.0)
    with pytest.raises(st.StepsError) as ei:
        st.steps_step(p, v, m, h, acc, 0.02, 0.001, st.Cosmology(), ctx=ctx)
    assert ei.value.code == st.STEPS_E_NOMEM
    torch.cuda.synchronize()
    assert torch.equal(p, p0) and torch.equal(v, v0)
    assert bool((acc == 1.0).all())
    del p, m, h, acc, v, p0, v0
    torch.cuda.empty_cache()
    ctx.set_tile()                          # back to automatic shapes
    ps = synth.config(1, n=500)
    got = st.steps_forces(dev(ps.pos), dev(ps.mass), dev(ps.soft), ctx=ctx)
    assert bool(torch.isfinite(got).all())
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_symmetric_shape_falls_back_when_scratch_is_short(st, prec):
    # N = 2^18: the automatic shape is a symmetric kernel, whose partial
    # sums take ~2 GB.  With all but ~700 MB of device memory held, that
    # allocation fails before any launch and the call runs the one-sided
    # kernel of the precision (FP64: matrix-core, ~0.43 GB of scratch;
    # mixed: ~0.2 GB) instead, to the same bar
    import torch
    ps = synth.config(2)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    acc = torch.zeros_like(p)
    ctx = st.Context(0, precision=prec)
    assert ctx.get_tile(ps.n)["variant"] == (14 if prec == "fp64" else 10)
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    try:
        hold = torch.empty(free - (700 << 20), dtype=torch.uint8, device="cuda")
    except RuntimeError:
        pytest.skip("could not hold the device memory")
    try:
        # less than the symmetric partials need (24 n Q + 48 C Q (Q - 1) / 2
        # bytes, Q = 171 chunks of C = 1536: 2.15 GB) is left, and more than
        # the one-sided kernel needs
        left = torch.cuda.mem_get_info()[0]
        assert (500 << 20) < left < 1.9e9, left
        st.steps_forces(p, m, h, acc=acc, ctx=ctx)
        torch.cuda.synchronize()
    finally:
        del hold
        torch.cuda.empty_cache()
    ctx.close()
    idx = np.random.default_rng(8).choice(ps.n, 64, replace=False)
    ref = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx)
    err = rel_err(host(acc)[:, idx], ref)
    if prec == "fp64":
        assert err.max() <= 1e-12
    else:
        assert np.median(err) <= 1e-5

