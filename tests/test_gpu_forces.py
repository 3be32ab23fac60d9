"""GPU parity of the force kernels (C ABI) against the FP64 oracle.

FP64 bar: per-particle relative force error <= 1e-12.  Mixed bar: median
relative error <= 1e-5 (the max is printed)."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import clustered, dev, host, rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


@pytest.fixture(scope="module")
def st():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1811_05903_amd as m
    m.load()
    return m


def _report(name, err):
    print("%s: n=%d median %.3e max %.3e" % (name, err.size, np.median(err),
                                            err.max()), flush=True)


def _gpu_forces(st, pos, mass, soft, ctx=None):
    return host(st.steps_forces(dev(pos), dev(mass), dev(soft), ctx=ctx))


@pytest.mark.parametrize("n", [2, 3, 17, 255, 256, 257, 1000, 5001])
def test_fp64_small_sets(st, n):
    ps = synth.config(1, n=n)
    ref = oracle.forces(ps.pos, ps.mass, ps.soft)
    got = _gpu_forces(st, ps.pos, ps.mass, ps.soft)
    err = rel_err(got, ref)
    _report("fp64 n=%d" % n, err)
    assert err.max() <= FP64_TOL


def test_n_zero_and_one(st):
    import torch
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    st.steps_forces(e, torch.empty(0, dtype=torch.float64, device="cuda"),
                    torch.empty(0, dtype=torch.float64, device="cuda"), acc=e)
    acc = torch.full((3, 1), 7.0, dtype=torch.float64, device="cuda")
    st.steps_forces(dev(np.ones((3, 1))), dev(np.ones(1)), dev(np.ones(1)), acc=acc)
    assert np.all(host(acc) == 0.0)


@pytest.mark.parametrize("zero_soft", [0.0, 0.3])
def test_fp64_softened_and_coincident(st, zero_soft):
    pos, mass, soft = clustered(3000, 17, zero_soft)
    ref = oracle.forces(pos, mass, soft)
    got = _gpu_forces(st, pos, mass, soft)
    err = rel_err(got, ref)
    _report("fp64 clustered zero_soft=%g" % zero_soft, err)
    assert np.all(np.isfinite(got))
    assert err.max() <= FP64_TOL


def _variants(st):
    out = []
    for prec in ("fp64", "mixed", "kahan"):
        ctx = st.Context(0, precision=prec)
        for r in (1, 2, 4, 8):
            for tj in (128, 256):
                for var in (0, 1, 2, 3, 6, 10, 14, 26, 30):
                    for js in (1, 3, 7):
                        try:
                            ctx.set_tile(r, tj, js, var)
                        except st.StepsError:
                            continue
                        out.append((prec, r, tj, var, js))
        ctx.close()
    return out


def test_every_launch_shape(st):
    # ragged n (not a multiple of any tile or block), several j-splits
    pos, mass, soft = clustered(1537, 23, 0.1)
    ref = oracle.forces(pos, mass, soft)
    shapes = _variants(st)
    # FP64: 4 r x 4 variants + two matrix-core tiles + the two symmetric
    # ones; mixed and Kahan: 4 r x 2 variants + the symmetric one, plain and
    # with the Newton step, at r = 2 and 4; 3 splits each (for the symmetric
    # kernels 1, 3 and 7 chunks, the last one a single particle)
    assert len(shapes) == (20 + 12 + 12) * 3
    ctxs = {p: st.Context(0, precision=p) for p in ("fp64", "mixed", "kahan")}
    for prec, r, tj, var, js in shapes:
        ctx = ctxs[prec]
        ctx.set_tile(r, tj, js, var)
        got = _gpu_forces(st, pos, mass, soft, ctx=ctx)
        err = rel_err(got, ref)
        tag = "%s r=%d tj=%d var=%d js=%d" % (prec, r, tj, var, js)
        if prec == "fp64":
            assert err.max() <= FP64_TOL, (tag, err.max())
        else:
            assert np.median(err) <= 1e-5, (tag, np.median(err))
            assert err.max() <= 1e-3, (tag, err.max())
    for c in ctxs.values():
        c.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_picks_a_compiled_shape_and_keeps_parity(st, prec, tmp_path):
    ps = synth.config(2, n=40000)
    ctx = st.Context(0, precision=prec)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    cache = str(tmp_path / "tune.json")
    tile = st.steps_autotune(p, m, h, ctx, cache=cache)
    assert tile["r"] in (1, 2, 4) and tile["jsplit"] >= 1
    assert ctx.get_tile(ps.n) == tile          # remembered for this n
    # a fresh context restores the shape from the file without timing
    ctx2 = st.Context(0, precision=prec)
    assert st.steps_autotune(p, m, h, ctx2, cache=cache) == tile
    assert ctx2.get_tile(ps.n) == tile
    ctx2.close()
    got = host(st.steps_forces(p, m, h, ctx=ctx))
    ctx.close()
    idx = np.random.default_rng(9).choice(ps.n, 64, replace=False)
    err = rel_err(got[:, idx], oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx))
    if prec == "fp64":
        assert err.max() <= FP64_TOL
    else:
        assert np.median(err) <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_full_size_includes_symmetric(st, prec, tmp_path):
    # at N = 2^18 the candidates include the symmetric kernel of the
    # precision (variant 14 or 10, chunk counts Q/2 and Q); the tuned shape
    # keeps parity on sampled rows
    ps = synth.config(2)
    ctx = st.Context(0, precision=prec)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    tile = st.steps_autotune(p, m, h, ctx, cache=str(tmp_path / "t.json"))
    print("tuned at 2^18 (%s):" % prec, tile, flush=True)
    assert tile["variant"] in ((0, 3, 6, 14, 30) if prec == "fp64" else (0, 2, 10, 26))
    got = host(st.steps_forces(p, m, h, ctx=ctx))
    ctx.close()
    idx = np.random.default_rng(11).choice(ps.n, 128, replace=False)
    err = rel_err(got[:, idx], oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx))
    if prec == "fp64":
        assert err.max() <= FP64_TOL
    else:
        assert np.median(err) <= 1e-5


@pytest.mark.parametrize("tj", [128, 256])
@pytest.mark.parametrize("n", [40000, None])
def test_matrix_core_kernel_parity(st, n, tj):
    # the matrix-core FP64 kernel (variant 6) on stereographic sets large
    # enough that most (wave, tile) blocks take the Gram path: all rows at
    # n = 40000, 256 sampled rows at N = 2^18
    ps = synth.config(2, n=n) if n else synth.config(2)
    ctx = st.Context(0, precision="fp64")
    ctx.set_tile(1, tj, 16, 6)
    got = _gpu_forces(st, ps.pos, ps.mass, ps.soft, ctx)
    again = _gpu_forces(st, ps.pos, ps.mass, ps.soft, ctx)
    ctx.close()
    assert np.array_equal(got, again)
    idx = np.arange(ps.n) if n else \
        np.random.default_rng(4).choice(ps.n, 256, replace=False)
    err = rel_err(got[:, idx], oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx))
    _report("fp64 matrix-core tj=%d n=%d" % (tj, ps.n), err)
    assert err.max() <= FP64_TOL


@pytest.mark.parametrize("q", [2, 3, 8, 0])
@pytest.mark.parametrize("kind", ["stereo", "clustered"])
@pytest.mark.parametrize("var", [14, 30])
def test_symmetric_kernel_parity(st, kind, q, var):
    # variants 14 and 30 (two lane layouts of the far blocks): each pair
    # between two chunks evaluated once and applied to both particles.
    # Ragged n; q chunks (0: the built-in count); the clustered set puts near
    # and softened blocks between chunks (the direct loop of the j-side), the
    # stereographic one mostly matrix-core blocks
    if kind == "stereo":
        ps = synth.config(2, n=20001)
        pos, mass, soft = ps.pos, ps.mass, ps.soft
    else:
        pos, mass, soft = clustered(9000, 37, 0.1)
    ctx = st.Context(0, precision="fp64")
    ctx.set_tile(1, 256, q, var)
    got = _gpu_forces(st, pos, mass, soft, ctx)
    again = _gpu_forces(st, pos, mass, soft, ctx)
    tile = ctx.get_tile(mass.size)
    ctx.close()
    assert np.array_equal(got, again)
    assert tile["variant"] == var and tile["jsplit"] >= 1
    err = rel_err(got, oracle.forces(pos, mass, soft))
    _report("fp64 symmetric v%d %s q=%d (jsplit %d)" % (var, kind, q, tile["jsplit"]), err)
    assert np.all(np.isfinite(got))
    assert err.max() <= FP64_TOL


@pytest.mark.parametrize("r,q", [(2, 2), (4, 3), (2, 8), (4, 0)])
@pytest.mark.parametrize("kind", ["stereo", "clustered"])
@pytest.mark.parametrize("prec", ["mixed", "kahan"])
@pytest.mark.parametrize("var", [10, 26])
def test_symmetric_mixed_kernel_parity(st, prec, kind, r, q, var):
    # variants 10 and 26 (the latter with a Newton step on r^-3): FP32 pairs,
    # one weight per pair for both particles, FP64 or Kahan FP32
    # accumulation; ragged n, q chunks (0: the built-in count), r particles
    # per lane; the clustered set has softened and coincident pairs between
    # chunks.  Mixed bar, and bitwise repeats
    if kind == "stereo":
        ps = synth.config(2, n=20001)
        pos, mass, soft = ps.pos, ps.mass, ps.soft
    else:
        pos, mass, soft = clustered(9000, 37, 0.1)
    ctx = st.Context(0, precision=prec)
    ctx.set_tile(r, 256, q, var)
    got = _gpu_forces(st, pos, mass, soft, ctx)
    again = _gpu_forces(st, pos, mass, soft, ctx)
    tile = ctx.get_tile(mass.size)
    ctx.close()
    assert np.array_equal(got, again)
    assert tile["variant"] == var
    err = rel_err(got, oracle.forces(pos, mass, soft))
    _report("%s symmetric v%d %s r=%d q=%d (jsplit %d)"
            % (prec, var, kind, r, q, tile["jsplit"]), err)
    assert np.all(np.isfinite(got))
    assert np.median(err) <= 1e-5
    assert err.max() <= 1e-3


@pytest.mark.parametrize("prec", ["mixed", "kahan"])
def test_symmetric_mixed_default_full_size_sampled(st, prec):
    # N = 2^18 + 37 in the default mixed shape (the symmetric kernel, ragged
    # last chunk); the last 40 rows and 216 others
    n = 262144 + 37
    ps = synth.config(2, n=n)
    ctx = st.Context(0, precision=prec)
    assert ctx.get_tile(n)["variant"] == 10
    got = _gpu_forces(st, ps.pos, ps.mass, ps.soft, ctx)
    ctx.close()
    rng = np.random.default_rng(7)
    idx = np.concatenate([np.arange(n - 40, n), rng.choice(n - 40, 216, replace=False)])
    err = rel_err(got[:, idx], oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx))
    _report("%s symmetric ragged n=%d" % (prec, n), err)
    assert np.median(err) <= 1e-5
    assert err.max() <= 1e-3


def test_symmetric_kernel_ragged_default_shape(st):
    # N = 2^18 + 37 in the default shape (the symmetric kernel with a ragged
    # last chunk and a partial last tile); the last 40 rows and 88 others
    n = 262144 + 37
    ps = synth.config(2, n=n)
    ctx = st.Context(0, precision="fp64")
    assert ctx.get_tile(n)["variant"] in (14, 30)
    got = _gpu_forces(st, ps.pos, ps.mass, ps.soft, ctx)
    ctx.close()
    rng = np.random.default_rng(6)
    idx = np.concatenate([np.arange(n - 40, n), rng.choice(n - 40, 88, replace=False)])
    err = rel_err(got[:, idx], oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx))
    _report("fp64 symmetric ragged n=%d" % n, err)
    assert err.max() <= FP64_TOL


@pytest.mark.parametrize("var", [14, 30])
def test_symmetric_kernel_full_size_sampled(st, var):
    # N = 2^18 with the built-in chunk count; oracle on 256 sampled rows
    ps = synth.config(2)
    ctx = st.Context(0, precision="fp64")
    ctx.set_tile(1, 256, 0, var)
    got = _gpu_forces(st, ps.pos, ps.mass, ps.soft, ctx)
    ctx.close()
    idx = np.random.default_rng(5).choice(ps.n, 256, replace=False)
    err = rel_err(got[:, idx], oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx))
    _report("fp64 symmetric v%d config2 sampled" % var, err)
    assert err.max() <= FP64_TOL


def test_determinism_bitwise(st):
    ps = synth.config(1, n=4096)
    for prec in ("fp64", "mixed", "kahan"):
        ctx = st.Context(0, precision=prec)
        a = _gpu_forces(st, ps.pos, ps.mass, ps.soft, ctx)
        b = _gpu_forces(st, ps.pos, ps.mass, ps.soft, ctx)
        assert np.array_equal(a, b), prec
        ctx.close()


def test_context_on_user_streams(st):
    # one context on two user streams in turn, the second call larger so that
    # its scratch is reallocated after the stream switch: oracle parity on the
    # first, and the second equal bitwise to the same call on the null stream
    import torch
    small, big = synth.config(1, n=3000), synth.config(2, n=40000)
    ps_, ms_, hs_ = dev(small.pos), dev(small.mass), dev(small.soft)
    pb, mb, hb = dev(big.pos), dev(big.mass), dev(big.soft)
    null_ctx = st.Context(0, precision="fp64")
    want = host(st.steps_forces(pb, mb, hb, ctx=null_ctx))
    null_ctx.close()
    torch.cuda.synchronize()
    ctx = st.Context(0, precision="fp64")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        a = st.steps_forces(ps_, ms_, hs_, ctx=ctx)
    with torch.cuda.stream(s2):
        b = st.steps_forces(pb, mb, hb, ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    err = rel_err(host(a), oracle.forces(small.pos, small.mass, small.soft))
    assert err.max() <= FP64_TOL
    assert np.array_equal(host(b), want)


def test_default_context_c_entry_point(st):
    # steps_forces (no ctx) through the raw C symbol on the null stream
    import torch
    ps = synth.config(1, n=700)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    acc = torch.zeros((3, 700), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    rc = st.load().steps_forces(ctypes.c_void_p(p.data_ptr()),
                                ctypes.c_void_p(m.data_ptr()),
                                ctypes.c_void_p(h.data_ptr()), 700,
                                ctypes.c_void_p(acc.data_ptr()))
    assert rc == 0
    torch.cuda.synchronize()
    err = rel_err(host(acc), oracle.forces(ps.pos, ps.mass, ps.soft))
    assert err.max() <= FP64_TOL


@pytest.mark.parametrize("prec", ["mixed", "kahan"])
def test_mixed_config1(st, prec):
    ps = synth.config(1, n=4096)
    ref = oracle.forces(ps.pos, ps.mass, ps.soft)
    ctx = st.Context(0, precision=prec)
    got = _gpu_forces(st, ps.pos, ps.mass, ps.soft, ctx)
    ctx.close()
    err = rel_err(got, ref)
    _report("%s config1" % prec, err)
    assert np.median(err) <= 1e-5


def test_full_size_config2_sampled(st):
    # N = 2^18 in the default launch shape; oracle on 256 sampled particles
    ps = synth.config(2)
    got = _gpu_forces(st, ps.pos, ps.mass, ps.soft)
    idx = np.random.default_rng(2).choice(ps.n, 256, replace=False)
    ref = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx)
    err = rel_err(got[:, idx], ref)
    _report("fp64 config2 sampled", err)
    assert err.max() <= FP64_TOL


def test_full_size_config3_sampled_all_modes(st):
    # N = 2^21, default launch shapes; oracle on 64 sampled particles
    ps = synth.config(3)
    idx = np.random.default_rng(3).choice(ps.n, 64, replace=False)
    ref = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    for prec in ("fp64", "mixed", "kahan"):
        ctx = st.Context(0, precision=prec)
        got = host(st.steps_forces(p, m, h, ctx=ctx))[:, idx]
        ctx.close()
        err = rel_err(got, ref)
        _report("%s config3 sampled" % prec, err)
        if prec == "fp64":
            assert err.max() <= FP64_TOL
        else:
            assert np.median(err) <= 1e-5


def test_full_size_config5_sampled_all_modes(st):
    # N = 2^22 (the largest workload), default launch shapes; oracle on 64
    # sampled particles
    ps = synth.config(5)
    idx = np.random.default_rng(5).choice(ps.n, 64, replace=False)
    ref = oracle.forces(ps.pos, ps.mass, ps.soft, idx=idx)
    p, m, h = dev(ps.pos), dev(ps.mass), dev(ps.soft)
    for prec in ("fp64", "mixed", "kahan"):
        print("config5 %s" % prec, flush=True)
        ctx = st.Context(0, precision=prec)
        got = host(st.steps_forces(p, m, h, ctx=ctx))[:, idx]
        tile = ctx.get_tile(ps.n)
        ctx.close()
        err = rel_err(got, ref)
        _report("%s config5 sampled %s" % (prec, tile), err)
        if prec == "fp64":
            assert err.max() <= FP64_TOL
        else:
            assert np.median(err) <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pair_momentum_vanishes(st, prec):
    # Eq. 8's pair sum is antisymmetric (Newton's third law), so
    # sum_i m_i S_i = 0 up to rounding; the bound is relative to the
    # magnitude sum_i m_i |S_i|, on a clustered set that exercises every
    # kernel branch and the culled fast loop.
    pos, mass, soft = clustered(6000, 41, 0.1)
    ctx = st.Context(0, precision=prec)
    got = _gpu_forces(st, pos, mass, soft, ctx)
    ctx.close()
    net = np.abs((mass * got).sum(axis=1))
    scale = (mass * np.abs(got)).sum(axis=1)
    rel = (net / scale).max()
    print("%s pair momentum %.3e" % (prec, rel), flush=True)
    assert rel <= (1e-13 if prec == "fp64" else 1e-5)


def test_potential_parity(st):
    pos, mass, soft = clustered(2000, 31, 0.2)
    ref = oracle.potential(pos, mass, soft)
    got = host(st.steps_potential(dev(pos), dev(mass), dev(soft)))
    err = np.abs(got - ref) / np.abs(ref)
    _report("potential", err)
    assert err.max() <= FP64_TOL
