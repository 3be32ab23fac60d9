"""CPU-side checks of the C ABI: libsteps.so loads, exports every function
include/steps.h declares, and its host-only entry points (background
cosmology, argument validation) behave -- no device compute is called."""
import ctypes
import math
import os
import re

import pytest

import oracle
import paper_1811_05903_amd as st
from paper_1811_05903_amd import build as stbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "steps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(steps_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(st.LIB_PATH):
        stbuild.build()
    return st.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert len(declared) >= 20
    assert sorted(st.EXPORTS) == declared
    raw = ctypes.CDLL(st.LIB_PATH)
    for name in declared:
        assert hasattr(raw, name), name


def test_version(lib):
    assert "gfx950" in st.steps_version()


def test_constants_agree_with_oracle(lib):
    assert st.steps_G() == pytest.approx(oracle.G(), rel=1e-15)
    assert st.steps_kms_to_mpc_per_gyr() == pytest.approx(
        oracle.kms_to_mpc_per_gyr(), rel=1e-15)


@pytest.mark.parametrize("a,da", [(0.02, 0.98), (0.02, 1e-4), (0.5, -0.3),
                                  (0.1, 0.9)])
def test_library_dt_closed_form_and_oracle(lib, a, da):
    kms = st.steps_kms_to_mpc_per_gyr()
    om, ol, h0 = 0.3089, 0.6911, 67.74 * kms
    t = lambda x: 2 / (3 * h0 * math.sqrt(ol)) * math.asinh(math.sqrt(ol / om) * x ** 1.5)
    got = st.steps_dt(st.Cosmology(67.74, om, ol), a, da)
    assert got == pytest.approx(t(a + da) - t(a), rel=1e-13)
    ref = oracle.dt(a, da, oracle.Cosmology(67.74, om, ol))
    assert got == pytest.approx(ref, rel=1e-13)


def test_library_dt_curved_radiation(lib):
    c = st.Cosmology(70.0, 0.25, 0.5, omega_r=1e-4)   # open + radiation
    oc = oracle.Cosmology(70.0, 0.25, 0.5, omega_r=1e-4)
    for a, da in [(0.01, 0.5), (0.3, 0.7)]:
        assert st.steps_dt(c, a, da) == pytest.approx(oracle.dt(a, da, oc), rel=1e-13)
    for a in (0.05, 1.0, 3.0):
        assert st.steps_hubble(c, a) == pytest.approx(oracle.hubble(a, oc), rel=1e-14)


def test_newtonian_mode_dt_is_da(lib):
    c = st.Cosmology(newtonian_test=True)
    assert st.steps_dt(c, 3.0, 0.25) == 0.25
    assert st.steps_hubble(c, 1.0) == 0.0


@pytest.mark.parametrize("bad", [
    dict(H0=-1.0), dict(H0=float("nan")), dict(G=-1.0),
    dict(omega_m=float("inf")),
])
def test_invalid_cosmology_rejected(lib, bad):
    kw = dict(H0=70.0, omega_m=0.3, omega_l=0.7)
    kw.update(bad)
    with pytest.raises(st.StepsError) as ei:
        st.steps_dt(st.Cosmology(**kw), 0.1, 0.1)
    assert ei.value.code == st.STEPS_E_INVAL


def test_negative_h2_rejected(lib):
    # closed universe with a turnaround: H^2 < 0 at large a
    c = st.Cosmology(70.0, 2.0, 0.0, omega_k=-1.0)
    with pytest.raises(st.StepsError) as ei:
        st.steps_dt(c, 0.5, 2.0)
    assert ei.value.code == st.STEPS_E_INVAL
    with pytest.raises(st.StepsError):
        st.steps_dt(st.Cosmology(70.0, 0.3, 0.7), 0.1, -0.2)   # a + da <= 0


def test_bad_mode_and_flags(lib):
    k = st.Cosmology().to_c()
    k.mode = 7
    out = ctypes.c_double()
    assert lib.steps_dt(ctypes.byref(k), 0.1, 0.1, ctypes.byref(out)) == st.STEPS_E_INVAL
    k = st.Cosmology().to_c()
    k.flags = 2
    assert lib.steps_dt(ctypes.byref(k), 0.1, 0.1, ctypes.byref(out)) == st.STEPS_E_INVAL
    assert b"flag" in lib.steps_last_error()
    # reversed gravity leaves the background (H, dt) as it is
    ref = ctypes.c_double()
    k = st.Cosmology().to_c()
    assert lib.steps_dt(ctypes.byref(k), 0.1, 0.1, ctypes.byref(ref)) == st.STEPS_OK
    k.flags = st.STEPS_REVERSED_GRAVITY
    assert lib.steps_dt(ctypes.byref(k), 0.1, 0.1, ctypes.byref(out)) == st.STEPS_OK
    assert out.value == ref.value


def test_null_arguments_rejected_before_device_use(lib):
    assert lib.steps_ctx_create(0, None) == st.STEPS_E_INVAL
    assert lib.steps_ctx_set_precision(None, 0) == st.STEPS_E_INVAL
    assert lib.steps_sync(None) == st.STEPS_E_INVAL
    assert lib.steps_ctx_destroy(None) == st.STEPS_OK
    assert lib.steps_forces_ctx(None, None, None, None, 4, None) == st.STEPS_E_INVAL


def test_null_context_rejected_by_newer_entry_points(lib):
    d = ctypes.c_double()
    i64 = ctypes.c_int64()
    k = st.Cosmology().to_c()
    t = st.steps_tile(1, 128, 1, 0)
    out = (ctypes.c_double * 7)()
    E = st.STEPS_E_INVAL
    assert lib.steps_kinetic_ctx(None, None, None, 4, 1.0, out) == E
    assert lib.steps_energy_ctx(None, None, None, None, None, 4, 1.0, ctypes.byref(k), out) == E
    assert lib.steps_adaptive_dt_ctx(None, None, None, None, None, 4, 1.0, ctypes.byref(k),
                                     1e-2, 1.0, ctypes.byref(d), ctypes.byref(d)) == E
    assert lib.steps_run_adaptive_ctx(None, None, None, None, None, 4, None, 0.1, 0.2,
                                      ctypes.byref(k), 1e-2, 1.0, 10, ctypes.byref(i64),
                                      ctypes.byref(d)) == E
    assert lib.steps_ctx_set_periodic(None, 10.0, 1) == E
    assert lib.steps_ctx_set_tuned(None, 100, ctypes.byref(t)) == E
    assert lib.steps_autotune(None, None, None, None, 4, None, ctypes.byref(t)) == E
    assert lib.steps_batch_tile(None, ctypes.byref(t)) == E
