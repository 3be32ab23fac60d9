"""The C ABI from plain C: tests/c_client/steps_client.c is built with gcc
against include/steps.h and libsteps.so, run as a child process, and its
results compared with the oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1811_05903_amd")


def test_plain_c_client(tmp_path):
    exe = str(tmp_path / "steps_client")
    build = subprocess.run(
        ["gcc", "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
         "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
         os.path.join(ROOT, "tests", "c_client", "steps_client.c"), "-o", exe,
         "-L" + PKG, "-lsteps", "-L/opt/rocm/lib", "-lamdhip64",
         "-Wl,-rpath," + PKG, "-Wl,-rpath,/opt/rocm/lib"],
        capture_output=True, text=True, timeout=120)
    assert build.returncode == 0, build.stderr
    out = str(tmp_path / "out.bin")
    run = subprocess.run([exe, "2000", out], capture_output=True, text=True, timeout=120)
    print(run.stdout, run.stderr)
    assert run.returncode == 0, run.stderr
    raw = open(out, "rb").read()
    n = int(np.frombuffer(raw[:8], dtype=np.int64)[0])
    d = np.frombuffer(raw[8:], dtype=np.float64)
    cut = np.cumsum([0, 3 * n, 3 * n, n, n, 3 * n, 5, 3 * n, 3 * n, 3 * n])
    pos, vel, mass, soft, S0, scal, pos1, vel1, S1 = (
        d[cut[k]:cut[k + 1]] for k in range(9))
    pos, vel, S0 = pos.reshape(3, n), vel.reshape(3, n), S0.reshape(3, n)
    pos1, vel1, S1 = pos1.reshape(3, n), vel1.reshape(3, n), S1.reshape(3, n)
    ref = oracle.forces(pos, mass, soft)
    rel = np.linalg.norm(S0 - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert rel.max() <= 1e-12
    a, da, H0, om, ol = scal
    c = oracle.Cosmology(H0=H0, omega_m=om, omega_l=ol, omega_k=0.0)
    p, v, S = pos.copy(), vel.copy(), ref.copy()
    oracle.kdk_step(p, v, mass, soft, S, a, da, c)
    assert np.max(np.abs(pos1 - p) / soft) < 1e-12
    relv = np.linalg.norm(vel1 - v, axis=0) / np.linalg.norm(v, axis=0)
    assert relv.max() < 1e-12
    rels = np.linalg.norm(S1 - S, axis=0) / np.linalg.norm(S, axis=0)
    assert rels.max() <= 1e-12
