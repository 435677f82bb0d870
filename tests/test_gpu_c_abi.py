"""The C ABI from plain C on the GPU: tests/c/abi_demo.c (library-owned
workspaces, null stream) steps a disc in FP64 and FP32, checks the documented
errors, and writes its FP64 fields, which must equal bitwise those of the same
solve through the Python binding (torch workspace and stream)."""
import math
import os
import subprocess

import numpy as np
import pytest

from c_abi_build import build_demo

pytestmark = pytest.mark.gpu


def test_c_program_matches_binding(tmp_path):
    from paper_2110_12448_amd import pfiso
    from paper_2110_12448_amd import workloads as wl
    exe = str(tmp_path / "abi_demo")
    rc, err = build_demo(exe)
    assert rc == 0, err
    out = str(tmp_path / "fields.bin")
    print("gpu case: C ABI demo", flush=True)
    r = subprocess.run([exe, out], capture_output=True, text=True, timeout=100)
    print(r.stdout, r.stderr)
    assert r.returncode == 0
    raw = np.fromfile(out, dtype=np.float64)
    n = 96 * 96
    c_psi, c_U = raw[:n].reshape(96, 96), raw[n:].reshape(96, 96)
    a = 10.0 * math.pi / 180.0
    rot = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0],
                    [0.0, 0.0, 1.0]])[None]
    i = np.arange(96)
    X, Y = np.meshgrid(i * 0.8 - 48 * 0.8, i * 0.8 - 48 * 0.8, indexing="xy")
    prob = dict(dim=2, nx=96, ny=96, nz=1, w=wl.ISO_2D, k=0.15, eps4=0.02, D=2.0, lam=0.0,
                h=0.8, dt=0.8 * 0.64 / 8.0, Vp=0.0, lT=0.0, y0=0.0, bc=(0, 0, 0), frame=0,
                shift_row=0, rot=rot, psi0=8.0 - np.sqrt(X * X + Y * Y),
                U0=np.full((96, 96), -0.55), grain=np.zeros((96, 96), dtype=np.int8),
                antitrapping=0, two_point=0, dynamic_grains=0)
    s = pfiso.Solver(prob, precision=pfiso.PF_F64, scheme=pfiso.PF_SCHEME_ISO)
    s.step(200)
    phi, U, psi, _ = s.read_fields()
    s.close()
    assert np.array_equal(psi, c_psi) and np.array_equal(U, c_U)
