"""The C ABI driven from plain C (tests/c_api/lbm_c_run.c, built by build()), with no Python
between the caller and the library: its diagnostics and on-axis E_z after 40 steps of C1's grid
and driver (no density noise) equal, bit for bit, those of the same run through the ctypes
binding, and in FP64 the oracle's to 1e-10."""
import json
import os
import subprocess

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import lbm_oracle as O

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2201_05473_amd", "_lib", "lbm_c_run")
KEYS = ("charge", "field_energy", "gauss_max", "umax")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2201_05473_amd import load_library
    load_library()


@pytest.mark.parametrize("storage", [wl.F64, wl.F32, wl.F16N])
def test_c_client_matches_binding_and_oracle(storage):
    if not os.path.exists(EXE):   # build() makes it; a host-only gcc line of under a second
        from paper_2201_05473_amd.build import build_c_client
        build_c_client()
    print(f"[c api] storage={storage}, 40 steps", flush=True)
    out = subprocess.run([EXE, "40", str(storage)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    c = json.loads(out.stdout)
    from paper_2201_05473_amd import Lattice
    cfg = wl.config("C1", noise_amp=0.0, storage=storage)
    lat = Lattice(cfg)
    lat.step(40)
    d = lat.diagnostics()
    ez = lat.fields()[0].cpu().numpy()
    lat.close()
    assert (c["step"], c["shifts"], c["nonfinite"]) == (d["step"], d["shifts"], 0)
    for key in KEYS:
        assert c[key] == d[key], key
    assert c["ez_axis"] == [float(ez[0, 40]), float(ez[0, 80]), float(ez[0, 120])]
    if storage == wl.F64:
        S, P = O.run(cfg, 40)
        r = O.diagnostics(S, P)
        for key in ("charge", "field_energy", "umax"):
            assert abs(c[key] - r[key]) <= 1e-10 * abs(r[key]), key
        ref = S.Ez.numpy()[0, [40, 80, 120]]
        assert np.abs(np.array(c["ez_axis"]) - ref).max() <= 1e-10 * np.abs(S.Ez.numpy()).max()
