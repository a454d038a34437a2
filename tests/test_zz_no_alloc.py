"""lbm_diagnostics_noalloc (partial sums in the library's fixed device array) against
lbm_diagnostics (partial sums in the context's workspace): bit for bit, through the C ABI, on two
calls in a row, the second on a smaller lattice, then again on the first."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _lattice(nz, nr, steps, **extra):
    from paper_2201_05473_amd import Lattice
    cfg = wl.config(None, nz=nz, nr=nr, dz=0.05, dr=0.05, moving_window=1, nb=0.2, sigma_z=0.3,
                    sigma_r=0.3, zd0=nz * 0.05 - 1.5, ramp_kind=2, ramp_start=nz * 0.05 - 3.0,
                    ramp_len=1.0, noise_amp=1e-3, seed=9, **extra)
    lat = Lattice(cfg, wl.density_perturbation(cfg))
    lat.step(steps)
    return lat


def _check(lat):
    from paper_2201_05473_amd.binding import lbm_diagnostics, lbm_diagnostics_noalloc
    ref = lbm_diagnostics(lat.ctx)
    got = lbm_diagnostics_noalloc(lat.ctx)
    print("[no-alloc]", lat.nz, lat.nr, ref, flush=True)
    assert got == ref, (got, ref)
    assert ref["charge"] > 0.0 and ref["field_energy"] > 0.0 and ref["nonfinite"] == 0


@pytest.mark.parametrize("storage", [wl.F64, wl.F32])
def test_noalloc_diagnostics_match(storage):
    # 1,200 x 300 = 360,000 sites: 1,407 blocks of 256 sites (below the 2,048 the scratch holds)
    big = _lattice(1200, 300, 12, storage=storage)
    _check(big)
    # smaller lattice second: the scratch keeps the first call's partials beyond its blocks
    small = _lattice(70, 9, 7, storage=storage)
    _check(small)
    # a lattice that needs the stride (4096 x 256 = 4,096 blocks' worth of sites), then the first
    # one again after more steps
    strided = _lattice(4096, 256, 3, storage=storage)
    _check(strided)
    big.step(5)
    _check(big)
    for lat in (big, small, strided):
        lat.close()
