"""The strip references used by the full-size GPU tests, checked against whole-grid oracle steps:
on C2's 512 x 128 copy (and on C3's physics on a 512 x 96 grid), a strip stepped as a problem of
its own reproduces the whole grid's step at every compared column, for a plain step and for a
window-shift step, at the grid's front and rear edges and around the driver."""
import numpy as np
import pytest

import workloads as wl
from oracle import lbm_oracle as O
from strips import MARGIN, group_errors, state_array, strip_reference


def whole_step(cfg, k0):
    P = O.Params(cfg)
    S = O.initial_state(P)
    S.k = k0
    return state_array(O.step(S, P), P)


CASES = {
    "C2s": wl.config("C2s", storage=wl.F64),
    # C3's driver and ramp (n_b = 1, sigma = 0.3, ramp just ahead of the driver) on a short grid
    "C3_short": dict(wl.config("C3", storage=wl.F64), nz=512, nr=96,
                     zd0=512 * 0.02 - 4.0, ramp_start=512 * 0.02 - 2.8),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("k0", [0, 4])
def test_strip_reference_matches_whole_grid(name, k0):
    cfg = CASES[name]
    nz = cfg["nz"]
    full = whole_step(cfg, k0)
    driver_col = int(round(cfg["zd0"] / cfg["dz"]))
    strips = ((nz - 96, 96), (0, 48), (driver_col - 40, 80))
    for c0, w in strips:
        ref, a, b = strip_reference(cfg, c0, w, k0)
        assert b - a >= w - 2 * MARGIN
        got = full[:, :, a:b]
        err = group_errors(ref, got).max()
        assert err < 1e-12, (name, k0, c0, err)
        # the strips are not trivial: plasma or driver field inside each compared part
        if c0 != 0:
            assert np.abs(got[27:33]).max() > 1e-6
