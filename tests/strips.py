"""Oracle references on column strips of a large grid.

One step of the scheme reaches a bounded number of columns (the pull of Eq. (6), the lagged
moments of the axisymmetric source, the Yee update of Eq. (5)), so the oracle run on a strip of
columns as a problem of its own gives the full grid's values away from the strip's cut edges.
The strip keeps every row (axis to outer edge), and its driver centre and ramp start move with
the strip's offset, so that each column sees the same background density and driver as in the
full grid.  This lets full-size GPU runs be checked against the oracle at sizes the oracle
cannot step whole in a test.
"""
import numpy as np

from oracle import lbm_oracle as O

MARGIN = 10   # columns next to a cut edge that are not compared

# Planes of the state view that share a physical scale: density populations, momentum
# populations (n p_z and n p_r lattices), density moment, momentum moments, the three fields.
GROUPS = [range(0, 9), range(9, 27), range(27, 28), range(28, 30), range(30, 33)]


def group_errors(st, ref):
    """Max-norm error of each plane relative to the largest reference value of its group, so
    that a plane that is zero up to round-off in the reference (E_z right after the
    Gauss-consistent initial state, where the discrete curl of B cancels the driver current)
    does not make the norm ill-posed.  Arrays of other than 33 planes form one group."""
    errs = np.zeros(ref.shape[0])
    groups = GROUPS if ref.shape[0] == 33 else [range(ref.shape[0])]
    for g in groups:
        den = max(np.abs(ref[c]).max() for c in g)
        for c in g:
            num = np.abs(st[c] - ref[c]).max()
            errs[c] = num / den if den > 0 else num
    return errs


def strip_config(cfg, c0, w):
    """The strip [c0, c0 + w) of the grid described by cfg."""
    h = cfg["dz"]
    return dict(cfg, nz=w, zd0=cfg["zd0"] - c0 * h, ramp_start=cfg["ramp_start"] - c0 * h)


def state_array(S, P):
    """The 33 planes of an oracle state in the layout of the C ABI's state view."""
    return np.concatenate([S.g.reshape(27, P.nr, P.nz).numpy(), S.M.numpy(),
                           np.stack([S.Ez.numpy(), S.Er.numpy(), S.B.numpy()])])


def strip_reference(cfg, c0, w, k0, margin=MARGIN):
    """One oracle step of the strip [c0, c0 + w) from the initial state with the step counter at
    k0.  Returns (reference planes, first column, end column) in the full grid's window order:
    the cut edges lose `margin` columns, the grid's own edges none."""
    nz = cfg["nz"]
    P = O.Params(strip_config(cfg, c0, w))
    S = O.initial_state(P)
    S.k = k0
    S = O.step(S, P)
    lo = margin if c0 > 0 else 0
    hi = w if c0 + w == nz else w - margin
    return state_array(S, P)[:, :, lo:hi], c0 + lo, c0 + hi
