"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test names the pin it implements; together they are chosen so that a plausible mistake in
the oracle (a coefficient, a sign, an index, a time level, a boundary rule) fails at least one.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import lbm_oracle as O
from oracle import scalar_ref as SR
from oracle import units as U

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F64 = torch.float64


def _run(cfg, nsteps, n_pert=None, p_init=None):
    P = O.Params(cfg)
    S = O.initial_state(P, n_pert, p_init)
    for _ in range(nsteps):
        S = O.step(S, P)
    return S, P


# ---------------------------------------------------------------------------------------------
# P_eq: equilibrium moments (Eq. (8), Eq. (9) under reading R1, D2Q9 set R4)
# ---------------------------------------------------------------------------------------------

def test_equilibrium_moments():
    g = torch.Generator().manual_seed(0)
    A = torch.rand(200, generator=g, dtype=F64) * 3
    uz = (torch.rand(200, generator=g, dtype=F64) - 0.5) * 0.4
    ur = (torch.rand(200, generator=g, dtype=F64) - 0.5) * 0.4
    f = O.equilibrium(A, uz, ur)
    xz = torch.tensor([x[0] for x in O.XI], dtype=F64)[:, None]
    xr = torch.tensor([x[1] for x in O.XI], dtype=F64)[:, None]
    assert torch.allclose(f.sum(0), A, rtol=0, atol=1e-14)
    assert torch.allclose((xz * f).sum(0), A * uz, rtol=0, atol=1e-14)
    assert torch.allclose((xr * f).sum(0), A * ur, rtol=0, atol=1e-14)
    # second moments A (c_s^2 I + u u) with c_s^2 = 1/3 (consistent with Eq. (12))
    assert torch.allclose((xz * xz * f).sum(0), A * (1 / 3 + uz * uz), rtol=0, atol=1e-14)
    assert torch.allclose((xr * xr * f).sum(0), A * (1 / 3 + ur * ur), rtol=0, atol=1e-14)
    assert torch.allclose((xz * xr * f).sum(0), A * uz * ur, rtol=0, atol=1e-14)
    assert abs(sum(O.W) - 1.0) < 1e-15


def test_printed_equilibrium_coefficients_violate_moments():
    """Reading R1: Eq. (9) as printed (1/3, 1/18, 1/6) does not return A u as its first moment,
    contradicting Eq. (8); this is why the standard coefficients are used."""
    A, uz = 1.0, 0.1
    f = [w * A * (1 + xz * uz / 3 + (xz * uz) ** 2 / 18 - uz * uz / 6) for (xz, _), w in zip(O.XI, O.W)]
    first = sum(xz * fi for (xz, _), fi in zip(O.XI, f))
    assert abs(first - A * uz) > 0.5 * A * uz


# ---------------------------------------------------------------------------------------------
# P_brute: vectorised oracle vs the scalar per-site loop
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("variant", [
    dict(),
    dict(moving_window=1),
    dict(periodic=1),
    dict(periodic=3, fields_on=0, cyl_on=0),
    dict(ramp_kind=2, ramp_start=0.1, ramp_len=0.2, moving_window=1),
    dict(ramp_kind=1, ramp_start=0.3, ramp_len=0.3, n_floor=1e-3),
    dict(collision=1, trt_magic=0.1, moving_window=1),
    dict(collision=2, ramp_kind=2, ramp_start=0.1, ramp_len=0.2),
    dict(collision=3, mrt_se=1.3, mrt_seps=0.6, mrt_sq=1.7, mrt_spi=1.2, moving_window=1),
])
def test_brute_force_agreement(variant):
    cfg = wl.config(None, nz=8, nr=4, dz=0.1, dr=0.1, nb=0.3, sigma_z=0.2, sigma_r=0.15, zd0=0.4,
                    noise_amp=0.05, seed=3, **variant)
    P = O.Params(cfg)
    S = O.initial_state(P, wl.density_perturbation(cfg), wl.random_momentum(cfg, 0.3, seed=2))
    G = SR.Grid(cfg)
    st = SR.from_tensors(S)
    for _ in range(7):
        S = O.step(S, P)
        st = SR.step(G, st)
    for a, b in zip(st[:5], (S.g, S.M, S.Ez, S.Er, S.B)):
        assert float((torch.tensor(a, dtype=F64) - b).abs().max()) < 1e-14
    assert (st[5], st[6]) == (S.k, S.s)


# ---------------------------------------------------------------------------------------------
# P_rest: a uniform plasma at rest with no driver is a fixed point (ghosts, axis, window)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("collision", [0, 1, 2, 3])
def test_rest_is_fixed_point(collision):
    cfg = wl.config(None, nz=32, nr=12, moving_window=1, n0=1.0, nb=0.0, collision=collision,
                    mrt_se=1.3, mrt_seps=0.6, mrt_sq=1.7, mrt_spi=1.2)
    P = O.Params(cfg)
    S0 = O.initial_state(P)
    S = S0
    for _ in range(12):
        S = O.step(S, P)
    assert S.s == 2
    assert float((S.g - S0.g).abs().max()) < 1e-15
    assert float((S.M - S0.M).abs().max()) < 1e-15
    for X in (S.Ez, S.Er, S.B):
        assert float(X.abs().max()) == 0.0


# ---------------------------------------------------------------------------------------------
# P_mass: per-site post-collision moments, and global conservation when streaming is a permutation
# ---------------------------------------------------------------------------------------------

def test_post_collision_populations_sum_to_moments():
    cfg = wl.config(None, nz=24, nr=10, nb=0.2, sigma_z=0.3, sigma_r=0.3, zd0=0.6, noise_amp=0.01,
                    seed=4, moving_window=1)
    S, _ = _run(cfg, 9, wl.density_perturbation(cfg), wl.random_momentum(cfg, 0.1))
    assert float((S.g.sum(1) - S.M).abs().max()) < 1e-14


def test_global_conservation_periodic():
    cfg = wl.config(None, nz=20, nr=14, periodic=3, fields_on=0, cyl_on=0, noise_amp=0.2, seed=9)
    P = O.Params(cfg)
    S = O.initial_state(P, wl.density_perturbation(cfg), wl.random_momentum(cfg, 0.2, seed=5))
    tot0 = S.M.sum(dim=(1, 2))
    for _ in range(60):
        S = O.step(S, P)
    tot = S.M.sum(dim=(1, 2))
    assert float((tot - tot0).abs().max()) < 1e-12 * float(tot0[0])
    # and the density actually moved (the test is not vacuous)
    assert float((S.M[0] - O.initial_state(P, wl.density_perturbation(cfg)).M[0]).abs().max()) > 1e-3


# ---------------------------------------------------------------------------------------------
# P_k0: uniform cold plasma oscillation, exact discrete map of the symplectic coupling
# (Eqs. (4), (5), R2, R5, R8, R13)
# ---------------------------------------------------------------------------------------------

def test_plasma_oscillation_exact_map():
    """p' = p - h E, E' = E + h beta(p'): with E^{-1} = 0 and p = eps the stored E^{k-1} after k
    steps is eps sin(k theta) / sqrt(1 - h^2/4), theta = 2 asin(h/2) (relativistic terms O(eps^2))."""
    cfg = wl.config(None, nz=16, nr=8, dz=0.05, dr=0.05, periodic=1, nb=0.0, tau=0.8)
    eps = 1e-6
    P = O.Params(cfg)
    S = O.initial_state(P, None, wl.uniform_momentum(cfg, pz=eps))
    h = P.dt
    th = 2 * math.asin(h / 2)
    worst = 0.0
    for _ in range(400):
        S = O.step(S, P)
        ref = eps * math.sin(S.k * th) / math.sqrt(1 - h * h / 4)
        worst = max(worst, float((S.Ez - ref).abs().max()) / eps)
    assert worst < 1e-10
    assert float(S.Er.abs().max()) < 1e-20 and float(S.M[2].abs().max()) < 1e-20


# ---------------------------------------------------------------------------------------------
# P_k: momentum diffusion with field coupling (Eq. (11) with D of Eq. (12))
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("tau", [0.8, 1.2])
def test_momentum_diffusion_wave(tau):
    """p_z = eps sin(kz): continuum solution E_z = (eps/w) exp(-D k^2 t/2) sin(w t) sin(kz),
    w = sqrt(1 - D^2 k^4/4); discretisation errors O((k dz)^2) and O(dt)."""
    cfg = wl.config(None, nz=64, nr=4, dz=0.05, dr=0.05, periodic=1, nb=0.0, tau=tau)
    eps = 1e-6
    S, P = _run(cfg, 600, None, wl.sine_momentum_z(cfg, eps, 1))
    kk = 2 * math.pi / (64 * 0.05)
    om = math.sqrt(1 - P.D ** 2 * kk ** 4 / 4)
    z = (torch.arange(64, dtype=F64) + 0.5) * 0.05
    t = (S.k - 0.5) * P.dt
    ref = eps / om * math.exp(-P.D * kk * kk * t / 2) * math.sin(om * t) * torch.sin(kk * z)
    assert float((S.Ez[0] - ref).abs().max()) < 0.02 * float(ref.abs().max())


# ---------------------------------------------------------------------------------------------
# P_D: diffusivity of Eq. (12) from the variance growth of a bump (Cartesian, fields off)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("tau,collision,magic", [(0.6, 0, 0.25), (0.8, 0, 0.25), (0.6, 1, 0.25),
                                                 (0.8, 1, 1.0 / 12.0), (0.6, 2, 0.25), (0.6, 3, 0.0),
                                                 (0.8, 3, 0.0)])
def test_diffusivity(tau, collision, magic):
    """For TRT, the regularised operator and MRT (R29) D depends on tau alone: with tau = 0.6 and
    Lambda = 1/4 the even rate is tau_plus = 3, which would give a five times larger D if the two
    rates were swapped; MRT runs with energy, energy-square, heat-flux and stress rates
    1.3, 0.6, 1.7, 1.2, none of them 1/tau."""
    n = 96
    cfg = wl.config(None, nz=n, nr=n, dz=0.05, dr=0.05, periodic=3, fields_on=0, cyl_on=0,
                    nb=0.0, tau=tau, collision=collision, trt_magic=magic,
                    mrt_se=1.3, mrt_seps=0.6, mrt_sq=1.7, mrt_spi=1.2)
    P = O.Params(cfg)
    zc, rc = 48 * 0.05, 48.5 * 0.05
    S = O.initial_state(P, wl.gaussian_bump(cfg, 0.1, 0.2, 0.2, zc=zc, rc=rc))
    z = torch.arange(n, dtype=F64) * 0.05
    r = (torch.arange(n, dtype=F64) + 0.5) * 0.05

    def variances(S):
        d = S.M[0] - 1.0
        m0 = d.sum()
        return float((d * (z[None, :] - zc) ** 2).sum() / m0), float((d * (r[:, None] - rc) ** 2).sum() / m0)

    snaps = {}
    for k in range(1, 201):
        S = O.step(S, P)
        if k in (50, 200):
            snaps[k] = variances(S)
    span = 150 * P.dt
    Dz = (snaps[200][0] - snaps[50][0]) / (2 * span)
    Dr = (snaps[200][1] - snaps[50][1]) / (2 * span)
    assert abs(Dz / P.D - 1) < 1e-6 and abs(Dr / P.D - 1) < 1e-6


# ---------------------------------------------------------------------------------------------
# P_cyl: axisymmetric diffusion term of Eq. (13) (reading R10)
# ---------------------------------------------------------------------------------------------

def test_cylindrical_diffusion():
    """Radial Gaussian, uniform in z: delta n = a (s0^2/s^2) exp(-r^2/2 s^2), s^2 = s0^2 + 2 D t."""
    cfg = wl.config(None, nz=4, nr=64, dz=0.05, dr=0.05, periodic=1, fields_on=0, cyl_on=1,
                    nb=0.0, tau=0.8)
    s0, a = 0.3, 0.1
    S, P = _run(cfg, 300, wl.gaussian_bump(cfg, a, None, s0))
    r = (torch.arange(64, dtype=F64) + 0.5) * 0.05
    s2 = s0 * s0 + 2 * P.D * S.k * P.dt
    ref = a * (s0 * s0 / s2) * torch.exp(-r * r / (2 * s2))
    assert float((S.M[0, :, 0] - 1.0 - ref).abs().max()) < 0.01 * a
    # without the cylindrical term the same run is the 1D (slab) solution, far from the reference
    cfg0 = dict(cfg, cyl_on=0)
    S0, _ = _run(cfg0, 300, wl.gaussian_bump(cfg0, a, None, s0))
    assert float((S0.M[0, :, 0] - 1.0 - ref).abs().max()) > 0.05 * a


def _radial_bump_error(h, lam, steps, nr, r_offset=0.5):
    """Max-norm error of the radial Gaussian of test_cylindrical_diffusion after `steps` steps
    against the exact axisymmetric heat kernel, on rows of width h with c dt / dz = lam; r_offset
    moves the radius the source term divides by (0.5: the row centres r_j = (j + 1/2) dr)."""
    cfg = wl.config(None, nz=4, nr=nr, dz=h, dr=h, c_dt_over_dz=lam, periodic=1, fields_on=0, cyl_on=1,
                    nb=0.0, tau=0.8)
    s0, a = 0.3, 0.1
    P = O.Params(cfg)
    if r_offset != 0.5:
        P.r = (P.jj + r_offset) * P.h   # a mistake planted in the oracle's source term
    S = O.initial_state(P, wl.gaussian_bump(cfg, a, None, s0))
    for _ in range(steps):
        S = O.step(S, P)
    r = (torch.arange(nr, dtype=F64) + 0.5) * h
    s2 = s0 * s0 + 2 * P.D * S.k * P.dt
    ref = a * (s0 * s0 / s2) * torch.exp(-r * r / (2 * s2))
    return float((S.M[0, :, 0] - 1.0 - ref).abs().max())


def test_cylindrical_diffusion_converges_at_second_order():
    """Reading R10's stencil: refining dr by 2 with c dt / dz halved (diffusive scaling: D and the
    time span fixed, four times the steps) cuts the error against the exact axisymmetric heat
    kernel by more than 2.5 at each refinement (measured 3.75 and 2.85), as a consistent
    second-order radial term does.  The same runs with the source term dividing by (j + 1) dr
    instead of the row centre (a plausible slip) converge at first order (ratios 1.6 and 1.8) and
    end 70 times further off; so does (j + 1/4) dr."""
    levels = ((0.1, 0.4, 75, 32), (0.05, 0.2, 300, 64), (0.025, 0.1, 1200, 128))
    e = [_radial_bump_error(*lv) for lv in levels]
    assert e[0] / e[1] > 2.5 and e[1] / e[2] > 2.5, e
    assert e[2] < 3e-5, e
    bad = [_radial_bump_error(*lv, r_offset=1.0) for lv in levels]
    assert not (bad[0] / bad[1] > 2.5 and bad[1] / bad[2] > 2.5 and bad[2] < 3e-5), bad


def test_radial_flow_continuity():
    """Uniform density with p_r = eps r: dn/dt = -(1/r) d(r n u_r)/dr = -2 eps away from the axis
    (Eq. (3)); half of it comes from the -A u_r / r source."""
    for cyl, rate in ((1, -2.0), (0, -1.0)):
        cfg = wl.config(None, nz=4, nr=32, dz=0.05, dr=0.05, periodic=1, fields_on=0, cyl_on=cyl,
                        nb=0.0, tau=0.8)
        eps = 1e-4
        S, P = _run(cfg, 20, None, wl.linear_radial_momentum(cfg, eps))
        d = (S.M[0, 4:16, 0] - 1.0) / (S.k * P.dt) / eps
        assert float((d - rate).abs().max()) < 0.01 * abs(rate)


def test_axis_mirror_equivalence():
    """Axis rule R11: a slab that is mirror-symmetric about r = 0 (n, n p_z even, n p_r odd), run
    Cartesian and periodic over 2 nr rows, equals the half domain with the axis ghost after one
    step from equilibrium (the ghost equilibrium then equals the mirrored population exactly)."""
    nr, nz = 6, 10
    half = wl.config(None, nz=nz, nr=nr, dz=0.1, dr=0.1, periodic=1, fields_on=0, cyl_on=0, nb=0.0)
    rng = np.random.default_rng(3)
    n_h = 0.2 * (rng.random((nr, nz)) - 0.5)
    p_h = 0.2 * (rng.random((2, nr, nz)) - 0.5)
    full = dict(half, nr=2 * nr, periodic=3)
    n_f = np.concatenate([n_h[::-1], n_h])
    p_f = np.concatenate([p_h[:, ::-1], p_h], axis=1)
    p_f[1, :nr] *= -1.0
    Sh, _ = _run(half, 1, n_h, p_h)
    Sf, _ = _run(full, 1, n_f, p_f)
    # rows below nr - 1 (the outer edge of the half domain reaches only its last row in one step)
    assert float((Sh.M[:, :-1] - Sf.M[:, nr:-1]).abs().max()) < 1e-15
    assert float((Sh.g[:, :, :-1] - Sf.g[:, :, nr:-1]).abs().max()) < 1e-15


# ---------------------------------------------------------------------------------------------
# P_divcurl: Yee operators incl. the axis (R12): div_h curl_h = 0
# ---------------------------------------------------------------------------------------------

def test_div_curl_identity():
    cfg = wl.config(None, nz=20, nr=10, dz=0.1, dr=0.1, nb=0.0, periodic=1)
    P = O.Params(cfg)
    g = torch.Generator().manual_seed(1)
    Ez, Er, B = (torch.randn(P.nr, P.nz, generator=g, dtype=F64) for _ in range(3))
    M = torch.stack([1 + 0.1 * torch.randn(P.nr, P.nz, generator=g, dtype=F64),
                     0.3 * torch.randn(P.nr, P.nz, generator=g, dtype=F64),
                     0.3 * torch.randn(P.nr, P.nz, generator=g, dtype=F64)])
    Mp = O.padded_moments(M, P, 0)
    Ez1, Er1, _ = O.field_update(Ez, Er, B, Mp, 0, 0, P)
    h, jj = P.h, P.jj

    def div(Ez, Er):
        return (Ez - torch.roll(Ez, 1, -1)) / h + \
            ((jj + 1) * Er - jj * torch.cat([torch.zeros(1, P.nz, dtype=F64), Er[:-1]])) / ((jj + 0.5) * h)

    Jz, Jr = O.current(Mp, P)
    Jzf = 0.5 * (Jz[1:-1, 1:-1] + Jz[1:-1, 2:])
    Jrf = 0.5 * (Jr[1:-1, 1:-1] + Jr[2:, 1:-1])
    lhs = (div(Ez1, Er1) - div(Ez, Er)) / P.dt
    rhs = div(Jzf, Jrf)
    assert float((lhs - rhs).abs().max()) < 1e-10 * float(B.abs().max() / h)


# ---------------------------------------------------------------------------------------------
# P_vac: driver field in vacuum moves rigidly at c (Faraday sign R2, J_b, window kinematics)
# ---------------------------------------------------------------------------------------------

def test_vacuum_driver_field():
    cfg = wl.config(None, nz=128, nr=48, dz=0.05, dr=0.05, moving_window=1, n0=0.0, nb=0.1,
                    sigma_z=0.5, sigma_r=0.5, zd0=3.2, tau=0.8)
    S, P = _run(cfg, 300)
    z = (S.s + P.ii) * P.h
    assert S.s == 60
    assert O.rel_err(S.Er, O.gauss_field(z, (S.k - 1) * P.dt, P)) < 5e-3
    assert O.rel_err(S.B, O.gauss_field(z + 0.5 * P.h, (S.k - 0.5) * P.dt, P)) < 5e-3
    assert float(S.Ez.abs().max()) < 5e-3 * float(S.Er.abs().max())
    assert float(S.M.abs().max()) == 0.0


def test_comoving_fluid_cancels_radial_force():
    """Lorentz force (Eq. (4), R8): in the driver's field (B_theta = E_r at beta_b = 1) a tenuous
    fluid moving with beta_z -> 1 feels -(E_r - beta_z B_theta) = -(1 - beta_z) E_r; a fluid at
    rest feels -E_r.  A sign error in the magnetic term would give (1 + beta_z) instead."""
    out = {}
    for pz in (0.0, 10.0):
        cfg = wl.config(None, nz=96, nr=32, dz=0.05, dr=0.05, moving_window=1, n0=1e-9,
                        n_floor=1e-15, nb=0.1, sigma_z=0.5, sigma_r=0.4, zd0=96 * 0.05 - 2.4)
        S, P = _run(cfg, 100, None, wl.uniform_momentum(cfg, pz=pz))
        i = int((P.zd0 + (S.k - 1) * P.dt) / P.h - S.s)
        out[pz] = float((S.M[2] / S.M[0])[2:8, i].abs().max())
    beta = 10 / math.sqrt(101)
    assert out[0.0] > 1e-3
    assert out[10.0] / out[0.0] < 3 * (1 - beta)


# ---------------------------------------------------------------------------------------------
# Initial state: discrete Gauss law (R18), perturbation, window
# ---------------------------------------------------------------------------------------------

def test_initial_gauss_law_exact():
    cfg = wl.config("C1", noise_amp=0.0)
    P = O.Params(cfg)
    S = O.initial_state(P)
    G = O.gauss_residual(S, P)
    assert float(G.abs().max()) < 1e-15
    # the driver's field is really there
    assert float(S.Er.abs().max()) > 1e-3


def test_initial_perturbation_applied():
    cfg = wl.config("C1")
    P = O.Params(cfg)
    pert = wl.density_perturbation(cfg)
    S = O.initial_state(P, pert)
    assert np.allclose(S.M[0].numpy(), 1.0 + pert, rtol=0, atol=1e-15)
    assert np.abs(pert).max() <= 1e-6 and np.abs(pert).max() > 0.9e-6


def test_ramp_profiles():
    for kind in (1, 2):
        cfg = wl.config(None, ramp_kind=kind, ramp_start=2.0, ramp_len=4.0, n0=1.5)
        P = O.Params(cfg)
        z = torch.tensor([0.0, 2.0, 4.0, 6.0, 100.0], dtype=F64)
        n = O.n_background(z, P)
        assert abs(float(n[2]) - 0.75) < 1e-15           # half density mid-ramp
        assert abs(float(n[4]) - 1.5) < 1e-12            # plateau
        assert float(n[0]) < 0.1 and float(n[1]) < 0.3   # (near) vacuum before the ramp
        assert bool((n[1:] >= n[:-1]).all())
    P = O.Params(wl.config(None, ramp_kind=1, ramp_start=2.0, ramp_len=4.0, n0=1.5))
    assert float(O.n_background(torch.tensor(2.0, dtype=F64), P)) == 0.0


def test_window_equals_fixed_domain():
    """R15: a run with the moving window equals, column for column in the lab frame, a run on a
    longer fixed domain, away from the rear edge (uniform plasma ahead, so the fresh columns are
    what the fixed run holds there)."""
    base = dict(dz=0.05, dr=0.05, nb=0.05, sigma_z=0.3, sigma_r=0.4, ramp_kind=0, tau=0.8)
    cA = wl.config(None, nz=96, nr=24, moving_window=1, zd0=96 * 0.05 - 3.0, **base)
    cB = wl.config(None, nz=116, nr=24, moving_window=0, zd0=96 * 0.05 - 3.0, **base)
    SA, _ = _run(cA, 40)
    SB, _ = _run(cB, 40)
    s, lo = SA.s, 42
    assert s == 8
    for name in ("g", "M", "Ez", "Er", "B"):
        a = getattr(SA, name)[..., lo:]
        b = getattr(SB, name)[..., s + lo:s + 96]
        assert float((a - b).abs().max()) <= 1e-14 * max(float(b.abs().max()), 1e-300)


def test_objective_interpolates_witness_position():
    cfg = wl.config(None, nz=64, nr=8, moving_window=1, zd0=2.5)
    P = O.Params(cfg)
    S = O.initial_state(P)
    S.k, S.s = 23, 4
    zE = (S.s + P.ii + 0.5) * P.h
    S.Ez = (0.3 * zE + 0.1) * torch.ones(P.nr, 1, dtype=F64)
    zstar = P.zd0 + (S.k - 1) * P.dt - 1.0
    assert abs(float(O.objective(S, P, 1.0)) - (0.3 * zstar + 0.1)) < 1e-14


# ---------------------------------------------------------------------------------------------
# P_lin: linear wake of a weak Gaussian driver (physics check, not parity)
# ---------------------------------------------------------------------------------------------

@pytest.mark.slow
def test_linear_wake_closed_form():
    """Cold-fluid linear theory: E_z(xi, r) = n_b R(r) int_xi^inf cos(x - xi) exp(-x^2/2 sz^2) dx,
    R(r) = int_0^inf r' I0(r<) K0(r>) exp(-r'^2/2 sr^2) dr'.

    The driver starts in vacuum and enters the plasma through a tanh ramp (a driver switched on
    inside the plasma, or a short entrance, launches a forward-moving transient that travels with
    it and only slowly falls behind); after 32 plasma periods of propagation at small diffusivity
    the wake behind the driver is compared on the first two rows."""
    from scipy import integrate, special
    h, nz, nr = 0.1, 160, 48
    zd0 = nz * h - 4.0
    cfg = wl.config("C1", noise_amp=0.0, tau=0.51, nz=nz, nr=nr, dz=h, dr=h, moving_window=1,
                    zd0=zd0, ramp_kind=2, ramp_start=zd0 + 2.0, ramp_len=2.0)
    S, P = _run(cfg, 1600)
    sz = sr = 0.5

    def R_of(r):
        f = lambda rp: rp * special.i0(min(r, rp)) * special.k0(max(r, rp)) * math.exp(-rp * rp / (2 * sr * sr))
        return integrate.quad(f, 0, r, limit=200)[0] + integrate.quad(f, r, 12 * sr, limit=200)[0]

    zd = P.zd0 + (S.k - 1) * P.dt
    for j in (0, 5):
        Rr = R_of((j + 0.5) * h)
        amp = 0.01 * Rr * math.sqrt(2 * math.pi) * sz * math.exp(-sz * sz / 2)
        worst = 0.0
        for i in range(P.nz):
            xi = (S.s + i + 0.5) * P.h - zd
            if -3.0 <= xi <= 1.0:
                ref = 0.01 * Rr * integrate.quad(
                    lambda x: math.cos(x - xi) * math.exp(-x * x / (2 * sz * sz)), xi, 12 * sz, limit=200)[0]
                worst = max(worst, abs(float(S.Ez[j, i]) - ref))
        assert worst < 0.05 * amp


# ---------------------------------------------------------------------------------------------
# P_units: values printed in the paper (golden fixtures)
# ---------------------------------------------------------------------------------------------

def test_normalized_charge_reproduces_paper():
    with open(os.path.join(GOLDEN, "paper_setup.json")) as fh:
        g = json.load(fh)
    sz, sx = g["sigma_z_um"] * 1e-6, g["sigma_xy_um"] * 1e-6
    for q_nC, qt in zip(g["charges_nC"], g["qtilde"]):
        alpha = U.peak_density_ratio(q_nC * 1e-9, sx, sx, sz, g["n0_cm3"])
        assert abs(U.normalized_charge(alpha, sx, sx, sz, g["n0_cm3"]) / qt - 1) < 5e-3
    kp = U.plasma_wavenumber(g["n0_cm3"])
    # the paper's grid in normalised units: k_p dz ~ 0.0047 and c dt / dz ~ 0.176
    assert abs(kp * g["dz_um"] * 1e-6 - 0.0047) < 1e-4
    assert abs(U.C_LIGHT * g["dt_fs"] * 1e-15 / (g["dz_um"] * 1e-6) - 0.1763) < 1e-3


def test_table1_gain_column():
    with open(os.path.join(GOLDEN, "table1.json")) as fh:
        t = json.load(fh)
    for f, l, gain in zip(t["fct_ks"], t["lbm_ks"], t["gain_percent"]):
        assert abs(U.gain_percent(f, l) - gain) < 0.01


# --- bubble length (Sec. IV, Fig. 4; reading R28) -----------------------------------------------

def test_bubble_length_counts_depleted_sites_by_hand():
    """A hand-made density row: 7 sites clearly below n* n_bg, one exactly at it (not counted),
    ramp sites in vacuum (n_bg = 0, not counted), and a z-range that cuts the depleted region."""
    cfg = wl.config(None, nz=40, nr=4, dz=0.1, dr=0.1, ramp_kind=1, ramp_start=0.5, ramp_len=0.5, n0=2.0)
    P = O.Params(cfg)
    z = torch.arange(40, dtype=torch.float64) * 0.1
    nbg = O.n_background(z, P)
    n = nbg.repeat(4, 1).clone()
    assert float(nbg[4]) == 0.0 and float(nbg[12]) == 2.0
    n[1, 20:27] = 0.5 * nbg[20:27]               # depleted: 7 sites
    n[1, 27] = 0.95 * nbg[27]                    # exactly at the threshold: not counted
    n[1, 0:5] = -1.0                             # below threshold but in vacuum: not counted
    n[2, 10:30] = 0.0                            # another row: not counted on row 1
    assert O.bubble_length(n, 0, P, row=1) == (7, 7 * 0.1)
    assert O.bubble_length(n, 0, P, row=1, z_from=2.25, z_to=2.55)[0] == 3   # sites 23, 24, 25
    assert O.bubble_length(n, 0, P, row=2)[0] == 20
    # the window shift moves the lab positions: with s = 10 the depleted sites sit in n0 plasma
    assert O.bubble_length(n, 10, P, row=1, z_from=3.0)[0] == 7


def test_bubble_length_of_a_uniform_rest_plasma_is_zero():
    cfg = wl.config(None, nz=30, nr=5, dz=0.05)
    P = O.Params(cfg)
    S = O.initial_state(P)
    n = O.moments_out(S, P)[0]
    assert O.bubble_length(n, 0, P, row=0)[0] == 0


# --- collision operators other than BGK (Sec. IV remark; reading R29) ---------------------------

def _moments9(f):
    """The nine D2Q9 moments of [9][...] populations: A, j_z, j_r, Pi_zz, Pi_rr, Pi_zr, q_z, q_r, m4
    (q_z = sum xi_z xi_r^2 f, q_r = sum xi_r xi_z^2 f, m4 = sum xi_z^2 xi_r^2 f); they determine f."""
    out = []
    for a, b in ((0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (1, 2), (2, 1), (2, 2)):
        out.append(sum((xz ** a) * (xr ** b) * f[q] for q, (xz, xr) in enumerate(O.XI)))
    return torch.stack(out)


@pytest.mark.parametrize("collision", [0, 1, 2, 3])
def test_collision_relaxes_each_moment_at_its_rate(collision):
    """Spatially uniform random populations on a doubly periodic lattice with fields and sources
    off: streaming is the identity, so one step is one collision.  The moment-space statement of
    each operator: BGK relaxes all eight non-conserved moments with 1/tau; TRT relaxes the odd
    ones (j, q) with 1/tau and the even ones (Pi, m4) with 1/tau_plus; the regularised operator
    relaxes j with 1/tau, sets Pi and m4 to equilibrium and sets q to q_eq + (1 - 1/tau) j_neq / 3
    (the q-moment of the first-order Hermite term, since sum w xi_z^2 xi_r^2 = 1/9).  MRT, stated
    in these raw moments through identities on the nine velocities (|xi|^4 = |xi|^2 + 2 xi_z^2
    xi_r^2 and xi_z^3 = xi_z): j relaxes with 1/tau; Pi_zz + Pi_rr (= (e + 4 rho)/3) with s_e;
    Pi_zz - Pi_rr and Pi_zr with s_pi; q_z = (q_z^MRT + 2 j_z)/3 and m4 = (eps + 2 e + 4 rho)/9
    each with the mix of rates that gives."""
    tau, magic = 0.7, 0.09
    s_e, s_eps, s_q, s_pi = 1.3, 0.6, 1.7, 1.2
    cfg = wl.config(None, nz=3, nr=3, periodic=3, fields_on=0, cyl_on=0, tau=tau,
                    collision=collision, trt_magic=magic, mrt_se=s_e, mrt_seps=s_eps, mrt_sq=s_q,
                    mrt_spi=s_pi)
    P = O.Params(cfg)
    S = O.initial_state(P)
    gen = torch.Generator().manual_seed(11)
    g0 = (0.05 + torch.rand(3, 9, dtype=F64, generator=gen))[:, :, None, None].expand(3, 9, 3, 3)
    S.g = g0.reshape(27, 3, 3).clone().reshape(S.g.shape)
    S.M = g0.sum(1).clone()
    S1 = O.step(S, P)
    g1 = S1.g.reshape(3, 9, 3, 3)
    tau_p = 0.5 + magic / (tau - 0.5) if collision == 1 else tau
    for kk in range(3):
        m0 = _moments9(g0[kk])
        A = [g0[c].sum(0) for c in range(3)]
        bz, br, _ = O.velocity(torch.stack(A), P)
        meq = _moments9(O.equilibrium(m0[0], P.lam * bz, P.lam * br))
        m1 = _moments9(g1[kk])
        expect = m0.clone()
        odd, even = [1, 2, 6, 7], [3, 4, 5, 8]
        if collision == 2:
            expect[1:3] = m0[1:3] - (m0[1:3] - meq[1:3]) / tau
            expect[even] = meq[even]
            expect[6:8] = meq[6:8] + (1 - 1 / tau) * (m0[1:3] - meq[1:3]) / 3
        elif collision == 3:
            d = m0 - meq
            jn = (1 - 1 / tau) * d[1:3]                              # flux
            tr = (1 - s_e) * (d[3] + d[4])                          # Pi_zz + Pi_rr
            df = (1 - s_pi) * (d[3] - d[4])                         # Pi_zz - Pi_rr
            expect[1:3] = meq[1:3] + jn
            expect[3] = meq[3] + 0.5 * (tr + df)
            expect[4] = meq[4] + 0.5 * (tr - df)
            expect[5] = meq[5] + (1 - s_pi) * d[5]
            qm = (1 - s_q) * (3 * d[6:8] - 2 * d[1:3])              # the MRT heat fluxes
            expect[6:8] = meq[6:8] + (qm + 2 * jn) / 3
            e_n = 3 * (d[3] + d[4])
            eps_n = 9 * d[8] - 2 * e_n
            expect[8] = meq[8] + ((1 - s_eps) * eps_n + 2 * (1 - s_e) * e_n) / 9
        else:
            expect[odd] = m0[odd] - (m0[odd] - meq[odd]) / tau
            expect[even] = m0[even] - (m0[even] - meq[even]) / tau_p
        assert float((m1 - expect).abs().max()) < 1e-14, (kk, m1 - expect)
        # the test is not vacuous: the populations were far from equilibrium
        assert float((m0[3:] - meq[3:]).abs().max()) > 0.05


def test_trt_with_lambda_of_bgk_is_bgk():
    """Lambda = (tau - 1/2)^2 makes tau_plus = tau: TRT must then reproduce BGK over a coupled,
    driven, windowed run."""
    tau = 0.7
    base = dict(nz=40, nr=10, dz=0.05, dr=0.05, nb=0.8, sigma_z=0.3, sigma_r=0.3, zd0=1.5, tau=tau,
                moving_window=1, noise_amp=0.02, seed=5)
    cfg_b = wl.config(None, **base)
    cfg_t = wl.config(None, collision=1, trt_magic=(tau - 0.5) ** 2, **base)
    Sb, _ = _run(cfg_b, 30, wl.density_perturbation(cfg_b))
    St, _ = _run(cfg_t, 30, wl.density_perturbation(cfg_t))
    for a, b in ((Sb.g, St.g), (Sb.M, St.M), (Sb.Ez, St.Ez), (Sb.B, St.B)):
        assert float((a - b).abs().max()) < 1e-13 * max(1.0, float(a.abs().max()))
    cfg_o = wl.config(None, collision=1, trt_magic=0.25, **base)
    So, _ = _run(cfg_o, 30, wl.density_perturbation(cfg_o))
    assert float((Sb.g - So.g).abs().max()) > 1e-6


def test_mrt_reduces_to_bgk_and_trt():
    """MRT with every rate 1/tau is BGK, and with s_e = s_eps = s_pi = 1/tau_plus, s_q = 1/tau it
    is TRT (R29), over a coupled, driven, windowed run; rates off those values differ from both."""
    tau, magic = 0.7, 0.09
    tau_p = 0.5 + magic / (tau - 0.5)
    base = dict(nz=40, nr=10, dz=0.05, dr=0.05, nb=0.8, sigma_z=0.3, sigma_r=0.3, zd0=1.5, tau=tau,
                moving_window=1, noise_amp=0.02, seed=5)
    runs = {}
    for name, extra in (("bgk", dict()), ("trt", dict(collision=1, trt_magic=magic)),
                        ("mrt_bgk", dict(collision=3, mrt_se=1 / tau, mrt_seps=1 / tau, mrt_sq=1 / tau,
                                         mrt_spi=1 / tau)),
                        ("mrt_trt", dict(collision=3, mrt_se=1 / tau_p, mrt_seps=1 / tau_p, mrt_sq=1 / tau,
                                         mrt_spi=1 / tau_p)),
                        ("mrt", dict(collision=3, mrt_se=1.3, mrt_seps=0.6, mrt_sq=1.7, mrt_spi=1.2))):
        cfg = wl.config(None, **base, **extra)
        runs[name], _ = _run(cfg, 30, wl.density_perturbation(cfg))
    for a, b in (("bgk", "mrt_bgk"), ("trt", "mrt_trt")):
        for x, y in ((runs[a].g, runs[b].g), (runs[a].M, runs[b].M), (runs[a].Ez, runs[b].Ez)):
            assert float((x - y).abs().max()) < 1e-13 * max(1.0, float(x.abs().max())), (a, b)
    for a in ("bgk", "trt"):
        assert float((runs[a].g - runs["mrt"].g).abs().max()) > 1e-6


def test_collision_operators_conserve_per_site():
    for collision in (1, 2, 3):
        cfg = wl.config(None, nz=24, nr=10, nb=0.4, sigma_z=0.3, sigma_r=0.3, zd0=0.6, noise_amp=0.01,
                        seed=4, moving_window=1, collision=collision,
                        mrt_se=1.3, mrt_seps=0.6, mrt_sq=1.7, mrt_spi=1.2)
        S, _ = _run(cfg, 9, wl.density_perturbation(cfg), wl.random_momentum(cfg, 0.1))
        assert float((S.g.sum(1) - S.M).abs().max()) < 1e-14


# --- particle driver (Sec. II, Eq. (1); reading R30) ---------------------------------------------

def _quadrature_bunch(cfg, nzq=64, nrq=48, nphi=4, beta_z_gamma=1e4):
    """A smooth bi-Gaussian bunch as a dense deterministic quadrature: particles on a polar grid
    (rings of nphi particles at radii (m + 1/2) dq_r, slices at z spacing dq_z), each carrying the
    rigid driver's density times its quadrature volume, all at p_z = beta_z_gamma, positions at
    t = -dt (the rigid driver's centre then)."""
    sr, sz, nb = cfg["sigma_r"], cfg["sigma_z"], cfg["nb"]
    dt = cfg["c_dt_over_dz"] * cfg["dz"]
    zc = cfg["zd0"] - dt
    dqz = 8.0 * sz / nzq / 4.0
    dqr = 4.0 * sr / nrq / 2.0
    zs = zc + (np.arange(4 * nzq) - 2 * nzq + 0.5) * dqz
    rs = (np.arange(2 * nrq) + 0.5) * dqr
    phis = (np.arange(nphi) + 0.25) * 2.0 * np.pi / nphi
    Z, R, PH = np.meshgrid(zs, rs, phis, indexing="ij")
    Z, R, PH = Z.ravel(), R.ravel(), PH.ravel()
    dens = nb * np.exp(-(Z - zc) ** 2 / (2 * sz * sz)) * np.exp(-R ** 2 / (2 * sr * sr))
    vol = R * dqr * dqz * (2.0 * np.pi / nphi)
    out = np.zeros((7, Z.size))
    out[0], out[1], out[2] = R * np.cos(PH), R * np.sin(PH), Z
    out[5] = beta_z_gamma
    out[6] = dens * vol
    return out


def test_boris_uniform_magnetic_field_rotates_exactly():
    """Pure B along z: |p| is conserved to round-off and each step rotates p_perp by exactly
    2 atan(|B| dt / (2 gamma)) (the Boris rotation angle), clockwise for the electron charge."""
    p = torch.tensor([[0.3], [0.0], [0.7]], dtype=F64)
    E = torch.zeros(3, 1, dtype=F64)
    B = torch.tensor([[0.0], [0.0], [0.9]], dtype=F64)
    dt = 0.05
    gam = math.sqrt(1.0 + float((p * p).sum()))
    ang = 2.0 * math.atan(0.9 * dt / (2.0 * gam))
    q = p.clone()
    for k in range(1, 101):
        q = O.boris(q, E, B, dt)
        phi = math.atan2(float(q[1, 0]), float(q[0, 0]))
        expect = math.remainder(+k * ang, 2 * math.pi)   # dp/dt = -beta x B: positive rotation
        assert abs(math.remainder(phi - expect, 2 * math.pi)) < 1e-12
    assert abs(float((q * q).sum()) - float((p * p).sum())) < 1e-14
    assert abs(float(q[2, 0]) - 0.7) < 1e-15


def test_boris_uniform_electric_field_kicks_exactly():
    p = torch.tensor([[0.1], [-0.2], [3.0]], dtype=F64)
    E = torch.tensor([[0.02], [0.01], [-0.5]], dtype=F64)
    q = p.clone()
    for _ in range(40):
        q = O.boris(q, E, torch.zeros(3, 1, dtype=F64), 0.01)
    assert float((q - (p - 40 * 0.01 * E)).abs().max()) < 1e-14


def _rand_particles(P, n, seed, r_max):
    g = torch.Generator().manual_seed(seed)
    z = (2.0 + (P.nz - 5) * torch.rand(n, generator=g, dtype=F64)) * P.h
    r = r_max * torch.rand(n, generator=g, dtype=F64)
    return z, r, torch.rand(n, generator=g, dtype=F64)


def test_deposit_conserves_charge_and_is_the_transpose_of_gather():
    cfg = wl.config(None, nz=40, nr=12, dz=0.1, dr=0.1)
    P = O.Params(cfg)
    z, r, w = _rand_particles(P, 500, 3, 0.9)
    vol_c = 2 * math.pi * P.r * P.h * P.h
    vol_e = 2 * math.pi * P.r_edge * P.h * P.h
    for zoff, edge, vol in ((0.0, False, vol_c), (0.5, False, vol_c), (0.0, True, vol_e), (0.5, True, vol_e)):
        n = O.deposit(w, z, r, 0, P, zoff, edge)
        if not edge:   # the centre rows keep every share (the fold); the edge rows drop the axis share
            assert abs(float((n * vol).sum()) - float(w.sum())) < 1e-12 * float(w.sum())
        F = torch.rand(P.nr, P.nz, generator=torch.Generator().manual_seed(7), dtype=F64)
        lhs = float((F * n * vol).sum())
        rhs = float((w * O.gather(F, z, r, 0, P, zoff, edge)).sum())
        assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_gather_reproduces_linear_fields():
    cfg = wl.config(None, nz=40, nr=12, dz=0.1, dr=0.1)
    P = O.Params(cfg)
    z, r, _ = _rand_particles(P, 300, 5, 1.0)
    zc = (P.ii + 0.5) * P.h
    # E_z-type (centre rows) field a + b z + c r, away from the fold (r >= dr / 2)
    F = 0.3 + 0.7 * zc - 1.1 * P.r
    keep = r >= 0.5 * P.h
    got = O.gather(F, z, r, 0, P, 0.5, False)[keep]
    assert float((got - (0.3 + 0.7 * z - 1.1 * r)[keep]).abs().max()) < 1e-13
    # E_r-type (edge rows, zero on the axis) field r (a + b z): exact down to the axis
    F = P.r_edge * (0.4 - 0.2 * P.ii * P.h)
    got = O.gather(F, z, r, 0, P, 0.0, True)
    assert float((got - r * (0.4 - 0.2 * z)).abs().max()) < 1e-13


def test_deposit_brute_force():
    cfg = wl.config(None, nz=12, nr=5, dz=0.1, dr=0.1)
    P = O.Params(cfg)
    z, r, w = _rand_particles(P, 40, 9, 0.45)
    for zoff, edge in ((0.5, False), (0.0, True)):
        ref = np.zeros((P.nr, P.nz))
        for zz, rr, ww in zip(z.tolist(), r.tolist(), w.tolist()):
            u = zz / P.h - zoff
            v = rr / P.h - (1.0 if edge else 0.5)
            i0, j0 = math.floor(u), math.floor(v)
            if not (1 <= i0 <= P.nz - 3 and -1 <= j0 <= P.nr - 2):
                continue
            for di, wz in ((0, 1 - (u - i0)), (1, u - i0)):
                for dj, wr in ((0, 1 - (v - j0)), (1, v - j0)):
                    j = j0 + dj
                    if j < 0:
                        if edge:
                            continue
                        j = 0
                    rn = (j + (1.0 if edge else 0.5)) * P.h
                    ref[j, i0 + di] += ww * wz * wr / (2 * math.pi * rn * P.h * P.h)
        got = O.deposit(w, z, r, 0, P, zoff, edge).numpy()
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_particle_bunch_reproduces_the_rigid_driver_current():
    """A dense smooth bunch at gamma = 1e4 (quadrature spacing dz/4): the deposited J_bz at
    t_{-1/2} equals the rigid driver's n_b(z - t) at the E_z points of rows j >= 1 to the linear
    shape's O(dz^2) smoothing (2 % of the peak).  Row 0 collects the share folded from below the
    axis: a smooth density comes out 13/12 times its axis value (R30), here to 3 %."""
    cfg = wl.config(None, nz=80, nr=24, dz=0.05, dr=0.05, nb=0.3, sigma_z=0.4, sigma_r=0.3, zd0=2.0,
                    driver=1)
    P = O.Params(cfg)
    b = torch.as_tensor(_quadrature_bunch(cfg), dtype=F64)
    _, Jbz, Jbr = O.bunch_move(b, 0, 0, P)
    ref = O.driver_density((P.ii + 0.5) * P.h, P.r, -0.5 * P.dt, P)
    assert float((Jbz[1:] - ref[1:]).abs().max()) < 0.02 * float(ref.max())
    peak = int(torch.argmax(ref[0]))
    assert abs(float(Jbz[0, peak] / ref[0, peak]) - 13.0 / 12.0) < 0.03
    assert float(Jbr.abs().max()) < 1e-12


def test_particle_driver_wake_matches_the_rigid_driver():
    """The rigid driver is the gamma -> infinity limit of the particle driver: over 60 coupled steps
    with the window moving, the fields and density of the two runs agree to the projection's
    smoothing (3 % of the wake amplitudes), and the bunch stays unchanged in shape (gamma = 1e4)."""
    base = dict(nz=100, nr=28, dz=0.05, dr=0.05, nb=0.3, sigma_z=0.4, sigma_r=0.3, zd0=2.6,
                moving_window=1)   # the whole bunch (4 sigma) inside the window
    cfg_r = wl.config(None, **base)
    cfg_p = wl.config(None, driver=1, **base)
    Sr, P = _run(cfg_r, 60)
    b = _quadrature_bunch(cfg_p)
    Sp, _ = O.run(cfg_p, 60, bunch=b)
    for a, c in ((Sp.Ez, Sr.Ez), (Sp.Er, Sr.Er), (Sp.B, Sr.B), (Sp.M[0] - Sr.M[0], None)):
        if c is None:
            continue
        assert float((a - c).abs().max()) < 0.03 * float(c.abs().max())
    dn_p = Sp.M[0] - 1.0
    dn_r = Sr.M[0] - 1.0
    assert float((dn_p - dn_r).abs().max()) < 0.03 * float(dn_r.abs().max())
    assert float(Sp.bunch[6].min()) > 0.0                      # no particle lost
    assert (Sp.k, Sp.s) == (60, 12)


def test_particle_driver_initial_gauss_law_is_exact():
    cfg = wl.config(None, nz=60, nr=16, dz=0.05, dr=0.05, nb=0.3, sigma_z=0.4, sigma_r=0.3, zd0=1.5, driver=1)
    P = O.Params(cfg)
    b = wl.bunch(cfg, 3000, seed=2)
    S = O.initial_state(P, None, None, b)
    assert float(S.Er.abs().max()) > 1e-3
    assert float(O.gauss_residual(S, P).abs().max()) < 1e-14


def test_free_particle_moves_exactly_and_is_lost_at_the_window_edge():
    """Fields off: positions advance by dt p / gamma per step; a particle heading out of the
    columns [1, nz - 2] is frozen with zero weight once its stencil would leave them."""
    cfg = wl.config(None, nz=30, nr=8, dz=0.1, dr=0.1, driver=1, fields_on=0)
    P = O.Params(cfg)
    b = torch.zeros(7, 2, dtype=F64)
    b[0:3, 0] = torch.tensor([0.05, 0.02, 1.0])
    b[3:6, 0] = torch.tensor([0.0, 0.0, 2.0])
    b[0:3, 1] = torch.tensor([0.03, 0.0, 0.5])
    b[3:6, 1] = torch.tensor([0.0, 0.0, -3.0])
    b[6] = 1.0
    S = O.initial_state(P, None, None, b)
    v0 = 2.0 / math.sqrt(5.0)
    for k in range(30):
        S = O.step(S, P)
        assert abs(float(S.bunch[2, 0]) - (1.0 + (k + 1) * P.dt * v0)) < 1e-13
    assert float(S.bunch[6, 0]) == 1.0
    assert float(S.bunch[6, 1]) == 0.0        # the backward particle left through the rear edge
    z1 = float(S.bunch[2, 1])
    assert 0.15 <= z1 < 0.15 + 0.02           # frozen where its midpoint stencil still fit column 1


# ---------------------------------------------------------------------------------------------
# FP64 diagnostics (charge of Sec. IV's set-up, field energy of Eq. (5)'s fields on the Yee grid
# of reading R12, Gauss residual of reading R18) against closed forms.  Each sum is checked on a
# state where only one term is non-zero, so a missing 2 pi, a power of dz, or r_edge in place of
# r (or the reverse) changes one of the results by a factor.
# ---------------------------------------------------------------------------------------------

def _diag_state(nz=13, nr=7, h=0.05, **cfg_extra):
    cfg = wl.config(None, nz=nz, nr=nr, dz=h, dr=h, nb=0.0, **cfg_extra)
    P = O.Params(cfg)
    S = O.initial_state(P)
    return S, P


@pytest.mark.parametrize("n0", [1.0, 0.37])
def test_diagnostic_charge_of_uniform_plasma(n0):
    """Uniform density n0 on nr x nz cells: sum_j 2 pi (j + 1/2) dr dr dz nz n0 and
    sum_j (2 j + 1) = nr^2 give pi (nr dr)^2 (nz dz) n0, the volume of the cylinder."""
    nz, nr, h = 13, 7, 0.05
    S, P = _diag_state(nz, nr, h, n0=n0)
    d = O.diagnostics(S, P)
    exact = math.pi * (nr * h) ** 2 * (nz * h) * n0
    assert abs(d["charge"] - exact) <= 1e-13 * exact
    assert d["field_energy"] == 0.0 and d["umax"] == 0.0 and d["nonfinite"] == 0


def test_diagnostic_energy_of_uniform_axial_field():
    """E_z = e everywhere (E_z lives on the fluid rows r_j = (j + 1/2) dr): the energy is
    1/2 e^2 times the cylinder's volume pi (nr dr)^2 (nz dz)."""
    nz, nr, h, e = 11, 6, 0.04, 0.3
    S, P = _diag_state(nz, nr, h)
    S.Ez = torch.full((nr, nz), e, dtype=F64)
    d = O.diagnostics(S, P)
    exact = 0.5 * e * e * math.pi * (nr * h) ** 2 * (nz * h)
    assert abs(d["field_energy"] - exact) <= 1e-13 * exact


@pytest.mark.parametrize("which", ["Er", "B"])
def test_diagnostic_energy_of_uniform_edge_field(which):
    """E_r = b (or B_theta = b) everywhere: both live on the edges r = (j + 1) dr, so the energy is
    1/2 b^2 sum_j 2 pi (j + 1) dr^3 nz = 1/2 b^2 pi dr^3 nz nr (nr + 1), not the cylinder's
    volume (which E_z on the rows (j + 1/2) dr would give)."""
    nz, nr, h, b = 9, 5, 0.07, -0.8
    S, P = _diag_state(nz, nr, h)
    S.Er = torch.zeros(nr, nz, dtype=F64)
    S.B = torch.zeros(nr, nz, dtype=F64)
    setattr(S, which, torch.full((nr, nz), b, dtype=F64))
    d = O.diagnostics(S, P)
    exact = 0.5 * b * b * math.pi * h ** 3 * nz * nr * (nr + 1)
    assert abs(d["field_energy"] - exact) <= 1e-13 * exact
    cyl = 0.5 * b * b * math.pi * (nr * h) ** 2 * (nz * h)
    assert abs(d["field_energy"] - cyl) > 0.1 * exact


@pytest.mark.parametrize("pz,pr", [(0.3, 0.0), (2.0, -1.5), (0.0, 0.05)])
def test_diagnostic_umax_of_uniform_momentum(pz, pr):
    """Uniform momentum p: beta = |p| / sqrt(1 + |p|^2) (Eq. (2)), lattice speed
    (c dt / dz) |beta| (reading R6)."""
    nz, nr = 10, 4
    cfg = wl.config(None, nz=nz, nr=nr, dz=0.05, dr=0.05, nb=0.0)
    P = O.Params(cfg)
    p_init = np.stack([np.full((nr, nz), pz), np.full((nr, nz), pr)])
    S = O.initial_state(P, None, p_init)
    d = O.diagnostics(S, P)
    p2 = pz * pz + pr * pr
    exact = cfg["c_dt_over_dz"] * math.sqrt(p2 / (1.0 + p2))
    assert abs(d["umax"] - exact) <= 1e-14


def test_diagnostic_gauss_residual_of_linear_fields():
    """Reading R18 defines the residual as div_h E - (n_bg - n - n_b) with the finite-volume
    divergence of the Yee grid.  E_r = a r_edge / 2 on the edges has discrete divergence exactly a
    on every row, the axis row included (((j + 1)^2 - j^2) a dr / 2 over (j + 1/2) dr), and
    E_z = b (i + 1/2) dz has d/dz exactly b.  With n = n_bg the residual is a + b everywhere it
    is defined (columns i >= 1); with n = n_bg - a - b it vanishes."""
    nz, nr, h, a, b = 12, 6, 0.05, 0.7, -0.25
    S, P = _diag_state(nz, nr, h)
    S.Er = (a * 0.5 * P.r_edge).expand(nr, nz).clone()
    S.Ez = (b * (P.ii + 0.5) * h).expand(nr, nz).clone()
    S.B = torch.zeros(nr, nz, dtype=F64)
    G = O.gauss_residual(S, P)
    assert G.shape == (nr, nz - 1)
    assert torch.allclose(G, torch.full_like(G, a + b), rtol=0, atol=1e-13)
    assert abs(O.diagnostics(S, P)["gauss_max"] - abs(a + b)) <= 1e-13
    S.M = S.M.clone()
    S.M[0] = S.M[0] - (a + b)
    assert float(O.gauss_residual(S, P).abs().max()) <= 1e-13


def test_diagnostic_gauss_residual_counts_the_driver():
    """The driver's density enters the residual with the electrons' sign (both are electrons):
    a state with no field, n = n_bg and a driver gives residual n_b at each site (i >= 1)."""
    nz, nr, h = 12, 6, 0.05
    cfg = wl.config(None, nz=nz, nr=nr, dz=h, dr=h, nb=0.4, sigma_z=0.1, sigma_r=0.1, zd0=0.3)
    P = O.Params(cfg)
    S = O.initial_state(P)
    S.Ez = torch.zeros(nr, nz, dtype=F64)
    S.Er = torch.zeros(nr, nz, dtype=F64)
    G = O.gauss_residual(S, P)
    nb = O.driver_density(P.ii * h, P.r, -P.dt, P)
    assert torch.allclose(G, nb[:, 1:], rtol=0, atol=1e-14)


def test_diagnostic_counts_nonfinite_values():
    S, P = _diag_state()
    assert O.diagnostics(S, P)["nonfinite"] == 0
    S.Ez = S.Ez.clone()
    S.Ez[2, 3] = float("nan")
    assert O.diagnostics(S, P)["nonfinite"] == 1
