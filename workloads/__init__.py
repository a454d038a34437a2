"""Synthetic workloads for the lattice-Boltzmann plasma-wakefield step.

This module holds only workload descriptions and seeded random draws: grid sizes, physical
parameters of the rigid driver and of the plasma profile, run lengths, and the initial density
perturbation.  It contains none of the method's arithmetic (no equilibrium, no forcing, no field
update, no profile evaluation), so that the FP64 oracle and the GPU path can both take their
inputs from it without sharing any computation.

Units are the normalised plasma units of Sec. IV of the paper: lengths in 1/k_p, times in
1/omega_p, densities in units of the plateau density, c = 1.

Presets (sizes and physics follow the paper's set-up of Sec. IV, scaled to the GPU workloads):

  C1   256 x 64,    dz=0.05, tau=0.8, FP64,  uniform plasma, weak driver (n_b=0.01, sigma=0.5),
       +-1e-6 seeded density noise, 500 steps, fixed window.
  C2   2048 x 512,  dz=0.02, FP32, linear entrance ramp of length 10 starting 4 sigma_z ahead
       of the driver, n_b=0.1, sigma_z=1, sigma_r=0.5, moving window, 10,000 steps.
  C2s  the 512 x 128 copy of C2 (same dz, driver, tau; window shortened) used for CPU checks.
  C3   4096 x 1024, dz=0.02, n_b=1, sigma=0.3, tau in {0.6, 0.8, 1.0}, FP64/FP32/FP16, 5,000 steps.
  C4   1024 x 256,  dz=0.05, FP32, tanh ramp, 2,000 steps, witness 4 behind the driver.
  C4s  the 128 x 32 copy of C4 used for the CPU adjoint.
  C5   8192 x 2048, dz=0.02, FP32, tanh ramp of seed-drawn length in [5, 20], 20,000 steps.
  P    the paper's finest grid (Sec. IV, Table 1): 600 x 100 um in cells of 0.25 um at
       n0 = 1e16 cm^-3 (1/k_p = 53.14 um), so 2400 x 400 with dz = 0.0047.  The paper's
       dt_c = 0.147 fs gives c dt/dz = 0.1763; the moving window here shifts one column every
       1/(c dt/dz) steps, which must be an integer, so c dt/dz = 1/6 (dt = 0.139 fs), and 2 mm of
       propagation is 48,000 steps (45,383 at the paper's dt).  Driver sigma_z = 17.7 um
       (0.333), sigma_r = 8.9 um (0.1675), n_b = 0.678 (Q~ = 0.1; 3.39 and 6.78 for Q~ = 0.5
       and 1), uniform plasma, moving window, FP32, tau = 0.8 (the paper takes the smallest
       stable D and does not give it).  The driver sits 200 um behind the window's front edge.
"""
from __future__ import annotations

import copy

import numpy as np

F64, F32, F16, F16N = 0, 1, 2, 3   # F16N: FP16 populations stored off their site's equilibrium
BGK, TRT, REG, MRT = 0, 1, 2, 3
RIGID, PARTICLES = 0, 1

# Field names and order of the C configuration struct (see include/lbmpwfa.h).
CONFIG_FIELDS = (
    "nz", "nr", "dz", "dr", "c_dt_over_dz", "tau", "storage",
    "moving_window", "periodic", "fields_on", "cyl_on",
    "n0", "ramp_kind", "ramp_start", "ramp_len",
    "nb", "sigma_z", "sigma_r", "zd0", "n_floor", "check_every", "fp64_math",
    "collision", "trt_magic", "driver", "max_particles",
    "mrt_se", "mrt_seps", "mrt_sq", "mrt_spi", "resort_every", "bunch_streaming",
)

_BASE = dict(
    nz=64, nr=16, dz=0.05, dr=0.05, c_dt_over_dz=0.2, tau=0.8, storage=F64,
    moving_window=0, periodic=0, fields_on=1, cyl_on=1,
    n0=1.0, ramp_kind=0, ramp_start=0.0, ramp_len=1.0,
    nb=0.0, sigma_z=0.5, sigma_r=0.5, zd0=0.0, n_floor=1e-10, check_every=0, fp64_math=0,
    collision=0, trt_magic=0.25, driver=0, max_particles=0,
    mrt_se=1.0, mrt_seps=1.0, mrt_sq=1.0, mrt_spi=1.0, resort_every=0, bunch_streaming=0,
    # workload-level fields (not part of the C struct)
    noise_amp=0.0, seed=0, nsteps=1, z_behind=4.0,
)


def _window_driver(nz, dz, sigma_z, ahead=8.0):
    """Driver centre placed `ahead` (in units of 1/k_p) behind the front edge of the window."""
    return nz * dz - ahead


def _preset(name):
    b = dict(_BASE)
    if name == "C1":
        b.update(nz=256, nr=64, dz=0.05, dr=0.05, tau=0.8, storage=F64,
                 n0=1.0, ramp_kind=0, nb=0.01, sigma_z=0.5, sigma_r=0.5, zd0=4.0,
                 noise_amp=1e-6, seed=20220114, nsteps=500)
    elif name in ("C2", "C2s"):
        nz, nr = (2048, 512) if name == "C2" else (512, 128)
        zd0 = _window_driver(nz, 0.02, 1.0)
        b.update(nz=nz, nr=nr, dz=0.02, dr=0.02, tau=0.8, storage=F32, moving_window=1,
                 n0=1.0, ramp_kind=1, ramp_start=zd0 + 4.0, ramp_len=10.0,
                 nb=0.1, sigma_z=1.0, sigma_r=0.5, zd0=zd0, n_floor=1e-6, nsteps=10000)
    elif name == "C3":
        zd0 = _window_driver(4096, 0.02, 0.3, ahead=4.0)
        b.update(nz=4096, nr=1024, dz=0.02, dr=0.02, tau=0.8, storage=F32, moving_window=1,
                 n0=1.0, ramp_kind=1, ramp_start=zd0 + 1.2, ramp_len=1.0,
                 nb=1.0, sigma_z=0.3, sigma_r=0.3, zd0=zd0, n_floor=1e-6, nsteps=5000)
    elif name in ("C4", "C4s"):
        if name == "C4":
            nz, nr, dz = 1024, 256, 0.05
        else:
            nz, nr, dz = 128, 32, 0.1
        zd0 = _window_driver(nz, dz, 0.5, ahead=4.0)
        b.update(nz=nz, nr=nr, dz=dz, dr=dz, tau=0.8, storage=F32, moving_window=1,
                 n0=1.0, ramp_kind=2, ramp_start=zd0 + 2.0, ramp_len=10.0 if name == "C4" else 4.0,
                 nb=0.1, sigma_z=0.5, sigma_r=0.5, zd0=zd0, n_floor=1e-6,
                 nsteps=2000 if name == "C4" else 200, z_behind=4.0)
    elif name == "C5":
        zd0 = _window_driver(8192, 0.02, 0.5, ahead=5.0)
        rng = np.random.default_rng(5)
        b.update(nz=8192, nr=2048, dz=0.02, dr=0.02, tau=0.8, storage=F32, moving_window=1,
                 n0=1.0, ramp_kind=2, ramp_start=zd0 + 2.0, ramp_len=float(rng.uniform(5.0, 20.0)),
                 nb=0.5, sigma_z=0.5, sigma_r=0.25, zd0=zd0, n_floor=1e-6, nsteps=20000,
                 seed=5)
    elif name == "P":
        b.update(nz=2400, nr=400, dz=0.0047, dr=0.0047, c_dt_over_dz=1.0 / 6.0, tau=0.8, storage=F32,
                 moving_window=1, n0=1.0, ramp_kind=0, nb=0.678, sigma_z=0.333, sigma_r=0.1675,
                 zd0=_window_driver(2400, 0.0047, 0.333, ahead=3.764), n_floor=1e-6, nsteps=48000)
    else:
        raise KeyError(f"unknown workload preset {name!r}")
    return b


PRESET_NAMES = ("C1", "C2", "C2s", "C3", "C4", "C4s", "C5", "P")


def config(name: str | None = None, **overrides) -> dict:
    """A workload configuration: a preset (or the small base case) with overrides applied."""
    cfg = copy.deepcopy(_preset(name) if name else dict(_BASE))
    for k, v in overrides.items():
        if k not in cfg:
            raise KeyError(f"unknown configuration field {k!r}")
        cfg[k] = v
    return cfg


def density_perturbation(cfg: dict) -> np.ndarray | None:
    """Seeded relative density perturbation, shape [nr][nz], uniform in [-amp, amp).

    The initial electron density is n_bg(z) * (1 + perturbation).  Returns None when the
    configured amplitude is zero."""
    amp = float(cfg.get("noise_amp", 0.0))
    if amp == 0.0:
        return None
    rng = np.random.Generator(np.random.PCG64(int(cfg.get("seed", 0))))
    u = rng.random((int(cfg["nr"]), int(cfg["nz"])))
    return amp * (2.0 * u - 1.0)


def uniform_momentum(cfg: dict, pz: float = 0.0, pr: float = 0.0) -> np.ndarray:
    """Initial momentum field [2][nr][nz] that is uniform in space."""
    out = np.zeros((2, int(cfg["nr"]), int(cfg["nz"])))
    out[0] = pz
    out[1] = pr
    return out


def sine_momentum_z(cfg: dict, eps: float, mode: int = 1) -> np.ndarray:
    """Initial momentum p_z = eps * sin(k z_i), k = 2 pi mode / (nz dz), on cell centres z_i = i dz."""
    nz, nr, dz = int(cfg["nz"]), int(cfg["nr"]), float(cfg["dz"])
    k = 2.0 * np.pi * mode / (nz * dz)
    z = np.arange(nz) * dz
    out = np.zeros((2, nr, nz))
    out[0] = eps * np.sin(k * z)[None, :]
    return out


def linear_radial_momentum(cfg: dict, eps: float) -> np.ndarray:
    """Initial momentum p_r = eps * r_j on cell centres r_j = (j + 1/2) dr."""
    nz, nr, dr = int(cfg["nz"]), int(cfg["nr"]), float(cfg["dr"])
    r = (np.arange(nr) + 0.5) * dr
    out = np.zeros((2, nr, nz))
    out[1] = eps * r[:, None]
    return out


def random_momentum(cfg: dict, amp: float, seed: int = 1) -> np.ndarray:
    """Seeded random momentum field [2][nr][nz], uniform in [-amp, amp)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return amp * (2.0 * rng.random((2, int(cfg["nr"]), int(cfg["nz"]))) - 1.0)


def gaussian_bump(cfg: dict, amp: float, sz: float | None, sr: float | None,
                  zc: float | None = None, rc: float = 0.0) -> np.ndarray:
    """Relative density perturbation amp*exp(-(z-zc)^2/2sz^2 - (r-rc)^2/2sr^2) on cell centres.

    sz or sr set to None drops that factor (a bump uniform along that direction)."""
    nz, nr, dz = int(cfg["nz"]), int(cfg["nr"]), float(cfg["dz"])
    z = np.arange(nz) * dz
    r = (np.arange(nr) + 0.5) * dz
    if zc is None:
        zc = z[nz // 2]
    fz = np.ones(nz) if sz is None else np.exp(-(z - zc) ** 2 / (2 * sz * sz))
    fr = np.ones(nr) if sr is None else np.exp(-(r - rc) ** 2 / (2 * sr * sr))
    return amp * fr[:, None] * fz[None, :]


def bunch(cfg: dict, n: int, gamma: float = 5000.0, emittance: float = 0.0, energy_spread: float = 0.0,
          seed: int = 5) -> np.ndarray:
    """Seeded bi-Gaussian macroparticle bunch, [7][n]: x, y, z, p_x, p_y, p_z, w.

    Positions: Gaussian with rms sigma_r in x and y and sigma_z in z around (0, 0, zd0 - dt), the
    rigid driver's centre at t = -dt (dt = c_dt_over_dz * dz; for gamma >> 1 the bunch moves at
    c).  Momenta at t = -dt/2: p_z = gamma (1 + energy_spread N(0, 1)) (p_z ~ gamma for the
    electrons of the bunch), p_x and p_y Gaussian with rms emittance / sigma_r (the normalised
    rms emittance in units of 1/k_p).  Weights: equal, so that the bunch holds the electrons of the
    rigid driver's peak density n_b over its volume, n_b (2 pi)^(3/2) sigma_r^2 sigma_z, in units
    of n_0 / k_p^3 (the paper's bunch of Sec. IV is of this shape: gamma = 5000, a 74 mm mrad
    emittance and a 0.01 % energy spread).
    """
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    sr, sz = float(cfg["sigma_r"]), float(cfg["sigma_z"])
    dt = float(cfg["c_dt_over_dz"]) * float(cfg["dz"])
    out = np.zeros((7, n))
    out[0] = sr * rng.standard_normal(n)
    out[1] = sr * rng.standard_normal(n)
    out[2] = float(cfg["zd0"]) - dt + sz * rng.standard_normal(n)
    pt = emittance / sr if sr > 0 else 0.0
    out[3] = pt * rng.standard_normal(n)
    out[4] = pt * rng.standard_normal(n)
    out[5] = gamma * (1.0 + energy_spread * rng.standard_normal(n))
    out[6] = float(cfg["nb"]) * (2.0 * np.pi) ** 1.5 * sr * sr * sz / n
    return out
