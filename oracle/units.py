"""Unit helpers for the paper's physical set-up (Sec. IV, Eq. (15) and the set-up paragraph).

TEST INFRASTRUCTURE ONLY (used by the unit pins; the product path does not need SI units).

Eq. (15) prints the normalised charge as (2 pi)^{3/2} sigma_x sigma_y sigma_z alpha k_p^{-3}, which
is not dimensionless; with k_p^{+3} (reading R3) it equals N_b k_p^3 / n_0 for a bi-Gaussian bunch of
N_b electrons and peak density ratio alpha = n_b / n_0, and reproduces the paper's values.
"""
from __future__ import annotations

import math

E_CHARGE = 1.602176634e-19      # C
EPS0 = 8.8541878128e-12         # F/m
M_E = 9.1093837015e-31          # kg
C_LIGHT = 299792458.0           # m/s


def plasma_wavenumber(n0_cm3: float) -> float:
    """k_p = omega_p / c in 1/m for an electron density n0 in cm^-3."""
    n = n0_cm3 * 1e6
    return math.sqrt(n * E_CHARGE ** 2 / (EPS0 * M_E)) / C_LIGHT


def peak_density_ratio(charge_C: float, sx_m: float, sy_m: float, sz_m: float, n0_cm3: float) -> float:
    """alpha = n_b / n_0 of a bi-Gaussian bunch of the given charge and rms sizes."""
    nb = charge_C / E_CHARGE / ((2 * math.pi) ** 1.5 * sx_m * sy_m * sz_m)
    return nb / (n0_cm3 * 1e6)


def normalized_charge(alpha: float, sx_m: float, sy_m: float, sz_m: float, n0_cm3: float) -> float:
    """Eq. (15) with the dimensionless reading: (2 pi)^{3/2} sigma_x sigma_y sigma_z alpha k_p^3."""
    kp = plasma_wavenumber(n0_cm3)
    return (2 * math.pi) ** 1.5 * sx_m * sy_m * sz_m * alpha * kp ** 3


def gain_percent(t_fct: float, t_lbm: float) -> float:
    """Table 1 gain column: (FCT - LBM) / FCT in percent."""
    return 100.0 * (t_fct - t_lbm) / t_fct
