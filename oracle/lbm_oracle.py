"""FP64 CPU oracle of the lattice-Boltzmann plasma-wakefield step.

TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct definition that the GPU
path is checked against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.  It shares no code with the GPU path.

What is computed follows G. Parise et al., "Lattice Boltzmann simulations of Plasma Wakefield
Acceleration" (arXiv:2201.05473):

  * cold-fluid plasma electrons, Sec. II, Eq. (2) (cold-fluid equations) rewritten in the
    axisymmetric conservative form Eq. (3) with A = (n, n p_z, n p_r), u = c beta and the
    Lorentz source F of Eq. (4);
  * Maxwell's equations Eq. (5) on a Yee (FDTD) grid, with J_e = n beta_e and J_b = n_b beta_b;
  * one D2Q9 lattice per transported scalar A (end of Sec. III), each evolved with the discrete
    Boltzmann equation Eq. (6), the BGK collision Eq. (7), moments Eq. (8), the equilibrium
    Eq. (9), the source Eq. (10), the diffusivity Eq. (12) and the axisymmetric target Eq. (13);
  * boundary populations set to the equilibrium of the boundary moments, Eq. (14), with axis
    symmetry and free flux (Sec. II, paragraph after Eq. (4));
  * the moving window (Sec. II, end).

Normalised units: t omega_p, x k_p, n / n_0, p / (m_e c), e E / (m_e c omega_p), e B / (m_e omega_p),
c = 1.  In these units the electron momentum equation reads dp/dt = -(E + beta x B), Ampere's law
dE/dt = curl B + n_e beta_e + n_b beta_b and Faraday's law dB/dt = -curl E.

Readings of the paper (where it is silent, garbled or inconsistent):

  R1  Eq. (9) is printed with coefficients 1/3, 1/18, 1/6; its zeroth and first moments then do
      not reproduce Eq. (8).  The standard D2Q9 form with c_s^2 = 1/3 is used:
      f_eq_i = w_i A (1 + 3 xi.u + 4.5 (xi.u)^2 - 1.5 u.u), consistent with Eq. (12).
  R2  Faraday's law is printed as dB/dt = +curl E; the standard -curl E is used.
  R4  The D2Q9 table (Fig. 2) is missing; the standard set and weights are used (XI, W below).
  R5  Eq. (6) adds S_i per step while Eq. (10) defines S_i = w_i F with F a rate; the source per
      step is w_i F dt (lattice units, dt_lattice = 1, tau dimensionless).
  R6  The lattice advects with u* = beta * (c dt / dz), which is below c_s = 1/sqrt(3).
  R7  The advecting velocity of all three lattices is beta_e computed from the moments of the
      n and n p lattices (beta = p / gamma, p = A_1,2 / A_0); first moments are not used.
  R8  (beta x B)_z = beta_r B_theta and (beta x B)_r = -beta_z B_theta (axisymmetric TM fields).
  R9  The same scalar operator of Eq. (13) is used for all three lattices.
  R10 The axisymmetric source is F_cyl = -A beta_r / r + D (dA/dr) / r, with dA/dr a central
      difference of the previous step's post-collision moments.
  R11 Ghost (boundary) populations are f_eq of ghost moments: axis mirror with parity (+, +, -),
      copy of the adjacent cell at the outer and rear edges, unperturbed plasma at rest at the
      window front (copy when the window is off).  Corners compose the z rule then the r rule.
  R12 Radially half-shifted Yee grid: E_z at (i+1/2, j), E_r at (i, r=(j+1) dr), B_theta at
      (i+1/2, r=(j+1) dr); E at integer times, B at half-integer times.
  R13 The fluid is kicked with E^n and B^n = (B^{n-1/2} + B^{n+1/2}) / 2; the next Ampere update
      uses the post-kick current (symplectic Euler coupling).
  R15 The window moves one cell every m = 1/(c dt/dz) steps; the new front column is plasma at
      rest at the background density with E = B = 0.
  R17 Fields use zero-gradient ghosts at the outer, rear and front edges; E_r and B_theta vanish
      on the axis.
  R19 Where A_0 <= n_floor the momentum, velocity, current and Lorentz force are zero.
  R23 Ramp shapes: linear n0 clamp((z - z_p)/L, 0, 1) and tanh n0 (1 + tanh(2 (z - z_p)/L - 1)) / 2.
  R28 Bubble length (Sec. IV, Fig. 4): sites of one row, in a given lab z-range, whose density is
      below n* = 0.95 times the local background (vacuum sites excluded), times dz.
  R29 Collision operators other than BGK (Sec. IV names BGK as the simplest choice and leaves
      others to future work without naming one).  Three are offered; all keep the equilibrium of
      Eq. (9) and add the source of Eq. (10) unchanged after relaxing:
        TRT  two relaxation times: the non-equilibrium part f - f_eq is split into its even and
             odd parts under xi -> -xi; the odd part (which carries the flux, hence D) relaxes
             with tau, the even part with tau_plus = 1/2 + Lambda / (tau - 1/2) for a given
             Lambda (Lambda = (tau - 1/2)^2 gives BGK back);
        REG  regularised BGK for an advected scalar: f - f_eq is replaced by its first-order
             Hermite projection w_i xi_i . j_neq / c_s^2, j_neq = sum_i xi_i (f_i - f_eq_i),
             before relaxing with tau (every non-equilibrium moment above the first is dropped);
        MRT  multiple relaxation times: f - f_eq is expanded in the nine moments of D2Q9 given by
             the polynomials 1, 3|xi|^2 - 4, (9|xi|^4 - 21|xi|^2 + 8)/2, xi_z, (3|xi|^2 - 5) xi_z,
             xi_r, (3|xi|^2 - 5) xi_r, xi_z^2 - xi_r^2, xi_z xi_r (density, energy, energy
             square, flux and heat flux in z and r, two stresses; orthogonal on the nine
             velocities), and each moment relaxes with its own rate: the flux moments with 1/tau,
             energy, energy square, heat flux and stresses with given rates s_e, s_eps, s_q,
             s_pi in (0, 2) (the density moment of f - f_eq is zero).  s_e = s_eps = s_pi =
             1/tau_plus with s_q = 1/tau is TRT; all four equal to 1/tau is BGK.
      All three relax the first moment exactly as BGK does, so D of Eq. (12) is unchanged.
  R30 Particle driver (Sec. II: the bunch as macroparticles obeying Eq. (1), coupled through the
      currents projected on the grid).  Macroparticles in 3D Cartesian (x, y, z, p_x, p_y, p_z)
      with weights w (electrons, in units of n_0 / k_p^3).  State after k steps: positions at
      t_{k-1}, momenta at t_{k-1/2}.  Step k: positions move by dt p/gamma to t_k; the current
      w beta at the midpoint is J_b(t_{k-1/2}) of Ampere's law (z and r components); after the
      fields and the fluid, a Boris push with E^k and B^k = (B^{k-1/2} + B^{k+1/2})/2 at the
      new position gives the momenta at t_{k+1/2}.  Projection and interpolation are linear in
      z onto the field's own points and linear in r between its rows: rows r_j = (j + 1/2) dr
      for E_z and densities (the row below the axis folds onto row 0), rows (j + 1) dr for E_r
      and B_theta (their axis value is zero; a share below the first row is dropped).  A node's
      density is its share of w over the annular volume 2 pi r dz dr of the node (charge is
      conserved exactly; rows j >= 1 are exact for a uniform density, row 0 collects 13/12 of
      it because of the fold, as linear weighting in cylindrical geometry does).  A particle
      whose stencil at the midpoint or at the new position (in the window frames before and
      after the step's shift) leaves columns [1, nz - 2] or the rows is lost: its weight is set
      to zero and it no longer moves.  The initial field is the discrete Gauss field of the
      deposited bunch density (positions at t = -dt for E_r, at t = -dt/2 for B_theta, with
      B_theta = E_r as for the rigid driver).

Pins.  tests/test_oracle_pins.py checks this module against closed forms, invariants and brute
force.  The stencil of the axisymmetric source (R10) is pinned by the exact radial heat kernel
and by second-order convergence to it under refinement (a source dividing by another radius
converges at first order).  Three readings have no closed form to check them against and are
pinned only through invariants (a plasma at rest stays at rest, axis mirror symmetry,
conservation): the exact time lag of that source (the previous step's moments; the current ones
would converge at the same order), the time level of the ghost moments (R11), and the
equilibrium ghosts at the axis row.  For those the module is the definition: parity unpinned.

State after k completed steps (k = 0 is the initial state):
    g  [3][9][nr][nz]   post-collision populations of step k-1 (raw values, not deviations)
    M  [3][nr][nz]      their moments A*_k = A_k + dt F_k of step k-1
    Ez [nr][nz]         E_z^{k-1} at (z_i + dz/2, r_j)
    Er [nr][nz]         E_r^{k-1} at (z_i, (j+1) dr)
    B  [nr][nz]         B_theta^{k-1/2} at (z_i + dz/2, (j+1) dr)
    k, s                step count and window shift count; z_i = (s + i) dz, r_j = (j + 1/2) dr

One step k -> k+1:
    1  Ampere   E^k = E^{k-1} + dt (curl B^{k-1/2} + J*_face(M) + J_b(t_{k-1/2}))
    2  Faraday  B^{k+1/2} = B^{k-1/2} - dt curl E^k
    3  fluid    pull-stream, moments, fields at the site, Lorentz + axisymmetric source, BGK
    4  window   shift by one cell when (k+1) is a multiple of m
"""
from __future__ import annotations

import math

import torch

DT = torch.float64

# D2Q9 velocity set (xi_z, xi_r) and weights (R4; Fig. 2 of the paper is not available).
XI = ((0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1))
W = (4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0)
# Index of the opposite direction, xi_{OPP[q]} = -xi_q.
OPP = tuple(XI.index((-xz, -xr)) for (xz, xr) in XI)
# Collision operators (R29).
BGK, TRT, REG, MRT = 0, 1, 2, 3


def mrt_basis():
    """[9][9] rows of the D2Q9 moment basis of R29 (MRT), each row a polynomial in xi evaluated on
    the nine velocities: density, energy, energy square, flux z, heat flux z, flux r, heat flux r,
    normal stress, shear stress."""
    rows = []
    for poly in (lambda z, r, q2: 1.0,
                 lambda z, r, q2: 3.0 * q2 - 4.0,
                 lambda z, r, q2: (9.0 * q2 * q2 - 21.0 * q2 + 8.0) / 2.0,
                 lambda z, r, q2: z,
                 lambda z, r, q2: (3.0 * q2 - 5.0) * z,
                 lambda z, r, q2: r,
                 lambda z, r, q2: (3.0 * q2 - 5.0) * r,
                 lambda z, r, q2: z * z - r * r,
                 lambda z, r, q2: z * r):
        rows.append([poly(z, r, z * z + r * r) for (z, r) in XI])
    return torch.tensor(rows, dtype=DT)
# Mirror parity of (n, n p_z, n p_r) across the axis r = 0 (R11).
PARITY = (1.0, 1.0, -1.0)


def _t(x):
    return x if isinstance(x, torch.Tensor) else torch.tensor(float(x), dtype=DT)


class Params:
    """Run parameters and the quantities derived from them.

    The four parameters that gradients are taken with respect to (n0, ramp_len, sigma_r, nb)
    are held as 0-dim float64 tensors, so autograd can differentiate the whole run."""

    def __init__(self, cfg: dict, theta: dict | None = None):
        self.nz, self.nr = int(cfg["nz"]), int(cfg["nr"])
        self.driver = int(cfg.get("driver", 0))    # 0 rigid bi-Gaussian, 1 macroparticles (R30)
        self.h = float(cfg["dz"])
        if abs(float(cfg["dr"]) - self.h) > 1e-12 * self.h:
            raise ValueError("the lattice needs dz == dr")
        self.lam = float(cfg["c_dt_over_dz"])
        self.dt = self.lam * self.h
        self.tau = float(cfg["tau"])
        if not self.tau > 0.5:
            raise ValueError("tau must exceed 1/2")
        # Eq. (12) in lattice units, converted to normalised units: D = (tau - 1/2)/3 dz^2/dt.
        self.D = (self.tau - 0.5) / 3.0 * self.h * self.h / self.dt
        self.collision = int(cfg.get("collision", BGK))
        if self.collision not in (BGK, TRT, REG, MRT):
            raise ValueError("unknown collision operator")
        # MRT rates of the nine moments (R29): density (any; its non-equilibrium part is zero),
        # energy, energy square, flux z, heat flux z, flux r, heat flux r, two stresses
        s_e, s_eps, s_q, s_pi = (float(cfg.get(k, 1.0)) for k in ("mrt_se", "mrt_seps", "mrt_sq", "mrt_spi"))
        if self.collision == MRT and not all(0.0 < v < 2.0 for v in (s_e, s_eps, s_q, s_pi)):
            raise ValueError("MRT rates must lie in (0, 2)")
        self.mrt_rates = (0.0, s_e, s_eps, 1.0 / self.tau, s_q, 1.0 / self.tau, s_q, s_pi, s_pi)
        self.tau_plus = self.tau
        if self.collision == TRT:
            magic = float(cfg.get("trt_magic", 0.25))
            if not magic > 0.0:
                raise ValueError("the TRT parameter Lambda must be positive")
            self.tau_plus = 0.5 + magic / (self.tau - 0.5)
        self.window = bool(cfg.get("moving_window", 0))
        per = int(cfg.get("periodic", 0))
        self.per_z, self.per_r = bool(per & 1), bool(per & 2)
        self.fields_on = bool(cfg.get("fields_on", 1))
        self.cyl_on = bool(cfg.get("cyl_on", 1))
        if self.per_r and (self.fields_on or self.cyl_on):
            raise ValueError("periodic r needs fields_on = 0 and cyl_on = 0")
        if self.per_z and self.window:
            raise ValueError("periodic z and the moving window exclude each other")
        self.m = 0
        if self.window:
            self.m = int(round(1.0 / self.lam))
            if abs(self.m * self.lam - 1.0) > 1e-9:
                raise ValueError("the moving window needs 1/(c dt/dz) to be an integer")
        self.ramp_kind = int(cfg.get("ramp_kind", 0))
        self.ramp_start = float(cfg.get("ramp_start", 0.0))
        self.sigma_z = float(cfg.get("sigma_z", 1.0))
        self.zd0 = float(cfg.get("zd0", 0.0))
        self.n_floor = float(cfg.get("n_floor", 1e-10))
        theta = theta or {}
        self.n0 = _t(theta.get("n0", cfg.get("n0", 1.0)))
        self.ramp_len = _t(theta.get("ramp_len", cfg.get("ramp_len", 1.0)))
        self.sigma_r = _t(theta.get("sigma_r", cfg.get("sigma_r", 1.0)))
        self.nb = _t(theta.get("nb", cfg.get("nb", 0.0)))
        # grid index vectors: j down the rows, i along the columns
        self.jj = torch.arange(self.nr, dtype=DT)[:, None]
        self.ii = torch.arange(self.nz, dtype=DT)[None, :]
        self.r = (self.jj + 0.5) * self.h            # fluid rows and E_z rows
        self.r_edge = (self.jj + 1.0) * self.h       # E_r and B_theta rows


# ---------------------------------------------------------------------------------------------
# Plasma profile and driver (Sec. IV set-up; ramp shapes are reading R23)
# ---------------------------------------------------------------------------------------------

def n_background(z, P: Params):
    """Unperturbed plasma (ion) density at lab positions z."""
    z = _t(z) if not isinstance(z, torch.Tensor) else z
    if P.ramp_kind == 0:
        return P.n0 * torch.ones_like(z)
    x = (z - P.ramp_start) / P.ramp_len
    if P.ramp_kind == 1:
        return P.n0 * torch.clamp(x, 0.0, 1.0)
    if P.ramp_kind == 2:
        return P.n0 * 0.5 * (1.0 + torch.tanh(2.0 * x - 1.0))
    raise ValueError("unknown ramp kind")


def driver_density(z, r, t: float, P: Params):
    """Rigid bi-Gaussian driver moving at c: n_b exp(-(z - z_d(t))^2/2 sz^2 - r^2/2 sr^2)."""
    zd = P.zd0 + t
    return P.nb * torch.exp(-(z - zd) ** 2 / (2.0 * P.sigma_z ** 2)) \
        * torch.exp(-r ** 2 / (2.0 * P.sigma_r ** 2))


def gauss_field(z, t: float, P: Params):
    """Radial field of the driver alone from the discrete Gauss law (vacuum, E_z = 0).

    Finite-volume form of (1/r) d(r E_r)/dr = -n_b on the rows j: E_r at r = (j+1) dr is
    -(dr / (j+1)) * sum_{j' <= j} (j' + 1/2) n_b(r_j').  For beta_b = 1, B_theta = E_r."""
    nb = driver_density(z, P.r, t, P)
    cum = torch.cumsum((P.jj + 0.5) * nb, dim=0)
    return -P.h * cum / (P.jj + 1.0)


# ---------------------------------------------------------------------------------------------
# Particle driver: macroparticles of Eq. (1) and their projection on the grid (reading R30)
# ---------------------------------------------------------------------------------------------

def _stencil(z, r, s: int, P: Params, zoff: float, edge: bool):
    """Linear weights of lab positions (z, r) onto the nodes z = (s + i + zoff) dz and the rows
    r_j = (j + 1/2) dr (edge False) or (j + 1) dr (edge True).  Returns (i0, fz, j0, fr): node
    pairs (i0, i0 + 1) with weights (1 - fz, fz) and (j0, j0 + 1) with (1 - fr, fr)."""
    u = z / P.h - s - zoff
    v = r / P.h - (1.0 if edge else 0.5)
    i0 = torch.floor(u)
    j0 = torch.floor(v)
    return i0.long(), u - i0, j0.long(), v - j0


def _inside(z, r, s: int, P: Params, zoff: float, edge: bool):
    """The stencil lies in columns [1, nz - 2] and in the rows (row -1 is the fold or the axis)."""
    i0, _, j0, _ = _stencil(z, r, s, P, zoff, edge)
    return (i0 >= 1) & (i0 + 1 <= P.nz - 2) & (j0 >= -1) & (j0 + 1 <= P.nr - 1)


def deposit(val, z, r, s: int, P: Params, zoff: float, edge: bool):
    """Node densities [nr][nz] of the particle quantities val (weights included): each share over
    the node's annular volume 2 pi r_node dz dr (R30).  Particles whose stencil is not inside
    contribute nothing."""
    ok = _inside(z, r, s, P, zoff, edge)
    i0, fz, j0, fr = _stencil(z[ok], r[ok], s, P, zoff, edge)
    v = val[ok]
    out = torch.zeros(P.nr, P.nz, dtype=DT)
    for di, wz in ((0, 1.0 - fz), (1, fz)):
        for dj, wr in ((0, 1.0 - fr), (1, fr)):
            j = j0 + dj
            if edge:
                keep = j >= 0                    # the axis node of E_r / J_r carries nothing
            else:
                keep = torch.ones_like(j, dtype=torch.bool)
                j = torch.clamp(j, min=0)        # the row below the axis folds onto row 0
            out.index_put_((j[keep], (i0 + di)[keep]), (v * wz * wr)[keep], accumulate=True)
    rnode = (P.jj + (1.0 if edge else 0.5)) * P.h
    return out / (2.0 * math.pi * rnode * P.h * P.h)


def gather(F, z, r, s: int, P: Params, zoff: float, edge: bool):
    """F [nr][nz] interpolated at the particles with the same weights as deposit; E_r and
    B_theta (edge rows) are zero on the axis, E_z (centre rows) is even across it.  Only
    meaningful for particles whose stencil is inside."""
    i0, fz, j0, fr = _stencil(z, r, s, P, zoff, edge)
    i0 = torch.clamp(i0, 0, P.nz - 2)
    out = torch.zeros_like(z)
    for di, wz in ((0, 1.0 - fz), (1, fz)):
        for dj, wr in ((0, 1.0 - fr), (1, fr)):
            j = torch.clamp(j0 + dj, -1, P.nr - 1)
            val = F[torch.clamp(j, min=0), i0 + di]
            if edge:
                val = torch.where(j >= 0, val, torch.zeros_like(val))
            out = out + wz * wr * val
    return out


def boris(p, E, B, dt: float):
    """Boris push for dp/dt = -(E + beta x B) (Eq. (1) with the electron charge, normalised):
    half electric kick, rotation about B through 2 atan(|B| dt / (2 gamma)), half kick.
    p, E, B: [3][N] Cartesian."""
    pm = p - 0.5 * dt * E
    gam = torch.sqrt(1.0 + (pm * pm).sum(0))
    t = -0.5 * dt * B / gam
    pp = pm + torch.cross(pm, t, dim=0)
    sv = 2.0 * t / (1.0 + (t * t).sum(0))
    return pm + torch.cross(pp, sv, dim=0) - 0.5 * dt * E


def _beta(p):
    return p / torch.sqrt(1.0 + (p * p).sum(0))


def bunch_move(bunch, k: int, s: int, P: Params):
    """Particle part of step k before the fields: positions from t_{k-1} to t_k, and the
    driver current J_b(t_{k-1/2}) = sum w beta at the midpoints on the E_z and E_r points.
    Returns (bunch', J_bz, J_br)."""
    x, p, w = bunch[0:3], bunch[3:6], bunch[6]
    beta = _beta(p)
    xn = x + P.dt * beta
    xm = 0.5 * (x + xn)
    rm = torch.sqrt(xm[0] ** 2 + xm[1] ** 2)
    rn = torch.sqrt(xn[0] ** 2 + xn[1] ** 2)
    ok = w != 0.0
    for zz, rr, zoff, edge in ((xm[2], rm, 0.5, False), (xm[2], rm, 0.0, True),
                               (xn[2], rn, 0.5, False), (xn[2], rn, 0.0, True), (xn[2], rn, 0.5, True)):
        ok = ok & _inside(zz, rr, s, P, zoff, edge)
    out = bunch.clone()
    out[0:3] = torch.where(ok, xn, x)
    out[6] = torch.where(ok, w, torch.zeros_like(w))
    wl = out[6]
    br = torch.where(rm > 0.0, (xm[0] * beta[0] + xm[1] * beta[1]) / torch.where(rm > 0.0, rm, 1.0),
                     torch.zeros_like(rm))
    Jbz = deposit(wl * beta[2], xm[2], rm, s, P, 0.5, False)
    Jbr = deposit(wl * br, xm[2], rm, s, P, 0.0, True)
    return out, Jbz, Jbr


def bunch_push(bunch, Ez1, Er1, B0, B1, s: int, P: Params):
    """Particle part of step k after the fields: momenta from t_{k-1/2} to t_{k+1/2} with E^k and
    B^k = (B^{k-1/2} + B^{k+1/2})/2 at the positions at t_k (arrays in the frame before the
    step's window shift).  Lost particles (w = 0) keep their momenta."""
    x, p, w = bunch[0:3], bunch[3:6], bunch[6]
    r = torch.sqrt(x[0] ** 2 + x[1] ** 2)
    ez = gather(Ez1, x[2], r, s, P, 0.5, False)
    er = gather(Er1, x[2], r, s, P, 0.0, True)
    bt = 0.5 * (gather(B0, x[2], r, s, P, 0.5, True) + gather(B1, x[2], r, s, P, 0.5, True))
    safe = torch.where(r > 0.0, r, torch.ones_like(r))
    cx = torch.where(r > 0.0, x[0] / safe, torch.zeros_like(r))
    cy = torch.where(r > 0.0, x[1] / safe, torch.zeros_like(r))
    E = torch.stack([er * cx, er * cy, ez])
    B = torch.stack([-bt * cy, bt * cx, torch.zeros_like(bt)])
    pn = boris(p, E, B, P.dt)
    out = bunch.clone()
    out[3:6] = torch.where(w != 0.0, pn, p)
    return out


def bunch_density(bunch, s: int, P: Params, zoff: float, t_ahead: float = 0.0):
    """Bunch density on the nodes z = (s + i + zoff) dz, rows r_j, with the positions moved by
    t_ahead along their velocities."""
    x = bunch[0:3] + t_ahead * _beta(bunch[3:6])
    r = torch.sqrt(x[0] ** 2 + x[1] ** 2)
    return deposit(bunch[6], x[2], r, s, P, zoff, False)


def bunch_gauss_field(nb, P: Params):
    """E_r of the discrete Gauss law for the density nb [nr][nz] (as gauss_field)."""
    cum = torch.cumsum((P.jj + 0.5) * nb, dim=0)
    return -P.h * cum / (P.jj + 1.0)


# ---------------------------------------------------------------------------------------------
# Lattice pieces: equilibrium Eq. (9) (reading R1), velocity from moments (R7, R19)
# ---------------------------------------------------------------------------------------------

def equilibrium(A, uz, ur):
    """Eq. (9) with the standard D2Q9 coefficients: [9][...] populations of scalar A at velocity u."""
    usq = uz * uz + ur * ur
    out = []
    for (xz, xr), w in zip(XI, W):
        cu = xz * uz + xr * ur
        out.append(w * A * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq))
    return torch.stack(out)


def collide(f, feq, P: Params):
    """Relaxation of [9][...] populations f toward feq, without the source: Eq. (7) (BGK) or one
    of the operators of reading R29."""
    neq = f - feq
    if P.collision == BGK:
        return f - neq / P.tau
    if P.collision == TRT:
        mirrored = neq[list(OPP)]
        even = 0.5 * (neq + mirrored)
        odd = 0.5 * (neq - mirrored)
        return f - even / P.tau_plus - odd / P.tau
    if P.collision == MRT:
        # expand neq in the orthogonal basis, relax each moment with its rate, transform back
        B = mrt_basis()                                        # [moment][q]
        norm2 = (B * B).sum(dim=1)
        shape = (9,) + (1,) * (f.dim() - 1)
        moments = torch.tensordot(B, neq, dims=([1], [0]))     # [moment][...]
        rates = torch.tensor(P.mrt_rates, dtype=DT).reshape(shape)
        return f - torch.tensordot(B.t(), rates * moments / norm2.reshape(shape), dims=([1], [0]))
    # REG: keep only the first-order Hermite part of neq, w_i xi_i . j_neq / c_s^2 (c_s^2 = 1/3)
    shape = (9,) + (1,) * (f.dim() - 1)
    xz = torch.tensor([x[0] for x in XI], dtype=DT).reshape(shape)
    xr = torch.tensor([x[1] for x in XI], dtype=DT).reshape(shape)
    w = torch.tensor(W, dtype=DT).reshape(shape)
    jz = (xz * neq).sum(dim=0)
    jr = (xr * neq).sum(dim=0)
    return feq + (1.0 - 1.0 / P.tau) * 3.0 * w * (xz * jz + xr * jr)


def velocity(M, P: Params):
    """beta_e = p / sqrt(1 + p^2), p = (A_1, A_2) / A_0 (Eq. (2) third line); zero where A_0 <= floor."""
    n = M[0]
    live = n > P.n_floor
    safe = torch.where(live, n, torch.ones_like(n))
    pz = torch.where(live, M[1] / safe, torch.zeros_like(n))
    pr = torch.where(live, M[2] / safe, torch.zeros_like(n))
    gam = torch.sqrt(1.0 + pz * pz + pr * pr)
    return pz / gam, pr / gam, live


def current(M, P: Params):
    """Electron current J_e = n_e beta_e of Eq. (5) (sign absorbed as in the paper)."""
    bz, br, _ = velocity(M, P)
    return M[0] * bz, M[0] * br


# ---------------------------------------------------------------------------------------------
# Ghost ring (R11, R17)
# ---------------------------------------------------------------------------------------------

def padded_moments(M, P: Params, s: int):
    """Moments on the ring i in [-1, nz], j in [-1, nr]: shape [3][nr+2][nz+2]."""
    nr = P.nr
    if P.per_z:
        rear, front = M[:, :, -1:], M[:, :, :1]
    else:
        rear = M[:, :, :1]
        if P.window:
            zf = _t((s + P.nz) * P.h)
            nf = n_background(zf, P)
            col = torch.zeros(3, nr, 1, dtype=DT)
            front = torch.cat([nf * torch.ones(1, nr, 1, dtype=DT), col[1:]], dim=0)
        else:
            front = M[:, :, -1:]
    Mz = torch.cat([rear, M, front], dim=2)
    if P.per_r:
        below, above = Mz[:, -1:, :], Mz[:, :1, :]
    else:
        par = torch.tensor(PARITY, dtype=DT)[:, None, None]
        below, above = Mz[:, :1, :] * par, Mz[:, -1:, :]
    return torch.cat([below, Mz, above], dim=1)


def padded_populations(g, Mp, P: Params):
    """Populations on the ring [3][9][nr+2][nz+2]: the interior is g; a ghost position that is a
    periodic image copies the wrapped populations, any other ghost is f_eq of the ghost moments
    (Eq. (14))."""
    bz, br, _ = velocity(Mp, P)
    uz, ur = P.lam * bz, P.lam * br
    gp = torch.stack([equilibrium(Mp[k], uz, ur) for k in range(3)])
    gp = gp.clone()
    gp[:, :, 1:-1, 1:-1] = g
    if P.per_z:
        gp[:, :, 1:-1, 0] = g[:, :, :, -1]
        gp[:, :, 1:-1, -1] = g[:, :, :, 0]
    if P.per_r:
        gp[:, :, 0, 1:-1] = g[:, :, -1, :]
        gp[:, :, -1, 1:-1] = g[:, :, 0, :]
    if P.per_z and P.per_r:
        gp[:, :, 0, 0] = g[:, :, -1, -1]
        gp[:, :, 0, -1] = g[:, :, -1, 0]
        gp[:, :, -1, 0] = g[:, :, 0, -1]
        gp[:, :, -1, -1] = g[:, :, 0, 0]
    return gp


def _left(X, P: Params):
    """X at column i-1: periodic wrap or zero-gradient copy at the rear edge."""
    if P.per_z:
        return torch.roll(X, 1, dims=-1)
    return torch.cat([X[..., :1], X[..., :-1]], dim=-1)


def _right(X, P: Params):
    """X at column i+1: periodic wrap or zero-gradient copy at the front edge."""
    if P.per_z:
        return torch.roll(X, -1, dims=-1)
    return torch.cat([X[..., 1:], X[..., -1:]], dim=-1)


def _below_axis_zero(X):
    """X at row j-1 with X = 0 below the first row (E_r and B_theta vanish on the axis)."""
    return torch.cat([torch.zeros_like(X[:1]), X[:-1]], dim=0)


def _above_copy(X):
    """X at row j+1 with a zero-gradient copy beyond the outer edge."""
    return torch.cat([X[1:], X[-1:]], dim=0)


# ---------------------------------------------------------------------------------------------
# Field update: Eq. (5), Yee scheme (R2, R12, R13, R17)
# ---------------------------------------------------------------------------------------------

def field_update(Ez, Er, B, Mp, k: int, s: int, P: Params, Jb=None):
    """Ampere then Faraday: returns (E_z^k, E_r^k, B^{k+1/2}) from (E^{k-1}, B^{k-1/2}, A*^{k-1}).
    Jb: the particle driver's (J_bz, J_br) at t_{k-1/2} (R30); None for the rigid driver."""
    h, dt = P.h, P.dt
    jj = P.jj
    # (curl B)_z = (1/r) d(r B)/dr at E_z points; the r = 0 edge flux vanishes.
    curl_z = ((jj + 1.0) * B - jj * _below_axis_zero(B)) / ((jj + 0.5) * h)
    # (curl B)_r = -dB/dz at E_r points
    curl_r = -(B - _left(B, P)) / h
    Jz, Jr = current(Mp, P)
    Jz_face = 0.5 * (Jz[1:-1, 1:-1] + Jz[1:-1, 2:])
    Jr_face = 0.5 * (Jr[1:-1, 1:-1] + Jr[2:, 1:-1])
    if Jb is None:
        zE = (s + P.ii + 0.5) * h
        Jbz, Jbr = driver_density(zE, P.r, (k - 0.5) * dt, P), 0.0
    else:
        Jbz, Jbr = Jb
    Ez1 = Ez + dt * (curl_z + Jz_face + Jbz)
    Er1 = Er + dt * (curl_r + Jr_face + Jbr)
    # dB_theta/dt = dE_z/dr - dE_r/dz
    B1 = B + dt * ((_above_copy(Ez1) - Ez1) / h - (_right(Er1, P) - Er1) / h)
    return Ez1, Er1, B1


def fields_at_sites(Ez1, Er1, B0, B1, P: Params):
    """E^k and B^k = (B^{k-1/2} + B^{k+1/2})/2 averaged onto the fluid sites (R12, R13)."""
    Ebar_z = 0.5 * (_left(Ez1, P) + Ez1)
    Ebar_r = 0.5 * (_below_axis_zero(Er1) + Er1)
    Bs = B0 + B1
    Bs_l = _left(Bs, P)
    Bbar = (Bs + Bs_l + _below_axis_zero(Bs) + _below_axis_zero(Bs_l)) / 8.0
    return Ebar_z, Ebar_r, Bbar


# ---------------------------------------------------------------------------------------------
# Fluid update: Eqs. (6)-(10), (13), (14)
# ---------------------------------------------------------------------------------------------

def fluid_update(g, Mp, Ebar_z, Ebar_r, Bbar, P: Params):
    """One collide-stream step of the three lattices; returns (g', A*)."""
    nz, nr = P.nz, P.nr
    gp = padded_populations(g, Mp, P)
    # Eq. (6) in pull form: f_i(x) = g_i(x - xi_i)
    f = torch.stack([torch.stack([gp[kk, q, 1 - xr:1 - xr + nr, 1 - xz:1 - xz + nz]
                                  for q, (xz, xr) in enumerate(XI)]) for kk in range(3)])
    A = f.sum(dim=1)                                    # Eq. (8), zeroth moments
    bz, br, live = velocity(A, P)
    uz, ur = P.lam * bz, P.lam * br                      # R6
    n = A[0]
    zero = torch.zeros_like(n)
    # Eq. (4): F = -e n (E + c beta x B); R8 for the cross product
    Fz = -(Ebar_z + br * Bbar)
    Fr = -(Ebar_r - bz * Bbar)
    F = [zero, torch.where(live, n * Fz, zero), torch.where(live, n * Fr, zero)]
    if P.cyl_on:
        # Eq. (13): -A u_r / r + D (dA/dr) / r, with the lagged radial gradient (R10)
        dAdr = (Mp[:, 2:, 1:-1] - Mp[:, :-2, 1:-1]) / (2.0 * P.h)
        F = [F[kk] - A[kk] * br / P.r + P.D * dAdr[kk] / P.r for kk in range(3)]
    w = torch.tensor(W, dtype=DT)[:, None, None]
    gnew, Mnew = [], []
    for kk in range(3):
        feq = equilibrium(A[kk], uz, ur)
        # Eq. (7) BGK relaxation (or R29) plus the source of Eq. (10) per step (R5)
        gnew.append(collide(f[kk], feq, P) + w * P.dt * F[kk])
        Mnew.append(A[kk] + P.dt * F[kk])
    return torch.stack(gnew), torch.stack(Mnew)


# ---------------------------------------------------------------------------------------------
# State, step, run
# ---------------------------------------------------------------------------------------------

class State:
    __slots__ = ("g", "M", "Ez", "Er", "B", "k", "s", "bunch")

    def __init__(self, g, M, Ez, Er, B, k=0, s=0, bunch=None):
        self.g, self.M, self.Ez, self.Er, self.B, self.k, self.s = g, M, Ez, Er, B, k, s
        self.bunch = bunch   # [7][N]: x, y, z, p_x, p_y, p_z, w (R30), or None

    def clone(self):
        return State(self.g.clone(), self.M.clone(), self.Ez.clone(), self.Er.clone(),
                     self.B.clone(), self.k, self.s, None if self.bunch is None else self.bunch.clone())


def initial_state(P: Params, n_pert=None, p_init=None, bunch=None) -> State:
    """Plasma at its local equilibrium with density n_bg(z)(1 + n_pert) and momentum p_init,
    the driver's discrete Gauss field E_r^{-1} at t = -dt and B^{-1/2} at t = -dt/2, E_z = 0.
    bunch: [7][N] macroparticles (positions at t = -dt, momenta at t = -dt/2) for the particle
    driver (R30)."""
    z = P.ii * P.h
    nbg = n_background(z, P) * torch.ones(P.nr, 1, dtype=DT)
    n = nbg if n_pert is None else nbg * (1.0 + torch.as_tensor(n_pert, dtype=DT))
    if p_init is None:
        A1 = torch.zeros_like(n)
        A2 = torch.zeros_like(n)
    else:
        p = torch.as_tensor(p_init, dtype=DT)
        A1, A2 = n * p[0], n * p[1]
    M = torch.stack([n, A1, A2])
    bz, br, _ = velocity(M, P)
    g = torch.stack([equilibrium(M[kk], P.lam * bz, P.lam * br) for kk in range(3)])
    zeros = torch.zeros(P.nr, P.nz, dtype=DT)
    bt = None if bunch is None else torch.as_tensor(bunch, dtype=DT).clone()
    if P.fields_on and P.driver == 1:
        if bt is None:
            Er, B = zeros.clone(), zeros.clone()
        else:
            Er = bunch_gauss_field(bunch_density(bt, 0, P, 0.0), P)
            B = bunch_gauss_field(bunch_density(bt, 0, P, 0.5, 0.5 * P.dt), P)
    elif P.fields_on:
        Er = gauss_field(z, -P.dt, P)
        B = gauss_field(z + 0.5 * P.h, -0.5 * P.dt, P)
    else:
        Er, B = zeros.clone(), zeros.clone()
    return State(g, M, zeros.clone(), Er, B, 0, 0, bt if P.driver == 1 else None)


def shift_due(k: int, P: Params) -> bool:
    """Whether the window moves at the end of step k (R15)."""
    return P.window and (k + 1) % P.m == 0


def step(S: State, P: Params) -> State:
    """Advance the state by one step (module docstring, steps 1-4)."""
    Mp = padded_moments(S.M, P, S.s)
    bunch, Jb = S.bunch, None
    if bunch is not None:
        bunch, Jbz, Jbr = bunch_move(bunch, S.k, S.s, P)
        Jb = (Jbz, Jbr)
    if P.fields_on:
        Ez1, Er1, B1 = field_update(S.Ez, S.Er, S.B, Mp, S.k, S.s, P, Jb)
        Ebz, Ebr, Bb = fields_at_sites(Ez1, Er1, S.B, B1, P)
    else:
        Ez1, Er1, B1 = S.Ez, S.Er, S.B
        Ebz = Ebr = Bb = torch.zeros(P.nr, P.nz, dtype=DT)
    g1, M1 = fluid_update(S.g, Mp, Ebz, Ebr, Bb, P)
    if bunch is not None:
        bunch = bunch_push(bunch, Ez1, Er1, S.B, B1, S.s, P)
    s = S.s
    if shift_due(S.k, P):
        nf = n_background(_t((s + P.nz) * P.h), P)
        w = torch.tensor(W, dtype=DT)[:, None, None]
        fresh_g = torch.zeros(3, 9, P.nr, 1, dtype=DT)
        fresh_g = torch.cat([(w * nf * torch.ones(1, P.nr, 1, dtype=DT))[None],
                             fresh_g[1:]], dim=0)
        fresh_M = torch.cat([nf * torch.ones(1, P.nr, 1, dtype=DT),
                             torch.zeros(2, P.nr, 1, dtype=DT)], dim=0)
        zc = torch.zeros(P.nr, 1, dtype=DT)
        g1 = torch.cat([g1[..., 1:], fresh_g], dim=-1)
        M1 = torch.cat([M1[..., 1:], fresh_M], dim=-1)
        Ez1 = torch.cat([Ez1[:, 1:], zc], dim=-1)
        Er1 = torch.cat([Er1[:, 1:], zc], dim=-1)
        B1 = torch.cat([B1[:, 1:], zc], dim=-1)
        s += 1
    return State(g1, M1, Ez1, Er1, B1, S.k + 1, s, bunch)


def run(cfg: dict, nsteps: int, n_pert=None, p_init=None, theta=None, callback=None, bunch=None):
    """Initial state plus nsteps steps; returns (final state, Params)."""
    P = Params(cfg, theta)
    S = initial_state(P, n_pert, p_init, bunch)
    for _ in range(nsteps):
        S = step(S, P)
        if callback is not None:
            callback(S, P)
    return S, P


# ---------------------------------------------------------------------------------------------
# Outputs and diagnostics
# ---------------------------------------------------------------------------------------------

def moments_out(S: State, P: Params):
    """[3][nr][nz]: n, J_z, J_r of the last step's post-collision moments."""
    Jz, Jr = current(S.M, P)
    return torch.stack([S.M[0], Jz, Jr])


def fields_out(S: State):
    """[3][nr][nz]: E_z, E_r, B_theta of the state."""
    return torch.stack([S.Ez, S.Er, S.B])


def gauss_residual(S: State, P: Params):
    """div_h E - (n_i - n_e - n_b) at the fluid sites with i >= 1 (reading R18): E^{k-1}, the
    electron density A*_0, ions at n_bg(z), driver at t_{k-1}."""
    h = P.h
    jj = P.jj
    div = (S.Ez - _left(S.Ez, P)) / h \
        + ((jj + 1.0) * S.Er - jj * _below_axis_zero(S.Er)) / ((jj + 0.5) * h)
    z = (S.s + P.ii) * h
    if P.driver == 1:
        nb = torch.zeros_like(S.M[0]) if S.bunch is None else bunch_density(S.bunch, S.s, P, 0.0)
    else:
        nb = driver_density(z, P.r, (S.k - 1) * P.dt, P)
    rho = n_background(z, P) - S.M[0] - nb
    return (div - rho)[:, 1:]


def diagnostics(S: State, P: Params) -> dict:
    """FP64 sums: electron charge in the window, field energy, max |Gauss residual|,
    max |u*| (lattice units) and whether any state value is non-finite."""
    h = P.h
    vol = 2.0 * math.pi * P.r * h * h
    charge = (vol * S.M[0]).sum()
    energy = 0.5 * (2.0 * math.pi * h * h * (P.r * S.Ez ** 2 + P.r_edge * S.Er ** 2
                                             + P.r_edge * S.B ** 2)).sum()
    bz, br, _ = velocity(S.M, P)
    umax = P.lam * torch.sqrt(bz * bz + br * br).max()
    G = gauss_residual(S, P)
    finite = all(bool(torch.isfinite(x).all()) for x in (S.M, S.Ez, S.Er, S.B))
    return dict(charge=float(charge), field_energy=float(energy),
                gauss_max=float(G.abs().max()) if G.numel() else 0.0,
                umax=float(umax), nonfinite=int(not finite), step=S.k, shifts=S.s)


def bubble_length(n, s: int, P: Params, row: int, n_star: float = 0.95, z_from: float = -math.inf,
                  z_to: float = math.inf):
    """Bubble length of Sec. IV (Fig. 4): the number of sites whose electron density lies below
    the threshold n* times the unperturbed density, times dz.  Reading R28: the sites are those of
    one row (the paper takes longitudinal profiles at a fixed radius) at lab positions
    z_i = (s + i) dz in [z_from, z_to], the threshold is relative to the local background n_bg(z_i)
    (so a density ramp is not counted), sites in vacuum (n_bg = 0) are excluded and the comparison
    is strict.  n: the electron density [nr][nz] (raw, FP64).  Returns (count, count * dz)."""
    z = (s + torch.arange(P.nz, dtype=DT)) * P.h
    nbg = n_background(z, P)
    sel = (z >= z_from) & (z <= z_to) & (nbg > 0.0) & (n[row] < n_star * nbg)
    count = int(sel.sum())
    return count, count * P.h


def objective(S: State, P: Params, z_behind: float):
    """Witness objective: E_z on the first row, linearly interpolated in z at z_d - z_behind,
    where z_d is the driver centre at the time level of the state's E (t_{k-1})."""
    zstar = P.zd0 + (S.k - 1) * P.dt - z_behind
    x = zstar / P.h - S.s - 0.5
    i0 = int(math.floor(x))
    if not (0 <= i0 < P.nz - 1):
        raise ValueError("witness position outside the window")
    w = x - i0
    return (1.0 - w) * S.Ez[0, i0] + w * S.Ez[0, i0 + 1]


def rel_err(x, ref) -> float:
    """Max-norm error relative to the max-norm of the reference (reading R24)."""
    x = torch.as_tensor(x, dtype=DT)
    ref = torch.as_tensor(ref, dtype=DT)
    den = float(ref.abs().max())
    num = float((x - ref).abs().max())
    return num / den if den > 0 else num
