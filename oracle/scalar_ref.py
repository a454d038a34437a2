"""Scalar per-site re-statement of the oracle step, for tiny grids only.

TEST INFRASTRUCTURE ONLY (pin "brute force": the vectorised oracle in lbm_oracle.py must agree
with this loop-by-loop version to round-off).  Everything here is plain Python floats, one site
and one population at a time, with the boundary rules written as explicit per-position
functions instead of padded arrays.  The definitions are the same ones listed in the header of
lbm_oracle.py (Eqs. (4)-(14) of the paper plus readings R1-R23 and R29).
"""
from __future__ import annotations

import math

XI = ((0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1))
W = (4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36)


class Grid:
    def __init__(self, cfg):
        self.nz, self.nr = int(cfg["nz"]), int(cfg["nr"])
        self.h = float(cfg["dz"])
        self.lam = float(cfg["c_dt_over_dz"])
        self.dt = self.lam * self.h
        self.tau = float(cfg["tau"])
        self.D = (self.tau - 0.5) / 3 * self.h ** 2 / self.dt
        self.coll = int(cfg.get("collision", 0))          # 0 BGK, 1 TRT, 2 regularised, 3 MRT (R29)
        self.tau_p = self.tau
        if self.coll == 1:
            self.tau_p = 0.5 + float(cfg.get("trt_magic", 0.25)) / (self.tau - 0.5)
        s_e, s_eps, s_q, s_pi = (float(cfg.get(k, 1.0)) for k in ("mrt_se", "mrt_seps", "mrt_sq", "mrt_spi"))
        self.mrt = (0.0, s_e, s_eps, 1.0 / self.tau, s_q, 1.0 / self.tau, s_q, s_pi, s_pi)
        self.window = bool(cfg.get("moving_window", 0))
        per = int(cfg.get("periodic", 0))
        self.pz, self.pr = bool(per & 1), bool(per & 2)
        self.fields = bool(cfg.get("fields_on", 1))
        self.cyl = bool(cfg.get("cyl_on", 1))
        self.m = int(round(1 / self.lam)) if self.window else 0
        self.kind = int(cfg.get("ramp_kind", 0))
        self.zp = float(cfg.get("ramp_start", 0.0))
        self.L = float(cfg.get("ramp_len", 1.0))
        self.n0 = float(cfg.get("n0", 1.0))
        self.nb = float(cfg.get("nb", 0.0))
        self.sz = float(cfg.get("sigma_z", 1.0))
        self.sr = float(cfg.get("sigma_r", 1.0))
        self.zd0 = float(cfg.get("zd0", 0.0))
        self.floor = float(cfg.get("n_floor", 1e-10))

    def nbg(self, z):
        if self.kind == 0:
            return self.n0
        x = (z - self.zp) / self.L
        if self.kind == 1:
            return self.n0 * min(max(x, 0.0), 1.0)
        return self.n0 * 0.5 * (1 + math.tanh(2 * x - 1))

    def driver(self, z, r, t):
        return self.nb * math.exp(-(z - self.zd0 - t) ** 2 / (2 * self.sz ** 2)
                                  - r ** 2 / (2 * self.sr ** 2))


def moment_poly(m, z, r):
    """Value of the m-th D2Q9 moment polynomial of R29 (MRT) at the velocity (z, r)."""
    q2 = z * z + r * r
    return (1.0, 3 * q2 - 4, (9 * q2 * q2 - 21 * q2 + 8) / 2, z, (3 * q2 - 5) * z, r, (3 * q2 - 5) * r,
            z * z - r * r, z * r)[m]


def feq(q, A, uz, ur):
    cu = XI[q][0] * uz + XI[q][1] * ur
    return W[q] * A * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (uz * uz + ur * ur))


def beta(G, M3):
    n, a1, a2 = M3
    if not n > G.floor:
        return 0.0, 0.0, False
    pz, pr = a1 / n, a2 / n
    gam = math.sqrt(1 + pz * pz + pr * pr)
    return pz / gam, pr / gam, True


def ghost_M(G, M, s, i, j):
    """Moments at ring position (i, j): z rule first, then r rule."""
    nz, nr = G.nz, G.nr
    if 0 <= i < nz:
        col = [[M[k][jj][i] for jj in range(nr)] for k in range(3)]
    elif i == -1:
        src = nz - 1 if G.pz else 0
        col = [[M[k][jj][src] for jj in range(nr)] for k in range(3)]
    else:  # i == nz
        if G.pz:
            col = [[M[k][jj][0] for jj in range(nr)] for k in range(3)]
        elif G.window:
            nf = G.nbg((s + nz) * G.h)
            col = [[nf] * nr, [0.0] * nr, [0.0] * nr]
        else:
            col = [[M[k][jj][nz - 1] for jj in range(nr)] for k in range(3)]
    if 0 <= j < nr:
        return [col[k][j] for k in range(3)]
    if j == -1:
        if G.pr:
            return [col[k][nr - 1] for k in range(3)]
        return [col[0][0], col[1][0], -col[2][0]]
    if G.pr:
        return [col[k][0] for k in range(3)]
    return [col[k][nr - 1] for k in range(3)]


def pulled(G, g, M, s, k, q, i, j):
    """f_q of lattice k at site (i, j): g_q at (i - xi_z, j - xi_r) or its ghost value."""
    a, b = i - XI[q][0], j - XI[q][1]
    out_z = not (0 <= a < G.nz)
    out_r = not (0 <= b < G.nr)
    if (out_z and not G.pz) or (out_r and not G.pr):
        Mg = ghost_M(G, M, s, a, b)
        bz, br, _ = beta(G, Mg)
        return feq(q, Mg[k], G.lam * bz, G.lam * br)
    return g[k][q][b % G.nr][a % G.nz]


def J_at(G, M, s, i, j):
    Mg = ghost_M(G, M, s, i, j)
    bz, br, _ = beta(G, Mg)
    return Mg[0] * bz, Mg[0] * br


def Bval(G, B, i, j):
    """B_theta with its ghost rules: zero on the axis row, rear copy or periodic wrap."""
    if j < 0:
        return 0.0
    if i < 0:
        i = G.nz - 1 if G.pz else 0
    return B[j][i]


def step(G, st):
    g, M, Ez, Er, B, k, s = st
    nz, nr, h, dt = G.nz, G.nr, G.h, G.dt
    Ez1 = [row[:] for row in Ez]
    Er1 = [row[:] for row in Er]
    B1 = [row[:] for row in B]
    if G.fields:
        for j in range(nr):
            for i in range(nz):
                rj = (j + 0.5) * h
                # (1/r) d(r B)/dr between the edges r = j h and r = (j + 1) h
                curl_z = ((j + 1) * h * Bval(G, B, i, j) - j * h * Bval(G, B, i, j - 1)) / (rj * h)
                Jz0, _ = J_at(G, M, s, i, j)
                Jz1, _ = J_at(G, M, s, i + 1, j)
                zE = (s + i + 0.5) * h
                Jb = G.driver(zE, rj, (k - 0.5) * dt)
                Ez1[j][i] = Ez[j][i] + dt * (curl_z + 0.5 * (Jz0 + Jz1) + Jb)
                curl_r = -(Bval(G, B, i, j) - Bval(G, B, i - 1, j)) / h
                _, Jr0 = J_at(G, M, s, i, j)
                _, Jr1 = J_at(G, M, s, i, j + 1)
                Er1[j][i] = Er[j][i] + dt * (curl_r + 0.5 * (Jr0 + Jr1))
        for j in range(nr):
            for i in range(nz):
                ez_up = Ez1[j + 1][i] if j + 1 < nr else Ez1[nr - 1][i]
                ip = (i + 1) % nz if G.pz else min(i + 1, nz - 1)
                B1[j][i] = B[j][i] + dt * ((ez_up - Ez1[j][i]) / h - (Er1[j][ip] - Er1[j][i]) / h)
    gn = [[[[0.0] * nz for _ in range(nr)] for _ in range(9)] for _ in range(3)]
    Mn = [[[0.0] * nz for _ in range(nr)] for _ in range(3)]
    for j in range(nr):
        for i in range(nz):
            f = [[pulled(G, g, M, s, kk, q, i, j) for q in range(9)] for kk in range(3)]
            A = [sum(f[kk]) for kk in range(3)]
            bz, br, live = beta(G, A)
            uz, ur = G.lam * bz, G.lam * br
            if G.fields:
                im = (i - 1) % nz if G.pz else max(i - 1, 0)
                Ebz = 0.5 * (Ez1[j][im] + Ez1[j][i])
                Ebr = 0.5 * ((Er1[j - 1][i] if j > 0 else 0.0) + Er1[j][i])
                Bb = 0.0
                for (a, b) in ((i, j), (i - 1, j), (i, j - 1), (i - 1, j - 1)):
                    Bb += Bval(G, B, a, b) + Bval(G, B1, a, b)
                Bb /= 8.0
            else:
                Ebz = Ebr = Bb = 0.0
            F = [0.0, 0.0, 0.0]
            if live:
                F[1] = A[0] * (-(Ebz + br * Bb))
                F[2] = A[0] * (-(Ebr - bz * Bb))
            if G.cyl:
                rj = (j + 0.5) * h
                up = ghost_M(G, M, s, i, j + 1)
                dn = ghost_M(G, M, s, i, j - 1)
                for kk in range(3):
                    F[kk] += -A[kk] * br / rj + G.D * (up[kk] - dn[kk]) / (2 * h) / rj
            for kk in range(3):
                fe = [feq(q, A[kk], uz, ur) for q in range(9)]
                neq = [f[kk][q] - fe[q] for q in range(9)]
                jz = sum(XI[q][0] * neq[q] for q in range(9))
                jr = sum(XI[q][1] * neq[q] for q in range(9))
                for q in range(9):
                    if G.coll == 0:
                        post = f[kk][q] - neq[q] / G.tau
                    elif G.coll == 1:
                        back = [p for p in range(9) if XI[p][0] == -XI[q][0] and XI[p][1] == -XI[q][1]][0]
                        even = 0.5 * (neq[q] + neq[back])
                        odd = 0.5 * (neq[q] - neq[back])
                        post = f[kk][q] - even / G.tau_p - odd / G.tau
                    elif G.coll == 3:
                        post = f[kk][q]
                        for m in range(9):
                            row = [moment_poly(m, XI[p][0], XI[p][1]) for p in range(9)]
                            nm = sum(row[p] * neq[p] for p in range(9))
                            post -= G.mrt[m] * nm / sum(v * v for v in row) * row[q]
                    else:
                        post = fe[q] + (1 - 1 / G.tau) * 3 * W[q] * (XI[q][0] * jz + XI[q][1] * jr)
                    gn[kk][q][j][i] = post + W[q] * dt * F[kk]
                Mn[kk][j][i] = A[kk] + dt * F[kk]
    if G.window and (k + 1) % G.m == 0:
        nf = G.nbg((s + nz) * h)
        for j in range(nr):
            for kk in range(3):
                for q in range(9):
                    row = gn[kk][q][j]
                    gn[kk][q][j] = row[1:] + [W[q] * nf if kk == 0 else 0.0]
                Mn[kk][j] = Mn[kk][j][1:] + [nf if kk == 0 else 0.0]
            Ez1[j] = Ez1[j][1:] + [0.0]
            Er1[j] = Er1[j][1:] + [0.0]
            B1[j] = B1[j][1:] + [0.0]
        s += 1
    return (gn, Mn, Ez1, Er1, B1, k + 1, s)


def from_tensors(S):
    """Convert an oracle State into nested lists."""
    return (S.g.tolist(), S.M.tolist(), S.Ez.tolist(), S.Er.tolist(), S.B.tolist(), S.k, S.s)
