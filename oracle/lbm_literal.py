"""Second FP64 oracle of the axisymmetric MRT lattice Boltzmann step (arXiv:1409.5929).

TEST INFRASTRUCTURE ONLY.  This module exists to check the first oracle
(``lbm_oracle.c``) on tiny grids: a literal, per-node, slow transcription of
the equations in plain Python and NumPy.  It shares no code, table or
constant with that oracle or with the GPU library; only the test suite may
import it.

How it differs from the C oracle, so that a slip in either shows up:
  - the matrix M of Eq. (18) is built from the polynomial definition of its
    rows (density, energy, energy square, momentum, energy flux, stress),
    not typed in as a table; its inverse is numpy.linalg.inv;
  - the equilibrium of a wall reconstruction is Eq. (32) itself, not
    M^{-1} m^eq (the two agree, pin P3);
  - streaming pulls: f_i(x, t+1) = f_i^+(x - e_i, t), the source found by
    wrap-around, the axis mirror or not at all (the slot is then NaN);
  - every node is a separate Python call; nothing is vectorised.

Points the paper leaves open are read exactly as in the C oracle and the
library (the same readings, written independently here):
  grid     row j at r = r0 + j, column k at z = k; wall nodes on rows 0,
           nr-1 and columns 0, nz-1 (Sec. 4 preamble);
  walls    non-equilibrium extrapolation (Sec. 4 preamble): the wall state
           (density of the fluid neighbour B, zero velocity, wall
           temperature) plus B's non-equilibrium part, then an ordinary
           collision at the wall state; B is the normal neighbour, the
           diagonal one at a corner; adiabatic walls copy T_B, isoflux walls
           (Sec. 4.4) add q'/k; a fixed-temperature radial wall wins at a
           corner;
  axis     cell-centred rows (r0 = 1/2) and a ghost row at r = -1/2 with
           f_i(-r) = -f_i*(r) for the r-weighted f and g_i(-r) = g_i*(r);
  inlet    (Sec. 4.1) column 0 takes u = (0, u_in), T_zmin (fixed) and B's
           density; the outlet column nz-1 takes B's u and T and rho = 1;
  source   Eq. (24) with the axisymmetric part a_r of F~ not divided by phi
           (src_printed = 0), or exactly as printed (src_printed = 1);
  start    f = M^{-1}(m^eq - S/2) at rho = 1 and the given u, g = g^eq
           (the change of variables before Eq. 15);
  porosity K(phi) = K_ref kappa(phi)/kappa(phi_ref), kappa = phi^3/(1-phi)^2
           (Eq. 8 with the particle diameter fixed), F_phi from Eq. (8) when
           the given value is negative;
  buoyancy +z, g beta dT = (Ma c_s)^2 / L when Ra > 0 (text before Eq. 39).
"""
from __future__ import annotations

import math

import numpy as np

# Eq. (14) with c = 1: the velocities in (r, z) order; Eq. (34) takes the first five.
E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
# Weights after Eq. (32); Eq. (36) with omega~_0 = 3/5.
OMEGA = [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4
OMEGA_T = [3.0 / 5.0] + [(1.0 - 3.0 / 5.0) / 4.0] * 4
CS2 = 1.0 / 3.0   # c_s^2, c_s = c / sqrt(3) (after Eq. 25)
CST2 = 1.0 / 5.0  # c_sT^2 (after Eq. 36)
DT = 1.0          # delta_t (Sec. 4 preamble)

SIDES = {"wall": 0, "axis": 1, "periodic": 2, "flow": 3}
THERMS = {"fixed": 0, "adiabatic": 1, "flux": 2}


def moment_matrix() -> np.ndarray:
    """M of Eq. (18): row a is the moment a evaluated on each velocity e_i,
    in the order of Eq. (17): 1, e = -4 + 3|e|^2, eps = 4 - 21/2 |e|^2 +
    9/2 |e|^4, e_r, q_r = (-5 + 3|e|^2) e_r, e_z, q_z = (-5 + 3|e|^2) e_z,
    e_r^2 - e_z^2, e_r e_z."""
    cols = []
    for er, ez in E:
        e2 = er * er + ez * ez
        cols.append([1.0, -4.0 + 3.0 * e2, 4.0 - 10.5 * e2 + 4.5 * e2 * e2, er,
                     (-5.0 + 3.0 * e2) * er, ez, (-5.0 + 3.0 * e2) * ez, er * er - ez * ez, er * ez])
    return np.array(cols, dtype=np.float64).T


def _kappa(ph):
    return ph ** 3 / (1.0 - ph) ** 2


class LiteralLattice:
    """One lattice; ``cfg`` uses the keys of ``oracle.Oracle``."""

    def __init__(self, cfg: dict, phi_field=None, init=None):
        c = dict(side_rmin="wall", side_rmax="wall", side_z="wall", therm_rmin="fixed",
                 therm_rmax="fixed", therm_z="adiabatic", r0=1.0, L=1.0, phi=1.0, Da=1e8,
                 F_phi=0.0, Ra=0.0, Pr=1.0, J=1.0, lam=1.0, Ma=0.1, tau_nu=0.0, accel_r=0.0,
                 accel_z=0.0, s_e=1.1, s_eps=1.1, s_q=1.2, s_j=1.0, src_printed=0, T_rmin=0.0,
                 T_rmax=0.0, T_zmin=0.0, T_zmax=0.0, T_ref=0.0, T_init=0.0, delta_T=0.0,
                 flux_rmin=0.0, flux_rmax=0.0, flux_zlo=-math.inf, flux_zhi=math.inf, u_in=0.0)
        c.update(cfg)
        for k in ("side_rmin", "side_rmax", "side_z"):
            c[k] = SIDES[c[k]] if isinstance(c[k], str) else int(c[k])
        for k in ("therm_rmin", "therm_rmax", "therm_z"):
            c[k] = THERMS[c[k]] if isinstance(c[k], str) else int(c[k])
        self.c = c
        self.nr, self.nz = int(c["nr"]), int(c["nz"])
        # Eq. (39), Eq. (31), Eq. (9)
        cs = math.sqrt(CS2)
        if c["tau_nu"] > 0:
            self.tau = c["tau_nu"]
        else:
            self.tau = 0.5 + c["Ma"] * c["J"] * c["L"] * math.sqrt(c["Pr"]) / (cs * DT * math.sqrt(c["Ra"]))
        self.tau_T = CS2 * c["lam"] * (self.tau - 0.5) / (CST2 * c["J"] * c["Pr"])
        self.nu_e = CS2 * (self.tau - 0.5) * DT
        self.nu = self.nu_e / c["J"]
        self.K_ref = c["Da"] * c["L"] ** 2
        dT = c["delta_T"] if c["delta_T"] != 0 else c["T_rmin"] - c["T_rmax"]
        self.gbeta = (c["Ma"] * cs) ** 2 / c["L"] / dT if c["Ra"] > 0 else 0.0
        # Eq. (23) with s_rho = 1 and s_nu = 1 / tau_nu
        self.Lam = np.diag([1.0, c["s_e"], c["s_eps"], c["s_j"], c["s_q"], c["s_j"], c["s_q"],
                            1.0 / self.tau, 1.0 / self.tau])
        self.M = moment_matrix()
        self.Minv = np.linalg.inv(self.M)
        nz, nr = self.nz, self.nr
        self.r = np.array([c["r0"] + j for j in range(nr)], dtype=np.float64)
        self.phi = np.full((nz, nr), float(c["phi"])) if phi_field is None else \
            np.array(phi_field, dtype=np.float64)
        self.K = np.full((nz, nr), self.K_ref)
        self.Fphi = np.full((nz, nr), float(c["F_phi"]))
        for k in range(nz):
            for j in range(nr):
                ph = self.phi[k, j]
                if phi_field is not None:
                    self.K[k, j] = self.K_ref * _kappa(ph) / _kappa(c["phi"])
                if c["F_phi"] < 0:
                    self.Fphi[k, j] = 1.75 / math.sqrt(150.0 * ph ** 3)  # Eq. (8)
        self.f = np.empty((nz, nr, 9))
        self.g = np.empty((nz, nr, 5))
        for k in range(nz):
            for j in range(nr):
                uz0 = init[0][k][j] if init is not None else 0.0
                ur0 = init[1][k][j] if init is not None else 0.0
                T0 = init[2][k][j] if init is not None else c["T_init"]
                meq = self.m_eq(self.r[j], 1.0, ur0, uz0, self.phi[k, j])
                S = self.S(k, j, 1.0, ur0, uz0, T0)
                self.f[k, j] = self.Minv @ (meq - 0.5 * DT * S)
                self.g[k, j] = [self.g_eq(i, T0, ur0, uz0) for i in range(5)]
        self.t = 0
        self.macros_all()

    # ---- geometry ----------------------------------------------------------
    def node_class(self, j, k):
        """(r_min wall, r_max wall, z_min boundary, z_max boundary) flags."""
        c = self.c
        zb = c["side_z"] in (0, 3)
        return (c["side_rmin"] == 0 and j == 0, c["side_rmax"] == 0 and j == self.nr - 1,
                zb and k == 0, zb and k == self.nz - 1)

    def mask(self, j, k):
        a, b, cz, d = self.node_class(j, k)
        return int(a) | 2 * int(b) | 4 * int(cz) | 8 * int(d) | 16 * int(self.c["side_rmin"] == 1 and j == 0)

    def is_boundary(self, j, k):
        return any(self.node_class(j, k))

    def owner(self, j, k):
        a, b, cz, d = self.node_class(j, k)
        return j + int(a) - int(b), k + int(cz) - int(d)

    # ---- the equations -------------------------------------------------------
    def G(self, T):
        """Eq. (7): (G_r, G_z)."""
        return self.c["accel_r"], self.gbeta * (T - self.c["T_ref"]) + self.c["accel_z"]

    def m_eq(self, r, rho, ur, uz, phi):
        """Eqs. (19)-(20)."""
        u2 = ur * ur + uz * uz
        return r * np.array([rho, -2.0 * rho + 3.0 * rho * u2 / phi, rho - 3.0 * rho * u2 / phi,
                             rho * ur, -rho * ur, rho * uz, -rho * uz,
                             rho * (ur * ur - uz * uz) / phi, rho * ur * uz / phi])

    def f_eq(self, r, rho, ur, uz, phi):
        """Eq. (32)."""
        out = np.empty(9)
        u2 = ur * ur + uz * uz
        for i, (er, ez) in enumerate(E):
            eu = er * ur + ez * uz
            out[i] = OMEGA[i] * r * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * phi * CS2 * CS2)
                                           - u2 / (2.0 * phi * CS2))
        return out

    def g_eq(self, i, T, ur, uz):
        """Eq. (35)."""
        er, ez = E[i]
        return OMEGA_T[i] * T * (1.0 + (er * ur + ez * uz) / CST2)

    def forces(self, k, j, ur, uz, T):
        """Eq. (6) and a_r of Eq. (25): (F_r, F_z, a_r)."""
        r, phi, K, Fp = self.r[j], self.phi[k, j], self.K[k, j], self.Fphi[k, j]
        Gr, Gz = self.G(T)
        um = math.sqrt(ur * ur + uz * uz)
        Fr = -phi * self.nu / K * ur - phi * Fp / math.sqrt(K) * um * ur + phi * Gr
        Fz = -phi * self.nu / K * uz - phi * Fp / math.sqrt(K) * um * uz + phi * Gz
        ar = CS2 * (1.0 - 2.0 * (self.tau - 0.5) * DT * ur / r) / r
        return Fr, Fz, ar

    def S(self, k, j, rho, ur, uz, T):
        """Eq. (24) with F~ of Eq. (25)."""
        r, phi = self.r[j], self.phi[k, j]
        Fr, Fz, ar = self.forces(k, j, ur, uz, T)
        Ftr, Ftz = Fr + ar, Fz
        if self.c["src_printed"]:
            a1 = 6.0 * (ur * Ftr + uz * Ftz) / phi
            a7 = 2.0 * (ur * Ftr - uz * Ftz) / phi
            a8 = (ur * Ftz + uz * Ftr) / phi
        else:  # a_r enters without the 1/phi of the porous-medium force
            a1 = 6.0 * ((ur * Fr + uz * Fz) / phi + ur * ar)
            a7 = 2.0 * ((ur * Fr - uz * Fz) / phi + ur * ar)
            a8 = (ur * Fz + uz * Fr) / phi + uz * ar
        return r * rho * np.array([0.0, a1, -a1, Ftr, -Ftr, Ftz, -Ftz, a7, a8])

    def fluid_macros(self, k, j):
        """Eqs. (38), (26), (29), (30), (28) at a fluid node: (rho, u_r, u_z, T)."""
        r, phi, K, Fp = self.r[j], self.phi[k, j], self.K[k, j], self.Fphi[k, j]
        f, g = self.f[k, j], self.g[k, j]
        T = float(np.sum(g))
        rho = float(np.sum(f)) / r
        Gr, Gz = self.G(T)
        er_f = sum(E[i][0] * f[i] for i in range(9))
        ez_f = sum(E[i][1] * f[i] for i in range(9))
        vr = (er_f + 0.5 * DT * r * phi * rho * Gr + 0.5 * DT * rho * CS2) / rho
        vz = (ez_f + 0.5 * DT * r * phi * rho * Gz) / rho
        lr0 = 0.5 * ((r * r + CS2 * (self.tau - 0.5) * DT * DT) / r + r * phi * 0.5 * DT * self.nu / K)
        lz0 = 0.5 * (r * r / r + r * phi * 0.5 * DT * self.nu / K)
        l1 = r * phi * 0.5 * DT * Fp / math.sqrt(K)
        vm = math.sqrt(vr * vr + vz * vz)
        ur = vr / (lr0 + math.sqrt(lr0 * lr0 + l1 * vm))
        uz = vz / (lz0 + math.sqrt(lz0 * lz0 + l1 * vm))
        return rho, ur, uz, T

    def wall_state(self, j, k):
        """Macroscopic state of a boundary node from its owner's (walls, isoflux
        window, inlet and outlet)."""
        c = self.c
        a, b, cz, d = self.node_class(j, k)
        jb, kb = self.owner(j, k)
        rhoB, urB, uzB, TB = self.mac[kb][jb]
        rho, ur, uz = rhoB, 0.0, 0.0
        if c["side_z"] == 3 and not (a or b):
            if cz:
                uz = c["u_in"]
            else:
                rho, ur, uz = 1.0, urB, uzB
        fixed = 0
        if a and c["therm_rmin"] == fixed:
            T = c["T_rmin"]
        elif b and c["therm_rmax"] == fixed:
            T = c["T_rmax"]
        elif cz and c["therm_z"] == fixed:
            T = c["T_zmin"]
        elif d and c["therm_z"] == fixed and c["side_z"] != 3:
            T = c["T_zmax"]
        else:
            T = TB
            heated = c["flux_zlo"] <= k <= c["flux_zhi"] and not ((cz or d) and c["therm_z"] == fixed)
            if heated and a and c["therm_rmin"] == 2:
                T = TB + c["flux_rmin"]
            elif heated and b and c["therm_rmax"] == 2:
                T = TB + c["flux_rmax"]
        return rho, ur, uz, T

    def macros_all(self):
        nz, nr = self.nz, self.nr
        self.mac = [[None] * nr for _ in range(nz)]
        for k in range(nz):
            for j in range(nr):
                if not self.is_boundary(j, k):
                    self.mac[k][j] = self.fluid_macros(k, j)
        for k in range(nz):
            for j in range(nr):
                if self.is_boundary(j, k):
                    self.mac[k][j] = self.wall_state(j, k)

    def collide(self, k, j):
        """Eqs. (21)-(22) and (33), (35), (37) at one node: (f^+, g^+)."""
        rho, ur, uz, T = self.mac[k][j]
        r, phi = self.r[j], self.phi[k, j]
        if self.is_boundary(j, k):
            # wall state's equilibrium plus the owner B's non-equilibrium part
            jb, kb = self.owner(j, k)
            rhoB, urB, uzB, TB = self.mac[kb][jb]
            f = self.f_eq(r, rho, ur, uz, phi) + (self.f[kb, jb] -
                                                  self.f_eq(self.r[jb], rhoB, urB, uzB, self.phi[kb, jb]))
            g = np.array([self.g_eq(i, T, ur, uz) + self.g[kb, jb][i] - self.g_eq(i, TB, urB, uzB)
                          for i in range(5)])
        else:
            f, g = self.f[k, j], self.g[k, j]
        m = self.M @ f
        mp = m - self.Lam @ (m - self.m_eq(r, rho, ur, uz, phi)) + DT * (np.eye(9) - 0.5 * self.Lam) @ \
            self.S(k, j, rho, ur, uz, T)
        fp = self.Minv @ mp
        gp = np.empty(5)
        for i in range(5):
            er = E[i][0]
            geq = self.g_eq(i, T, ur, uz)
            omega_g = (1.0 + er * self.tau_T * DT / r) / (self.tau_T + 0.5)
            psi = -(ur / r) * geq
            gp[i] = g[i] - omega_g * (g[i] - geq) + DT * psi
        return fp, gp

    def source_of(self, j, k, er, ez):
        """Node whose population moving along e = (er, ez) arrives at (j, k), as
        (j_s, k_s, mirrored) or None when it would come from outside."""
        c = self.c
        js, ks = j - er, k - ez
        if c["side_z"] == 2:
            ks %= self.nz
        if not 0 <= ks < self.nz:
            return None
        mirrored = False
        if js < 0 and c["side_rmin"] == 2:
            js %= self.nr
        elif js >= self.nr and c["side_rmax"] == 2:
            js %= self.nr
        elif js == -1 and c["side_rmin"] == 1:
            js, mirrored = 0, True  # the ghost row at r = -1/2 mirrors row 0
        if not 0 <= js < self.nr:
            return None
        return js, ks, mirrored

    def step(self, n: int = 1):
        for _ in range(n):
            nz, nr = self.nz, self.nr
            post = [[self.collide(k, j) for j in range(nr)] for k in range(nz)]
            fn = np.full((nz, nr, 9), np.nan)
            gn = np.full((nz, nr, 5), np.nan)
            for k in range(nz):
                for j in range(nr):
                    for i, (er, ez) in enumerate(E):
                        src = self.source_of(j, k, er, ez)
                        if src is None:
                            continue
                        js, ks, mir = src
                        if mir:  # f_i(-r) = -f_i*(r), i* = e_r reversed
                            istar = E.index((-er, ez))
                            fn[k, j, i] = -post[ks][js][0][istar]
                        else:
                            fn[k, j, i] = post[ks][js][0][i]
                        if i < 5:
                            gn[k, j, i] = post[ks][js][1][E.index((-er, ez)) if mir else i]
            self.f, self.g = fn, gn
            self.t += 1
            self.macros_all()

    def macros(self) -> dict:
        nz, nr = self.nz, self.nr
        out = {k: np.empty((nz, nr)) for k in ("rho", "ur", "uz", "T", "p")}
        out["mask"] = np.empty((nz, nr), dtype=np.uint8)
        for k in range(nz):
            for j in range(nr):
                rho, ur, uz, T = self.mac[k][j]
                out["rho"][k, j], out["ur"][k, j], out["uz"][k, j], out["T"][k, j] = rho, ur, uz, T
                out["p"][k, j] = rho * CS2 / self.phi[k, j]
                out["mask"][k, j] = self.mask(j, k)
        return out
