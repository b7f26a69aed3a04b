"""Seeded synthetic inputs shaped like the paper's test problems.

This module only states problems: grids, parameters, boundary choices and
seeded porosity fields.  It holds none of the lattice Boltzmann arithmetic, so
both the FP64 oracle and the GPU library can consume what it produces without
sharing any of the method's code.

A problem is a plain ``dict`` with these keys (lattice units, spacing 1):

  nr, nz                 grid: rows along r (index j), columns along z (index k)
  r0                     radius of row j = 0 (rows sit at r0 + j)
  L                      characteristic length of Eq. (9)
  side_rmin, side_rmax   "wall" | "axis" (r_min only) | "periodic"
  side_z                 "wall" | "periodic" | "flow" (inlet at z = 0, outlet at z = H)
  u_in                   inlet axial velocity of side_z = "flow"
  therm_rmin, therm_rmax, therm_z   "fixed" | "adiabatic" | "flux" (radial walls)
  T_rmin, T_rmax, T_zmin, T_zmax    wall temperatures of fixed walls
  flux_rmin, flux_rmax   q'/k of flux walls (a temperature gradient)
  flux_zlo, flux_zhi     heated window of flux walls, z = k (default: the whole wall)
  T_ref, T_init, delta_T reference temperature T_0 of Eq. (7), initial
                         temperature, temperature difference (0: T_rmin - T_rmax)
  phi, Da, F_phi         porosity (reference porosity with a field), Darcy
                         number, Forchheimer coefficient (negative: Ergun, Eq. 8)
  Ra, Pr, J, lam, Ma     Eq. (9) groups and the Mach number of Eq. (39)
  tau_nu                 > 0 overrides Eq. (39)
  accel_r, accel_z       external acceleration a of Eq. (7)
"""
from __future__ import annotations

import math

import numpy as np

ERGUN = -1.0  # F_phi < 0 selects the Ergun relation of Eq. (8)


def pipe(nr: int = 64, nz: int = 8, phi: float = 0.6, Da: float = 1e-2, Re: float = 10.0,
         tau_nu: float = 0.8, Pr: float = 1.0, F_phi: float = ERGUN, T_wall: float = 1.0,
         T_init: float = 0.0) -> dict:
    """Porous-pipe flow driven by an axial body force, periodic in z.

    Rows are cell-centred about the axis (r0 = 1/2); the wall row nr-1 sits at
    R = nr - 1/2, which is also the length scale L (the paper's pipe problem
    uses L = r_i).  The axial acceleration is chosen so that the mean velocity
    of the Brinkman-extended Darcy solution (Forchheimer term off) gives the
    requested Re = U R / nu.
    """
    from scipy.special import i0, i1

    R = nr - 0.5
    nu = (tau_nu - 0.5) / 3.0  # J = 1
    K = Da * R * R
    k = math.sqrt(phi / K)
    U = Re * nu / R
    mean_factor = 1.0 - 2.0 * float(i1(k * R)) / (k * R * float(i0(k * R)))
    accel = U * nu / (K * mean_factor)
    return dict(nr=nr, nz=nz, r0=0.5, L=R, side_rmin="axis", side_rmax="wall",
                side_z="periodic", therm_rmin="adiabatic", therm_rmax="fixed",
                therm_z="adiabatic", T_rmin=0.0, T_rmax=T_wall, T_zmin=0.0, T_zmax=0.0,
                T_ref=0.0, T_init=T_init, delta_T=T_wall - T_init, phi=phi, Da=Da,
                F_phi=F_phi, Ra=0.0, Pr=Pr, J=1.0, lam=1.0, Ma=0.1, tau_nu=tau_nu,
                accel_r=0.0, accel_z=accel)


def annulus(nr: int = 256, nz: int = 256, Rstar: float = 2.0, phi: float = 0.6,
            Da: float = 1e-4, Ra: float = 1e5, Pr: float = 1.0, F_phi: float = ERGUN,
            T_i: float = 1.0, T_o: float = 0.0, J: float = 1.0, lam: float = 1.0,
            Ma: float = 0.1) -> dict:
    """Natural convection between coaxial cylinders (Fig. 3 problem).

    Wall nodes lie on the walls: L = r_o - r_i = nr - 1, H = nz - 1,
    r_i = L / (R* - 1).  Hot inner wall, cold outer wall, adiabatic ends,
    T_0 = (T_i + T_o) / 2, interior starting at T_o and at rest.
    """
    L = nr - 1.0
    ri = L / (Rstar - 1.0)
    return dict(nr=nr, nz=nz, r0=ri, L=L, side_rmin="wall", side_rmax="wall",
                side_z="wall", therm_rmin="fixed", therm_rmax="fixed", therm_z="adiabatic",
                T_rmin=T_i, T_rmax=T_o, T_zmin=0.0, T_zmax=0.0, T_ref=0.5 * (T_i + T_o),
                T_init=T_o, delta_T=T_i - T_o, phi=phi, Da=Da, F_phi=F_phi, Ra=Ra, Pr=Pr,
                J=J, lam=lam, Ma=Ma, tau_nu=0.0, accel_r=0.0, accel_z=0.0)


def table2(Ra: float, nr: int = 100, nz: int = 200) -> dict:
    """Annulus without porous medium as in Sec. 4.2 / Table 2 (phi = 1, Da = 1e8)."""
    return annulus(nr=nr, nz=nz, Rstar=2.0, phi=1.0, Da=1e8, Ra=Ra, Pr=0.7, F_phi=0.0)


def developing_pipe(Da: float = 1e8, nr: int = 41, A: float = 16.0, Re: float = 100.0,
                    Pr: float = 0.7, u_in: float = 0.005, phi: float = 1.0, F_phi: float = 0.0,
                    T_in: float = 0.0, T_w: float = 1.0) -> dict:
    """Thermally developing flow in a pipe filled with porous medium (Sec. 4.1, Fig. 1).

    Rows are cell-centred about the axis (r0 = 1/2). The wall row nr-1 sits at
    r_i = nr - 1/2, which is also the length L of Re = L u_in / nu. The paper's
    "81 x 648" grid with A = H / r_i = 16 gives r_i = 40.5: nr = 41 rows here,
    i.e. 81 cells across the diameter. The pipe spans H = A r_i with columns at
    z = 0..H. Column 0 is the inlet (u_z = u_in, T = T_in) and column H the
    outlet (zero axial gradient). The wall is held at T_w.

    The paper gives no relaxation time for this problem. tau_nu follows from
    Re and u_in, whose default of 0.005 keeps the Darcy pressure drop at
    Da = 1e-3 near 1 % of the density. Ma = u_in / c_s makes the inlet
    velocity the velocity scale of the steady-state residual. With Ra = 0 and
    tau_nu given, Ma enters nothing else.
    """
    R = nr - 0.5
    H = A * R
    nz = int(round(H)) + 1
    nu = u_in * R / Re
    return dict(nr=nr, nz=nz, r0=0.5, L=R, side_rmin="axis", side_rmax="wall", side_z="flow",
                therm_rmin="adiabatic", therm_rmax="fixed", therm_z="fixed", T_rmin=0.0,
                T_rmax=T_w, T_zmin=T_in, T_zmax=0.0, T_ref=0.0, T_init=T_in,
                delta_T=T_w - T_in, phi=phi, Da=Da, F_phi=F_phi, Ra=0.0, Pr=Pr, J=1.0, lam=1.0,
                Ma=u_in * math.sqrt(3.0), tau_nu=0.5 + 3.0 * nu, accel_r=0.0, accel_z=0.0,
                u_in=u_in)


def plug_start(cfg: dict) -> np.ndarray:
    """Start fields (u_z, u_r, T) of a pipe problem: plug flow at u_in, T_init."""
    nz, nr = cfg["nz"], cfg["nr"]
    out = np.zeros((3, nz, nr))
    out[0] = cfg["u_in"]
    out[2] = cfg["T_init"]
    return out


def heater_annulus(Da: float, nr: int = 200, nz: int = 200, Ra: float = 1e7, Pr: float = 0.7,
                   phi: float = 0.9, F_phi: float = 0.0, Rstar: float = 2.0,
                   l_over_H: float = 0.4, h_over_H: float = 0.5, dT: float = 10.0,
                   T_o: float = 1.0, Ma: float = 0.1) -> dict:
    """Porous annulus with an isoflux heater on the inner wall (Sec. 4.4, Fig. 7).

    Wall nodes lie on the walls: L = r_o - r_i = nr - 1, H = nz - 1,
    r_i = L / (R* - 1).  The heater covers h - l/2 <= z <= h + l/2 of the
    inner wall with q'/k = dT / L (so that q' L / k = dT); the rest of the
    inner wall and both ends are adiabatic; the outer wall is held at T_o,
    which is also T_0 and the start temperature.  The defaults are the
    paper's: Ra = 1e7, Pr = 0.7, phi = 0.9, F_phi = 0, A = 1, R* = 2,
    l/H = 0.4, h/H = 0.5, dT = 10, T_o = 1 on a 200 x 200 grid.
    """
    L = nr - 1.0
    H = nz - 1.0
    ri = L / (Rstar - 1.0)
    return dict(nr=nr, nz=nz, r0=ri, L=L, side_rmin="wall", side_rmax="wall",
                side_z="wall", therm_rmin="flux", therm_rmax="fixed", therm_z="adiabatic",
                T_rmin=0.0, T_rmax=T_o, T_zmin=0.0, T_zmax=0.0, T_ref=T_o, T_init=T_o,
                delta_T=dT, flux_rmin=dT / L, flux_rmax=0.0,
                flux_zlo=(h_over_H - 0.5 * l_over_H) * H, flux_zhi=(h_over_H + 0.5 * l_over_H) * H,
                phi=phi, Da=Da, F_phi=F_phi, Ra=Ra, Pr=Pr, J=1.0, lam=1.0, Ma=Ma, tau_nu=0.0,
                accel_r=0.0, accel_z=0.0)


def porous_annulus_43(Ra_star: float, nr: int = 300, nz: int = 300, F_phi: float = ERGUN) -> dict:
    """Natural convection in a vertical annulus filled with porous medium (Sec. 4.3).

    R* = 5.338, A = 1, Pr = 1, phi = 0.3698, Da = 1.66e-6 and the Darcy-Rayleigh
    number Ra* = Ra Da, so Ra = Ra* / Da; hot inner wall, cold outer wall,
    adiabatic ends, on the paper's 300 x 300 grid by default.  The section does
    not set F_phi (Secs. 4.1 and 4.4 set it to 0 explicitly), so Eq. (8)'s Ergun
    value of the porosity applies.
    """
    return annulus(nr=nr, nz=nz, Rstar=5.338, phi=0.3698, Da=1.66e-6, Ra=Ra_star / 1.66e-6,
                   Pr=1.0, F_phi=F_phi)


def porosity_grf(nz: int, nr: int, seed: int = 1409, sigma: float = 8.0, mean: float = 0.6,
                 std: float = 0.15, lo: float = 0.3, hi: float = 0.95) -> np.ndarray:
    """Seeded Gaussian random porosity field, [nz, nr] float64.

    White N(0,1) noise from numpy's PCG64 with the given seed, a Gaussian
    filter of ``sigma`` cells (reflecting edges), standardised to zero mean and
    unit variance, then phi = clip(mean + std * xi, lo, hi).
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((nz, nr), dtype=np.float64)
    xi = gaussian_filter(xi, sigma=sigma, mode="reflect")
    xi = (xi - xi.mean()) / xi.std()
    return np.clip(mean + std * xi, lo, hi)


def variable_porosity_annulus(n: int = 8192, Ra: float = 1e6, Da: float = 1e-3,
                              seed: int = 1409):
    """The throughput problem: an n x n annulus (R* = 2, Pr = 1) with a seeded
    porosity field of mean 0.6 (also the reference porosity for K), Ergun
    Forchheimer coefficient from the local porosity.  Returns (problem, phi)."""
    cfg = annulus(nr=n, nz=n, Rstar=2.0, phi=0.6, Da=Da, Ra=Ra, Pr=1.0, F_phi=ERGUN)
    return cfg, porosity_grf(n, n, seed=seed)


def sweep(n_inst: int = 1024, seed: int = 1409, sizes=None) -> list:
    """Batched parameter sweep of annuli with uneven grids and parameters.

    Nr, Nz uniform on {32, 64, ..., 512}; Ra log-uniform on [1e3, 1e6];
    Da log-uniform on [1e-6, 1e-2]; phi uniform on [0.3, 0.95]; R* log-uniform
    on [1.2, 10]; Pr from {0.71, 1, 7}; Ergun Forchheimer coefficient.
    """
    rng = np.random.default_rng(seed)
    sizes = np.arange(32, 513, 32) if sizes is None else np.asarray(sizes)
    out = []
    for _ in range(n_inst):
        nr = int(rng.choice(sizes))
        nz = int(rng.choice(sizes))
        Ra = 10.0 ** rng.uniform(3.0, 6.0)
        Da = 10.0 ** rng.uniform(-6.0, -2.0)
        phi = float(rng.uniform(0.3, 0.95))
        Rstar = math.exp(rng.uniform(math.log(1.2), math.log(10.0)))
        Pr = float(rng.choice([0.71, 1.0, 7.0]))
        out.append(annulus(nr=nr, nz=nz, Rstar=Rstar, phi=phi, Da=Da, Ra=Ra, Pr=Pr,
                           F_phi=ERGUN))
    return out


# ---- warm-start network inputs -------------------------------------------------

def no_init_params(widths, seed: int = 1409) -> np.ndarray:
    """Seeded initial weights of the warm-start network, float32, packed layer
    by layer as W[cout][cin][k][k] then b[cout].  He-normal weights
    (std sqrt(2 / (cin k^2))), zero biases; the 1x1 output layer is scaled
    down by 10 so that the untrained network predicts nearly zero."""
    c1, c2, c3, c4 = widths
    shapes = [(6, c1, 3), (c1, c2, 3), (c2, c3, 3), (c3, c4, 3), (c4, c3, 3), (c3, c2, 3),
              (c2, c1, 3), (c1, 3, 1)]
    rng = np.random.default_rng(seed)
    out = []
    for i, (ci, co, k) in enumerate(shapes):
        std = np.sqrt(2.0 / (ci * k * k)) * (0.1 if i == len(shapes) - 1 else 1.0)
        out.append(rng.standard_normal(co * ci * k * k) * std)
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


U_SCALE = 0.1 / math.sqrt(3.0)  # characteristic velocity Ma c_s of the annulus problems


def no_features(cfg: dict) -> np.ndarray:
    """Six [nz, nr] feature planes of an annulus problem: normalised log10 Ra,
    log10 Da, porosity, log10 Pr, ln R*, and the radius r / r_o of each node."""
    nz, nr = int(cfg["nz"]), int(cfg["nr"])
    r0, L = float(cfg["r0"]), float(cfg["L"])
    rstar = (r0 + L) / r0
    vals = [(math.log10(cfg["Ra"]) - 4.5) / 1.5, (math.log10(cfg["Da"]) + 4.0) / 2.0,
            (cfg["phi"] - 0.625) / 0.325, math.log10(cfg["Pr"]), math.log(rstar) / math.log(10.0)]
    out = np.empty((6, nz, nr), dtype=np.float32)
    for i, v in enumerate(vals):
        out[i] = v
    out[5] = ((r0 + np.arange(nr)) / (r0 + L))[None, :]
    return out


def conduction_T(cfg: dict) -> np.ndarray:
    """Temperature of pure radial conduction between the walls,
    T = T_o + (T_i - T_o) ln(r_o / r) / ln R*, as an [nz, nr] plane."""
    nz, nr = int(cfg["nz"]), int(cfg["nr"])
    r0, L = float(cfg["r0"]), float(cfg["L"])
    r = r0 + np.arange(nr)
    prof = np.log((r0 + L) / r) / np.log((r0 + L) / r0)
    return np.repeat((cfg["T_rmax"] + (cfg["T_rmin"] - cfg["T_rmax"]) * prof)[None, :], nz, axis=0)


T_SCALE = 4.0  # departures of T from conduction are ~4x smaller than u / U


def velocity_scale(cfg: dict) -> float:
    """Expected size of the buoyant velocity of an annulus problem (lattice
    units).  In a porous layer the velocity is the Darcy velocity
    u_D = K g beta dT / nu; with K = Da L^2 (Eq. 9), g beta dT = U^2 / L and
    nu = U L sqrt(Pr / Ra) (Eq. 39 with J = 1) that is q U, q = Da sqrt(Ra / Pr),
    which spans six decades over the sweep distribution.  Where the medium
    barely resists (q large) the velocity stays near U = Ma c_s, hence
    U q / (1 + q)."""
    q = cfg["Da"] * math.sqrt(cfg["Ra"] / cfg["Pr"])
    return U_SCALE * q / (1.0 + q)


def no_targets(fields: dict, cfg: dict) -> np.ndarray:
    """Network targets of a field dict, float32 [3, nz, nr]: u_z and u_r over
    the problem's velocity_scale, and T_SCALE times the departure of T from
    radial conduction (so that a zero output is the conduction start)."""
    us = velocity_scale(cfg)
    return np.stack([fields["uz"] / us, fields["ur"] / us,
                     T_SCALE * (fields["T"] - conduction_T(cfg))]).astype(np.float32)


def no_fields(pred: np.ndarray, cfg: dict) -> np.ndarray:
    """Inverse of no_targets: start fields (u_z, u_r, T) [3, nz, nr] from a prediction."""
    us = velocity_scale(cfg)
    return np.stack([pred[0] * us, pred[1] * us,
                     pred[2] / T_SCALE + conduction_T(cfg)]).astype(np.float32)
