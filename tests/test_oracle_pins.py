"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: matrices the
paper prints, an equilibrium or forcing written in another published form,
conservation laws, and closed-form solutions of the macroscopic equations the
model is built to recover (Eqs. 1-5).
"""
import math
import os

import numpy as np
import pytest

import lbm_inputs as li
from tests.conftest import load_matrix

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1.0])
EZ = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1.0])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CS2 = 1.0 / 3.0


def _node_oracle(oracle_mod, **kw):
    cfg = dict(nr=3, nz=3, r0=1.0, tau_nu=0.8, phi=0.7, Da=1e-2, L=20.0, F_phi=0.3,
               accel_r=1e-4, accel_z=2e-4, Ra=1e4, Pr=0.8, T_rmin=1.0, T_rmax=0.0, T_ref=0.5)
    cfg.update(kw)
    return oracle_mod.Oracle(cfg)


def _random_node(rng, r):
    """Populations near an r-weighted equilibrium with a random perturbation."""
    ur, uz = rng.normal(0, 0.03, 2)
    eu = EX * ur + EZ * uz
    f = W * r * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ur * ur + uz * uz))
    f = f * (1 + 0.02 * rng.standard_normal(9))
    g = np.array([0.6, 0.1, 0.1, 0.1, 0.1]) * rng.uniform(0.2, 1.0) * (1 + 0.05 * rng.standard_normal(5))
    return f, g


# --- printed matrices (Eq. 18, Appendix A) ---------------------------------

def test_M_is_the_printed_matrix_and_orthogonal(oracle_mod):
    M, Minv = _node_oracle(oracle_mod).matrices()
    np.testing.assert_array_equal(M, load_matrix("M_eq18.txt"))
    np.testing.assert_array_equal(M @ M.T, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4.0]))
    np.testing.assert_allclose(M @ Minv, np.eye(9), atol=1e-15)


def test_streaming_matrices_match_appendix_A(oracle_mod):
    """C_j = M (e_j I) M^-1 as printed: pins M^-1 and the (r, z) velocity order."""
    M, Minv = _node_oracle(oracle_mod).matrices()
    np.testing.assert_allclose(M @ np.diag(EX) @ Minv, load_matrix("Cr_appA.txt"), atol=1e-15)
    np.testing.assert_allclose(M @ np.diag(EZ) @ Minv, load_matrix("Cz_appA.txt"), atol=1e-15)


# --- per-node identities ----------------------------------------------------

def test_equilibrium_moments_equal_eq32(oracle_mod):
    """M^-1 m^eq (Eqs. 19-20) equals the velocity-space equilibrium of Eq. (32)."""
    o = _node_oracle(oracle_mod)
    _, Minv = o.matrices()
    rng = np.random.default_rng(1)
    for _ in range(20):
        r = rng.uniform(0.5, 300)
        phi = rng.uniform(0.3, 1.0)
        f, g = _random_node(rng, r)
        n = o.node(r, phi, f, g)
        ur, uz, rho = n["ur"], n["uz"], n["rho"]
        eu = EX * ur + EZ * uz
        feq32 = W * r * rho * (1 + eu / CS2 + eu ** 2 / (2 * phi * CS2 ** 2)
                               - (ur * ur + uz * uz) / (2 * phi * CS2))
        np.testing.assert_allclose(Minv @ n["meq"], feq32, rtol=0, atol=1e-13 * r)


def _guo_forcing(r, rho, ur, uz, phi, Fr, Fz, ar, printed):
    """Velocity-space porous forcing (Guo-Zhao form) with F~ = F + a_r e_r.

    As printed, Eq. (24) is the moment-space image of this with u.F~ divided by
    phi throughout; the default reading divides only F by phi.
    """
    eu = EX * ur + EZ * uz
    Ftr = Fr + ar
    eF = EX * Ftr + EZ * Fz
    if printed:
        quad = eu * eF / phi
        lin = (ur * Ftr + uz * Fz) / phi
    else:
        quad = eu * (EX * Fr + EZ * Fz) / phi + eu * EX * ar
        lin = (ur * Fr + uz * Fz) / phi + ur * ar
    return W * r * rho * (eF / CS2 + quad / CS2 ** 2 - lin / CS2)


@pytest.mark.parametrize("printed", [0, 1])
def test_source_moments_are_guo_forcing(oracle_mod, printed):
    """M^-1 S (Eq. 24) equals the velocity-space porous forcing of Guo and Zhao."""
    o = _node_oracle(oracle_mod, src_printed=printed)
    _, Minv = o.matrices()
    rng = np.random.default_rng(2)
    for _ in range(20):
        r = rng.uniform(0.5, 50)
        phi = rng.uniform(0.3, 1.0)
        f, g = _random_node(rng, r)
        n = o.node(r, phi, f, g)
        Fr = n["Ftr"] - n["a_r"]
        ref = _guo_forcing(r, n["rho"], n["ur"], n["uz"], phi, Fr, n["Ftz"], n["a_r"], printed)
        np.testing.assert_allclose(Minv @ n["S"], ref, rtol=0, atol=1e-14 * r)


def test_collision_conserves_mass(oracle_mod):
    o = _node_oracle(oracle_mod)
    rng = np.random.default_rng(3)
    for _ in range(20):
        r = rng.uniform(0.5, 100)
        f, g = _random_node(rng, r)
        n = o.node(r, 0.6, f, g)
        assert abs(n["f_out"].sum() - f.sum()) <= 1e-13 * abs(f.sum())


@pytest.mark.parametrize("s_j", [1.0, 1.3])
def test_momentum_change_equals_force(oracle_mod, s_j):
    """With F_phi = 0, Eqs. (25)-(28) and (21) give m_3+ - m_3 = r rho F~_r and
    m_5+ - m_5 = r rho F~_z for any s_j."""
    o = _node_oracle(oracle_mod, F_phi=0.0, s_j=s_j)
    M, _ = o.matrices()
    rng = np.random.default_rng(4)
    for _ in range(20):
        r = rng.uniform(0.5, 100)
        phi = rng.uniform(0.3, 1.0)
        f, g = _random_node(rng, r)
        n = o.node(r, phi, f, g)
        dm = M @ n["f_out"] - M @ f
        scale = r * n["rho"]
        assert abs(dm[3] - scale * n["Ftr"]) <= 1e-13 * r
        assert abs(dm[5] - scale * n["Ftz"]) <= 1e-13 * r


def test_bgk_limit(oracle_mod):
    """With every rate equal to 1/tau the MRT step is BGK with the equilibrium
    of Eq. (32) and the forcing weighted by (1 - 1/(2 tau)) (text before Eq. 32)."""
    tau = 0.8
    o = _node_oracle(oracle_mod, tau_nu=tau, s_e=1 / tau, s_eps=1 / tau, s_q=1 / tau, s_j=1 / tau)
    rng = np.random.default_rng(5)
    for _ in range(10):
        r = rng.uniform(0.5, 100)
        phi = rng.uniform(0.3, 1.0)
        f, g = _random_node(rng, r)
        n = o.node(r, phi, f, g)
        # s_0 = 1 is irrelevant: m_0 = m_0^eq and S_0 = 0.
        ur, uz, rho = n["ur"], n["uz"], n["rho"]
        eu = EX * ur + EZ * uz
        feq = W * r * rho * (1 + 3 * eu + 4.5 * eu ** 2 / phi - 1.5 * (ur * ur + uz * uz) / phi)
        force = _guo_forcing(r, rho, ur, uz, phi, n["Ftr"] - n["a_r"], n["Ftz"], n["a_r"], 0)
        ref = f - (f - feq) / tau + (1 - 0.5 / tau) * force
        np.testing.assert_allclose(n["f_out"], ref, rtol=0, atol=1e-13 * r)


def test_thermal_equilibrium_is_fixed_point(oracle_mod):
    """At rest (u = 0) a temperature equilibrium is left unchanged by Eq. (33)."""
    o = _node_oracle(oracle_mod, accel_r=0.0, accel_z=0.0, Ra=0.0, T_ref=0.7)
    rng = np.random.default_rng(6)
    for _ in range(5):
        r = rng.uniform(0.5, 50)
        T = rng.uniform(0.1, 1.0)
        # populations whose Eq. (28) velocity vanishes: quiescent r-weighted state
        f = W * r
        f = f.copy()
        f[1] -= 0.25 * CS2  # sum e_r f = -rho c_s^2 / 2 gives u_r = 0 (Eq. 27)
        f[3] += 0.25 * CS2
        g = np.array([0.6, 0.1, 0.1, 0.1, 0.1]) * T
        n = o.node(r, 1.0, f, g)
        assert abs(n["ur"]) < 1e-15 and abs(n["uz"]) < 1e-15
        np.testing.assert_allclose(n["g_out"], g, rtol=0, atol=1e-15)


def test_initial_state_returns_given_velocity(oracle_mod):
    """Reading of the start: f = f^eq - S~/2 (the change of variables before
    Eq. 15) makes Eqs. (26)-(28) return the prescribed u and T (F_phi = 0)."""
    nr, nz = 9, 7
    rng = np.random.default_rng(8)
    init = np.stack([rng.normal(0, 0.02, (nz, nr)), rng.normal(0, 0.02, (nz, nr)),
                     rng.uniform(0, 1, (nz, nr))])
    cfg = dict(nr=nr, nz=nz, r0=3.0, L=8.0, side_z="periodic", phi=0.7, Da=1e-2, F_phi=0.0,
               Ra=1e4, Pr=1.0, T_rmin=1.0, T_rmax=0.0, T_ref=0.5, accel_z=1e-4)
    m = oracle_mod.Oracle(cfg, init=init).macros()
    fluid = m["mask"] == 0
    np.testing.assert_allclose(m["uz"][fluid], init[0][fluid], rtol=0, atol=1e-15)
    np.testing.assert_allclose(m["ur"][fluid], init[1][fluid], rtol=0, atol=1e-15)
    np.testing.assert_allclose(m["T"][fluid], init[2][fluid], rtol=0, atol=1e-15)
    np.testing.assert_allclose(m["rho"][fluid], 1.0, rtol=0, atol=1e-15)


# --- whole-lattice invariants -----------------------------------------------

def test_mass_conserved_on_periodic_lattice(oracle_mod):
    """Fully periodic lattice: collision conserves sum f, streaming permutes it."""
    nr, nz = 12, 10
    rng = np.random.default_rng(7)
    init = np.stack([rng.normal(0, 0.01, (nz, nr)), rng.normal(0, 0.01, (nz, nr)),
                     rng.uniform(0, 1, (nz, nr))])
    # The radial wrap joins rows of different radius: a benign viscosity and a
    # large r0 keep that jump small.  Only the mass bookkeeping is checked.
    cfg = dict(nr=nr, nz=nz, r0=400.0, L=10.0, side_rmin="periodic", side_rmax="periodic",
               side_z="periodic", phi=0.6, Da=1e-2, F_phi=-1.0, tau_nu=1.0, Pr=1.0,
               accel_z=1e-5, T_rmin=1.0, T_rmax=0.0, T_ref=0.5)
    o = oracle_mod.Oracle(cfg, init=init)
    f0, _ = o.populations()
    o.step(300)
    f1, _ = o.populations()
    assert np.isfinite(f1).all()
    assert abs(f1.sum() - f0.sum()) <= 1e-13 * abs(f0.sum())


def test_quiescent_annulus_stays_at_rest(oracle_mod):
    """Uniform temperature, no body force: the flow stays at rest up to the
    small spurious velocity the wall scheme leaves (level recorded)."""
    cfg = li.annulus(nr=17, nz=9, Rstar=2.0, phi=0.6, Da=1e-2, Ra=1e4, Pr=1.0, T_i=0.5, T_o=0.5)
    cfg["delta_T"] = 1.0
    o = oracle_mod.Oracle(cfg)
    o.step(3000)
    m = o.macros()
    assert np.abs(m["ur"]).max() < 1e-7 and np.abs(m["uz"]).max() < 1e-7
    np.testing.assert_allclose(m["T"], 0.5, rtol=0, atol=1e-12)


# --- closed-form solutions of the macroscopic model -------------------------

def _run_to_steady(o, tol, chunk=1000, max_steps=400_000, key="res_u"):
    while o.t < max_steps:
        o.snapshot()
        o.step(chunk)
        if o.residual()[key] < tol:
            break
    return o


def _pipe_error(oracle_mod, nr, phi=0.6, Da=1e-2, printed=0):
    from scipy.special import i0

    cfg = li.pipe(nr=nr, nz=2, phi=phi, Da=Da, Re=10.0, tau_nu=0.8, F_phi=0.0)
    cfg["src_printed"] = printed
    o = _run_to_steady(oracle_mod.Oracle(cfg), 1e-12)
    R, nu, a = nr - 0.5, 0.1, cfg["accel_z"]
    K = Da * R * R
    k = math.sqrt(phi / K)
    r = 0.5 + np.arange(nr)
    exact = a * K / nu * (1 - i0(k * r) / i0(k * R))
    uz = o.macros()["uz"][1]
    return np.linalg.norm(uz - exact) / np.linalg.norm(exact), o


def test_pipe_matches_brinkman_bessel_profile(oracle_mod):
    """Porous pipe, Forchheimer off: u_z(r) = (a K / nu)[1 - I0(kr)/I0(kR)],
    k^2 = phi / (J K), the fully developed solution of Eq. (3) with Eq. (6).
    Second-order convergence, 1e-3 relative L2 at Nr = 64."""
    errs = [_pipe_error(oracle_mod, nr)[0] for nr in (16, 32, 64)]
    assert errs[2] < 1e-3
    assert math.log2(errs[0] / errs[1]) > 1.5 and math.log2(errs[1] / errs[2]) > 1.5


def test_pipe_hagen_poiseuille_limit(oracle_mod):
    """phi -> 1, Da -> infinity: u_z = a (R^2 - r^2) / (4 nu_e)."""
    nr = 32
    cfg = li.pipe(nr=nr, nz=2, phi=1.0, Da=1e8, Re=10.0, tau_nu=0.8, F_phi=0.0)
    o = _run_to_steady(oracle_mod.Oracle(cfg), 1e-12)
    R, a = nr - 0.5, cfg["accel_z"]
    r = 0.5 + np.arange(nr)
    exact = a * (R * R - r * r) / (4 * 0.1)
    uz = o.macros()["uz"][1]
    assert np.linalg.norm(uz - exact) / np.linalg.norm(exact) < 2e-3


def test_printed_source_form_misses_porous_pipe(oracle_mod):
    """Eq. (24) as printed scales the axisymmetric correction a_r by 1/phi; at
    phi = 1 both forms agree up to rounding, at phi = 0.6 the printed form makes
    Hagen-Poiseuille flow 1.5 times too fast."""
    _, o0 = _pipe_error(oracle_mod, 16, phi=1.0, Da=1e8, printed=0)
    _, o1 = _pipe_error(oracle_mod, 16, phi=1.0, Da=1e8, printed=1)
    np.testing.assert_allclose(o0.macros()["uz"], o1.macros()["uz"], rtol=1e-12, atol=0)
    nr = 32
    cfg = li.pipe(nr=nr, nz=2, phi=0.6, Da=1e8, Re=10.0, tau_nu=0.8, F_phi=0.0)
    cfg["src_printed"] = 1
    o = _run_to_steady(oracle_mod.Oracle(cfg), 1e-12)
    R, a = nr - 0.5, cfg["accel_z"]
    r = 0.5 + np.arange(nr)
    exact = 0.6 * a * (R * R - r * r) / (4 * 0.1)
    ratio = o.macros()["uz"][1][:-1] / exact[:-1]
    assert abs(ratio.mean() - 1.5) < 0.01


def test_annular_poiseuille(oracle_mod):
    """Axial flow between cylinders, second-order convergence to
    u = phi a / (4 nu_e) [r_o^2 - r^2 + (r_o^2 - r_i^2) ln(r / r_o) / ln(r_o / r_i)]."""
    errs = []
    for nr in (9, 17, 33):
        ri = nr - 1.0
        ro = ri + nr - 1
        cfg = dict(nr=nr, nz=2, side_z="periodic", r0=ri, L=nr - 1.0, phi=0.8, Da=1e8,
                   F_phi=0.0, tau_nu=0.8, accel_z=1e-6)
        o = _run_to_steady(oracle_mod.Oracle(cfg), 1e-12)
        r = ri + np.arange(nr)
        exact = 0.8 * 1e-6 / (4 * 0.1) * (ro ** 2 - r ** 2 + (ro ** 2 - ri ** 2) * np.log(r / ro) / np.log(ro / ri))
        uz = o.macros()["uz"][1]
        errs.append(np.linalg.norm(uz - exact) / np.linalg.norm(exact))
    assert errs[2] < 3e-3
    assert math.log2(errs[0] / errs[1]) > 1.8 and math.log2(errs[1] / errs[2]) > 1.8


def test_annular_conduction_log_profile(oracle_mod):
    """No flow: T = ln(r_o / r) / ln R* (Eq. 12 with u = 0), second order; the
    Eq. (42) Nusselt numbers approach 1 / ln R* (first order: the wall scheme
    leaves an O(h^2) temperature jump that the r_i dT/dr of Eq. (42) amplifies)."""
    out = []
    for nr in (17, 33):
        cfg = li.annulus(nr=nr, nz=4, Rstar=2.0, phi=1.0, Da=1e8, Ra=0.0, Pr=0.5, F_phi=0.0)
        cfg["tau_nu"] = 0.8
        o = _run_to_steady(oracle_mod.Oracle(cfg), 1e-13, chunk=2000, key="res_T")
        r = cfg["r0"] + np.arange(nr)
        exact = np.log(r[-1] / r) / math.log(2.0)
        T = o.macros()["T"][1]
        out.append((np.abs(T - exact).max(), o.nusselt()))
    (e17, nu17), (e33, nu33) = out
    assert e33 < 1e-3 and math.log2(e17 / e33) > 1.8
    exact_nu = 1 / math.log(2.0)
    for a, b in zip(nu17, nu33):
        assert abs(b - exact_nu) < 0.04
        assert abs(a - exact_nu) / abs(b - exact_nu) > 1.6


@pytest.mark.parametrize("phi, G", [(0.45, 0.055), (0.75, 0.005)])
def test_uniform_porous_flow_obeys_ergun(oracle_mod, phi, G):
    """A body force G drives a uniform flow through a packed bed whose porosity
    phi differs from the reference porosity phi_ref = 0.6 (porosity field, Ergun
    F_phi).  At steady state Eq. (2) loses every gradient, so the drag of
    Eq. (6) must balance G; written in Ergun's own form with superficial velocity
    U and particle diameter d (fixed by K(phi_ref) = Da L^2), that is
    G = 150 nu (1 - phi)^2 U / (phi^3 d^2) + 1.75 (1 - phi) U^2 / (phi^3 d).
    This checks K(phi) and F_phi(phi) of Eq. (8) against the Ergun equation
    itself.  The Forchheimer part carries 18 % and 42 % of the drag here.
    A large r0 makes the radial wrap of the fully periodic lattice negligible."""
    phi_ref, L, Da = 0.6, 10.0, 1e-2
    cfg = dict(nr=3, nz=3, r0=1e6, L=L, side_rmin="periodic", side_rmax="periodic",
               side_z="periodic", phi=phi_ref, Da=Da, F_phi=-1.0, tau_nu=0.8, Ra=0.0, Pr=1.0,
               accel_z=G, T_rmin=0.0, T_rmax=0.0, T_ref=0.0, T_init=0.0)
    o = oracle_mod.Oracle(cfg, phi_field=np.full((3, 3), phi))
    nu = o.derived()["nu"]
    o.step(3000)
    U0 = o.macros()["uz"]
    o.step(100)
    m = o.macros()
    o.close()
    U = m["uz"].mean()
    assert np.abs(m["uz"] - U0).max() <= 1e-14 and np.ptp(m["uz"]) <= 1e-14
    assert 0.09 < U < 0.16
    d = math.sqrt(150.0 * (1.0 - phi_ref) ** 2 * Da * L * L / phi_ref ** 3)
    darcy = 150.0 * nu * (1.0 - phi) ** 2 * U / (phi ** 3 * d * d)
    forch = 1.75 * (1.0 - phi) * U * U / (phi ** 3 * d)
    assert forch > 0.15 * (darcy + forch)
    assert abs((darcy + forch) / G - 1.0) <= 1e-8


def test_pipe_conduction_mode_decays_through_the_axis(oracle_mod):
    """No flow in a pipe with its wall held at T = 0: the slowest conduction mode
    T = J0(lam r / R), lam the first zero of J0, keeps its shape and decays at
    alpha lam^2 / R^2 (Eq. 12 with u = 0 in cylindrical coordinates; alpha =
    c_sT^2 tau_T).  A slab of the same half-width would decay at alpha (pi/2)^2 / R^2,
    less than half as fast, so the rate checks the 1/r terms of the temperature
    lattice and the axis rows together.  The rate is taken between half and one
    and a half decay times, after the start transient, on R = 10.5, 20.5 and 40.5;
    its error must fall by more than 2.5 per grid doubling."""
    from scipy.special import j0

    lam = 2.404825557695773
    errs = []
    for nr in (11, 21, 41):
        cfg = li.pipe(nr=nr, nz=3, phi=1.0, Da=1e8, Re=0.0, tau_nu=0.8, Pr=1.0, F_phi=0.0, T_wall=0.0)
        cfg["accel_z"] = 0.0
        R = nr - 0.5
        r = 0.5 + np.arange(nr)
        mode = j0(lam * r[:-1] / R)
        init = np.zeros((3, 3, nr))
        init[2] = j0(lam * r / R)[None, :]
        o = oracle_mod.Oracle(cfg, init=init)
        alpha = 0.2 * o.derived()["tau_T"]
        rate = alpha * lam * lam / (R * R)
        t1, t2 = int(0.5 / rate), int(1.5 / rate)
        amps = []
        for n in (t1, t2 - t1):
            o.step(n)
            m = o.macros()
            T = m["T"][1, :-1]
            a = (T * mode).sum() / (mode * mode).sum()
            assert np.abs(T - a * mode).max() <= 0.02 * a  # the shape is kept
            assert np.abs(m["uz"]).max() <= 1e-15 and np.abs(m["ur"]).max() <= 1e-15
            amps.append(a)
        o.close()
        errs.append(abs(math.log(amps[0] / amps[1]) / (t2 - t1) / rate - 1.0))
    assert errs[0] <= 0.05 and errs[2] <= 0.006
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5


def test_oracle_steady_annulus_matches_table2():
    """The oracle's steady Nusselt numbers for the Sec. 4.2 annulus (R* = 2,
    A = 2, Pr = 0.7, no porous medium), stored in tests/golden/table2_nu_oracle.txt
    by make_nusselt_golden.py (which calls only the oracle), against the
    "Present" column of Table 2: within 0.3 % (0.23, 0.10, 0.04 % at Ra = 1e3,
    1e4, 1e5).  At steady state the heat entering at the inner wall leaves at
    the outer one, Nu_i = Nu_o (Eq. 42), up to the first-order wall error
    (1.3, 0.3, 0.5 % here; bound 1.5 %)."""
    printed = {1e3: 1.710, 1e4: 3.211, 1e5: 5.768}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_nu_oracle.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert sorted(float(r[0]) for r in rows) == sorted(printed)
    for ra, _, res, nu_i, nu_o in rows:
        ra, res, nu_i, nu_o = float(ra), float(res), float(nu_i), float(nu_o)
        assert res <= 1e-10
        assert abs(nu_i - printed[ra]) <= 0.003 * printed[ra], (ra, nu_i)
        assert abs(nu_i - nu_o) <= 0.015 * nu_i, (ra, nu_i, nu_o)


def test_derived_constants_eq39(oracle_mod):
    """Eq. (39) relaxation times and g beta dT = U^2 / L for the Table 2 cases."""
    for Ra, tn, tt in ((1e3, 0.9537, 1.080), (1e4, 0.6435, 0.342), (1e5, 0.5454, 0.108)):
        d = oracle_mod.Oracle(li.table2(Ra)).derived()
        assert abs(d["tau_nu"] - tn) < 1e-4 and abs(d["tau_T"] - tt) < 1e-3
        assert abs(d["gbeta"] - 0.01 / 3 / 99) < 1e-12


# --- steady-state residual ----------------------------------------------------

@pytest.mark.parametrize("du, dT", [((3e-4, -4e-4), 0.0), ((0.0, 0.0), 2e-3), ((1e-4, 0.0), 5e-4)])
def test_residual_of_a_uniform_change_is_its_rate(oracle_mod, du, dT):
    """The residual is the rms change per step since the snapshot, scaled by
    U = Ma c_s and dT.  Between the snapshot and a state n steps later whose
    fluid-node velocity differs by a constant vector du and temperature by a
    constant dT (a field changing linearly in time), it is exactly
    |du| / (n U) and |dT| / (n dT_ref), and res is the larger of the two.  The
    two states are start states (reading R8), whose fluid nodes return the
    given u and T (exactly with F_phi = 0)."""
    cfg = li.annulus(nr=12, nz=9, Ra=1e4, Da=1e-2, F_phi=0.0)
    nz, nr = cfg["nz"], cfg["nr"]
    rng = np.random.default_rng(7)
    a = np.stack([rng.normal(0, 0.01, (nz, nr)), rng.normal(0, 0.01, (nz, nr)), rng.uniform(0, 1, (nz, nr))])
    b = a.copy()
    b[0] += du[1]  # u_z
    b[1] += du[0]  # u_r
    b[2] += dT
    n = 37
    o = oracle_mod.Oracle(cfg, init=a)
    o.snapshot()
    o.step(n)
    ob = oracle_mod.Oracle(cfg, init=b)
    o.set_populations(*ob.populations())
    ob.close()
    r = o.residual()
    o.close()
    U = cfg["Ma"] * math.sqrt(CS2)
    want_u = math.hypot(*du) / (n * U)
    want_T = abs(dT) / (n * abs(cfg["delta_T"]))
    assert r["res_u"] == pytest.approx(want_u, rel=1e-9, abs=1e-15)
    assert r["res_T"] == pytest.approx(want_T, rel=1e-9, abs=1e-15)
    assert r["res"] == max(r["res_u"], r["res_T"])
