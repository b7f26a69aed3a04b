"""Pin of the C oracle's indexing and boundary handling by brute force: a second,
literal oracle (``oracle.lbm_literal``: per-node Python loops, M built from the
definition of its rows, pull streaming, Eq. 32 for wall equilibria) and the C
oracle advance the same tiny lattices with every side and thermal type; their
populations, fields and node classes agree to FP64 rounding after 10 steps.
"""
import numpy as np
import pytest

from oracle import lbm_literal as O2
from tests.conftest import load_matrix

STEPS = 10
TOL = 1e-13


def _cases():
    base = dict(r0=3.0, L=6.0, phi=0.6, Da=1e-2, F_phi=0.0, Pr=0.7, tau_nu=0.0, Ra=1e4,
                T_rmin=1.0, T_rmax=0.0, T_ref=0.5)
    out = [
        ("annulus, porosity field, Ergun", dict(base, F_phi=-1.0), True),
        ("printed source, fixed z walls", dict(base, src_printed=1, therm_z="fixed", T_zmin=0.2,
                                               T_zmax=0.8, F_phi=0.4, accel_r=1e-4), False),
        ("pipe: axis, periodic z", dict(r0=0.5, side_rmin="axis", side_z="periodic",
                                        therm_rmin="adiabatic", L=4.0, phi=0.8, Da=1e-1,
                                        tau_nu=0.8, accel_z=1e-3, T_rmax=1.0, T_init=0.0), False),
        ("closed cylinder: axis, fixed z walls", dict(r0=0.5, side_rmin="axis", therm_rmin="adiabatic",
                                                      therm_z="fixed", T_zmin=1.0, T_zmax=0.0,
                                                      T_rmax=0.0, delta_T=1.0, T_ref=0.5, L=5.0,
                                                      phi=0.7, Da=1e-2, F_phi=-1.0, Ra=1e4), True),
        ("periodic r and z", dict(r0=40.0, side_rmin="periodic", side_rmax="periodic",
                                  side_z="periodic", L=10.0, phi=0.6, Da=1e-2, F_phi=-1.0,
                                  tau_nu=1.0, accel_z=1e-4, T_rmin=1.0, T_rmax=0.0, T_ref=0.5), True),
        ("pipe inlet/outlet", dict(r0=0.5, side_rmin="axis", side_z="flow", therm_rmin="adiabatic",
                                   therm_z="fixed", T_zmin=0.0, T_rmax=1.0, delta_T=1.0, u_in=0.01,
                                   tau_nu=0.7, L=4.0, phi=0.9, Da=1e-1, F_phi=0.2), False),
        ("inner flux wall window", dict(base, therm_rmin="flux", flux_rmin=0.2, flux_zlo=2.0,
                                        flux_zhi=4.0, delta_T=1.0, T_ref=0.0), False),
        ("outer flux wall, adiabatic ends", dict(base, therm_rmax="flux", flux_rmax=0.3,
                                                 flux_zlo=0.0, flux_zhi=5.0), False),
    ]
    return out


def _start(rng, nz, nr):
    return np.stack([rng.normal(0, 0.02, (nz, nr)), rng.normal(0, 0.02, (nz, nr)),
                     rng.uniform(0, 1, (nz, nr))])


def _run_both(oracle_mod, cfg, phi, init, steps):
    o1 = oracle_mod.Oracle(cfg, phi_field=phi, init=init)
    o2 = O2.LiteralLattice(cfg, phi_field=phi, init=init)
    o1.step(steps)
    o2.step(steps)
    f1, g1 = o1.populations()
    m1 = o1.macros()
    o1.close()
    return (f1, g1, m1), (o2.f, o2.g, o2.macros())


def _compare(a, b, what):
    (f1, g1, m1), (f2, g2, m2) = a, b
    np.testing.assert_array_equal(m1["mask"], m2["mask"], err_msg=f"{what}: node classes")
    for name, x, y in (("f", f1, f2), ("g", g1, g2)):
        np.testing.assert_array_equal(np.isnan(x), np.isnan(y), err_msg=f"{what}: unset {name} slots")
        ok = ~np.isnan(x)
        err = np.abs(x[ok] - y[ok]).max() / np.abs(y[ok]).max()
        assert err <= TOL, (what, name, err)
    # rho, T, p relative to their size; u on the scale of the lattice speed
    # c = 1 that the populations carry (u_r comes out of a sum of terms of
    # order r w_i that cancel down to r rho u_r)
    for k in ("rho", "ur", "uz", "T", "p"):
        scale = 1.0 if k in ("ur", "uz") else max(np.abs(m2[k]).max(), 1e-300)
        err = np.abs(m1[k] - m2[k]).max() / scale
        assert err <= TOL, (what, k, err)


@pytest.mark.parametrize("grid", [(4, 6), (5, 7)], ids=["4x6", "5x7"])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_literal_oracle_equals_c_oracle(oracle_mod, case, grid):
    name, cfg, field = case
    nr, nz = grid
    cfg = dict(cfg, nr=nr, nz=nz)
    rng = np.random.default_rng(1409 + nr)
    phi = rng.uniform(0.4, 0.8, (nz, nr)) if field else None
    init = _start(rng, nz, nr)
    for steps in (0, STEPS):
        _compare(*_run_both(oracle_mod, cfg, phi, init, steps), f"{name} {nr}x{nz} n={steps}")


def test_literal_moment_matrix_is_the_printed_one():
    """M built from its rows' definitions is the matrix printed as Eq. (18)."""
    np.testing.assert_array_equal(O2.moment_matrix(), load_matrix("M_eq18.txt"))


def test_a_planted_sign_error_is_caught(oracle_mod, monkeypatch):
    """The comparison has teeth: flipping the sign of the axisymmetric term a_r
    of Eq. (25) in the literal oracle makes the two disagree far beyond
    rounding."""
    _, cfg, _ = _cases()[0]
    cfg = dict(cfg, nr=4, nz=6)
    rng = np.random.default_rng(3)
    phi = rng.uniform(0.4, 0.8, (6, 4))
    init = _start(rng, 6, 4)
    good = O2.LiteralLattice.forces

    def flipped(self, k, j, ur, uz, T):
        Fr, Fz, ar = good(self, k, j, ur, uz, T)
        return Fr, Fz, -ar

    monkeypatch.setattr(O2.LiteralLattice, "forces", flipped)
    a, b = _run_both(oracle_mod, cfg, phi, init, 3)
    err = np.nanmax(np.abs(a[0] - b[0])) / np.nanmax(np.abs(b[0]))
    assert err > 1e-4
