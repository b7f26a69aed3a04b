"""Shared comparison helpers of the GPU parity tests (no arithmetic of the method)."""
import numpy as np

# FP32 storage and arithmetic against the FP64 oracle: relative L2 of the
# velocity vector (u_z, u_r), of the density and temperature deviations and of
# the pressure output after a fixed number of steps.
TOL_FP32 = 1e-5


# Near rest FP32 resolves velocities only to about 1e-9 absolute; where a
# flow is slower than this floor (1 % of the characteristic velocity Ma c_s,
# Ma = 0.1) the velocity error is measured against the floor instead.
U_FLOOR = 0.01 * 0.1 / np.sqrt(3.0)

# Density and temperature are compared as deviations from the oracle field's
# mean (rho - rho_bar, T - T_bar): their totals carry a constant part (rho
# near 1, T near the reference temperature) that would swamp the physical
# signal in a relative norm.  Where a field barely varies (the density of a
# periodic pipe, a uniform temperature) its error is measured against a floor
# instead.  For the density the floor is the deviation rho' = u / c_s that a
# sound wave of 1 % of the characteristic velocity Ma c_s carries, 0.01 Ma:
# rho - 1 is a sum of populations whose size is set by the velocity, so FP32
# resolves it only to about 2^-24 u / c_s (1e-9 in slow pipe flow).  For the
# temperature it is 1e-3 of a unit temperature difference (FP32); 16-bit
# storage rounds T - T_s, so there the tests pass the temperature difference
# itself.
RHO_FLOOR = 0.01 * 0.1
T_FLOOR = 1e-3
# 16-bit storage rounds the velocity-sized populations to 2^-11 (FP16) or
# 2^-8 (BF16) of their size, stochastically, and the mass those roundings
# move does not decay (it is conserved): the density deviation is resolved
# only to that rounding of u / c_s, accumulated over the steps.  There the
# density floor is 10 % of the characteristic density scale Ma.
RHO_FLOOR_16 = 0.1 * 0.1


def tol_fp32(n: int) -> float:
    """FP32 bound after n steps.  Storage rounds each population deviation to
    2^-24 of its size every step and the roundings of successive steps are
    independent; the conserved part (mass) carries them on as a random walk.
    So beyond 100 steps the 1e-5 bound grows like sqrt(n / 100)."""
    return TOL_FP32 * max(1.0, (n / 100.0) ** 0.5)

FIELD_KEYS = ("uz", "ur", "p", "T", "mask", "drho", "rho")


def rho_deviation(d: dict):
    """rho - 1 in FP64 from a field dict: the GPU's "drho" (rho - 1 as the
    library computes it from its stored deviations) or the oracle's "rho"."""
    if "drho" in d:
        return np.asarray(d["drho"], dtype=np.float64)
    if "rho" in d:
        return np.asarray(d["rho"], dtype=np.float64) - 1.0
    return None


def window(d: dict, ks: slice, js: slice) -> dict:
    """The [ks, js] window of every field a dict holds."""
    return {k: d[k][ks, js] for k in FIELD_KEYS if k in d}


def _dev_error(a, b, floor):
    """Relative L2 of a - b against the deviation of b from its mean (or the floor)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.linalg.norm(b - b.mean()), floor * np.sqrt(b.size))
    return float(np.linalg.norm(a - b) / den)


def rel_errors(gpu: dict, orc: dict, u_floor: float = 0.0, t_floor: float = T_FLOOR,
               rho_floor: float = RHO_FLOOR) -> dict:
    du2 = np.sum((gpu["uz"] - orc["uz"]) ** 2 + (gpu["ur"] - orc["ur"]) ** 2)
    u2 = max(np.sum(orc["uz"] ** 2 + orc["ur"] ** 2), orc["uz"].size * u_floor ** 2)
    out = {"u": float(np.sqrt(du2 / u2)) if u2 > 0 else float(np.sqrt(du2))}
    n = np.linalg.norm(orc["p"])
    out["p"] = float(np.linalg.norm(gpu["p"] - orc["p"]) / n) if n > 0 else float(np.linalg.norm(gpu["p"]))
    rg, ro = rho_deviation(gpu), rho_deviation(orc)
    if rg is not None and ro is not None:
        out["rho"] = _dev_error(rg, ro, rho_floor)
    out["T"] = _dev_error(gpu["T"], orc["T"], t_floor)
    return out


def assert_parity(gpu: dict, orc: dict, tol=TOL_FP32, label="", u_floor=0.0):
    np.testing.assert_array_equal(gpu["mask"], orc["mask"], err_msg=f"{label}: node classes differ")
    assert "drho" in gpu or "rho" in gpu, f"{label}: no density deviation to compare"
    e = rel_errors(gpu, orc, u_floor)
    print(f"{label}: rel L2 u {e['u']:.2e} rho-rho_bar {e['rho']:.2e} T-T_bar {e['T']:.2e} "
          f"p {e['p']:.2e}", flush=True)
    for k, v in e.items():
        assert v <= tol, f"{label}: {k} rel L2 {v:.3e} > {tol:.1e}"
    return e
