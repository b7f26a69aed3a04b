"""Shared comparison helpers of the GPU parity tests (no arithmetic of the method)."""
import numpy as np

# FP32 storage and arithmetic against the FP64 oracle: relative L2 of the
# velocity vector (u_z, u_r), of p and of T after a fixed number of steps.
TOL_FP32 = 1e-5


# Near rest FP32 resolves velocities only to about 1e-9 absolute; where a
# flow is slower than this floor (1 % of the characteristic velocity Ma c_s,
# Ma = 0.1) the velocity error is measured against the floor instead.
U_FLOOR = 0.01 * 0.1 / np.sqrt(3.0)


def rel_errors(gpu: dict, orc: dict, u_floor: float = 0.0) -> dict:
    du2 = np.sum((gpu["uz"] - orc["uz"]) ** 2 + (gpu["ur"] - orc["ur"]) ** 2)
    u2 = max(np.sum(orc["uz"] ** 2 + orc["ur"] ** 2), orc["uz"].size * u_floor ** 2)
    out = {"u": float(np.sqrt(du2 / u2)) if u2 > 0 else float(np.sqrt(du2))}
    for k in ("p", "T"):
        n = np.linalg.norm(orc[k])
        out[k] = float(np.linalg.norm(gpu[k] - orc[k]) / n) if n > 0 else float(np.linalg.norm(gpu[k]))
    return out


def assert_parity(gpu: dict, orc: dict, tol=TOL_FP32, label="", u_floor=0.0):
    np.testing.assert_array_equal(gpu["mask"], orc["mask"], err_msg=f"{label}: node classes differ")
    e = rel_errors(gpu, orc, u_floor)
    print(f"{label}: rel L2 u {e['u']:.2e} p {e['p']:.2e} T {e['T']:.2e}", flush=True)
    for k, v in e.items():
        assert v <= tol, f"{label}: {k} rel L2 {v:.3e} > {tol:.1e}"
    return e
