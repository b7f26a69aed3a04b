"""Writes table2_nu_oracle.txt: steady mean Nusselt numbers of the Table 2
annulus (Sec. 4.2) computed by the FP64 oracle alone.

The oracle steps the 100 x 200 problem and checks every 1000 steps; it stops
once the mean change per step over the last 1000 steps (velocity in units of
Ma c_s, temperature in units of dT) is at most 1e-10, then records Nu_i and
Nu_o (Eq. 42).  Run from the repository root: python tests/golden/make_nusselt_golden.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lbm_inputs as li  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table2_nu_oracle.txt")
TOL, CHECK, MAX_STEPS = 1e-10, 1000, 1_000_000


def main():
    oracle.build(force=False)
    lines = ["# Steady Nu_i, Nu_o of the Table 2 annulus (Sec. 4.2) from the FP64 oracle,",
             f"# stopped at mean change per step <= {TOL:g} over {CHECK} steps.",
             "# Written by make_nusselt_golden.py.  Columns: Ra, steps, residual, Nu_i, Nu_o."]
    for ra in (1e3, 1e4, 1e5):
        o = oracle.Oracle(li.table2(ra))
        t0 = time.time()
        res = 1.0
        while o.t < MAX_STEPS:
            o.snapshot()
            o.step(CHECK)
            res = o.residual()["res"]
            if res <= TOL:
                break
        nu_i, nu_o = o.nusselt()
        print(f"Ra={ra:g}: t={o.t} res={res:.3e} Nu_i={nu_i:.8f} Nu_o={nu_o:.8f} ({time.time() - t0:.0f} s)",
              flush=True)
        lines.append(f"{ra:g} {o.t} {res:.3e} {nu_i:.10f} {nu_o:.10f}")
        o.close()
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
