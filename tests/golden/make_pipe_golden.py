"""Writes pipe_nu_oracle.txt: local Nusselt numbers of the thermally developing
pipe flow (Sec. 4.1) at steady state, computed by the FP64 oracle alone.

The geometry is the paper's (A = H / r_i = 16) at a quarter and at half its
resolution: r_i = 10.5 and 20.5 (11 and 21 rows with the wall row).  Pr = 0.7,
phi = 1, F_phi = 0, plug-flow start.  Re = 25 with L = r_i, so that flow and
temperature are fully developed over the last part of the pipe; the paper's
Re = 100 leaves the clear pipe short of thermal development at this length.
u_in = 0.0025 keeps the density drop along the pipe, and the spurious T div u
sink that a weakly compressible flow puts into the temperature equation,
small.  Two Darcy numbers are run: none (Da = 1e8, a clear pipe) and
Da = 1e-2.  Every 1000 steps the mean change per step over those steps is
checked, with u_in and T_w - T_in as scales.  The run stops at 1e-10 and
records, at every column, Nu (Eq. 40) and T_b with the mixing-cup and with
the area-mean bulk temperature.
Run from the repository root: python tests/golden/make_pipe_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lbm_inputs as li  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pipe_nu_oracle.txt")
TOL, CHECK, MAX_STEPS = 1e-10, 1000, 4_000_000
CASES = [(nr, da) for nr in (11, 21) for da in (1e8, 1e-2)]


def config(Da, nr=21):
    return li.developing_pipe(Da=Da, nr=nr, Re=25.0, u_in=0.0025)


def main():
    oracle.build(force=False)
    lines = ["# Steady local Nu (Eq. 40) and T_b of the Sec. 4.1 pipe (A = 16, Re = 25,",
             "# Pr = 0.7, u_in = 0.0025) at r_i = 10.5 and 20.5 from the FP64 oracle,",
             f"# stopped at mean change per step <= {TOL:g} over {CHECK} steps.",
             "# Written by make_pipe_golden.py.  Per case: a line 'case nr Da steps residual',",
             "# then one line per column: k Nu_mix Tb_mix Nu_area Tb_area (mixing-cup and",
             "# area-mean bulk temperature)."]
    for nr, Da in CASES:
        cfg = config(Da, nr)
        o = oracle.Oracle(cfg, init=li.plug_start(cfg))
        t0 = time.time()
        res = 1.0
        while o.t < MAX_STEPS:
            o.snapshot()
            o.step(CHECK)
            res = o.residual()["res"]
            if o.t % 20000 == 0:
                print(f"nr={nr} Da={Da:g} t={o.t} res={res:.3e} ({time.time() - t0:.0f} s)", flush=True)
            if res <= TOL:
                break
        nu, tb = o.pipe_nusselt()
        nua, tba = o.pipe_nusselt(area=True)
        k = int(0.9 * (cfg["nz"] - 1))
        print(f"nr={nr} Da={Da:g}: t={o.t} res={res:.3e} Nu(z=0.9H)={nu[k]:.6f} (area {nua[k]:.6f}) "
              f"({time.time() - t0:.0f} s)", flush=True)
        lines.append(f"case {nr} {Da:g} {o.t} {res:.3e}")
        lines += [f"{i} {nu[i]:.10f} {tb[i]:.10f} {nua[i]:.10f} {tba[i]:.10f}"
                  for i in range(cfg["nz"])]
        o.close()
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
