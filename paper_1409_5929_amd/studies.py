"""The paper's steady validation problems, run on the GPU.

  python -m paper_1409_5929_amd.studies table1     # Sec. 4.1, thermally developing porous pipe
  python -m paper_1409_5929_amd.studies table2     # Sec. 4.2, annulus without porous medium
  python -m paper_1409_5929_amd.studies table3     # Sec. 4.4, porous annulus with a heater
  python -m paper_1409_5929_amd.studies sec43      # Sec. 4.3, porous annulus, Ra* = 200, 500, 2000

Every case of a table runs as one instance of a single batched handle: for
Tables 2 and 3 and Sec. 4.3 until its residual reaches the tolerance (or the
step cap), for Table 1 for a fixed number of flow-through times. Progress lines are printed
as the run goes, followed by a table of the measured and printed values.

For Table 1, each case runs on the paper's grid spacing (r_i = 40.5) and at
its Re = 100 (L = r_i), Pr = 0.7, from a plug-flow start, for a fixed number
of flow-through times. The Nusselt number (Eq. 40, mixing-cup bulk
temperature) is reported at z = 0.9 H. The paper's pipe length, A = 16, is
shorter than the clear pipe's thermal entry length at this Re (about
0.05 Re_D Pr D = 7 D = 0.9 H), so the default pipe is twice as long. The
inlet velocity 0.0025 keeps the Darcy pressure drop, and the spurious T div u
sink it causes in the temperature equation, small at Da = 1e-3.

Sec. 4.3 prints no numbers (its results are the curves of Figs. 5-6): the
study reports the mean Nusselt numbers of both walls and the temperature
profiles T(r) at z / H = 0.25, 0.5, 0.75 and 1.

For Table 3, max |psi| is reported in units of alpha_e L. Here
alpha_e = c_sT^2 tau_T is the effective thermal diffusivity (text after Eq. 38),
with tau_T from Eq. (39). The paper prints the values without their scale;
this scale matches them at Da = 1e-4 and 1e-2.
"""
from __future__ import annotations

import argparse
import time

import lbm_inputs as li

from . import lbm
from .lbm import Lattice

# Printed values: Table 1 (Present, ref. [6]), Table 2 ("Present" column) and
# Table 3 (Ref. [5], Present).
TABLE1 = {1e-3: (5.467, 5.428), 3e-3: (5.226, 5.188), 1e-2: (4.770, 4.791), 3e-2: (4.390, 4.353),
          1e-1: (3.977, 3.963), 0.5: (3.745, 3.731), 1e8: (3.674, 3.658)}
TABLE2 = {1e3: 1.710, 1e4: 3.211, 1e5: 5.768}
TABLE3 = {1e-6: dict(nu_ref=2.97, nu=2.92, psi_ref=0.28, psi=0.27),
          1e-4: dict(nu_ref=9.28, nu=9.21, psi_ref=5.44, psi=5.69),
          1e-2: dict(nu_ref=17.51, nu=17.09, psi_ref=16.09, psi=16.38)}


def alpha_e(cfg: dict) -> float:
    """alpha_e = c_sT^2 tau_T (text after Eq. 38) as the library derives it."""
    return lbm.derived(cfg)["alpha_e"]


def run_to_steady(cfgs, tol=1e-10, max_steps=40_000_000, check=2000, chunk=1_000_000,
                  log=print, temperature=False):
    """Run all problems in one handle until none is running. Returns, per case,
    the state, step count, residual, Nu_i, Nu_o, max |psi| (lattice units) and,
    with temperature=True, the temperature field."""
    lat = Lattice(cfgs, check_interval=check, tol=tol, max_steps=max_steps)
    t0 = time.time()
    try:
        while True:
            lat.step(chunk)
            r = lat.residual()
            info = [lat.info(i) for i in range(len(cfgs))]
            log(f"t={info[0]['t']:>10d} {time.time() - t0:7.1f} s  " + "  ".join(
                f"[{i}] {x['status'][:4]} res {r['res'][i]:.1e} Nu {r['nu_i'][i]:.4f}"
                for i, x in enumerate(info)))
            if all(x["status"] != "running" for x in info):
                break
        return [dict(status=info[i]["status"], t=info[i]["t"], res=float(r["res"][i]),
                     nu_i=float(r["nu_i"][i]), nu_o=float(r["nu_o"][i]),
                     psi_max=lat.stream_function(i, field=False)[1],
                     T=lat.fields(i)["T"] if temperature else None)
                for i in range(len(cfgs))]
    finally:
        lat.close()


def table1(A=32.0, u_in=0.0025, flow_throughs=3.0, log=print):
    """Fully developed pipe Nusselt numbers for the Darcy numbers of Table 1
    (1e8 stands for the pipe without porous medium)."""
    das = sorted(TABLE1)
    cfgs = [li.developing_pipe(Da=da, A=A, u_in=u_in) for da in das]
    H = cfgs[0]["nz"] - 1
    steps = int(flow_throughs * H / u_in)
    lat = Lattice(cfgs, init=[li.plug_start(c) for c in cfgs], check_interval=0)
    t0 = time.time()
    try:
        done, chunk = 0, 200_000
        while done < steps:
            n = min(chunk, steps - done)
            lat.step(n)
            done += n
            lat.sync()
            log(f"t={done:>9d} of {steps} {time.time() - t0:7.1f} s")
        k = int(0.9 * H)
        out = []
        for i, da in enumerate(das):
            nu, _ = lat.pipe_nusselt(i)
            nua, _ = lat.pipe_nusselt(i, area=True)
            out.append(dict(Da=da, nu=float(nu[k]), nu_area=float(nua[k]), nu_mid=float(nu[H // 2]),
                            steps=steps))
    finally:
        lat.close()
    log("Da      Nu(0.9H)  Nu(0.5H)  paper   ref.6   area-mean T_b")
    for o in out:
        p, ref = TABLE1[o["Da"]]
        log(f"{o['Da']:<7g} {o['nu']:.4f}    {o['nu_mid']:.4f}    {p:.3f}   {ref:.3f}   {o['nu_area']:.4f}")
    return out


def table2(log=print):
    ras = sorted(TABLE2)
    out = run_to_steady([li.table2(ra) for ra in ras], tol=1e-10, chunk=100_000, check=1000,
                        log=log)
    log("Ra      Nu_i     Nu_o     paper   steps      state")
    for ra, o in zip(ras, out):
        log(f"{ra:<7g} {o['nu_i']:.4f}  {o['nu_o']:.4f}  {TABLE2[ra]:.3f}   {o['t']:<10d} {o['status']}")
    return out


def table3(nr=200, nz=200, log=print):
    das = sorted(TABLE3)
    cfgs = [li.heater_annulus(Da=da, nr=nr, nz=nz) for da in das]
    out = run_to_steady(cfgs, log=log)
    log("Da      Nu        paper (ref.5)   |psi|max/(alpha_e L)  paper (ref.5)   Nu_o    steps     state")
    for da, c, o in zip(das, cfgs, out):
        p = TABLE3[da]
        psi = o["psi_max"] / (alpha_e(c) * c["L"])
        o["psi"] = psi
        log(f"{da:<7g} {o['nu_i']:.4f}   {p['nu']:.2f} ({p['nu_ref']:.2f})    {psi:8.4f}              "
            f"{p['psi']:.2f} ({p['psi_ref']:.2f})   {o['nu_o']:.4f}  {o['t']:<9d} {o['status']}")
    return out


def sec43(nr=300, nz=300, ra_stars=(200.0, 500.0, 2000.0), tol=1e-9, max_steps=30_000_000,
          log=print):
    """Sec. 4.3 annulus at the given Darcy-Rayleigh numbers: steady mean Nusselt
    numbers (Eq. 42) and the temperature profiles theta = (T - T_o) / (T_i - T_o)
    across the gap at z / H = 0.25, 0.5, 0.75 and 1 (the curves of Fig. 6)."""
    cfgs = [li.porous_annulus_43(ra, nr=nr, nz=nz) for ra in ra_stars]
    out = run_to_steady(cfgs, tol=tol, max_steps=max_steps, log=log, temperature=True)
    log("Ra*     Nu_i     Nu_o     steps      state")
    for ra, o in zip(ra_stars, out):
        log(f"{ra:<7g} {o['nu_i']:.4f}  {o['nu_o']:.4f}  {o['t']:<10d} {o['status']}")
    xs = [0.0, 0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0]
    log("theta at (r - r_i) / L = " + " ".join(f"{x:5.2f}" for x in xs))
    for ra, c, o in zip(ra_stars, cfgs, out):
        theta = (o["T"] - c["T_rmax"]) / (c["T_rmin"] - c["T_rmax"])
        o["theta"] = {}
        for zh in (0.25, 0.5, 0.75, 1.0):
            k = int(round(zh * (nz - 1)))
            row = [float(theta[k, int(round(x * (nr - 1)))]) for x in xs]
            o["theta"][zh] = row
            log(f"Ra*={ra:<6g} z/H={zh:<4g} " + " ".join(f"{v:5.3f}" for v in row))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("table", choices=["table1", "table2", "table3", "sec43"])
    ap.add_argument("--grid", type=int, default=200, help="table3: nr = nz (paper: 200)")
    ap.add_argument("--A", type=float, default=32.0, help="table1: pipe length over r_i (paper: 16)")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.table == "table1":
        table1(A=a.A, log=log)
    elif a.table == "table2":
        table2(log)
    elif a.table == "sec43":
        sec43(log=log)
    else:
        table3(a.grid, a.grid, log)


if __name__ == "__main__":
    main()
