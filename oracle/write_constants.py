"""Write the van der Waals constants that the synthetic workloads use as inputs.

    python -m oracle.write_constants

Calls only the oracle (oracle/thermo.py).  Output:
paper_2002_09217_amd/data/vdw_constants.json with
  * the coexistence densities (Maxwell's equal-area rule, main text, Fig. 2) for
    T/T_cr = 0.850, 0.855, ..., 0.995 with the paper's a = 2/49, b = 2/21, R = 1;
  * the post-shock state behind a shock with pressure ratio 3 running into saturated
    vapour at T/T_cr = 0.95, delta = 1/3 (Rankine-Hugoniot, App. E);
  * the shock-tube states the paper prints in reduced units (p/p_cr, rho/rho_cr) -- the
    anomalous case of the main text (Fig. 4, delta = 0.0125) and the two cases of
    App. E -- with the temperature of each state from the van der Waals EoS.
"""
from __future__ import annotations

import json
import os

from oracle.thermo import VdW

# (p_L, rho_L, p_R, rho_R) in reduced units and delta: main text, Fig. 4 caption
# (anomalous shock), and App. E, table of shock-tube conditions (cases I and II)
SHOCK_TUBES = {
    "anomalous": (1.09, 0.879, 0.885, 0.562, 0.0125),
    "case_I": (1.6077, 1.01, 0.8957, 0.594, 0.329),
    "case_II": (3.00, 1.818, 0.575, 0.275, 0.0125),
}

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "paper_2002_09217_amd", "data", "vdw_constants.json")


def compute() -> dict:
    g = VdW()
    table = {"T_over_Tcr": [], "rho_v": [], "rho_l": [], "p_sat": []}
    for i in range(30):
        tr = round(0.85 + 0.005 * i, 3)
        rv, rl, ps = g.maxwell(tr * g.T_cr)
        table["T_over_Tcr"].append(tr)
        table["rho_v"].append(rv)
        table["rho_l"].append(rl)
        table["p_sat"].append(ps)
    amb = VdW(delta=1.0 / 3.0)
    rv, rl, ps = amb.maxwell(0.95 * amb.T_cr)
    sh = amb.hugoniot_direct(rv, ps, 3.0 * ps)
    shock = {"T_over_Tcr": 0.95, "delta": 1.0 / 3.0, "pressure_ratio": 3.0, "rho0": rv, "p0": ps,
             "rho_liquid": rl, "rho1": sh["rho1"], "u1": sh["u1"], "p1": sh["p1"], "T1": sh["T1"],
             "shock_speed": sh["s"], "mach": sh["Ms"]}
    tubes = {}
    for name, (pl, rl_, pr, rr, d) in SHOCK_TUBES.items():
        gd = VdW(delta=d)
        states = []
        for p_r, rho_r in ((pl, rl_), (pr, rr)):
            rho, p = rho_r * gd.rho_cr, p_r * gd.p_cr
            states.append({"rho": rho, "p": p, "T": gd.T_of_p(rho, p)})
        tubes[name] = {"delta": d, "left": states[0], "right": states[1]}
    return {"a": g.a, "b": g.b, "R": g.R, "rho_cr": g.rho_cr, "T_cr": g.T_cr, "p_cr": g.p_cr,
            "coexistence": table, "shock": shock, "shock_tubes": tubes}


def main():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    with open(OUT, "w") as fh:
        json.dump(compute(), fh, indent=1)
        fh.write("\n")
    print(OUT)


if __name__ == "__main__":
    main()
