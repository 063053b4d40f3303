"""Writes tests/golden/tiny_step.json: the FP64 oracle's outputs for a tiny
seeded case (64 gas + 48 dm particles), and tests/golden/tiny_recon.json:
the same case with the reconstructed viscosity and the compatible energy
update of a kick of RECON_DT.  Calls only the oracle; the stored values
guard the oracle against unintended changes of its arithmetic."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2510_03557_amd import workloads  # noqa: E402


def case():
    return workloads.random_uniform(64, 48, 2024, n_ngb=40.0, h_spread=0.1,
                                    h_rule="global")


RECON_DT = 1e-3


def recon_outputs():
    wl = case()
    out = oracle.step(wl, brute=True, recon=True)
    r = oracle.compatible_update(wl, out, RECON_DT, recon=True, brute=True)
    return {"dv": out["dv"], "a_hydro": out["a_hydro"], "dudt": out["dudt"],
            "dudt_compatible": r["dudt"], "u1": r["u1"]}


def main():
    out = oracle.step(case(), brute=True)
    keep = {k: np.asarray(v).tolist() for k, v in out.items()
            if k not in ("degenerate", "dv")}
    with open(os.path.join(HERE, "tiny_step.json"), "w") as f:
        json.dump({"case": "random_uniform(64, 48, 2024, n_ngb=40, "
                           "h_spread=0.1, h_rule=global)", "outputs": keep}, f)
    keep = {k: np.asarray(v).tolist() for k, v in recon_outputs().items()}
    with open(os.path.join(HERE, "tiny_recon.json"), "w") as f:
        json.dump({"case": "random_uniform(64, 48, 2024, n_ngb=40, "
                           "h_spread=0.1, h_rule=global), reconstructed "
                           "viscosity, compatible kick of 1e-3",
                   "outputs": keep}, f)


if __name__ == "__main__":
    main()
