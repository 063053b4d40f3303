"""Writes tests/golden/tiny_step.json: the FP64 oracle's outputs for a tiny
seeded case (64 gas + 48 dm particles).  Calls only the oracle; the stored
values guard the oracle against unintended changes of its arithmetic."""
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


def main():
    out = oracle.step(case(), brute=True)
    keep = {k: np.asarray(v).tolist() for k, v in out.items()
            if k != "degenerate"}
    with open(os.path.join(HERE, "tiny_step.json"), "w") as f:
        json.dump({"case": "random_uniform(64, 48, 2024, n_ngb=40, "
                           "h_spread=0.1, h_rule=global)", "outputs": keep}, f)


if __name__ == "__main__":
    main()
