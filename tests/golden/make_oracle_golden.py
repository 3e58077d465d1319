"""Writes tiny16_oracle.json: the FP64 oracle's E_xx, sigma_xx and per-pair
energies for the tiny cubic workload (12 bohr, 60^3, 16 orbitals).  Calls only
the oracle and the input generator."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2011_07209_amd import synth  # noqa: E402


def main():
    cfg = synth.CONFIGS["tiny16"]
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    P = oracle.make_params(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, cfg.stencil_n, cfg.cg_tol)
    res = oracle.evaluate(P, phi, orbs.centres)
    out = {
        "workload": "tiny16: cubic 12 bohr, 60^3, 16 orbitals, R_pair 8, R_PE 5, R_ME 7, l_max 6, n 1, tol 1e-10",
        "E": res["E"],
        "sigma": res["sigma"].tolist(),
        "D_abs_sum": float(np.abs(res["D"]).sum()),
        "D_dot_phi": float(np.sum(res["D"] * phi)),
        "pairs": [[p.i, p.j, p.E, p.cg_iters, p.n_pe, p.n_me] for p in res["pairs"]],
    }
    with open(os.path.join(HERE, "tiny16_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
