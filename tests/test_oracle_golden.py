"""The oracle reproduces its stored tiny-workload result (written by
tests/golden/make_oracle_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

import oracle
from paper_2011_07209_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_tiny16_matches_stored_oracle_result():
    with open(os.path.join(HERE, "golden", "tiny16_oracle.json")) as f:
        g = json.load(f)
    cfg = synth.CONFIGS["tiny16"]
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    P = oracle.make_params(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, cfg.stencil_n, cfg.cg_tol)
    res = oracle.evaluate(P, phi, orbs.centres)
    assert abs(res["E"] / g["E"] - 1) < 1e-12
    np.testing.assert_allclose(res["sigma"], np.array(g["sigma"]), rtol=1e-10, atol=1e-14)
    assert [(p.i, p.j) for p in res["pairs"]] == [(p[0], p[1]) for p in g["pairs"]]
    assert abs(np.abs(res["D"]).sum() / g["D_abs_sum"] - 1) < 1e-10
