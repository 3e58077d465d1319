"""Fluctuating cells on the GPU (Sec. III B 2): a plan keeps its
proto-subdomains (grid offsets, so fixed scaled coordinates and point counts)
while exx_set_cell changes the cell.  Checked against the oracle run with the
same frozen offset sets (h_geom = the plan's cell) and the new physical cell,
against the strain derivative of E_xx, and for re-assembly against a fresh
plan.  FP64 bars as in the parity tests."""
import math

import numpy as np
import pytest
import torch

from paper_2011_07209_amd import exx, synth

from gpu_util import oracle_eval, rel1
from test_gpu_general import _cell, _cfg
from test_gpu_parity import TOL_D, TOL_E, TOL_S

pytestmark = pytest.mark.gpu

H0 = _cell(12.0, 12.5, 11.5, 80, 95, 100)
N0 = (48, 50, 46)
# with cell_fluctuation the ME sphere holds n steps along every nearest-neighbour
# direction (the longest, (1,1,1)-like, is 0.49 bohr here)
R_ME_FLUCT = 5.6
# The library lists pairs with the new cell, the oracle with the frozen one;
# a pair radius above every minimum-image distance keeps the same (all) pairs
# on both sides, whose grid centres agree (fixed crystal coordinates).
R_PAIR_ALL = 20.0
STRAIN = np.array([[0.012, 0.004, -0.003], [0.002, -0.008, 0.005], [-0.004, 0.003, 0.010]])


def _inputs(cfg):
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    dev = torch.device("cuda:0")
    return orbs, phi, torch.from_numpy(phi).to(dev), torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev)


def _eval(plan, orb_t, cen_t, want_D=True):
    dev = orb_t.device
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    S = torch.zeros(9, dtype=torch.float64, device=dev)
    D = torch.empty_like(orb_t) if want_D else None
    plan.eval(orb_t, cen_t, E, D, S)
    torch.cuda.synchronize()
    return E.item(), S.cpu().numpy().reshape(3, 3, order="F"), (D.cpu().numpy() if want_D else None), plan.stats()


def _oracle_strained(cfg, orbs, phi, h1):
    import oracle
    P = oracle.make_params(h1, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, cfg.stencil_n, cfg.cg_tol,
                           h_geom=cfg.h)
    return oracle.evaluate(P, phi, orbs.centres)


@pytest.mark.parametrize("start", ["triclinic", "cubic"])
def test_set_cell_matches_oracle_with_frozen_subdomains(start):
    h0 = H0 if start == "triclinic" else np.diag([12.0, 12.0, 12.0])
    N = N0 if start == "triclinic" else (48, 48, 48)
    cfg = _cfg(f"cell-{start}", h0, N, R_ME=R_ME_FLUCT, R_pair=R_PAIR_ALL, seed_index=120)
    orbs, phi, orb_t, cen_t = _inputs(cfg)
    h1 = (np.eye(3) + STRAIN) @ h0
    plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, stencil_n=cfg.stencil_n,
                    cg_tol=cfg.cg_tol, cell_fluctuation=1)
    try:
        plan.set_cell(h1)
        # the orbital centres move with the cell (fixed crystal coordinates)
        C1 = orbs.centres @ np.linalg.inv(h0).T @ h1.T
        cen_t.copy_(torch.from_numpy(np.ascontiguousarray(C1)).to(cen_t.device))
        E, S, D, st = _eval(plan, orb_t, cen_t)
    finally:
        plan.close()
    o = _oracle_strained(cfg, orbs, phi, h1)
    print(f"[set_cell {start}] E gpu={E:.15g} oracle={o['E']:.15g} strain={st['cell_strain']:.4f} "
          f"arms={st['n_arms']}", flush=True)
    assert abs(st["cell_strain"] - np.abs(h1 @ np.linalg.inv(h0) - np.eye(3)).max()) < 1e-14
    assert st["reassemblies"] == 0 and st["n_arms"] == 6 and st["n_unconverged"] == 0
    assert st["n_pairs"] == len(o["pairs"]) == cfg.n_orb * (cfg.n_orb + 1) // 2
    assert rel1(E, o["E"]) <= TOL_E
    assert rel1(S, o["sigma"]) <= TOL_S
    assert rel1(D, o["D"]) <= TOL_D
    # the EXX contribution to the internal pressure (eq. pxx_working) equals
    # E/(3V) up to the discretization gap of the virial identity
    Pi, p = exx.exx_pressure(h1, S)
    V = abs(np.linalg.det(h1))
    assert abs(p - E / (3 * V)) <= 3e-3 * abs(E / (3 * V)), (p, E / (3 * V))


def test_orthorhombic_plan_follows_isotropic_scaling():
    """Without cell_fluctuation an orthorhombic plan keeps its axis-stencil
    tables and accepts orthorhombic cells only (isotropic NpT in a cubic cell)."""
    h0 = np.diag([12.0, 12.0, 12.0])
    cfg = synth.custom(key="iso", grid=(48, 48, 48), n_orb=6, R_pair=R_PAIR_ALL, R_PE=4.0, R_ME=5.2, l_max=5,
                       cg_tol=1e-12, seed_index=121)
    orbs, phi, orb_t, cen_t = _inputs(cfg)
    h1 = 1.015 * h0
    plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, stencil_n=cfg.stencil_n,
                    cg_tol=cfg.cg_tol)
    try:
        plan.set_cell(h1)
        cen_t.copy_(torch.from_numpy(np.ascontiguousarray(1.015 * orbs.centres)).to(cen_t.device))
        E, S, D, st = _eval(plan, orb_t, cen_t)
        with pytest.raises(exx.ExxError) as ei:
            plan.set_cell(h0 @ (np.eye(3) + STRAIN))
        assert ei.value.status == exx.EXX_EINVAL
    finally:
        plan.close()
    o = _oracle_strained(cfg, orbs, phi, h1)
    assert st["n_arms"] == 3
    assert rel1(E, o["E"]) <= TOL_E
    assert rel1(S, o["sigma"]) <= TOL_S
    assert rel1(D, o["D"]) <= TOL_D


def test_sigma_is_the_strain_derivative_through_set_cell():
    """sigma^{a al} = dE/dh_{a al} (eq. sxx_working) checked with the library
    alone: central differences of E_xx over exx_set_cell, orbitals fixed in
    crystal coordinates (phi -> phi sqrt(V0/V)), at discretization level."""
    # the grid and radii of the oracle's strain-derivative pin (spacing ~0.2
    # bohr): sigma and the derivative of the discrete E agree to the
    # discretization level established there
    cfg = _cfg("cell-fd", H0, (60, 62, 58), n_orb=3, R_PE=4.5, R_ME=6.2, R_pair=R_PAIR_ALL, cg_tol=1e-13,
               seed_index=122)
    orbs, phi, orb_t, cen_t = _inputs(cfg)
    plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, stencil_n=cfg.stencil_n,
                    cg_tol=cfg.cg_tol, cell_fluctuation=1)
    V0 = abs(np.linalg.det(H0))
    eps = 1e-4 * 12.0
    try:
        _, S0, _, _ = _eval(plan, orb_t, cen_t, want_D=False)
        smax = np.abs(S0).max()
        for (a, al) in [(0, 0), (0, 1), (2, 0), (1, 2)]:
            Es = []
            for sgn in (1, -1):
                h = H0.copy()
                h[a, al] += sgn * eps
                plan.set_cell(h)
                orb_t.copy_(torch.from_numpy(phi * math.sqrt(V0 / abs(np.linalg.det(h)))).to(orb_t.device))
                C = orbs.centres @ np.linalg.inv(H0).T @ h.T
                cen_t.copy_(torch.from_numpy(np.ascontiguousarray(C)).to(cen_t.device))
                Es.append(_eval(plan, orb_t, cen_t, want_D=False)[0])
            fd = (Es[0] - Es[1]) / (2 * eps)
            print(f"[cell fd] ({a},{al}) fd={fd:.10g} sigma={S0[a, al]:.10g}", flush=True)
            assert abs(fd - S0[a, al]) <= 3e-4 * smax
    finally:
        plan.close()


def test_reassembly_equals_a_fresh_plan():
    """Past reassemble_strain the proto-subdomains are rebuilt at the new cell:
    results equal those of a plan made at that cell."""
    cfg = _cfg("cell-re", H0, N0, R_ME=R_ME_FLUCT, seed_index=123)
    orbs, phi, orb_t, cen_t = _inputs(cfg)
    h1 = (np.eye(3) + 2.0 * STRAIN) @ H0
    C1 = orbs.centres @ np.linalg.inv(H0).T @ h1.T
    cen_t.copy_(torch.from_numpy(np.ascontiguousarray(C1)).to(cen_t.device))
    opt = dict(stencil_n=cfg.stencil_n, cg_tol=cfg.cg_tol, cell_fluctuation=1, reassemble_strain=0.01)
    plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, **opt)
    fresh = exx.Plan(h1, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, **opt)
    try:
        n_before = plan.geometry()["n_pe"]
        plan.set_cell(h1)
        E1, S1, D1, st1 = _eval(plan, orb_t, cen_t)
        E2, S2, D2, st2 = _eval(fresh, orb_t, cen_t)
        assert st1["reassemblies"] == 1 and st1["cell_strain"] == 0.0
        assert plan.geometry() == fresh.geometry() and plan.geometry()["n_pe"] != n_before
        assert E1 == E2 and np.array_equal(S1, S2)
        assert rel1(D1, D2) <= 1e-14
    finally:
        plan.close()
        fresh.close()
