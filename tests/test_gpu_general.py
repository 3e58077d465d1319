"""General (non-orthogonal) cells on the GPU (Sec. III B 1, Sec. III C 1-2):
the HIP path through the C ABI against the FP64 oracle on the same seeded
inputs, with the bars of the orthorhombic parity tests (FP64: relative 1-norm
error <= 1e-9 on E_xx, <= 1e-8 on D_xx and sigma_xx; mixed: 1e-6 Ha per
molecule-equivalent on E_xx, 1e-6 relative on sigma_xx and D_xx).

The cells cover the three stencil families of the paper's lattice-symmetry
study: one auxiliary direction inside the sweep plane (hexagonal), one that
needs a permuted sweep axis (monoclinic, unique axis b), arms that leave the
sweep plane with padded columns (triclinic, rhombohedral)."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2011_07209_amd import exx, synth

from gpu_util import gpu_eval, oracle_eval, rel1
from test_gpu_parity import MIXED_D, MIXED_E_PER_MOLECULE, MIXED_S, TOL_D, TOL_E, TOL_S, _check_mixed, _compare

pytestmark = pytest.mark.gpu


def _cell(a, b, c, al, be, ga):
    al, be, ga = np.radians([al, be, ga])
    L1 = np.array([a, 0.0, 0.0])
    L2 = np.array([b * np.cos(ga), b * np.sin(ga), 0.0])
    cx = c * np.cos(be)
    cy = c * (np.cos(al) - np.cos(be) * np.cos(ga)) / np.sin(ga)
    return np.column_stack([L1, L2, [cx, cy, np.sqrt(c * c - cx * cx - cy * cy)]])


def _cfg(key, h, grid, **kw):
    base = dict(n_orb=7, R_pair=7.0, R_PE=4.0, R_ME=5.2, l_max=5, stencil_n=3, cg_tol=1e-12, seed_index=60)
    base.update(kw)
    return synth.custom(key=key, cell=tuple(np.linalg.norm(h, axis=0)), grid=grid,
                        hmat=tuple(np.asarray(h).flatten("F")), **base)


CELLS = {
    "hexagonal": (_cell(12.0, 12.0, 12.0, 90, 90, 120), (48, 48, 48)),
    "monoclinic": (_cell(12.0, 12.0, 12.0, 90, 105, 90), (48, 48, 48)),
    "triclinic": (_cell(12.0, 12.5, 11.5, 80, 95, 100), (48, 50, 46)),
    "rhombohedral": (_cell(12.0, 12.0, 12.0, 113, 113, 113), (48, 48, 48)),
}


@pytest.mark.parametrize("name", sorted(CELLS))
def test_general_cell_fp64_parity(name):
    h, N = CELLS[name]
    cfg = _cfg(f"gen-{name}", h, N, seed_index=61 + sorted(CELLS).index(name))
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    print(f"[{name}] arms {exx.exx_nk_stencil(h, N)['u'].tolist()}", flush=True)
    _compare(cfg, orbs, phi)


def _tri_big():
    h, N = _cell(12.0, 12.5, 11.5, 80, 95, 100), (60, 62, 58)
    return _cfg("gen-tri-big", h, N, n_orb=5, R_PE=5.0, R_ME=6.3, seed_index=70)


_ORACLE_CACHE = {}


def _oracle_cached(cfg, orbs, phi):
    if cfg.key not in _ORACLE_CACHE:
        _ORACLE_CACHE[cfg.key] = oracle_eval(cfg, orbs, phi)
    return _ORACLE_CACHE[cfg.key]


@pytest.mark.parametrize("threads", [512, 1024])
def test_general_cell_cg_variants(threads):
    """Both workgroup sizes on spheres of ~2000 columns (several columns per
    thread), triclinic cell with three arms leaving the sweep plane."""
    cfg = _tri_big()
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g = gpu_eval(cfg, orbs, phi, solve_threads=threads)
    o = _oracle_cached(cfg, orbs, phi)
    print(f"[tri-big {threads}] E gpu={g['E']:.15g} oracle={o['E']:.15g} iters max={g['stats']['cg_iter_max']} "
          f"threads={g['stats']['solve_threads']}", flush=True)
    assert g["stats"]["solve_threads"] == threads
    assert [tuple(x) for x in g["pairs"]["ij"]] == [(p.i, p.j) for p in o["pairs"]]
    assert g["stats"]["n_unconverged"] == 0
    assert rel1(g["E"], o["E"]) <= TOL_E
    assert rel1(g["sigma"], o["sigma"]) <= TOL_S
    assert rel1(g["D"], o["D"]) <= TOL_D


@pytest.mark.parametrize("threads", [512, 1024])
def test_general_cell_cg_variants_mixed(threads):
    """Mixed precision on the same spheres (four columns per thread with 512
    threads, two with 1024).  The tilted-arm CG runs fused sweeps (pass B with
    the next pass A, Ap kept in a vector between them) wherever the next
    residual norm is clear of the update and stop thresholds."""
    cfg = _tri_big()
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g = gpu_eval(cfg, orbs, phi, solve_threads=threads, precision=exx.EXX_PREC_MIXED)
    o = _oracle_cached(cfg, orbs, phi)
    print(f"[tri-big mixed {threads}] E gpu={g['E']:.15g} oracle={o['E']:.15g} iters max={g['stats']['cg_iter_max']}",
          flush=True)
    assert g["stats"]["solve_threads"] == threads
    assert [tuple(x) for x in g["pairs"]["ij"]] == [(p.i, p.j) for p in o["pairs"]]
    _check_mixed(g, o, cfg.n_orb)
    # every pair converged to the FP64 criterion: its E within the mixed bound
    # of the oracle's
    Eo = np.array([p.E for p in o["pairs"]])
    assert np.abs(g["pairs"]["E"] - Eo).max() <= 1e-6 * np.abs(Eo).max()


@pytest.mark.parametrize("n", [1, 2, 3])
def test_general_cell_fused_tilted_sweeps_per_stencil_order(n):
    """The fused tilted-arm sweeps (mixed, 512 and 1024 threads) for each
    stencil order."""
    h, N = CELLS["triclinic"]
    cfg = _cfg(f"gen-tri-fused-n{n}", h, N, stencil_n=n, R_ME=4.9 if n < 3 else 6.3, seed_index=84 + n)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    o = oracle_eval(cfg, orbs, phi)
    for threads in (512, 1024):
        g = gpu_eval(cfg, orbs, phi, solve_threads=threads, precision=exx.EXX_PREC_MIXED)
        assert g["stats"]["solve_threads"] == threads
        assert [tuple(x) for x in g["pairs"]["ij"]] == [(p.i, p.j) for p in o["pairs"]]
        _check_mixed(g, o, cfg.n_orb)


@pytest.mark.parametrize("name", ["triclinic", "monoclinic"])
def test_general_cell_mixed_precision(name):
    h, N = CELLS[name]
    cfg = _cfg(f"gen-mixed-{name}", h, N, seed_index=75)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED)
    o = oracle_eval(cfg, orbs, phi)
    assert [tuple(x) for x in g["pairs"]["ij"]] == [(p.i, p.j) for p in o["pairs"]]
    _check_mixed(g, o, cfg.n_orb)


@pytest.mark.parametrize("n", [1, 2])
def test_general_cell_lower_order_stencils(n):
    h, N = CELLS["triclinic"]
    cfg = _cfg(f"gen-tri-n{n}", h, N, stencil_n=n, R_ME=4.9, seed_index=80 + n)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    _compare(cfg, orbs, phi)


def test_sheared_cubic_general_path_matches_orthorhombic_path():
    """The same lattice described by h0 (orthorhombic kernels) and by h0 M (M
    unimodular: the general kernels, with the NK construction recovering the
    cubic axes) gives the same E_xx and D_xx on the GPU, to rounding."""
    N = 48
    h0 = np.diag([12.0, 12.0, 12.0])
    M = np.array([[1, 1, 0], [0, 1, 0], [0, 0, 1]])
    cfg0 = synth.custom(key="cubic", grid=(N, N, N), n_orb=6, R_pair=7.0, R_PE=4.0, R_ME=5.2, l_max=5, cg_tol=1e-12,
                        seed_index=90)
    orbs = synth.make_orbitals(cfg0)
    phi0 = synth.fill_orbitals(cfg0, orbs)
    n1, n2 = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    src = (n1 + n2) % N
    phi1 = np.ascontiguousarray(phi0[:, :, n2, src])
    cfg1 = _cfg("sheared", h0 @ M, (N, N, N), n_orb=6, seed_index=90)
    g0 = gpu_eval(cfg0, orbs, phi0)
    g1 = gpu_eval(cfg1, orbs, phi1)
    print(f"[sheared] E cubic={g0['E']:.15g} sheared={g1['E']:.15g}", flush=True)
    assert [tuple(x) for x in g0["pairs"]["ij"]] == [tuple(x) for x in g1["pairs"]["ij"]]
    assert rel1(g1["E"], g0["E"]) <= 1e-11
    assert rel1(g1["D"], np.ascontiguousarray(g0["D"][:, :, n2, src])) <= 1e-9
    # sigma' = sigma M^-T: rows x and z use the same first-derivative stencils
    want = g0["sigma"] @ np.linalg.inv(M).T
    np.testing.assert_allclose(g1["sigma"][[0, 2]], want[[0, 2]], rtol=0, atol=1e-10 * np.abs(want).max())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_general_cell_warm_start_over_displaced_steps(prec):
    """Warm starts in the triclinic cell; mixed: the fused tilted-arm sweeps
    from a warm-started residual."""
    h, N = CELLS["triclinic"]
    cfg = _cfg("gen-warm", h, N, seed_index=95)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    dev = torch.device("cuda:0")
    orb_t = torch.from_numpy(phi).to(dev)
    cen_t = torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    S = torch.zeros(9, dtype=torch.float64, device=dev)
    D = torch.empty_like(orb_t)
    plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, stencil_n=cfg.stencil_n,
                    cg_tol=cfg.cg_tol, max_pairs=64, warm_start=1,
                    precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64)
    # FP64: the parity bars; mixed: 1e-6 Ha per molecule-equivalent in E, 1e-6 relative in sigma and D
    tol_S, tol_D = (TOL_S, TOL_D) if prec == "fp64" else (MIXED_S, MIXED_D)
    try:
        iters = []
        for step in range(2):
            if step:
                orbs = synth.displace(cfg, orbs, step, amplitude=0.05)
                phi = synth.fill_orbitals(cfg, orbs)
                orb_t.copy_(torch.from_numpy(phi).to(dev))
                cen_t.copy_(torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev))
            plan.eval(orb_t, cen_t, E, D, S)
            torch.cuda.synchronize()
            st = plan.stats()
            o = oracle_eval(cfg, orbs, phi)
            iters.append(st["cg_iter_sum"])
            print(f"[gen warm {prec}] step {step}: warm {st['warm_pairs']}/{st['n_pairs']} iters "
                  f"{st['cg_iter_sum']} E rel {rel1(E.item(), o['E']):.2e}", flush=True)
            assert st["n_unconverged"] == 0
            assert (st["warm_pairs"] == 0) if step == 0 else (st["warm_pairs"] >= 0.75 * st["n_pairs"])
            if prec == "fp64":
                assert rel1(E.item(), o["E"]) <= TOL_E
            else:
                assert abs(E.item() - o["E"]) <= MIXED_E_PER_MOLECULE * cfg.n_orb / 4
            assert rel1(S.cpu().numpy().reshape(3, 3, order="F"), o["sigma"]) <= tol_S
            assert rel1(D.cpu().numpy(), o["D"]) <= tol_D
        assert iters[1] < iters[0]
    finally:
        plan.close()


@pytest.mark.parametrize("name", ["hexagonal", "monoclinic"])
def test_general_cell_quad_layout(name):
    """Cells whose one auxiliary direction is a diagonal of the sweep plane and
    whose columns need no padding run the quad layout (runs of four columns,
    the diagonal arm read from the neighbouring runs' vectors): mixed by
    default, FP64 when asked, both against the oracle."""
    h, N = CELLS[name]
    cfg = _cfg(f"gen-quad-{name}", h, N, seed_index=77)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    o = oracle_eval(cfg, orbs, phi)
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED)
    print(f"[quad {name}] layout {g['stats']['cg_layout']} E gpu={g['E']:.15g} oracle={o['E']:.15g}", flush=True)
    assert g["stats"]["cg_layout"] == 2
    assert [tuple(x) for x in g["pairs"]["ij"]] == [(p.i, p.j) for p in o["pairs"]]
    _check_mixed(g, o, cfg.n_orb)
    f = gpu_eval(cfg, orbs, phi, cg_layout=2)
    assert f["stats"]["cg_layout"] == 2 and f["stats"]["n_unconverged"] == 0
    assert rel1(f["E"], o["E"]) <= TOL_E
    assert rel1(f["sigma"], o["sigma"]) <= TOL_S
    assert rel1(f["D"], o["D"]) <= TOL_D


def test_quad_layout_warm_start_over_displaced_steps():
    """Warm start on a general cell in the quad layout (hexagonal, mixed): the
    previous solution is moved through the 3D slot map, dead slots start at
    zero, and each step meets the mixed bars against the oracle."""
    h, N = CELLS["hexagonal"]
    cfg = _cfg("gen-quad-warm", h, N, seed_index=96)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    dev = torch.device("cuda:0")
    orb_t = torch.from_numpy(phi).to(dev)
    cen_t = torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    S = torch.zeros(9, dtype=torch.float64, device=dev)
    D = torch.empty_like(orb_t)
    plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, stencil_n=cfg.stencil_n,
                    cg_tol=cfg.cg_tol, max_pairs=64, warm_start=1, precision=exx.EXX_PREC_MIXED)
    try:
        iters = []
        for step in range(2):
            if step:
                orbs = synth.displace(cfg, orbs, step, amplitude=0.05)
                phi = synth.fill_orbitals(cfg, orbs)
                orb_t.copy_(torch.from_numpy(phi).to(dev))
                cen_t.copy_(torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev))
            plan.eval(orb_t, cen_t, E, D, S)
            torch.cuda.synchronize()
            st = plan.stats()
            o = oracle_eval(cfg, orbs, phi)
            iters.append(st["cg_iter_sum"])
            print(f"[quad warm] step {step}: layout {st['cg_layout']} warm {st['warm_pairs']}/{st['n_pairs']} "
                  f"iters {st['cg_iter_sum']}", flush=True)
            assert st["cg_layout"] == 2 and st["n_unconverged"] == 0
            assert (st["warm_pairs"] == 0) if step == 0 else (st["warm_pairs"] >= 0.75 * st["n_pairs"])
            assert abs(E.item() - o["E"]) <= 1e-6 * cfg.n_orb / 4
            assert rel1(S.cpu().numpy().reshape(3, 3, order="F"), o["sigma"]) <= 1e-6
            assert rel1(D.cpu().numpy(), o["D"]) <= 1e-6
        assert iters[1] < iters[0]
    finally:
        plan.close()
