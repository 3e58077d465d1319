"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the
same seeded inputs.  Bar for the plain FP64 path: relative 1-norm error
(eq. error_exx / error_sxx form) <= 1e-9 on E_xx and <= 1e-8 on D_xx and
sigma_xx; both sides solve to ||r|| <= 1e-12 ||b|| so that the CG stopping
point does not dominate the comparison.

Bar for the mixed path (FP32 CG, split-BF16 moments): |dE_xx| <= 1e-6 Ha per
molecule-equivalent (4 orbitals), sigma_xx and D_xx within 1e-6 relative.
The FP64 bars do not apply there: the moments carry the split-BF16 product
error (about 2^-17 relative per term)."""
import dataclasses

import numpy as np
import pytest

from paper_2011_07209_amd import synth

from gpu_util import gpu_eval, oracle_eval, rel1, subset_config

pytestmark = pytest.mark.gpu

TOL_E, TOL_D, TOL_S = 1e-9, 1e-8, 1e-8
MIXED_E_PER_MOLECULE, MIXED_D, MIXED_S = 1e-6, 1e-6, 1e-6


def _check_mixed(g, o, n_orb):
    dE = g["E"] - o["E"]
    print(f"  mixed: dE={dE:.3e} Ha ({dE / (n_orb / 4):.3e} per molecule-eq) "
          f"sigma rel={rel1(g['sigma'], o['sigma']):.3e} D rel={rel1(g['D'], o['D']):.3e}", flush=True)
    assert g["stats"]["n_unconverged"] == 0
    assert abs(dE) <= MIXED_E_PER_MOLECULE * n_orb / 4
    assert rel1(g["sigma"], o["sigma"]) <= MIXED_S
    assert rel1(g["D"], o["D"]) <= MIXED_D


def _compare(cfg, orbs, phi, want_D=True, **opt):
    g = gpu_eval(cfg, orbs, phi, want_D=want_D, **opt)
    o = oracle_eval(cfg, orbs, phi, want_D=want_D, **{k: v for k, v in opt.items()
                                                      if k in ("sample_seed", "sample_frac")})
    print(f"[{cfg.key}] pairs gpu={len(g['pairs']['E'])} oracle={len(o['pairs'])} E gpu={g['E']:.15g} "
          f"oracle={o['E']:.15g} iters max={g['stats']['cg_iter_max']}", flush=True)
    assert [tuple(x) for x in g["pairs"]["ij"]] == [(p.i, p.j) for p in o["pairs"]]
    assert g["stats"]["n_unconverged"] == 0
    assert rel1(g["E"], o["E"]) <= TOL_E, (g["E"], o["E"])
    assert rel1(g["sigma"], o["sigma"]) <= TOL_S, (g["sigma"], o["sigma"])
    if want_D:
        assert rel1(g["D"], o["D"]) <= TOL_D
    # per pair
    Eo = np.array([p.E for p in o["pairs"]])
    So = np.array([list(p.sigma) for p in o["pairs"]])
    scale = np.abs(Eo).max()
    assert np.abs(g["pairs"]["E"] - Eo).max() <= TOL_E * scale
    assert np.abs(g["pairs"]["sigma"] - So).max() <= TOL_S * np.abs(So).max()
    return g, o


def test_tiny16_fp64_parity():
    cfg = dataclasses.replace(synth.CONFIGS["tiny16"], cg_tol=1e-12)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    _compare(cfg, orbs, phi)


@pytest.mark.parametrize("n", [2, 3])
def test_small_cell_higher_order_stencils(n):
    cfg = synth.custom(key=f"small-n{n}", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46), n_orb=7, R_pair=7.0, R_PE=3.9,
                       R_ME=5.3, l_max=5, stencil_n=n, cg_tol=1e-12, seed_index=40 + n)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    _compare(cfg, orbs, phi)


def test_single_orbital_self_pair():
    cfg = synth.custom(key="single", grid=(48, 48, 48), n_orb=1, R_PE=4.0, R_ME=5.5, stencil_n=3, cg_tol=1e-12)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g, o = _compare(cfg, orbs, phi)
    assert len(o["pairs"]) == 1


def test_centres_on_cell_faces_and_corners():
    """Subdomains that wrap through the periodic boundary on every axis."""
    cfg = synth.custom(key="wrap", grid=(48, 48, 48), n_orb=4, R_PE=4.0, R_ME=5.5, stencil_n=3, cg_tol=1e-12)
    orbs = synth.make_orbitals(cfg)
    orbs = dataclasses.replace(orbs, centres=np.array([[0.01, 0.02, 11.99], [11.9, 0.3, 0.2],
                                                       [0.4, 11.7, 11.8], [6.0, 0.0, 6.0]]))
    phi = synth.fill_orbitals(cfg, orbs)
    _compare(cfg, orbs, phi)


def test_pair_sample_subset_matches():
    cfg = dataclasses.replace(synth.CONFIGS["tiny16"], cg_tol=1e-12)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g, o = _compare(cfg, orbs, phi, sample_seed=1234567, sample_frac=0.3)
    assert 0 < len(o["pairs"]) < 100


def test_variable_radius_classes():
    cfg = synth.custom(key="classes", grid=(48, 48, 48), n_orb=6, R_pair=7.0, R_PE=4.0, R_ME=5.5, stencil_n=2,
                       cg_tol=1e-12, R_PE_classes=(3.0, 0.5, 3), R_orb_range=(3.0, 4.0), seed_index=77)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g, o = _compare(cfg, orbs, phi)
    assert len({p.R_PE for p in o["pairs"]}) >= 2


def test_float32_orbitals_fp64_path():
    """FP32 orbital storage, FP64 arithmetic: parity against the oracle on the
    same (FP32-rounded) orbital values; D is accumulated in FP32."""
    cfg = dataclasses.replace(synth.CONFIGS["tiny16"], cg_tol=1e-12)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs).astype(np.float32).astype(np.float64)
    import torch
    g = gpu_eval(cfg, orbs, phi, dtype=torch.float32)
    o = oracle_eval(cfg, orbs, phi)
    assert rel1(g["E"], o["E"]) <= TOL_E
    assert rel1(g["sigma"], o["sigma"]) <= TOL_S
    assert rel1(g["D"], o["D"]) <= 1e-6   # FP32 storage of D


def test_repeat_is_bitwise_deterministic_for_E_and_sigma():
    cfg, orbs = subset_config("tiny16", 8)
    phi = synth.fill_orbitals(cfg, orbs)
    a = gpu_eval(cfg, orbs, phi, want_D=False)
    b = gpu_eval(cfg, orbs, phi, want_D=False)
    assert a["E"] == b["E"]
    assert np.array_equal(a["sigma"], b["sigma"])
    assert np.array_equal(a["pairs"]["iters"], b["pairs"]["iters"])


# ---------------------------------------------------------------------------
# mixed precision: FP32 CG with FP64 dots, reliable updates and FP64 stop test

@pytest.mark.parametrize("tol", [1e-10, 1e-12])
def test_mixed_precision_tiny16(tol):
    """Mixed path against the FP64 oracle, at two CG tolerances: the reliable
    updates and the FP64 true-residual stop reach either one."""
    cfg = dataclasses.replace(synth.CONFIGS["tiny16"], cg_tol=tol)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    from paper_2011_07209_amd import exx
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED)
    o = oracle_eval(cfg, orbs, phi)
    print(f"[mixed tol={tol}] E gpu={g['E']:.15g} oracle={o['E']:.15g} "
          f"iters max={g['stats']['cg_iter_max']} updates max={g['stats']['refine_passes_max']}", flush=True)
    assert g["stats"]["max_rel_residual"] <= tol
    _check_mixed(g, o, cfg.n_orb)


@pytest.mark.parametrize("n", [1, 3])
def test_mixed_precision_small_cell(n):
    cfg = synth.custom(key=f"mixed-n{n}", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46), n_orb=7, R_pair=7.0, R_PE=3.9,
                       R_ME=5.3, l_max=5, stencil_n=n, cg_tol=1e-12, seed_index=50 + n)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    from paper_2011_07209_amd import exx
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED)
    o = oracle_eval(cfg, orbs, phi)
    _check_mixed(g, o, cfg.n_orb)


def test_mixed_precision_far_pair_with_vanishing_density():
    """A pair whose density is ~1e-40 (below the FP32 normal range): the mixed
    solve works in units of ||b|| and the BF16 moments in units of the pair's
    power-of-two density scale, so it comes out like any other pair."""
    cfg = synth.custom(key="far", cell=(24.0, 24.0, 24.0), grid=(96, 96, 96), n_orb=2, R_pair=10.0, R_PE=4.0,
                       R_ME=5.0, l_max=4, stencil_n=3, cg_tol=1e-10)
    orbs = synth.OrbitalSet(np.array([[7.05, 12.0, 12.0], [16.95, 12.0, 12.0]]), np.array([2.2, 2.0]),
                            np.array([[0.1, 0.0, 0.2], [0.0, -0.2, 0.1]]))
    phi = synth.fill_orbitals(cfg, orbs)
    from paper_2011_07209_amd import exx
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED)
    o = oracle_eval(cfg, orbs, phi)
    assert len(o["pairs"]) == 3
    assert g["stats"]["n_unconverged"] == 0, g["pairs"]
    Eo = np.array([p.E for p in o["pairs"]])
    assert abs(Eo[1]) < 1e-60      # the cross pair is vanishingly small
    for k in range(3):
        assert abs(g["pairs"]["E"][k] - Eo[k]) <= 1e-7 * abs(Eo[k]), (k, g["pairs"]["E"][k], Eo[k])


@pytest.mark.parametrize("layout,threads,depth", [(1, 1024, 1), (1, 1024, 2), (1, 512, 1), (1, 512, 2),
                                                  (2, 1024, 1), (2, 1024, 2), (2, 768, 1), (2, 768, 2),
                                                  (2, 512, 1), (2, 512, 2)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_every_solve_variant(layout, threads, depth, prec):
    """Each CG variant the autotuner may pick (layout: single columns or runs
    of four, workgroup size x load depth, in both precisions; runs of four:
    one per thread with 768 and 1024 threads, two with 512, with fused
    sweeps in mixed plans of 512 and 768 threads) gives the oracle's
    result."""
    cfg = synth.custom(key=f"var-{layout}-{threads}-{depth}-{prec}", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46),
                       n_orb=5, R_pair=7.0, R_PE=3.9, R_ME=5.3, l_max=4, stencil_n=3, cg_tol=1e-12, seed_index=60)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    from paper_2011_07209_amd import exx
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64,
                 solve_threads=threads, solve_depth=depth, cg_layout=layout)
    o = oracle_eval(cfg, orbs, phi)
    print(f"[layout {layout} {threads}x{depth} {prec}] E gpu={g['E']:.15g} oracle={o['E']:.15g}", flush=True)
    assert g["stats"]["cg_layout"] == layout
    assert (g["stats"]["solve_threads"], g["stats"]["solve_depth"]) == (threads, depth)
    if prec == "mixed":
        _check_mixed(g, o, cfg.n_orb)
        return
    assert g["stats"]["n_unconverged"] == 0
    assert rel1(g["E"], o["E"]) <= TOL_E
    assert rel1(g["sigma"], o["sigma"]) <= TOL_S
    assert rel1(g["D"], o["D"]) <= TOL_D


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotuned_solve(prec):
    """With autotune on, the first evaluation times the CG variants on a sample
    of its pairs, keeps the fastest, and still returns the oracle's result."""
    cfg = dataclasses.replace(synth.CONFIGS["tiny16"], cg_tol=1e-12)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    from paper_2011_07209_amd import exx
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64,
                 autotune=1)
    o = oracle_eval(cfg, orbs, phi)
    assert g["stats"]["solve_threads"] in (512, 768, 1024) and g["stats"]["solve_depth"] in (1, 2)
    assert g["stats"]["tune_ms"] > 0
    if prec == "mixed":
        _check_mixed(g, o, cfg.n_orb)
        return
    assert rel1(g["E"], o["E"]) <= TOL_E
    assert rel1(g["sigma"], o["sigma"]) <= TOL_S
    assert rel1(g["D"], o["D"]) <= TOL_D


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_separate_self_radii(prec):
    """Self pairs on their own PE and ME spheres (R_PE_self, R_ME_self), one
    sphere class of their own, against the oracle with the same radii."""
    import oracle
    cfg = synth.custom(key=f"selfr-{prec}", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46), n_orb=7, R_pair=7.0,
                       R_PE=3.9, R_ME=5.3, l_max=5, stencil_n=3, cg_tol=1e-12, seed_index=81)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    from paper_2011_07209_amd import exx
    g = gpu_eval(cfg, orbs, phi, R_PE_self=3.3, R_ME_self=4.6,
                 precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64)
    P = oracle.make_params(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, cfg.stencil_n, cfg.cg_tol,
                           R_PE_self=3.3, R_ME_self=4.6)
    o = oracle.evaluate(P, phi, orbs.centres)
    assert g["stats"]["n_classes"] == 2
    assert [tuple(x) for x in g["pairs"]["ij"]] == [(p.i, p.j) for p in o["pairs"]]
    if prec == "mixed":
        _check_mixed(g, o, cfg.n_orb)
        return
    assert g["stats"]["n_unconverged"] == 0
    assert rel1(g["E"], o["E"]) <= TOL_E
    assert rel1(g["sigma"], o["sigma"]) <= TOL_S
    assert rel1(g["D"], o["D"]) <= TOL_D
    Eo = np.array([p.E for p in o["pairs"]])
    assert np.abs(g["pairs"]["E"] - Eo).sum() <= TOL_E * np.abs(Eo).sum()


@pytest.mark.parametrize("n", [1, 2])
def test_quad_layout_lower_order_stencils(n):
    """The quad layout with the n = 1 and n = 2 stencils (the run's x
    neighbours reach 1 or 2 points into the neighbour vectors), FP64 path."""
    from paper_2011_07209_amd import exx
    cfg = synth.custom(key=f"quad-n{n}", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46), n_orb=5, R_pair=7.0, R_PE=3.9,
                       R_ME=5.3, l_max=4, stencil_n=n, cg_tol=1e-12, seed_index=70 + n)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g, _ = _compare(cfg, orbs, phi, cg_layout=2)
    assert g["stats"]["cg_layout"] == 2


def test_quad_layout_variable_radius_classes():
    """Three sphere classes, each in its own padded run layout, mixed path."""
    from paper_2011_07209_amd import exx
    cfg = synth.custom(key="quad-classes", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46), n_orb=7, R_pair=7.0, R_PE=3.9,
                       R_ME=5.3, l_max=4, stencil_n=3, cg_tol=1e-12, seed_index=83, R_PE_classes=(3.0, 0.45, 3),
                       R_orb_range=(3.0, 3.9))
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED)
    o = oracle_eval(cfg, orbs, phi)
    assert g["stats"]["cg_layout"] == 2 and g["stats"]["n_classes"] >= 2
    assert [tuple(x) for x in g["pairs"]["ij"]] == [(p.i, p.j) for p in o["pairs"]]
    _check_mixed(g, o, cfg.n_orb)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_quad_layout_fused_sweeps(n):
    """Mixed quad layout in a 768-thread workgroup (the default where a sphere
    has at most 768 runs): pass B and the next pass A share one sweep, whose
    beta comes from |r - alpha Ap|^2 = |r|^2 - 2 alpha r.Ap + alpha^2 |Ap|^2.
    Same oracle result and nearly the same iteration count as the two passes
    of the 1024-thread kernel; the algorithmic bytes per iteration, which count
    six vector accesses per point for a fused sweep and eight for two passes,
    shrink by about a quarter."""
    from paper_2011_07209_amd import exx
    cfg = synth.custom(key=f"fused-n{n}", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46), n_orb=7, R_pair=7.0, R_PE=3.9,
                       R_ME=5.3, l_max=4, stencil_n=n, cg_tol=1e-12, seed_index=90 + n)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED)
    g2 = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED, solve_threads=1024)
    o = oracle_eval(cfg, orbs, phi)
    s, s2 = g["stats"], g2["stats"]
    print(f"[fused n={n}] iters {s['cg_iter_sum']} vs {s2['cg_iter_sum']} bytes/iter "
          f"{s['cg_alg_bytes'] / s['cg_iter_sum']:.4g} vs {s2['cg_alg_bytes'] / s2['cg_iter_sum']:.4g}", flush=True)
    assert s["cg_layout"] == 2 and s["solve_threads"] == 768
    assert s2["cg_layout"] == 2 and s2["solve_threads"] == 1024
    _check_mixed(g, o, cfg.n_orb)
    _check_mixed(g2, o, cfg.n_orb)
    assert abs(s["cg_iter_sum"] - s2["cg_iter_sum"]) <= 0.02 * s2["cg_iter_sum"] + s["n_pairs"]
    assert s["cg_alg_bytes"] / s["cg_iter_sum"] < 0.85 * s2["cg_alg_bytes"] / s2["cg_iter_sum"]


@pytest.mark.parametrize("threads", [0, 1024])
def test_mixed_quad_iteration_cap(threads):
    """With cg_max_iter below what the pairs need, the mixed quad-layout CG
    (768-thread fused sweeps by default, two passes at 1024 threads) stops
    every pair at the cap.  No fused sweep takes the last iteration, so the cap
    ends in a pass B and an FP64 true residual: every pair reports the cap,
    and the plan reports them unconverged (EXX_ENOCONV)."""
    import torch
    from paper_2011_07209_amd import exx
    cfg = synth.custom(key=f"cap-{threads}", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46), n_orb=5, R_pair=7.0,
                       R_PE=3.9, R_ME=5.3, l_max=4, stencil_n=3, cg_tol=1e-12, seed_index=97)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    dev = torch.device("cuda:0")
    cap = 30
    plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, stencil_n=cfg.stencil_n,
                    cg_tol=cfg.cg_tol, precision=exx.EXX_PREC_MIXED, cg_max_iter=cap, solve_threads=threads)
    try:
        orb_t = torch.from_numpy(phi).to(dev)
        cen_t = torch.from_numpy(orbs.centres).to(dev)
        plan.eval(orb_t, cen_t)
        torch.cuda.synchronize()
        with pytest.raises(exx.ExxError):
            plan.stats()
        st = plan.stats(allow_noconv=True)
        res = plan.pair_results()
    finally:
        plan.close()
    print(f"[cap {threads}] variant {st['solve_threads']} pairs {st['n_pairs']} unconverged {st['n_unconverged']} "
          f"iters max {st['cg_iter_max']} residual max {st['max_rel_residual']:.3e}", flush=True)
    assert st["cg_layout"] == 2 and st["solve_threads"] == (768 if threads == 0 else 1024)
    assert st["n_unconverged"] == st["n_pairs"] > 0
    assert st["n_cg_cap"] == st["n_pairs"] and st["n_cg_breakdown"] == 0 and st["n_cg_nonfinite"] == 0
    assert st["cg_restarts"] == 0
    assert st["cg_iter_max"] == cap and st["cg_iter_sum"] == cap * st["n_pairs"]
    assert np.all(np.asarray(res["iters"]) == cap)
    assert np.all(res["exit"] == exx.EXX_CG_CAP) and np.all(res["restarts"] == 0)
    assert st["max_rel_residual"] > cfg.cg_tol


def test_quad_layout_falls_back_for_wide_spheres():
    """A sphere of more than 1024 runs of four columns (R_PE 7.1 at spacing 0.2:
    3,969 columns in 1,044 runs): the default layout of a mixed plan falls back
    to single columns, and asking for runs is refused."""
    from paper_2011_07209_amd import exx
    h = np.diag([30.0, 30.0, 30.0])
    with pytest.raises(exx.ExxError):
        exx.Plan(h, (150, 150, 150), 6.0, 7.1, 8.5, 4, cg_layout=2, precision=exx.EXX_PREC_MIXED)
    cfg = synth.custom(key="quad-wide", cell=(30.0, 30.0, 30.0), grid=(150, 150, 150), n_orb=2, R_pair=6.0, R_PE=7.1,
                       R_ME=8.5, l_max=4, stencil_n=3, cg_tol=1e-10, seed_index=84)
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    g = gpu_eval(cfg, orbs, phi, want_D=False, precision=exx.EXX_PREC_MIXED)
    assert g["stats"]["cg_layout"] == 1
    assert g["stats"]["n_unconverged"] == 0


def test_layout_per_sphere_class():
    """Variable radii where the largest class (R_PE 7.1 at spacing 0.2: 1,044
    runs) does not fit the quad layout: that class keeps single columns, the
    others run quads (stats report both).  The mixed result meets the mixed
    bars against the FP64 path (single columns) on the same inputs."""
    from paper_2011_07209_amd import exx
    cfg = synth.custom(key="layout-classes", cell=(30.0, 30.0, 30.0), grid=(150, 150, 150), n_orb=6, R_pair=8.0,
                       R_PE=6.0, R_ME=9.0, l_max=4, stencil_n=3, cg_tol=1e-10, seed_index=85,
                       R_PE_classes=(5.0, 1.05, 3), R_orb_range=(5.0, 7.1))
    orbs = synth.make_orbitals(cfg)
    phi = synth.fill_orbitals(cfg, orbs)
    m = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_MIXED)
    f = gpu_eval(cfg, orbs, phi, precision=exx.EXX_PREC_FP64)
    radii = sorted({round(r, 6) for r in m["pairs"]["R_PE"]}) if "R_PE" in m["pairs"] else None
    print(f"[layout classes] layout={m['stats']['cg_layout']} classes={m['stats']['n_classes']} radii={radii} "
          f"E mixed={m['E']:.12f} fp64={f['E']:.12f}", flush=True)
    assert m["stats"]["cg_layout"] == 3 and f["stats"]["cg_layout"] == 1
    assert [tuple(x) for x in m["pairs"]["ij"]] == [tuple(x) for x in f["pairs"]["ij"]]
    assert m["stats"]["n_unconverged"] == 0 and f["stats"]["n_unconverged"] == 0
    assert abs(m["E"] - f["E"]) <= MIXED_E_PER_MOLECULE * cfg.n_orb / 4
    assert rel1(m["sigma"], f["sigma"]) <= MIXED_S
    assert rel1(m["D"], f["D"]) <= MIXED_D
