"""Parity at the full sizes of the water-like workloads (64, 128, 256 and 512
molecules), on outputs the oracle can compute one by one:

* per-pair E_xx and sigma_xx of sampled pairs, the oracle given only the two
  orbitals of the pair (copied back from the device, so it sees the exact
  inputs the kernels read);
* D_xx of one orbital, against the oracle run on that orbital and every
  orbital within R_pair of it (which holds all of its pairs);
* the virial identity over the whole set, and mixed against FP64 within the
  mixed-precision targets.

The 64-molecule set runs every pair in the launch configuration the benchmark
times.  The 256- and 512-molecule sets run a deterministic pair subset (the
same SplitMix64 rule on the device as in the oracle), the 256-molecule one as
graph replays over displaced centres, the 512-molecule one with FP32 orbitals
(113 GB) and l_max 8."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2011_07209_amd import exx, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = torch.device("cuda:0")
TOL_E, TOL_S, TOL_D = 1e-9, 1e-8, 1e-8


def _plan(cfg, **kw):
    opt = dict(stencil_n=cfg.stencil_n, cg_tol=cfg.cg_tol, workspace_gb=48.0)
    if cfg.R_PE_classes is not None:
        opt.update(R_PE_min=cfg.R_PE_classes[0], R_PE_step=cfg.R_PE_classes[1], R_PE_nclass=cfg.R_PE_classes[2])
    opt.update(kw)
    return exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, **opt)


def _oracle_params(cfg, **kw):
    return oracle.make_params(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, cfg.stencil_n, cfg.cg_tol,
                              R_PE_classes=cfg.R_PE_classes, **kw)


def _check_pairs(tag, cfg, orbs, orb_t, pr, picks):
    """Per-pair E and sigma of the picked rows of pair_results against the oracle."""
    P = _oracle_params(cfg)
    for k in picks:
        i, j = (int(x) for x in pr["ij"][k])
        idx = [i] if i == j else [i, j]
        phi2 = orb_t[idx].to(torch.float64).cpu().numpy()
        cen = orbs.centres[idx]
        R2 = None if orbs.R_orb is None or cfg.R_PE_classes is None else orbs.R_orb[idx]
        f = oracle.pair_fields(P, phi2, cen, 0, len(idx) - 1, R2)
        r = f["res"]
        print(f"[{tag}] pair ({i},{j}) gpu E={pr['E'][k]:.15g} oracle={r.E:.15g} iters {pr['iters'][k]}/{r.cg_iters}",
              flush=True)
        # both sides stop at ||r|| <= 1e-10 ||b||: the solution error is bounded by kappa * 1e-10
        assert abs(pr["E"][k] - r.E) <= TOL_E * abs(r.E) + 1e-14
        s_o = np.array(list(r.sigma))
        assert np.abs(pr["sigma"][k] - s_o).sum() <= TOL_S * np.abs(s_o).sum() + 1e-14


def _picks(pr, n, seed):
    rng = np.random.default_rng(seed)
    m = len(pr["E"])
    self_idx = [k for k in range(m) if pr["ij"][k, 0] == pr["ij"][k, 1]]
    return sorted(set(rng.choice(m, n, replace=False).tolist() + [self_idx[len(self_idx) // 2]]))


def _neighbourhood(cfg, orbs, i):
    L = np.asarray(cfg.cell)
    d = orbs.centres - orbs.centres[i]
    d -= L * np.round(d / L)
    return [i] + [j for j in np.flatnonzero((d * d).sum(1) <= cfg.R_pair ** 2 * (1 + 1e-12)).tolist() if j != i]


# ---------------------------------------------------------------------------
# 64 molecules: every pair, as the benchmark runs it

@pytest.fixture(scope="module")
def water64_run():
    cfg = synth.CONFIGS["water64"]
    orbs = synth.make_orbitals(cfg)
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    plan = _plan(cfg)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    S = torch.zeros(9, dtype=torch.float64, device=DEV)
    D = torch.empty_like(orb_t)
    plan.eval(orb_t, cen_t, E, D, S)
    torch.cuda.synchronize()
    pr = plan.pair_results()
    st = plan.stats()
    plan.close()
    print(f"[water64] pairs={st['n_pairs']} E={E.item():.12f} iters mean={st['cg_iter_sum'] / st['n_pairs']:.1f}",
          flush=True)
    yield cfg, orbs, orb_t, D, E.item(), S.cpu().numpy().reshape(3, 3, order="F"), pr, st
    del orb_t, D
    torch.cuda.empty_cache()


def test_water64_sampled_pairs_match_oracle(water64_run):
    cfg, orbs, orb_t, D, E, S, pr, st = water64_run
    assert st["n_unconverged"] == 0
    _check_pairs("water64", cfg, orbs, orb_t, pr, _picks(pr, 6, 64))


def test_water64_mixed_sampled_pairs_match_oracle():
    """The headline configuration as the benchmark runs it (mixed precision,
    autotuned CG variant, quad layout): sampled pairs against the oracle, per
    pair within the mixed bar (1e-6 relative on E_xx and sigma_xx)."""
    cfg = synth.CONFIGS["water64"]
    orbs = synth.make_orbitals(cfg)
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    plan = _plan(cfg, autotune=1, precision=exx.EXX_PREC_MIXED)
    try:
        E = torch.zeros(1, dtype=torch.float64, device=DEV)
        S = torch.zeros(9, dtype=torch.float64, device=DEV)
        plan.eval(orb_t, cen_t, E, None, S)
        torch.cuda.synchronize()
        pr = plan.pair_results()
        st = plan.stats()
    finally:
        plan.close()
    print(f"[water64 mixed] pairs={st['n_pairs']} layout={st['cg_layout']} variant={st['solve_threads']}x"
          f"{st['solve_depth']} E={E.item():.12f}", flush=True)
    assert st["n_unconverged"] == 0 and st["cg_layout"] == 2
    P = _oracle_params(cfg)
    for k in _picks(pr, 3, 65):
        i, j = (int(x) for x in pr["ij"][k])
        idx = [i] if i == j else [i, j]
        f = oracle.pair_fields(P, orb_t[idx].to(torch.float64).cpu().numpy(), orbs.centres[idx], 0, len(idx) - 1)
        r = f["res"]
        s_o = np.array(list(r.sigma))
        print(f"[water64 mixed] pair ({i},{j}) gpu E={pr['E'][k]:.15g} oracle={r.E:.15g}", flush=True)
        assert abs(pr["E"][k] - r.E) <= 1e-6 * abs(r.E) + 1e-14
        assert np.abs(pr["sigma"][k] - s_o).sum() <= 1e-6 * np.abs(s_o).sum() + 1e-14
    del orb_t
    torch.cuda.empty_cache()


def test_water64_D_of_one_orbital_matches_oracle(water64_run):
    cfg, orbs, orb_t, D, E, S, pr, st = water64_run
    i = 37
    nb = _neighbourhood(cfg, orbs, i)
    phi = orb_t[nb].cpu().numpy()
    o = oracle.evaluate(_oracle_params(cfg), phi, orbs.centres[nb], want_D=True)
    Dg = D[i].cpu().numpy()
    err = np.abs(Dg - o["D"][0]).sum() / np.abs(o["D"][0]).sum()
    print(f"[water64] D of orbital {i} ({len(nb)} orbitals, {len(o['pairs'])} pairs in the oracle run): rel {err:.3e}",
          flush=True)
    assert err <= TOL_D


def test_water64_virial_and_symmetry(water64_run):
    cfg, orbs, orb_t, D, E, S, pr, st = water64_run
    assert E < 0
    assert abs(np.sum(S * cfg.h) / -E - 1) < 2e-3   # continuum identity, discretization-level gap
    assert np.abs(S - S.T).max() <= 1e-3 * np.abs(S).max()
    assert abs(E - pr["E"].sum()) <= 1e-12 * abs(E)


# ---------------------------------------------------------------------------
# 128 molecules: every pair, FP64 and mixed

def test_water128_fp64_pairs_and_mixed_targets():
    cfg = synth.CONFIGS["water128"]
    orbs = synth.make_orbitals(cfg)
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    res = {}
    for prec in ("fp64", "mixed"):
        plan = _plan(cfg, precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64)
        E = torch.zeros(1, dtype=torch.float64, device=DEV)
        S = torch.zeros(9, dtype=torch.float64, device=DEV)
        D = torch.empty((4,) + tuple(orb_t.shape[1:]), dtype=torch.float64, device=DEV)
        sub = torch.tensor([0, 101, 202, 303], dtype=torch.int32, device=DEV)
        plan.eval(orb_t, cen_t, E, D, S, d_subset=sub)
        torch.cuda.synchronize()
        st = plan.stats()
        res[prec] = (E.item(), S.cpu().numpy(), D.cpu().numpy(), plan.pair_results(), st)
        plan.close()
        print(f"[water128] {prec}: pairs={st['n_pairs']} E={E.item():.12f} "
              f"iters mean={st['cg_iter_sum'] / st['n_pairs']:.1f}", flush=True)
        assert st["n_unconverged"] == 0
    _check_pairs("water128", cfg, orbs, orb_t, res["fp64"][3], _picks(res["fp64"][3], 3, 128))
    (Ea, Sa, Da, _, _), (Eb, Sb, Db, _, _) = res["mixed"], res["fp64"]
    n_mol = cfg.n_orb / 4
    print(f"[water128] mixed - fp64: dE/molecule={(Ea - Eb) / n_mol:.3e} "
          f"sigma rel={np.abs(Sa - Sb).sum() / np.abs(Sb).sum():.3e} D rel={np.abs(Da - Db).sum() / np.abs(Db).sum():.3e}",
          flush=True)
    assert abs(Ea - Eb) <= 1e-6 * n_mol
    assert np.abs(Sa - Sb).sum() <= 1e-6 * np.abs(Sb).sum()
    assert np.abs(Da - Db).sum() <= 1e-6 * np.abs(Db).sum()
    del orb_t
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# 256 molecules: variable sphere radii, graph replays over displaced centres

def test_water256_graph_replays_over_displaced_centres():
    cfg = synth.CONFIGS["water256"]
    frac = 1.0 / 32
    orbs = synth.make_orbitals(cfg)
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    R_t = torch.from_numpy(orbs.R_orb).to(DEV)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    S = torch.zeros(9, dtype=torch.float64, device=DEV)
    plan = _plan(cfg, max_pairs=4096, pair_sample_seed=2011072094, pair_sample_frac=frac, autotune=1)
    try:
        plan.eval(orb_t, cen_t, E, None, S, R_t)
        torch.cuda.synchronize()
        st = plan.stats()
        print(f"[water256] eager: pairs={st['n_pairs']} classes={st['n_classes']} E={E.item():.12f}", flush=True)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            plan.set_stream(side)
            with torch.cuda.graph(g, stream=side):
                plan.eval(orb_t, cen_t, E, None, S, R_t)
        torch.cuda.current_stream().wait_stream(side)
        plan.set_stream(torch.cuda.current_stream())
        for step in (1, 2):
            orbs = synth.displace(cfg, orbs, step)
            synth.fill_orbitals_device(cfg, orbs, DEV, out=orb_t)
            cen_t.copy_(torch.from_numpy(orbs.centres).to(DEV))
            g.replay()
            torch.cuda.synchronize()
            st = plan.stats()
            pr = plan.pair_results()
            print(f"[water256] replay {step}: pairs={st['n_pairs']} E={E.item():.12f}", flush=True)
            assert st["graph_recorded"] == 1 and st["n_unconverged"] == 0
            # the subset rule and the pair list of the displaced centres, from the oracle
            ol = oracle.pair_list(_oracle_params(cfg, sample_seed=2011072094, sample_frac=frac), orbs.centres,
                                  orbs.R_orb)
            assert [tuple(x) for x in pr["ij"]] == [(p.i, p.j) for p in ol]
            assert abs(E.item() - pr["E"].sum()) <= 1e-12 * abs(E.item())
        _check_pairs("water256", cfg, orbs, orb_t, pr, _picks(pr, 3, 256))
        del g
    finally:
        plan.close()
    del orb_t
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# 512 molecules: FP32 orbitals (113 GB), l_max 8, pair subset

def test_water512_fp32_orbitals_lmax8_subset():
    cfg = synth.CONFIGS["water512"]
    frac = 1.0 / 32
    orbs = synth.make_orbitals(cfg)
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)   # float32
    assert orb_t.dtype == torch.float32
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    print(f"[water512] orbitals on the device: {orb_t.numel() * 4 / 1e9:.1f} GB", flush=True)
    res = {}
    sub = torch.tensor([7, 1500], dtype=torch.int32, device=DEV)
    for prec in ("fp64", "mixed"):
        plan = _plan(cfg, precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64,
                     pair_sample_seed=2011072095, pair_sample_frac=frac)
        E = torch.zeros(1, dtype=torch.float64, device=DEV)
        S = torch.zeros(9, dtype=torch.float64, device=DEV)
        D = torch.empty((2,) + tuple(orb_t.shape[1:]), dtype=torch.float32, device=DEV)
        plan.eval(orb_t, cen_t, E, D, S, d_subset=sub)
        torch.cuda.synchronize()
        st = plan.stats()
        res[prec] = (E.item(), S.cpu().numpy(), D.double().cpu().numpy(), plan.pair_results(), st)
        plan.close()
        print(f"[water512] {prec}: pairs={st['n_pairs']} E={E.item():.12f} "
              f"iters mean={st['cg_iter_sum'] / st['n_pairs']:.1f}", flush=True)
        assert st["n_unconverged"] == 0
    _check_pairs("water512", cfg, orbs, orb_t, res["fp64"][3], _picks(res["fp64"][3], 3, 512))
    (Ea, Sa, Da, _, _), (Eb, Sb, Db, _, _) = res["mixed"], res["fp64"]
    n_mol = cfg.n_orb / 4 * frac   # molecule-equivalents the sampled pairs stand for
    print(f"[water512] mixed - fp64 on the subset: dE={Ea - Eb:.3e} Ha "
          f"sigma rel={np.abs(Sa - Sb).sum() / np.abs(Sb).sum():.3e} D rel={np.abs(Da - Db).sum() / np.abs(Db).sum():.3e}",
          flush=True)
    assert abs(Ea - Eb) <= 1e-6 * n_mol
    assert np.abs(Sa - Sb).sum() <= 1e-6 * np.abs(Sb).sum()
    # D is stored in FP32 in both paths: compare at FP32 storage resolution
    assert np.abs(Da - Db).sum() <= 1e-5 * np.abs(Db).sum()
    del orb_t
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# general cells (hexagonal, triclinic): every pair, autotuned as the benchmark
# runs them, FP64 against the oracle on sampled pairs and mixed against FP64

@pytest.mark.parametrize("key", ["hex64", "tri64"])
def test_general_cell_full_size(key):
    cfg = synth.CONFIGS[key]
    orbs = synth.make_orbitals(cfg)
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    sub = torch.tensor([0, 63, 128, 255], dtype=torch.int32, device=DEV)
    res = {}
    for prec in ("fp64", "mixed"):
        plan = _plan(cfg, autotune=1, precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64)
        E = torch.zeros(1, dtype=torch.float64, device=DEV)
        S = torch.zeros(9, dtype=torch.float64, device=DEV)
        D = torch.empty((4,) + tuple(orb_t.shape[1:]), dtype=torch.float64, device=DEV)
        plan.eval(orb_t, cen_t, E, D, S, d_subset=sub)
        torch.cuda.synchronize()
        st = plan.stats()
        res[prec] = (E.item(), S.cpu().numpy().reshape(3, 3, order="F"), D.cpu().numpy(), plan.pair_results(), st)
        plan.close()
        print(f"[{key}] {prec}: pairs={st['n_pairs']} arms={st['n_arms']} E={E.item():.12f} "
              f"iters mean={st['cg_iter_sum'] / st['n_pairs']:.1f} variant={st['solve_threads']}x{st['solve_depth']}",
              flush=True)
        assert st["n_unconverged"] == 0
    E, S, _, pr, st = res["fp64"]
    # the pair list (minimum image and R_pair in the general cell) is the oracle's
    ora = oracle.pair_list(_oracle_params(cfg), orbs.centres)
    assert [tuple(int(x) for x in ij) for ij in pr["ij"]] == [(p.i, p.j) for p in ora]
    assert st["n_arms"] == (4 if key == "hex64" else 6)
    # random pairs (mostly far apart), a self pair, and the two strongest
    # non-self pairs
    off = [k for k in range(len(pr["E"])) if pr["ij"][k, 0] != pr["ij"][k, 1]]
    strong = sorted(off, key=lambda k: abs(pr["E"][k]), reverse=True)[:2]
    _check_pairs(key, cfg, orbs, orb_t, pr, sorted(set(_picks(pr, 3, 64 + len(key)) + strong)))
    assert abs(np.sum(S * cfg.h) / -E - 1) < 2e-3   # virial identity, discretization-level gap
    # rotational invariance of E makes sigma h^T, i.e. the stress of eq.
    # pixx_working, symmetric (sigma itself is not, in a non-orthogonal cell)
    Pi, _ = exx.exx_pressure(cfg.h, S)
    assert np.abs(Pi - Pi.T).max() <= 1e-3 * np.abs(Pi).max()
    (Ea, Sa, Da, _, _), (Eb, Sb, Db, _, _) = res["mixed"], res["fp64"]
    n_mol = cfg.n_orb / 4
    print(f"[{key}] mixed - fp64: dE/molecule={(Ea - Eb) / n_mol:.3e} "
          f"sigma rel={np.abs(Sa - Sb).sum() / np.abs(Sb).sum():.3e} D rel={np.abs(Da - Db).sum() / np.abs(Db).sum():.3e}",
          flush=True)
    assert abs(Ea - Eb) <= 1e-6 * n_mol
    assert np.abs(Sa - Sb).sum() <= 1e-6 * np.abs(Sb).sum()
    assert np.abs(Da - Db).sum() <= 1e-6 * np.abs(Db).sum()
