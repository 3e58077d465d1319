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
from concurrent.futures import ThreadPoolExecutor

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


def _oracle_pairs(cfg, orbs, orb_t, ij_list):
    """The oracle's result for each pair (i, j), given only that pair's
    orbitals (copied back from the device, so it sees the exact values the
    kernels read); the pairs run in parallel host threads."""
    P = _oracle_params(cfg)
    jobs = []
    for i, j in ij_list:
        idx = [i] if i == j else [i, j]
        R2 = None if orbs.R_orb is None or cfg.R_PE_classes is None else orbs.R_orb[idx]
        jobs.append((idx, orb_t[idx].to(torch.float64).cpu().numpy(), R2))

    def one(job):
        idx, phi, R2 = job
        return oracle.pair_fields(P, phi, orbs.centres[idx], 0, len(idx) - 1, R2)["res"]

    with ThreadPoolExecutor(max_workers=min(16, max(1, len(jobs)))) as ex:
        return dict(zip(ij_list, ex.map(one, jobs)))


def _check_pairs(tag, cfg, orbs, orb_t, pr, picks, tol_E=TOL_E, tol_S=TOL_S):
    """Per-pair E and sigma of the picked rows of pair_results against the
    oracle: FP64 within 1e-9 (E) and 1e-8 (sigma) relative, the mixed path
    within its 1e-6 bar."""
    ij_list = [tuple(int(x) for x in pr["ij"][k]) for k in picks]
    ora = _oracle_pairs(cfg, orbs, orb_t, ij_list)
    for k, ij in zip(picks, ij_list):
        r = ora[ij]
        print(f"[{tag}] pair {ij} gpu E={pr['E'][k]:.15g} oracle={r.E:.15g} iters {pr['iters'][k]}/{r.cg_iters}",
              flush=True)
        # both sides stop at ||r|| <= 1e-10 ||b||: the solution error is bounded by kappa * 1e-10
        assert abs(pr["E"][k] - r.E) <= tol_E * abs(r.E) + 1e-14
        s_o = np.array(list(r.sigma))
        assert np.abs(pr["sigma"][k] - s_o).sum() <= tol_S * np.abs(s_o).sum() + 1e-14


def _picks(pr, n, seed, n_strong=5):
    """n random pairs (mostly far apart), the middle self pair and the n_strong
    non-self pairs of largest |E| (the ones that carry E_xx)."""
    rng = np.random.default_rng(seed)
    m = len(pr["E"])
    self_idx = [k for k in range(m) if pr["ij"][k, 0] == pr["ij"][k, 1]]
    cross = np.flatnonzero(pr["ij"][:, 0] != pr["ij"][:, 1])
    strong = cross[np.argsort(-np.abs(pr["E"][cross]))[:n_strong]].tolist()
    return sorted(set(rng.choice(m, n, replace=False).tolist() + [self_idx[len(self_idx) // 2]] + strong))


def _rel_max(a, b):
    """Largest pointwise difference relative to the largest |b| (one orbital's D)."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


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
    _check_pairs("water64", cfg, orbs, orb_t, pr, _picks(pr, 10, 64))


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
    _check_pairs("water64 mixed", cfg, orbs, orb_t, pr, _picks(pr, 10, 65), tol_E=1e-6, tol_S=1e-6)
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
    emax = _rel_max(Dg, o["D"][0])
    print(f"[water64] D of orbital {i} ({len(nb)} orbitals, {len(o['pairs'])} pairs in the oracle run): rel {err:.3e}, "
          f"max {emax:.3e}", flush=True)
    assert err <= TOL_D and emax <= TOL_D


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
    _check_pairs("water128", cfg, orbs, orb_t, res["fp64"][3], _picks(res["fp64"][3], 10, 128))
    _check_pairs("water128 mixed", cfg, orbs, orb_t, res["mixed"][3], _picks(res["mixed"][3], 10, 129),
                 tol_E=1e-6, tol_S=1e-6)
    (Ea, Sa, Da, _, _), (Eb, Sb, Db, _, _) = res["mixed"], res["fp64"]
    n_mol = cfg.n_orb / 4
    dmax = max(_rel_max(Da[r], Db[r]) for r in range(Da.shape[0]))
    print(f"[water128] mixed - fp64: dE/molecule={(Ea - Eb) / n_mol:.3e} "
          f"sigma rel={np.abs(Sa - Sb).sum() / np.abs(Sb).sum():.3e} D rel={np.abs(Da - Db).sum() / np.abs(Db).sum():.3e} "
          f"D max per orbital={dmax:.3e}", flush=True)
    assert abs(Ea - Eb) <= 1e-6 * n_mol
    assert np.abs(Sa - Sb).sum() <= 1e-6 * np.abs(Sb).sum()
    assert np.abs(Da - Db).sum() <= 1e-6 * np.abs(Db).sum()
    assert max(_rel_max(Da[r], Db[r]) for r in range(Da.shape[0])) <= 1e-6 and dmax <= 1e-6
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
        _check_pairs("water256", cfg, orbs, orb_t, pr, _picks(pr, 10, 256))
        del g
    finally:
        plan.close()
    del orb_t
    torch.cuda.empty_cache()


def _pair_class(cfg, orbs, i, j):
    """Sphere class of pair (i, j): the rung of (R_i + R_j) / 2 (self pairs: R_i)."""
    rmin, step, ncls = cfg.R_PE_classes
    k = round((0.5 * (orbs.R_orb[i] + orbs.R_orb[j]) - rmin) / step)
    return int(min(max(k, 0), ncls - 1))


def test_water256_mixed_graph_replays_warm_start_every_class():
    """The repeated-call case in mixed precision as the benchmark runs it:
    variable radii (9 sphere classes, quad layout with fused sweeps on the
    classes of at most 768 runs, columns on the widest), autotuned, recorded
    into a HIP graph and replayed over displaced centres with each pair's CG
    started from its previous solution.  After the replays, sampled pairs of
    every class (and the strongest ones) match the oracle within the mixed bar."""
    cfg = synth.CONFIGS["water256"]
    frac = 1.0 / 32
    orbs = synth.make_orbitals(cfg)
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    R_t = torch.from_numpy(orbs.R_orb).to(DEV)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    S = torch.zeros(9, dtype=torch.float64, device=DEV)
    plan = _plan(cfg, max_pairs=4096, pair_sample_seed=2011072094, pair_sample_frac=frac, autotune=1, warm_start=1,
                 precision=exx.EXX_PREC_MIXED)
    try:
        plan.eval(orb_t, cen_t, E, None, S, R_t)
        torch.cuda.synchronize()
        st = plan.stats()
        print(f"[water256 mixed] eager: pairs={st['n_pairs']} classes={st['n_classes']} layout={st['class_layout']} "
              f"threads={st['class_threads']} E={E.item():.12f}", flush=True)
        assert st["n_classes"] == 9 and 2 in st["class_layout"]
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
            print(f"[water256 mixed] replay {step}: pairs={st['n_pairs']} warm={st['warm_pairs']} "
                  f"iters mean={st['cg_iter_sum'] / st['n_pairs']:.1f} restarts={st['cg_restarts']} "
                  f"E={E.item():.12f}", flush=True)
            assert st["graph_recorded"] == 1 and st["n_unconverged"] == 0 and np.all(pr["exit"] == 0)
            assert st["warm_pairs"] > 0.9 * st["n_pairs"]
            ol = oracle.pair_list(_oracle_params(cfg, sample_seed=2011072094, sample_frac=frac), orbs.centres,
                                  orbs.R_orb)
            assert [tuple(x) for x in pr["ij"]] == [(p.i, p.j) for p in ol]
        del g
    finally:
        plan.close()
    # two pairs of every class, and the strongest pairs
    rng = np.random.default_rng(2561)
    by_class = {}
    for k, (i, j) in enumerate(pr["ij"]):
        by_class.setdefault(_pair_class(cfg, orbs, int(i), int(j)), []).append(k)
    assert sorted(by_class) == list(range(9))
    picks = set(_picks(pr, 0, 2562, n_strong=4))
    for c, ks in sorted(by_class.items()):
        picks |= set(rng.choice(ks, min(2, len(ks)), replace=False).tolist())
    _check_pairs("water256 mixed", cfg, orbs, orb_t, pr, sorted(picks), tol_E=1e-6, tol_S=1e-6)
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
    _check_pairs("water512", cfg, orbs, orb_t, res["fp64"][3], _picks(res["fp64"][3], 10, 512))
    _check_pairs("water512 mixed", cfg, orbs, orb_t, res["mixed"][3], _picks(res["mixed"][3], 10, 513),
                 tol_E=1e-6, tol_S=1e-6)
    (Ea, Sa, Da, _, _), (Eb, Sb, Db, _, _) = res["mixed"], res["fp64"]
    n_mol = cfg.n_orb / 4 * frac   # molecule-equivalents the sampled pairs stand for
    print(f"[water512] mixed - fp64 on the subset: dE={Ea - Eb:.3e} Ha "
          f"sigma rel={np.abs(Sa - Sb).sum() / np.abs(Sb).sum():.3e} D rel={np.abs(Da - Db).sum() / np.abs(Db).sum():.3e}",
          flush=True)
    assert abs(Ea - Eb) <= 1e-6 * n_mol
    assert np.abs(Sa - Sb).sum() <= 1e-6 * np.abs(Sb).sum()
    # D is stored in FP32 in both paths: compare at FP32 storage resolution
    assert np.abs(Da - Db).sum() <= 1e-5 * np.abs(Db).sum()
    assert max(_rel_max(Da[r], Db[r]) for r in range(Da.shape[0])) <= 1e-5
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
    _check_pairs(key, cfg, orbs, orb_t, pr, sorted(set(_picks(pr, 10, 64 + len(key)) + strong)))
    _check_pairs(key + " mixed", cfg, orbs, orb_t, res["mixed"][3], _picks(res["mixed"][3], 10, 65 + len(key)),
                 tol_E=1e-6, tol_S=1e-6)
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


def test_tri64_fused_tilted_sweeps_full_size():
    """tri64 mixed in 512-thread (six columns per thread) and 1024-thread
    (three) workgroups: the tilted-arm CG fuses each pass B with the next pass
    A, keeping Ap between sweeps.  Sampled pairs against the oracle, E against
    the FP64 path's value on the same pair list."""
    cfg = synth.CONFIGS["tri64"]
    orbs = synth.make_orbitals(cfg)
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    res = {}
    for prec, threads in (("mixed", 512), ("mixed1024", 1024), ("fp64", 1024)):
        plan = _plan(cfg, solve_threads=threads,
                     precision=exx.EXX_PREC_FP64 if prec == "fp64" else exx.EXX_PREC_MIXED)
        E = torch.zeros(1, dtype=torch.float64, device=DEV)
        plan.eval(orb_t, cen_t, E)
        torch.cuda.synchronize()
        st = plan.stats()
        print(f"[tri64 {prec} {threads}] E={E.item():.12f} iters mean={st['cg_iter_sum'] / st['n_pairs']:.1f} "
              f"solve {st['solve_ms']:.0f} ms threads={st['solve_threads']}", flush=True)
        assert st["n_unconverged"] == 0
        assert st["solve_threads"] == threads
        res[prec] = (E.item(), plan.pair_results())
        plan.close()
    Ef, pf = res["fp64"]
    for prec in ("mixed", "mixed1024"):
        Em, pm = res[prec]
        assert np.array_equal(pm["ij"], pf["ij"])
        assert abs(Em - Ef) <= 1e-6 * cfg.n_orb / 4
    _check_pairs("tri64 fused 512", cfg, orbs, orb_t, res["mixed"][1], _picks(res["mixed"][1], 8, 91), tol_E=1e-6,
                 tol_S=1e-6)
    _check_pairs("tri64 fused 1024", cfg, orbs, orb_t, res["mixed1024"][1], _picks(res["mixed1024"][1], 8, 92),
                 tol_E=1e-6, tol_S=1e-6)


# ---------------------------------------------------------------------------
# fused CG sweeps on a sphere of more than 700 runs of four columns

def _quad_runs(R, d):
    """Runs of four x-adjacent columns (starting at x = 4k on even rows, 4k + 2
    on odd rows) that the equatorial disc of a sphere of radius R on a cubic
    grid of spacing d needs: the quad layout's run count."""
    Rg = int(np.floor(R / d + 1e-9)) + 1
    r2 = R * R * (1 + 1e-12)
    n = 0
    for oy in range(-Rg, Rg + 1):
        s = 2 * (oy & 1)
        k = -((Rg + s + 3) // 4) - 1
        while 4 * k + s <= Rg:
            if any((x * d) ** 2 + (oy * d) ** 2 <= r2 for x in range(4 * k + s, 4 * k + s + 4)):
                n += 1
            k += 1
    return n


def test_fused_sweeps_on_a_760_run_sphere():
    """R_PE 5.9 on the 64-molecule grid: 760 runs, so the mixed plan takes
    768-thread workgroups whose CG fuses pass B with the next pass A.  Every
    pair of two molecules matches the oracle within the mixed bar, with the
    same iteration counts as the two-pass 1024-thread kernel and fewer bytes
    per iteration."""
    base = synth.CONFIGS["water64"]
    full = synth.make_orbitals(base)
    n = 8
    cfg = dataclasses.replace(base, n_orb=n, R_PE=5.9)
    orbs = synth.OrbitalSet(full.centres[:n], full.expo[:n], full.poly[:n])
    runs = _quad_runs(cfg.R_PE, cfg.cell[0] / cfg.grid[0])
    assert 700 <= runs <= 768, runs
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    out = {}
    for threads in (0, 1024):
        plan = _plan(cfg, precision=exx.EXX_PREC_MIXED, solve_threads=threads)
        try:
            E = torch.zeros(1, dtype=torch.float64, device=DEV)
            plan.eval(orb_t, cen_t, E)
            torch.cuda.synchronize()
            st = plan.stats()
            out[threads] = (E.item(), plan.pair_results(), st)
        finally:
            plan.close()
        print(f"[fused 760 runs] threads {st['class_threads']}: pairs {st['n_pairs']} iterations {st['cg_iter_sum']} "
              f"bytes/iteration/point {st['cg_alg_bytes'] / st['cg_iter_sum'] / 113000:.2f} E={E.item():.12f}",
              flush=True)
        assert st["n_unconverged"] == 0 and st["class_layout"] == [2]
    fused, plain = out[0][2], out[1024][2]
    assert fused["class_threads"] == [768] and plain["class_threads"] == [1024]
    assert abs(fused["cg_iter_sum"] - plain["cg_iter_sum"]) <= 0.02 * plain["cg_iter_sum"] + plain["n_pairs"]
    assert fused["cg_alg_bytes"] / fused["cg_iter_sum"] < 0.85 * plain["cg_alg_bytes"] / plain["cg_iter_sum"]
    pr = out[0][1]
    _check_pairs("fused 760 runs", cfg, orbs, orb_t, pr, list(range(len(pr["E"]))), tol_E=1e-6, tol_S=1e-6)
    del orb_t
    torch.cuda.empty_cache()


def test_two_run_fused_sweeps_on_the_64_molecule_sphere():
    """The 64-molecule sphere needs more than 768 runs (780), so the mixed
    plan runs it in 512-thread workgroups with two runs per thread, whose CG
    fuses pass B with the next pass A.  Every pair of two molecules matches
    the oracle within the mixed bar, with the same iteration counts as the
    two-pass 1024-thread kernel and fewer bytes per iteration."""
    base = synth.CONFIGS["water64"]
    full = synth.make_orbitals(base)
    n = 8
    cfg = dataclasses.replace(base, n_orb=n)
    orbs = synth.OrbitalSet(full.centres[:n], full.expo[:n], full.poly[:n])
    runs = _quad_runs(cfg.R_PE, cfg.cell[0] / cfg.grid[0])
    assert 768 < runs <= 1024, runs
    orb_t = synth.fill_orbitals_device(cfg, orbs, DEV)
    cen_t = torch.from_numpy(orbs.centres).to(DEV)
    out = {}
    for threads in (0, 1024):
        plan = _plan(cfg, precision=exx.EXX_PREC_MIXED, solve_threads=threads)
        try:
            E = torch.zeros(1, dtype=torch.float64, device=DEV)
            plan.eval(orb_t, cen_t, E)
            torch.cuda.synchronize()
            st = plan.stats()
            out[threads] = (E.item(), plan.pair_results(), st)
        finally:
            plan.close()
        print(f"[fused {runs} runs] threads {st['class_threads']}: pairs {st['n_pairs']} iterations "
              f"{st['cg_iter_sum']} bytes/iteration/point {st['cg_alg_bytes'] / st['cg_iter_sum'] / 120473:.2f} "
              f"E={E.item():.12f}", flush=True)
        assert st["n_unconverged"] == 0 and st["class_layout"] == [2]
    fused, plain = out[0][2], out[1024][2]
    assert fused["class_threads"] == [512] and plain["class_threads"] == [1024]
    assert abs(fused["cg_iter_sum"] - plain["cg_iter_sum"]) <= 0.02 * plain["cg_iter_sum"] + plain["n_pairs"]
    assert fused["cg_alg_bytes"] / fused["cg_iter_sum"] < 0.85 * plain["cg_alg_bytes"] / plain["cg_iter_sum"]
    pr = out[0][1]
    _check_pairs(f"fused {runs} runs", cfg, orbs, orb_t, pr, list(range(len(pr["E"]))), tol_E=1e-6, tol_S=1e-6)
    del orb_t
    torch.cuda.empty_cache()
