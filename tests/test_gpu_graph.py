"""Fixed pair capacity, HIP-graph recording and D subsets, through the C ABI.

A plan with a fixed capacity (max_pairs) enqueues exx_eval without host waits
and, after one eager call, without allocations, so the call can be recorded
into a graph and replayed on new orbital values held in the same buffers (the
repeated-evaluation use of an MD run).  Every replay is checked: against the
eager result of the same inputs, and after new inputs against the oracle."""
import numpy as np
import pytest
import torch

from paper_2011_07209_amd import exx, synth

from gpu_util import oracle_eval, rel1

pytestmark = pytest.mark.gpu

CFG = synth.custom(key="graph", cell=(11.0, 12.0, 10.5), grid=(50, 56, 46), n_orb=7, R_pair=7.0, R_PE=3.9,
                   R_ME=5.3, l_max=5, stencil_n=3, cg_tol=1e-12, seed_index=71)
TOL_E, TOL_D, TOL_S = 1e-9, 1e-8, 1e-8


def _plan(cfg, **kw):
    return exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, stencil_n=cfg.stencil_n,
                    cg_tol=cfg.cg_tol, **kw)


def _inputs(cfg, orbs):
    dev = torch.device("cuda:0")
    phi = synth.fill_orbitals(cfg, orbs)
    orb_t = torch.from_numpy(phi).to(dev)
    cen_t = torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev)
    return phi, orb_t, cen_t


def test_d_subset_rows_match_full_D():
    orbs = synth.make_orbitals(CFG)
    phi, orb_t, cen_t = _inputs(CFG, orbs)
    dev = orb_t.device
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    plan = _plan(CFG)
    try:
        D = torch.empty_like(orb_t)
        plan.eval(orb_t, cen_t, E, D)
        subset = [5, 0, 3]
        Ds = torch.full((3,) + tuple(orb_t.shape[1:]), float("nan"), dtype=torch.float64, device=dev)
        plan.eval(orb_t, cen_t, E, Ds, d_subset=torch.tensor(subset, dtype=torch.int32, device=dev))
        torch.cuda.synchronize()
        for s, i in enumerate(subset):
            # same contributions, atomics in a different order
            assert rel1(Ds[s].cpu().numpy(), D[i].cpu().numpy()) <= 1e-13, (s, i)
    finally:
        plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replay_matches_eager_then_oracle_on_new_inputs(prec):
    """Replays reproduce the eager call; after new inputs they match the
    oracle (mixed plans run the quad layout and are held to the mixed bars)."""
    orbs = synth.make_orbitals(CFG)
    phi, orb_t, cen_t = _inputs(CFG, orbs)
    dev = orb_t.device
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    S = torch.zeros(9, dtype=torch.float64, device=dev)
    D = torch.empty_like(orb_t)
    plan = _plan(CFG, max_pairs=64, autotune=1,
                 precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64)
    try:
        plan.eval(orb_t, cen_t, E, D, S)          # eager: sizes the workspace and runs the autotuner
        torch.cuda.synchronize()
        n_pairs = plan.stats()["n_pairs"]
        E0, S0, D0 = E.clone(), S.clone(), D.clone()
        print(f"[graph] eager E={E0.item():.15g} pairs={n_pairs}", flush=True)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            plan.set_stream(side)
            with torch.cuda.graph(g, stream=side):
                plan.eval(orb_t, cen_t, E, D, S)
        torch.cuda.current_stream().wait_stream(side)
        plan.set_stream(torch.cuda.current_stream())

        for rep in range(3):
            E.zero_()
            S.zero_()
            D.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            print(f"[graph] replay {rep}: E={E.item():.15g}", flush=True)
            assert E.item() == E0.item()
            assert torch.equal(S, S0)
            assert rel1(D.cpu().numpy(), D0.cpu().numpy()) <= 1e-13
            st = plan.stats()
            assert st["graph_recorded"] == 1 and st["n_pairs"] == n_pairs and st["n_unconverged"] == 0

        # new centres and orbital values in the same buffers, then the oracle
        orbs2 = synth.displace(CFG, orbs, 1, amplitude=0.25)
        phi2 = synth.fill_orbitals(CFG, orbs2)
        orb_t.copy_(torch.from_numpy(phi2).to(dev))
        cen_t.copy_(torch.from_numpy(np.ascontiguousarray(orbs2.centres)).to(dev))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o = oracle_eval(CFG, orbs2, phi2)
        pr = plan.pair_results()
        print(f"[graph] new inputs: E={E.item():.15g} oracle={o['E']:.15g} pairs={len(pr['E'])}", flush=True)
        assert [tuple(x) for x in pr["ij"]] == [(p.i, p.j) for p in o["pairs"]]
        if prec == "mixed":
            assert plan.stats()["cg_layout"] == 2
            assert abs(E.item() - o["E"]) <= 1e-6 * CFG.n_orb / 4
            assert rel1(S.cpu().numpy().reshape(3, 3, order="F"), o["sigma"]) <= 1e-6
            assert rel1(D.cpu().numpy(), o["D"]) <= 1e-6
        else:
            assert rel1(E.item(), o["E"]) <= TOL_E
            assert rel1(S.cpu().numpy().reshape(3, 3, order="F"), o["sigma"]) <= TOL_S
            assert rel1(D.cpu().numpy(), o["D"]) <= TOL_D
        del g
    finally:
        plan.close()


def test_recording_without_an_eager_call_is_refused():
    orbs = synth.make_orbitals(CFG)
    phi, orb_t, cen_t = _inputs(CFG, orbs)
    E = torch.zeros(1, dtype=torch.float64, device=orb_t.device)
    plan = _plan(CFG, max_pairs=64)
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with pytest.raises(exx.ExxError) as err:
            with torch.cuda.stream(side):
                plan.set_stream(side)
                with torch.cuda.graph(g, stream=side):
                    plan.eval(orb_t, cen_t, E)
        assert err.value.status == exx.EXX_EINVAL
        torch.cuda.synchronize()
    finally:
        plan.close()


def test_capacity_overflow_is_reported_and_keeps_the_first_pairs():
    orbs = synth.make_orbitals(CFG)
    phi, orb_t, cen_t = _inputs(CFG, orbs)
    E = torch.zeros(1, dtype=torch.float64, device=orb_t.device)
    o = oracle_eval(CFG, orbs, phi, want_D=False)
    cap = 5
    assert len(o["pairs"]) > cap
    plan = _plan(CFG, max_pairs=cap)
    try:
        plan.eval(orb_t, cen_t, E)
        with pytest.raises(exx.ExxError) as err:
            plan.stats()
        assert err.value.status == exx.EXX_ECAPACITY
        st = plan.stats(allow_capacity=True)
        assert st["pairs_kept"] == len(o["pairs"]) and st["n_pairs"] == cap
        pr = plan.pair_results()
        assert [tuple(x) for x in pr["ij"]] == [(p.i, p.j) for p in o["pairs"][:cap]]
        Eo = np.array([p.E for p in o["pairs"][:cap]])
        assert np.allclose(pr["E"], Eo, rtol=1e-9, atol=0)
    finally:
        plan.close()


# ---------------------------------------------------------------------------
# warm start: each solve starts from the pair's previous solution

@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_warm_start_over_displaced_steps_matches_cold_oracle(prec):
    """Three MD-like steps (0.05 bohr per step).  From the second step on,
    pairs start from their previous solution; every step still matches the
    oracle, which always starts from zero, and needs fewer CG iterations
    than the cold first step."""
    orbs = synth.make_orbitals(CFG)
    phi, orb_t, cen_t = _inputs(CFG, orbs)
    dev = orb_t.device
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    S = torch.zeros(9, dtype=torch.float64, device=dev)
    D = torch.empty_like(orb_t)
    plan = _plan(CFG, max_pairs=64, warm_start=1,
                 precision=exx.EXX_PREC_MIXED if prec == "mixed" else exx.EXX_PREC_FP64)
    try:
        iters = []
        for step in range(3):
            if step:
                orbs = synth.displace(CFG, orbs, step, amplitude=0.05)
                phi = synth.fill_orbitals(CFG, orbs)
                orb_t.copy_(torch.from_numpy(phi).to(dev))
                cen_t.copy_(torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev))
            plan.eval(orb_t, cen_t, E, D, S)
            torch.cuda.synchronize()
            st = plan.stats()
            o = oracle_eval(CFG, orbs, phi)
            iters.append(st["cg_iter_sum"])
            print(f"[warm {prec}] step {step}: warm pairs {st['warm_pairs']}/{st['n_pairs']} iters {st['cg_iter_sum']} "
                  f"E={E.item():.15g} oracle={o['E']:.15g}", flush=True)
            assert st["n_unconverged"] == 0
            # a displacement may create pairs or move a pair centre by more than one point
            if step == 0:
                assert st["warm_pairs"] == 0
            else:
                assert 0.75 * st["n_pairs"] <= st["warm_pairs"] <= st["n_pairs"]
            if prec == "fp64":
                assert rel1(E.item(), o["E"]) <= TOL_E
                assert rel1(S.cpu().numpy().reshape(3, 3, order="F"), o["sigma"]) <= TOL_S
                assert rel1(D.cpu().numpy(), o["D"]) <= TOL_D
            else:
                assert abs(E.item() - o["E"]) <= 1e-6 * CFG.n_orb / 4
                assert rel1(S.cpu().numpy().reshape(3, 3, order="F"), o["sigma"]) <= 1e-6
                assert rel1(D.cpu().numpy(), o["D"]) <= 1e-6
        assert iters[1] < iters[0] and iters[2] < iters[0]
    finally:
        plan.close()


def test_warm_start_in_graph_replays():
    """The warm-start history lives on the device (store parity, previous pair
    list), so graph replays carry it from one replay to the next."""
    orbs = synth.make_orbitals(CFG)
    phi, orb_t, cen_t = _inputs(CFG, orbs)
    dev = orb_t.device
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    S = torch.zeros(9, dtype=torch.float64, device=dev)
    plan = _plan(CFG, max_pairs=64, warm_start=1)
    try:
        plan.eval(orb_t, cen_t, E, None, S)
        torch.cuda.synchronize()
        cold = plan.stats()["cg_iter_sum"]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            plan.set_stream(side)
            with torch.cuda.graph(g, stream=side):
                plan.eval(orb_t, cen_t, E, None, S)
        torch.cuda.current_stream().wait_stream(side)
        plan.set_stream(torch.cuda.current_stream())
        for step in (1, 2):
            orbs = synth.displace(CFG, orbs, step, amplitude=0.05)
            phi = synth.fill_orbitals(CFG, orbs)
            orb_t.copy_(torch.from_numpy(phi).to(dev))
            cen_t.copy_(torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            st = plan.stats()
            o = oracle_eval(CFG, orbs, phi, want_D=False)
            print(f"[warm graph] replay {step}: warm pairs {st['warm_pairs']}/{st['n_pairs']} iters "
                  f"{st['cg_iter_sum']} (cold {cold}) E={E.item():.15g} oracle={o['E']:.15g}", flush=True)
            assert 0.75 * st["n_pairs"] <= st["warm_pairs"] <= st["n_pairs"] and st["cg_iter_sum"] < cold
            assert rel1(E.item(), o["E"]) <= TOL_E
            assert rel1(S.cpu().numpy().reshape(3, 3, order="F"), o["sigma"]) <= TOL_S
        del g
    finally:
        plan.close()
