"""exx_eval_noalloc (no device allocation; the workspace comes from the
library's static scratch array) against exx_eval on the same inputs, through
the C ABI: two calls in a row on one plan, the second with fewer orbitals, in
FP64 and in mixed precision.  E_xx, sigma_xx and D_xx agree within the FP64
parity bar (1e-9 relative on E, 1e-8 on sigma and D); the per-pair work is the
same kernels', so E and sigma come out bitwise equal and D (atomic adds)
within rounding.  The device's free memory is unchanged across each call."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2011_07209_amd import exx, synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _inputs(n):
    base = synth.CONFIGS["tiny16"]
    full = synth.make_orbitals(base)
    cfg = dataclasses.replace(base, n_orb=n)
    orbs = synth.OrbitalSet(full.centres[:n], full.expo[:n], full.poly[:n])
    phi = synth.fill_orbitals(cfg, orbs)
    return cfg, torch.from_numpy(phi).to(DEV), torch.from_numpy(orbs.centres).to(DEV)


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_exx_eval_on_two_calls(precision):
    prec = exx.EXX_PREC_MIXED if precision == "mixed" else exx.EXX_PREC_FP64
    cfg10, orb10, cen10 = _inputs(10)
    cfg6, orb6, cen6 = _inputs(6)
    opt = dict(stencil_n=cfg10.stencil_n, cg_tol=cfg10.cg_tol, precision=prec)
    ref_plan = exx.Plan(cfg10.h, cfg10.grid, cfg10.R_pair, cfg10.R_PE, cfg10.R_ME, cfg10.l_max, **opt)
    cap = ref_plan.count_pairs(cen10) + 8
    plan = exx.Plan(cfg10.h, cfg10.grid, cfg10.R_pair, cfg10.R_PE, cfg10.R_ME, cfg10.l_max, max_pairs=cap, **opt)
    try:
        for tag, orb_t, cen_t in (("10 orbitals", orb10, cen10), ("6 orbitals", orb6, cen6)):
            # reference through exx_eval
            E0 = torch.zeros(1, dtype=torch.float64, device=DEV)
            S0 = torch.zeros(9, dtype=torch.float64, device=DEV)
            D0 = torch.empty_like(orb_t)
            ref_plan.eval(orb_t, cen_t, E0, D0, S0)
            torch.cuda.synchronize()
            st0 = ref_plan.stats()
            # the same through exx_eval_noalloc
            E1 = torch.zeros(1, dtype=torch.float64, device=DEV)
            S1 = torch.zeros(9, dtype=torch.float64, device=DEV)
            D1 = torch.full_like(orb_t, float("nan"))
            torch.cuda.synchronize()
            free0, _ = torch.cuda.mem_get_info()
            plan.eval(orb_t, cen_t, E1, D1, S1, noalloc=True)
            torch.cuda.synchronize()
            free1, _ = torch.cuda.mem_get_info()
            st1 = plan.stats()
            pr1 = plan.pair_results()
            eE = abs(E1.item() - E0.item()) / abs(E0.item())
            eS = _rel(S1.cpu().numpy(), S0.cpu().numpy())
            eD = _rel(D1.cpu().numpy(), D0.cpu().numpy())
            print(f"[noalloc {precision}] {tag}: pairs {st1['n_pairs']}/{st0['n_pairs']} E={E1.item():.15g} "
                  f"ref={E0.item():.15g} relE={eE:.2e} relS={eS:.2e} relD={eD:.2e} free memory change "
                  f"{free0 - free1} bytes", flush=True)
            assert st1["n_pairs"] == st0["n_pairs"] > 0 and st1["n_unconverged"] == 0
            assert len(pr1["E"]) == st1["n_pairs"] and np.all(pr1["exit"] == exx.EXX_CG_CONVERGED)
            assert eE <= 1e-9 and eS <= 1e-8 and eD <= 1e-8
            assert np.isfinite(D1.cpu().numpy()).all()
            assert free1 == free0
    finally:
        plan.close()
        ref_plan.close()


def test_noalloc_refuses_plans_it_cannot_serve():
    """Without a fixed pair capacity, with warm-start stores, or with a pair
    capacity whose arrays exceed the scratch array: EXX_EINVAL, nothing run."""
    cfg, orb_t, cen_t = _inputs(4)
    base = dict(stencil_n=cfg.stencil_n, cg_tol=cfg.cg_tol)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    for kw in (dict(), dict(max_pairs=64, warm_start=1), dict(max_pairs=4_000_000)):
        plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, **base, **kw)
        try:
            with pytest.raises(exx.ExxError) as e:
                plan.eval(orb_t, cen_t, E, noalloc=True)
            assert e.value.status == exx.EXX_EINVAL
            print(f"[noalloc refused] {kw}: {e.value}", flush=True)
        finally:
            plan.close()
