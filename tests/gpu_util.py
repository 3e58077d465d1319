"""Helpers shared by the GPU tests: run the HIP path and the oracle on the
same seeded inputs and compare them."""
import dataclasses

import numpy as np
import torch

import oracle
from paper_2011_07209_amd import exx, synth


def rel1(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def subset_config(key, n_orb):
    base = synth.CONFIGS[key]
    full = synth.make_orbitals(base)
    cfg = dataclasses.replace(base, n_orb=n_orb)
    orbs = synth.OrbitalSet(full.centres[:n_orb], full.expo[:n_orb], full.poly[:n_orb],
                            None if full.R_orb is None else full.R_orb[:n_orb])
    return cfg, orbs


def gpu_eval(cfg, orbs, phi, want_D=True, dtype=torch.float64, **opt):
    """Runs exx_eval on cuda:0; returns dict(E, sigma (3x3 [a, al]), D, pairs, stats)."""
    dev = torch.device("cuda:0")
    kw = dict(stencil_n=cfg.stencil_n, cg_tol=cfg.cg_tol)
    if cfg.R_PE_classes is not None:
        kw.update(R_PE_min=cfg.R_PE_classes[0], R_PE_step=cfg.R_PE_classes[1], R_PE_nclass=cfg.R_PE_classes[2])
    for k, v in opt.items():
        kw[{"sample_seed": "pair_sample_seed", "sample_frac": "pair_sample_frac"}.get(k, k)] = v
    plan = exx.Plan(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, **kw)
    try:
        orb_t = torch.from_numpy(np.ascontiguousarray(phi)).to(dev, dtype)
        cen_t = torch.from_numpy(np.ascontiguousarray(orbs.centres)).to(dev, torch.float64)
        R_t = None
        if cfg.R_PE_classes is not None:
            R_t = torch.from_numpy(np.ascontiguousarray(orbs.R_orb)).to(dev, torch.float64)
        E = torch.zeros(1, dtype=torch.float64, device=dev)
        S = torch.zeros(9, dtype=torch.float64, device=dev)
        D = torch.empty_like(orb_t) if want_D else None
        plan.eval(orb_t, cen_t, E, D, S, R_t)
        torch.cuda.synchronize()
        out = {
            "E": float(E.item()),
            "sigma": S.cpu().numpy().reshape(3, 3, order="F"),
            "D": None if D is None else D.cpu().numpy(),
            "pairs": plan.pair_results(),
            "stats": plan.stats(allow_noconv=True),
        }
    finally:
        plan.close()
    return out


def oracle_eval(cfg, orbs, phi, want_D=True, **kw):
    P = oracle.make_params(cfg.h, cfg.grid, cfg.R_pair, cfg.R_PE, cfg.R_ME, cfg.l_max, cfg.stencil_n, cfg.cg_tol,
                           R_PE_classes=cfg.R_PE_classes, **kw)
    return oracle.evaluate(P, phi, orbs.centres, orbs.R_orb if cfg.R_PE_classes is not None else None, want_D)
