"""Host logic of general (non-orthogonal) cells, checked on the CPU: the
library's own Algorithm 1 / NK Laplacian (Sec. III C 2) and its general
proto-subdomains (Sec. III B 1) against the oracle, which is written
independently.  No device is needed: both entry points are host-only."""
import numpy as np
import pytest

import oracle
from paper_2011_07209_amd import exx, synth
from test_oracle_pins import _NK_CELLS, _cell


def _arms(S):
    return {tuple(int(x) for x in u): b for u, b in zip(S["u"], S["beta"])}


CELLS = dict(_NK_CELLS)
CELLS["orthorhombic"] = (np.diag([11.0, 12.5, 13.0]), (44, 50, 52))
CELLS["sheared_cubic"] = (np.diag([12.0, 12.0, 12.0]) @ np.array([[1, 1, 0], [0, 1, 0], [0, 0, 1]]), (48, 48, 48))
CELLS["monoclinic_unequal"] = (_cell(11.0, 12.0, 13.5, 90, 110, 90), (56, 60, 66))


@pytest.mark.parametrize("name", sorted(CELLS))
def test_library_nk_arms_match_the_oracle(name):
    h, N = CELLS[name]
    lib = exx.exx_nk_stencil(h, N)
    ora = oracle.nk_stencil(h, N)
    a, b = _arms(lib), _arms(ora)
    assert set(a) == set(b), (a, b)
    for k in a:
        assert abs(a[k] - b[k]) <= 1e-12 * max(1.0, abs(b[k])), (k, a[k], b[k])
    steps = {tuple(int(x) for x in u): s for u, s in zip(lib["u"], lib["step"])}
    for u, s in zip(ora["u"], ora["step"]):
        assert abs(steps[tuple(int(x) for x in u)] - s) <= 1e-13 * s


@pytest.mark.parametrize("name", ["hexagonal", "monoclinic", "triclinic", "rhombohedral", "sheared_cubic"])
def test_library_general_subdomains_match_the_oracle(name):
    """PE and ME point counts of the library's tables equal the oracle's masks;
    the Dirichlet count equals a brute-force count of the points outside PE
    reached along an arm or a lattice axis within n steps."""
    h, N = CELLS[name]
    n, R_PE, R_ME = 3, 3.0, 4.6
    cfg = synth.custom(cell=tuple(np.linalg.norm(h, axis=0)), grid=N, hmat=tuple(np.asarray(h).flatten("F")),
                       R_PE=R_PE, R_ME=R_ME, stencil_n=n, n_orb=1)
    P = oracle.make_params(cfg.h, cfg.grid, cfg.R_pair, R_PE, R_ME, cfg.l_max, n)
    K = oracle.box_dims(P)
    phi = np.zeros((1, N[2], N[1], N[0]))
    f = oracle.pair_fields(P, phi, np.array([[0.0, 0.0, 0.0]]), 0, 0)
    mask = f["mask"]
    pe = mask == 2
    lib = exx.exx_subdomain_counts(h, N, R_PE, R_ME, n)
    assert lib["n_pe"] == int(pe.sum())
    assert lib["n_me"] == int((mask > 0).sum())
    dirs = [tuple(u) for u in oracle.nk_stencil(h, N)["u"]]
    for e in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        if e not in dirs:
            dirs.append(e)
    reach = np.zeros_like(pe)
    Kx, Ky, Kz = K
    for u in dirs:
        for q in range(1, n + 1):
            for sgn in (1, -1):
                dx, dy, dz = (sgn * q * c for c in u)
                shifted = np.zeros_like(pe)
                src = pe[max(0, dz):pe.shape[0] + min(0, dz), max(0, dy):pe.shape[1] + min(0, dy),
                         max(0, dx):pe.shape[2] + min(0, dx)]
                shifted[max(0, -dz):pe.shape[0] + min(0, -dz), max(0, -dy):pe.shape[1] + min(0, -dy),
                        max(0, -dx):pe.shape[2] + min(0, -dx)] = src
                reach |= shifted
    assert lib["n_halo"] == int((reach & ~pe).sum())


def test_pressure_tensor_isotropic_closed_form():
    """For pure Gaussian densities sigma = -(E/3) h^-T in any cell (the
    closed form the oracle pins), so eq. pixx_working gives Pi = E/(3V) I and
    eq. pxx_working p_int = E/(3V) (eq. liq_press in the cubic case)."""
    for name in ("triclinic", "hexagonal", "orthorhombic"):
        h, _ = CELLS[name]
        E = -3.7
        sigma = -(E / 3.0) * np.linalg.inv(h).T
        Pi, p = exx.exx_pressure(h, sigma)
        V = abs(np.linalg.det(h))
        np.testing.assert_allclose(Pi, E / (3 * V) * np.eye(3), rtol=0, atol=1e-14 * abs(E / V))
        assert abs(p - E / (3 * V)) <= 1e-14 * abs(E / V)


def test_pressure_tensor_components():
    """Pi_ab = -(1/V) sum_al sigma^{a al} h_{b al}, written out by components."""
    rng = np.random.default_rng(3)
    h, _ = CELLS["triclinic"]
    sigma = rng.normal(size=(3, 3))
    Pi, p = exx.exx_pressure(h, sigma)
    V = abs(np.linalg.det(h))
    for a in range(3):
        for b in range(3):
            want = -sum(sigma[a, al] * h[b, al] for al in range(3)) / V
            assert abs(Pi[a, b] - want) <= 1e-14 * abs(sigma).max() * abs(h).max() / V
    assert abs(p - np.trace(Pi) / 3) <= 1e-15 * abs(Pi).max()
