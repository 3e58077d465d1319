"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/exx.h declares, matches the header's struct layouts, and rejects
invalid arguments before touching a device.  No compute call is made."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2011_07209_amd import exx, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exx.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(exx.LIB_PATH):
        pytest.skip("libexx.so not built")
    return exx.load()


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+[\s\*]+(exx_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "exx_plan" in names and "exx_eval" in names and len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(exx.SYMBOLS) == names


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "exx.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(exx_options), sizeof(exx_stats),'
                    ' offsetof(exx_options, pair_sample_seed), offsetof(exx_options, solve_groups),'
                    ' offsetof(exx_stats, moment_flops), offsetof(exx_stats, cg_restarts),'
                    ' offsetof(exx_stats, class_pairs), offsetof(exx_options, refine_delta),'
                    ' offsetof(exx_stats, class_refine_delta)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out == [ctypes.sizeof(exx.Options), ctypes.sizeof(exx.Stats), exx.Options.pair_sample_seed.offset,
                   exx.Options.solve_groups.offset, exx.Stats.moment_flops.offset, exx.Stats.cg_restarts.offset,
                   exx.Stats.class_pairs.offset, exx.Options.refine_delta.offset,
                   exx.Stats.class_refine_delta.offset]


def test_default_options(lib):
    o = exx.exx_default_options()
    assert o.stencil_n == 3 and o.precision == exx.EXX_PREC_FP64 and o.cg_tol == 1e-10
    assert o.cg_max_iter == 5000 and o.pair_sample_frac == 1.0 and o.R_PE_nclass == 0


@pytest.mark.parametrize("case", ["singular", "left_handed", "arm_reach", "rme", "lmax", "stencil", "grid", "tol",
                                  "layout", "quad_general", "threads_640"])
def test_plan_rejects_invalid_arguments(lib, case):
    h = np.diag([12.0, 12.0, 12.0])
    grid, R_pair, R_PE, R_ME, L = (60, 60, 60), 8.0, 5.0, 7.0, 6
    opt = exx.exx_default_options(stencil_n=1)
    if case == "singular":
        h[:, 1] = h[:, 0]
    elif case == "left_handed":
        h[0, 1] = 0.5
        h[:, 2] *= -1.0
    elif case == "arm_reach":
        # a triclinic cell whose longest NK arm is longer than the lattice
        # spacings: R_ME covers n axis steps but not n arm steps
        from test_oracle_pins import _cell
        h = _cell(12.0, 12.5, 11.5, 80, 95, 100)
        grid = (60, 62, 58)
        opt.stencil_n = 3
        axis = max(np.linalg.norm(h, axis=0) / np.asarray(grid))
        longest = max(exx.exx_nk_stencil(h, grid)["step"])
        assert longest > 1.05 * axis
        R_ME = R_PE + 3 * (axis + longest) / 2
    elif case == "rme":
        R_ME = 5.1
    elif case == "lmax":
        L = 9
    elif case == "stencil":
        opt.stencil_n = 4
    elif case == "grid":
        grid = (60, 0, 60)
    elif case == "tol":
        opt.cg_tol = 0.0
    elif case == "layout":
        opt.cg_layout = 3
    elif case == "quad_general":   # runs of four columns need arms inside the sweep plane
        from test_oracle_pins import _cell
        h = _cell(12.0, 12.5, 11.5, 80, 95, 100)
        grid = (60, 62, 58)
        opt.cg_layout = 2
    elif case == "threads_640":    # workgroups of 512, 768 or 1024 threads only
        opt.solve_threads = 640
    with pytest.raises(exx.ExxError) as ei:
        exx.exx_plan(h, grid, R_pair, R_PE, R_ME, L, opt)
    assert ei.value.status == exx.EXX_EINVAL
    assert exx.exx_last_error(None)


@pytest.mark.parametrize("R_PE,R_ME,n,grid,cell", [
    (5.0, 7.0, 1, (60, 60, 60), (12.0, 12.0, 12.0)),
    (4.0, 5.5, 3, (48, 50, 44), (12.0, 12.5, 11.0)),
    (3.1, 4.2, 2, (40, 40, 40), (10.0, 10.0, 10.0)),
])
def test_subdomain_counts_match_oracle(lib, R_PE, R_ME, n, grid, cell):
    """The plan's sphere tables hold exactly the oracle's PE and ME point sets."""
    h = np.diag(cell)
    c = exx.exx_subdomain_counts(h, grid, R_PE, R_ME, n)
    cfg = synth.custom(cell=cell, grid=grid, R_PE=R_PE, R_ME=R_ME, stencil_n=n)
    P = oracle.make_params(h, grid, 8.0, R_PE, R_ME, 2, n)
    N1, N2, N3 = grid
    phi = np.zeros((1, N3, N2, N1))
    f = oracle.pair_fields(P, phi, np.array([[1.0, 1.0, 1.0]]), 0, 0)
    assert c["n_pe"] == f["res"].n_pe == np.count_nonzero(f["mask"] == 2)
    assert c["n_me"] == f["res"].n_me
    # Dirichlet points: non-PE points within n axis steps of a PE point
    m = f["mask"] == 2
    reach = np.zeros_like(m)
    for q in range(1, n + 1):
        for ax in range(3):
            reach |= np.roll(m, q, axis=ax) | np.roll(m, -q, axis=ax)
    assert c["n_halo"] == np.count_nonzero(reach & ~m)
    assert cfg.n_orb > 0


def test_tiny_config_counts(lib):
    c = exx.exx_subdomain_counts(np.diag([12.0] * 3), (60, 60, 60), 5.0, 7.0, 1)
    assert c["n_pe"] == 65267
