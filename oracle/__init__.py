"""FP64 CPU oracle for the EXX pair kernel (arXiv:2011.07209) -- test infrastructure.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (``paper_2011_07209_amd``) never does,
and the two share no code.  The arithmetic lives in ``exx_oracle.c``; this
module builds it with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double * 9),
        ("h_geom", ctypes.c_double * 9),
        ("grid", ctypes.c_int * 3),
        ("R_pair", ctypes.c_double),
        ("R_PE", ctypes.c_double),
        ("R_ME", ctypes.c_double),
        ("l_max", ctypes.c_int),
        ("stencil_n", ctypes.c_int),
        ("cg_tol", ctypes.c_double),
        ("cg_max_iter", ctypes.c_int),
        ("R_PE_min", ctypes.c_double),
        ("R_PE_step", ctypes.c_double),
        ("R_PE_nclass", ctypes.c_int),
        ("sample_seed", ctypes.c_ulonglong),
        ("sample_frac", ctypes.c_double),
        ("n_threads", ctypes.c_int),
        ("R_PE_self", ctypes.c_double),
        ("R_ME_self", ctypes.c_double),
    ]


class PairResult(ctypes.Structure):
    _fields_ = [
        ("i", ctypes.c_int),
        ("j", ctypes.c_int),
        ("c", ctypes.c_int * 3),
        ("R_PE", ctypes.c_double),
        ("n_pe", ctypes.c_int),
        ("n_me", ctypes.c_int),
        ("cg_iters", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("rel_res", ctypes.c_double),
        ("true_rel_res", ctypes.c_double),
        ("E", ctypes.c_double),
        ("sigma", ctypes.c_double * 9),
        ("shell_rho_v", ctypes.c_double),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        lib.oracle_eval.restype = ctypes.c_long
        lib.oracle_eval.argtypes = [P(Params), ctypes.c_int, dp, dp, dp, dp, dp, dp, P(PairResult), ctypes.c_long]
        lib.oracle_pair_list.restype = ctypes.c_long
        lib.oracle_pair_list.argtypes = [P(Params), ctypes.c_int, dp, dp, P(PairResult), ctypes.c_long]
        lib.oracle_pair_fields.restype = ctypes.c_int
        lib.oracle_pair_fields.argtypes = [P(Params), ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp, dp,
                                           P(ctypes.c_ubyte), P(PairResult)]
        lib.oracle_box_dims.restype = None
        lib.oracle_box_dims.argtypes = [P(Params), P(ctypes.c_int)]
        lib.oracle_ylm.restype = None
        lib.oracle_ylm.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        lib.oracle_stencil_weights.restype = None
        lib.oracle_stencil_weights.argtypes = [ctypes.c_int, dp, dp]
        lib.oracle_apply_A.restype = ctypes.c_int
        lib.oracle_apply_A.argtypes = [P(ctypes.c_int), dp, ctypes.c_int, P(ctypes.c_ubyte), dp, dp]
        lib.oracle_nk_stencil.restype = ctypes.c_int
        lib.oracle_nk_stencil.argtypes = [dp, P(ctypes.c_int), P(ctypes.c_int), dp, dp, P(ctypes.c_int), dp]
        lib.oracle_apply_arms.restype = ctypes.c_int
        lib.oracle_apply_arms.argtypes = [P(ctypes.c_int), ctypes.c_int, ctypes.c_int, P(ctypes.c_int), dp,
                                          P(ctypes.c_ubyte), dp, dp]
        lib.oracle_cg_mask.restype = ctypes.c_int
        lib.oracle_cg_mask.argtypes = [P(ctypes.c_int), dp, ctypes.c_int, P(ctypes.c_ubyte), dp, ctypes.c_double,
                                       ctypes.c_int, dp, P(ctypes.c_int), dp]
        _lib = lib
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(h, grid, R_pair, R_PE, R_ME, l_max, stencil_n, cg_tol=1e-10, cg_max_iter=5000, h_geom=None,
                R_PE_classes=None, sample_seed=0, sample_frac=1.0, n_threads=0, R_PE_self=0.0,
                R_ME_self=0.0) -> Params:
    """h: 3x3 array with h[:, al] = L_al (Cartesian columns)."""
    p = Params()
    h = np.asarray(h, dtype=np.float64)
    hg = h if h_geom is None else np.asarray(h_geom, dtype=np.float64)
    p.h[:] = list(h.flatten(order="F"))
    p.h_geom[:] = list(hg.flatten(order="F"))
    p.grid[:] = [int(g) for g in grid]
    p.R_pair, p.R_PE, p.R_ME = float(R_pair), float(R_PE), float(R_ME)
    p.l_max, p.stencil_n = int(l_max), int(stencil_n)
    p.cg_tol, p.cg_max_iter = float(cg_tol), int(cg_max_iter)
    if R_PE_classes is not None:
        rmin, step, ncls = R_PE_classes
        p.R_PE_min, p.R_PE_step, p.R_PE_nclass = float(rmin), float(step), int(ncls)
    p.sample_seed = int(sample_seed) & 0xFFFFFFFFFFFFFFFF
    p.sample_frac = float(sample_frac)
    p.n_threads = int(n_threads)
    p.R_PE_self, p.R_ME_self = float(R_PE_self), float(R_ME_self)
    return p


_ERR = {-1: "invalid argument", -2: "no three admissible NK auxiliary directions",
        -3: "R_ME < R_PE + n*max stencil step", -4: "out of memory"}


def _check(rc):
    if rc < 0:
        raise ValueError("oracle: " + _ERR.get(int(rc), str(rc)))
    return rc


def pair_list(params: Params, centres, R_orb=None):
    lib = _load()
    c = np.ascontiguousarray(centres, dtype=np.float64)
    ro = None if R_orb is None else np.ascontiguousarray(R_orb, dtype=np.float64)
    n = _check(lib.oracle_pair_list(ctypes.byref(params), c.shape[0], _dp(c), _dp(ro), None, 0))
    out = (PairResult * max(n, 1))()
    lib.oracle_pair_list(ctypes.byref(params), c.shape[0], _dp(c), _dp(ro), out, n)
    return [out[k] for k in range(n)]


def evaluate(params: Params, orbitals, centres, R_orb=None, want_D=True):
    """Returns dict(E, sigma (3x3, sigma[a, al]), D or None, pairs=list of PairResult)."""
    lib = _load()
    orb = np.ascontiguousarray(orbitals, dtype=np.float64)
    c = np.ascontiguousarray(centres, dtype=np.float64)
    ro = None if R_orb is None else np.ascontiguousarray(R_orb, dtype=np.float64)
    n_orb = c.shape[0]
    assert orb.shape[0] == n_orb
    npair = _check(lib.oracle_pair_list(ctypes.byref(params), n_orb, _dp(c), _dp(ro), None, 0))
    E = np.zeros(1)
    sig = np.zeros(9)
    D = np.zeros_like(orb) if want_D else None
    pr = (PairResult * max(npair, 1))()
    n = _check(lib.oracle_eval(ctypes.byref(params), n_orb, _dp(orb), _dp(c), _dp(ro), _dp(E), _dp(D), _dp(sig),
                               pr, npair))
    return {
        "E": float(E[0]),
        "sigma": sig.reshape(3, 3, order="F"),
        "D": D,
        "pairs": [pr[k] for k in range(n)],
    }


def box_dims(params: Params):
    lib = _load()
    K = (ctypes.c_int * 3)()
    lib.oracle_box_dims(ctypes.byref(params), K)
    return tuple(K)


def pair_fields(params: Params, orbitals, centres, i, j, R_orb=None):
    """Fields of one pair on its local box, shaped [z, y, x] (offset = index - K)."""
    lib = _load()
    K = box_dims(params)
    shape = (2 * K[2] + 1, 2 * K[1] + 1, 2 * K[0] + 1)
    orb = np.ascontiguousarray(orbitals, dtype=np.float64)
    c = np.ascontiguousarray(centres, dtype=np.float64)
    ro = None if R_orb is None else np.ascontiguousarray(R_orb, dtype=np.float64)
    rho = np.zeros(shape)
    v = np.zeros(shape)
    mask = np.zeros(shape, dtype=np.uint8)
    res = PairResult()
    rc = lib.oracle_pair_fields(ctypes.byref(params), c.shape[0], _dp(orb), _dp(c), _dp(ro), int(i), int(j),
                                _dp(rho), _dp(v), mask.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                                ctypes.byref(res))
    _check(rc)
    return {"K": K, "rho": rho, "v": v, "mask": mask, "res": res}


def ylm(lmax, x, y, z):
    lib = _load()
    out = np.zeros((lmax + 1) ** 2)
    lib.oracle_ylm(int(lmax), float(x), float(y), float(z), _dp(out))
    return out


def stencil_weights(n):
    lib = _load()
    w2 = np.zeros(4)
    w1 = np.zeros(4)
    lib.oracle_stencil_weights(int(n), _dp(w2), _dp(w1))
    return w2, w1


def apply_A(K, spacing, n, mask, p):
    """-(axis-stencil Laplacian) on the mask==2 points of a [z, y, x] box of half-widths K=(Kx,Ky,Kz)."""
    lib = _load()
    Kc = (ctypes.c_int * 3)(*K)
    sp = np.ascontiguousarray(spacing, dtype=np.float64)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    q = np.zeros_like(pp)
    _check(lib.oracle_apply_A(Kc, _dp(sp), int(n), m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), _dp(pp), _dp(q)))
    return q


def cg_mask(K, spacing, n, mask, b, tol=1e-12, max_iter=10000):
    lib = _load()
    Kc = (ctypes.c_int * 3)(*K)
    sp = np.ascontiguousarray(spacing, dtype=np.float64)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(bb)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0)
    rc = lib.oracle_cg_mask(Kc, _dp(sp), int(n), m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), _dp(bb),
                            float(tol), int(max_iter), _dp(x), ctypes.byref(it), ctypes.byref(rel))
    _check(rc)
    return x, it.value, rel.value


def nk_stencil(h, grid):
    """NK Laplacian arms of cell h (3x3, columns L_al) on a grid: dict with
    u (k x 3 integer steps), beta, step (length of u), coef = beta / step^2, and
    the three directions Algorithm 1 accepted (aux, k x 3) with their weights b."""
    lib = _load()
    hh = np.ascontiguousarray(np.asarray(h, dtype=np.float64).flatten(order="F"))
    N = (ctypes.c_int * 3)(*[int(g) for g in grid])
    u = (ctypes.c_int * 18)()
    aux = (ctypes.c_int * 9)()
    beta = np.zeros(6)
    step = np.zeros(6)
    b = np.zeros(3)
    n = _check(lib.oracle_nk_stencil(_dp(hh), N, u, _dp(beta), _dp(step), aux, _dp(b)))
    U = np.array(list(u), dtype=np.int64).reshape(6, 3)[:n]
    return {"u": U, "beta": beta[:n].copy(), "step": step[:n].copy(), "coef": beta[:n] / step[:n] ** 2,
            "aux": np.array(list(aux), dtype=np.int64).reshape(3, 3), "b": b}


def apply_arms(K, n, u, coef, mask, p):
    """-(sum over arms of coef * second difference along u) on the mask==2 points of a [z, y, x] box."""
    lib = _load()
    Kc = (ctypes.c_int * 3)(*K)
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.int32).reshape(-1))
    cc = np.ascontiguousarray(coef, dtype=np.float64)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    q = np.zeros_like(pp)
    _check(lib.oracle_apply_arms(Kc, int(n), len(cc), uu.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(cc),
                                 m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), _dp(pp), _dp(q)))
    return q
