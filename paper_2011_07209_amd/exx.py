"""Thin ctypes binding of libexx.so (declared in include/exx.h).

Argument marshalling only: every step of the evaluation runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the HIP stream.
The names mirror the C ABI.  If the library has not been built, the first
call raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch  # loaded first so that the library binds to the same HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexx.so")

EXX_OK, EXX_EINVAL, EXX_ENOMEM, EXX_ENOCONV, EXX_EDEVICE, EXX_ECAPACITY = range(6)
EXX_F64, EXX_F32 = 0, 1
EXX_PREC_FP64, EXX_PREC_MIXED = 0, 1
EXX_CG_CONVERGED, EXX_CG_CAP, EXX_CG_BREAKDOWN, EXX_CG_NONFINITE = range(4)
CG_EXIT_NAMES = {0: "converged", 1: "cap", 2: "breakdown", 3: "nonfinite"}
_STATUS = {0: "EXX_OK", 1: "EXX_EINVAL", 2: "EXX_ENOMEM", 3: "EXX_ENOCONV", 4: "EXX_EDEVICE", 5: "EXX_ECAPACITY"}


class ExxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("stencil_n", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("cg_tol", ctypes.c_double),
        ("cg_max_iter", ctypes.c_int),
        ("R_PE_min", ctypes.c_double),
        ("R_PE_step", ctypes.c_double),
        ("R_PE_nclass", ctypes.c_int),
        ("pair_sample_seed", ctypes.c_ulonglong),
        ("pair_sample_frac", ctypes.c_double),
        ("max_pairs", ctypes.c_longlong),
        ("workspace_gb", ctypes.c_double),
        ("solve_groups", ctypes.c_int),
        ("solve_threads", ctypes.c_int),
        ("solve_depth", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("warm_start", ctypes.c_int),
        ("R_PE_self", ctypes.c_double),
        ("R_ME_self", ctypes.c_double),
        ("cell_fluctuation", ctypes.c_int),
        ("reassemble_strain", ctypes.c_double),
        ("cg_layout", ctypes.c_int),
        ("refine_delta", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_longlong),
        ("cg_iter_sum", ctypes.c_longlong),
        ("cg_iter_max", ctypes.c_int),
        ("n_unconverged", ctypes.c_int),
        ("n_classes", ctypes.c_int),
        ("refine_passes_max", ctypes.c_int),
        ("max_rel_residual", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("eval_ms", ctypes.c_double),
        ("cg_alg_bytes", ctypes.c_double),
        ("moment_flops", ctypes.c_double),
        ("n_evals", ctypes.c_longlong),
        ("solve_launches", ctypes.c_longlong),
        ("solve_ms_total", ctypes.c_double),
        ("cg_alg_bytes_total", ctypes.c_double),
        ("eval_ms_total", ctypes.c_double),
        ("solve_threads", ctypes.c_int),
        ("solve_depth", ctypes.c_int),
        ("tune_ms", ctypes.c_double),
        ("moment_ms", ctypes.c_double),
        ("moment_mfma_flops", ctypes.c_double),
        ("pairs_kept", ctypes.c_longlong),
        ("graph_recorded", ctypes.c_int),
        ("warm_pairs", ctypes.c_longlong),
        ("cell_strain", ctypes.c_double),
        ("reassemblies", ctypes.c_int),
        ("n_arms", ctypes.c_int),
        ("cg_layout", ctypes.c_int),
        ("n_cg_cap", ctypes.c_int),
        ("n_cg_breakdown", ctypes.c_int),
        ("n_cg_nonfinite", ctypes.c_int),
        ("cg_restarts", ctypes.c_longlong),
        ("t_pairlist_ms", ctypes.c_double),
        ("t_reduce_ms", ctypes.c_double),
        ("class_threads", ctypes.c_int * 16),
        ("class_depth", ctypes.c_int * 16),
        ("class_layout", ctypes.c_int * 16),
        ("class_pairs", ctypes.c_longlong * 16),
        ("class_refine_delta", ctypes.c_double * 16),
    ]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v)[:self.n_classes] if isinstance(v, ctypes.Array) else v
        return d


SYMBOLS = ["exx_default_options", "exx_plan", "exx_set_stream", "exx_eval", "exx_eval_noalloc", "exx_count_pairs",
           "exx_pair_results",
           "exx_stats_fetch", "exx_plan_geometry", "exx_subdomain_counts", "exx_nk_stencil", "exx_set_cell",
           "exx_pressure", "exx_destroy", "exx_last_error"]

_lib = None


def load():
    """Loads libexx.so; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc for gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, dp, ip, llp = ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int), P(ctypes.c_longlong)
    lib.exx_default_options.restype = None
    lib.exx_default_options.argtypes = [P(Options)]
    lib.exx_plan.restype = ctypes.c_int
    lib.exx_plan.argtypes = [dp, ip, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, P(Options),
                             P(vp)]
    lib.exx_set_stream.restype = ctypes.c_int
    lib.exx_set_stream.argtypes = [vp, vp]
    lib.exx_eval.restype = ctypes.c_int
    lib.exx_eval.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, ctypes.c_int, vp, vp, vp]
    lib.exx_eval_noalloc.restype = ctypes.c_int
    lib.exx_eval_noalloc.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, ctypes.c_int, vp, vp, vp]
    lib.exx_count_pairs.restype = ctypes.c_int
    lib.exx_count_pairs.argtypes = [vp, ctypes.c_int, vp, vp, llp]
    lib.exx_pair_results.restype = ctypes.c_int
    lib.exx_pair_results.argtypes = [vp, ctypes.c_longlong, ip, dp, dp, ip, dp, ip, ip, llp]
    lib.exx_stats_fetch.restype = ctypes.c_int
    lib.exx_stats_fetch.argtypes = [vp, P(Stats)]
    lib.exx_plan_geometry.restype = ctypes.c_int
    lib.exx_plan_geometry.argtypes = [vp, ctypes.c_int, llp, llp, llp]
    lib.exx_subdomain_counts.restype = ctypes.c_int
    lib.exx_subdomain_counts.argtypes = [dp, ip, ctypes.c_double, ctypes.c_double, ctypes.c_int, llp, llp, llp]
    lib.exx_nk_stencil.restype = ctypes.c_int
    lib.exx_nk_stencil.argtypes = [dp, ip, ip, ip, dp, dp]
    lib.exx_set_cell.restype = ctypes.c_int
    lib.exx_set_cell.argtypes = [vp, dp]
    lib.exx_pressure.restype = ctypes.c_int
    lib.exx_pressure.argtypes = [dp, dp, dp, dp]
    lib.exx_destroy.restype = ctypes.c_int
    lib.exx_destroy.argtypes = [vp]
    lib.exx_last_error.restype = ctypes.c_char_p
    lib.exx_last_error.argtypes = [vp]
    _lib = lib
    return lib


def exx_last_error(plan=None) -> str:
    s = load().exx_last_error(plan)
    return s.decode() if s else ""


def _check(status: int, plan=None):
    if status != EXX_OK:
        raise ExxError(status, exx_last_error(plan))


def exx_default_options(**kw) -> Options:
    o = Options()
    load().exx_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def exx_plan(h, grid, R_pair, R_PE, R_ME, l_max, opt: Optional[Options] = None):
    """h: 3x3 (h[:, al] = L_al) or 9 column-major values; returns the plan handle."""
    import numpy as np
    hv = np.asarray(h, dtype=np.float64)
    hv = hv.flatten(order="F") if hv.shape == (3, 3) else hv.reshape(9)
    hc = (ctypes.c_double * 9)(*hv.tolist())
    gc = (ctypes.c_int * 3)(*[int(x) for x in grid])
    out = ctypes.c_void_p()
    st = load().exx_plan(hc, gc, float(R_pair), float(R_PE), float(R_ME), int(l_max),
                         ctypes.byref(opt) if opt is not None else None, ctypes.byref(out))
    _check(st, None)
    return out.value


def exx_set_stream(plan, stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _check(load().exx_set_stream(plan, ctypes.c_void_p(handle)), plan)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def exx_eval(plan, orbitals: torch.Tensor, centres: torch.Tensor, E_xx: torch.Tensor,
             D_xx: Optional[torch.Tensor] = None, sigma: Optional[torch.Tensor] = None,
             R_PE_orb: Optional[torch.Tensor] = None, d_subset: Optional[torch.Tensor] = None,
             noalloc: bool = False):
    """Enqueues one evaluation; tensors are device tensors laid out as in exx.h.
    noalloc: through exx_eval_noalloc (no device allocation; workspace in the
    library's scratch array)."""
    if orbitals.dtype == torch.float64:
        dt = EXX_F64
    elif orbitals.dtype == torch.float32:
        dt = EXX_F32
    else:
        raise ExxError(EXX_EINVAL, "orbitals must be float64 or float32")
    for name, t in (("orbitals", orbitals), ("centres", centres), ("E_xx", E_xx), ("D_xx", D_xx),
                    ("sigma", sigma), ("R_PE_orb", R_PE_orb), ("d_subset", d_subset)):
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ExxError(EXX_EINVAL, f"{name} must be a contiguous device tensor")
    if centres.dtype != torch.float64 or E_xx.dtype != torch.float64:
        raise ExxError(EXX_EINVAL, "centres and E_xx must be float64")
    n_orb = orbitals.shape[0]
    n_subset = 0
    if d_subset is not None:
        if d_subset.dtype != torch.int32:
            raise ExxError(EXX_EINVAL, "d_subset must be int32")
        n_subset = d_subset.numel()
    rows = n_subset if d_subset is not None else n_orb
    if D_xx is not None and (D_xx.dtype != orbitals.dtype or D_xx.numel() != rows * (orbitals.numel() // n_orb)):
        raise ExxError(EXX_EINVAL, "D_xx must match the orbitals' dtype and hold one grid per requested orbital")
    if centres.numel() != 3 * n_orb:
        raise ExxError(EXX_EINVAL, "centres must be [n_orb, 3]")
    fn = load().exx_eval_noalloc if noalloc else load().exx_eval
    st = fn(plan, int(n_orb), _ptr(orbitals), dt, _ptr(centres), _ptr(R_PE_orb), _ptr(d_subset), int(n_subset),
            _ptr(E_xx), _ptr(D_xx), _ptr(sigma))
    _check(st, plan)


def exx_count_pairs(plan, centres: torch.Tensor, R_PE_orb: Optional[torch.Tensor] = None) -> int:
    """Pairs exx_eval would form for these centres (waits on the host)."""
    n = ctypes.c_longlong(0)
    _check(load().exx_count_pairs(plan, int(centres.shape[0]), _ptr(centres), _ptr(R_PE_orb), ctypes.byref(n)),
           plan)
    return n.value


def exx_pair_results(plan):
    """Per-pair results of the last evaluation as numpy arrays."""
    import numpy as np
    n = ctypes.c_longlong(0)
    lib = load()
    _check(lib.exx_pair_results(plan, 0, None, None, None, None, None, None, None, ctypes.byref(n)), plan)
    m = n.value
    ij = np.zeros(2 * max(m, 1), dtype=np.int32)
    E = np.zeros(max(m, 1))
    S = np.zeros(9 * max(m, 1))
    it = np.zeros(max(m, 1), dtype=np.int32)
    res = np.zeros(max(m, 1))
    ex = np.zeros(max(m, 1), dtype=np.int32)
    upd = np.zeros(max(m, 1), dtype=np.int32)
    P = ctypes.POINTER
    ip = P(ctypes.c_int)
    _check(lib.exx_pair_results(plan, m, ij.ctypes.data_as(ip), E.ctypes.data_as(P(ctypes.c_double)),
                                S.ctypes.data_as(P(ctypes.c_double)), it.ctypes.data_as(ip),
                                res.ctypes.data_as(P(ctypes.c_double)), ex.ctypes.data_as(ip), upd.ctypes.data_as(ip),
                                ctypes.byref(n)), plan)
    return {"ij": ij[:2 * m].reshape(m, 2), "E": E[:m], "sigma": S[:9 * m].reshape(m, 9), "iters": it[:m],
            "rel_res": res[:m], "exit": ex[:m] & 0xff, "restarts": ex[:m] >> 8, "updates": upd[:m]}


def exx_stats_fetch(plan, allow_noconv: bool = False, allow_capacity: bool = False) -> dict:
    s = Stats()
    st = load().exx_stats_fetch(plan, ctypes.byref(s))
    if not ((allow_noconv and st == EXX_ENOCONV) or (allow_capacity and st == EXX_ECAPACITY)):
        _check(st, plan)
    d = s.as_dict()
    d["status"] = st
    return d


def exx_plan_geometry(plan, cls: int = 0):
    a, b, c = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
    _check(load().exx_plan_geometry(plan, int(cls), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), plan)
    return {"n_pe": a.value, "n_halo": b.value, "n_me": c.value}


def exx_subdomain_counts(h, grid, R_PE, R_ME, stencil_n):
    import numpy as np
    hv = np.asarray(h, dtype=np.float64)
    hv = hv.flatten(order="F") if hv.shape == (3, 3) else hv.reshape(9)
    hc = (ctypes.c_double * 9)(*hv.tolist())
    gc = (ctypes.c_int * 3)(*[int(x) for x in grid])
    a, b, c = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
    _check(load().exx_subdomain_counts(hc, gc, float(R_PE), float(R_ME), int(stencil_n), ctypes.byref(a),
                                       ctypes.byref(b), ctypes.byref(c)), None)
    return {"n_pe": a.value, "n_halo": b.value, "n_me": c.value}


def exx_nk_stencil(h, grid):
    """The library's NK Laplacian for cell h: dict u (k x 3), beta, step."""
    import numpy as np
    hv = np.asarray(h, dtype=np.float64)
    hv = hv.flatten(order="F") if hv.shape == (3, 3) else hv.reshape(9)
    hc = (ctypes.c_double * 9)(*hv.tolist())
    gc = (ctypes.c_int * 3)(*[int(x) for x in grid])
    n = ctypes.c_int()
    u = (ctypes.c_int * 18)()
    beta = (ctypes.c_double * 6)()
    step = (ctypes.c_double * 6)()
    _check(load().exx_nk_stencil(hc, gc, ctypes.byref(n), u, beta, step), None)
    k = n.value
    return {"u": np.array(list(u), dtype=np.int64).reshape(6, 3)[:k], "beta": np.array(list(beta))[:k],
            "step": np.array(list(step))[:k]}


def _h9(h):
    import numpy as np
    hv = np.asarray(h, dtype=np.float64)
    hv = hv.flatten(order="F") if hv.shape == (3, 3) else hv.reshape(9)
    return (ctypes.c_double * 9)(*hv.tolist())


def exx_set_cell(plan, h):
    _check(load().exx_set_cell(plan, _h9(h)), plan)


def exx_pressure(h, sigma):
    """(Pi (3x3, [a, b]), p_int) from sigma (3x3 [a, al]) and the cell h."""
    import numpy as np
    Pi = (ctypes.c_double * 9)()
    p = ctypes.c_double()
    _check(load().exx_pressure(_h9(h), _h9(sigma), Pi, ctypes.byref(p)), None)
    return np.array(list(Pi)).reshape(3, 3, order="F"), p.value


def exx_destroy(plan):
    if plan:
        _check(load().exx_destroy(plan), None)


class Plan:
    """Owning wrapper: plan + stream binding + the three calls."""

    def __init__(self, h, grid, R_pair, R_PE, R_ME, l_max, **opts):
        self.opt = exx_default_options(**opts)
        self.handle = exx_plan(h, grid, R_pair, R_PE, R_ME, l_max, self.opt)
        exx_set_stream(self.handle)

    def eval(self, orbitals, centres, E_xx=None, D_xx=None, sigma=None, R_PE_orb=None, d_subset=None,
             noalloc=False):
        dev = orbitals.device
        if E_xx is None:
            E_xx = torch.zeros(1, dtype=torch.float64, device=dev)
        exx_eval(self.handle, orbitals, centres, E_xx, D_xx, sigma, R_PE_orb, d_subset, noalloc)
        return E_xx

    def set_stream(self, stream=None):
        """Binds the stream later calls enqueue on (default: torch's current stream)."""
        exx_set_stream(self.handle, stream)

    def count_pairs(self, centres, R_PE_orb=None):
        return exx_count_pairs(self.handle, centres, R_PE_orb)

    def pair_results(self):
        return exx_pair_results(self.handle)

    def stats(self, allow_noconv=False, allow_capacity=False):
        return exx_stats_fetch(self.handle, allow_noconv, allow_capacity)

    def set_cell(self, h):
        exx_set_cell(self.handle, h)

    def geometry(self, cls=0):
        return exx_plan_geometry(self.handle, cls)

    def close(self):
        if self.handle:
            exx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
