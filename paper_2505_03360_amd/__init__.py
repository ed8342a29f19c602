"""Python binding of the bz C ABI (include/bz.h).

Argument marshalling only: every step of the collision operator and of the
regime mask runs in the HIP library ``libbz.so``; torch tensors only provide
device memory and streams.  Importing works without a GPU (the host-only
entry points, e.g. plan construction, can be called); every call that
launches GPU work needs the library built for gfx950 and a visible GPU.
There is no CPU fallback: if libbz.so is missing, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbz.so")

BZ_OK, BZ_AGAIN = 0, 1
BZ_ERR_ARG, BZ_ERR_UNSUPPORTED, BZ_ERR_DEVICE, BZ_ERR_NOMEM, BZ_ERR_STATE, BZ_ERR_NUMERIC = -1, -2, -3, -4, -5, -6
BZ_FP64, BZ_FP32 = 0, 1
BZ_DIRS_EXPLICIT, BZ_DIRS_ICOSA6, BZ_DIRS_PRODUCT, BZ_DIRS_SPIRAL, BZ_DIRS_CIRCLE, BZ_DIRS_DESIGN = 0, 1, 2, 3, 4, 5
BZ_XF_AUTO, BZ_XF_FUSED, BZ_XF_PLAIN, BZ_XF_DFT_GEMM = 0, 1, 2, 3
BZ_SCATTER = 1
BZ_CELL_SOLID, BZ_CELL_FORCE_BOLTZMANN = 1, 2
BZ_REGIME_SOLID = 255

_c_double_p = ctypes.POINTER(ctypes.c_double)


class BzPlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("L", ctypes.c_double),
        ("R", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("kernel_c", ctypes.c_double),
        ("m", ctypes.c_int32),
        ("dir_kind", ctypes.c_int32),
        ("dirs", _c_double_p),
        ("weights", _c_double_p),
        ("a1", ctypes.c_int32),
        ("a2", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("transform", ctypes.c_int32),
        ("project", ctypes.c_int32),
        ("max_cells", ctypes.c_int32),
        ("chunks", ctypes.c_int32),
        ("slices", ctypes.c_int32),
        ("dealias", ctypes.c_int32),
        ("dim", ctypes.c_int32),
    ]


class BzMaskDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("mu0", ctypes.c_double), ("kappa0", ctypes.c_double),
        ("eta0", ctypes.c_double), ("eta1", ctypes.c_double), ("delta0", ctypes.c_double),
        ("laplacian_u_mode", ctypes.c_int32),
    ]


class BzServerDesc(ctypes.Structure):
    _fields_ = [("arena_dev", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("max_inflight", ctypes.c_int32), ("n_streams", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("slice_cells", ctypes.c_int32)]


class BzRequest(ctypes.Structure):
    _fields_ = [("plan", BzPlanDesc), ("f", ctypes.c_void_p), ("f_dtype", ctypes.c_int32),
                ("idx", ctypes.c_void_p), ("ncells", ctypes.c_int32), ("q", ctypes.c_void_p),
                ("flags", ctypes.c_int32), ("client_id", ctypes.c_int32), ("ready_event", ctypes.c_void_p)]


class BzResult(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("err", ctypes.c_int32), ("t_submit_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class BzServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("queued", ctypes.c_int32), ("inflight", ctypes.c_int32), ("plans_cached", ctypes.c_int32),
                ("arena_used", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("cells_per_s", ctypes.c_double)]


BZ_REQ_QUEUED, BZ_REQ_ADMITTED, BZ_REQ_DONE, BZ_REQ_FAILED = 0, 1, 2, 3


class BzStepBuffers(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_void_p), ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p),
                ("T", ctypes.c_void_p), ("eps", ctypes.c_void_p), ("regime_in", ctypes.c_void_p),
                ("l1dist", ctypes.c_void_p), ("cell_flags", ctypes.c_void_p), ("regime_out", ctypes.c_void_p),
                ("boltz_idx", ctypes.c_void_p), ("counts", ctypes.c_void_p), ("diag", ctypes.c_void_p),
                ("f", ctypes.c_void_p), ("f_dtype", ctypes.c_int32), ("q", ctypes.c_void_p),
                ("kinetic_moments", ctypes.c_int32), ("kin_idx", ctypes.c_void_p), ("kin_count", ctypes.c_void_p)]


class BzMomentsOut(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("rho", "u1", "u2", "u3", "T", "l1")]


class BzImexDesc(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("eps", ctypes.c_double), ("eps_cells", ctypes.c_void_p)]


class BzEsbgkDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("L", ctypes.c_double), ("beta", ctypes.c_double), ("mu0", ctypes.c_double)]


class BzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bz error {code}: {msg}")
        self.code = code


_LIB = None
ABI_VERSION = 5  # the struct layouts below match include/bz.h at this version

# (name, restype, argtypes) for every symbol declared in include/bz.h
_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t
SIGNATURES = [
    ("bz_abi_version", _I32, []),
    ("bz_last_error", ctypes.c_char_p, []),
    ("bz_plan_create", _I32, [ctypes.POINTER(BzPlanDesc), ctypes.POINTER(_VP)]),
    ("bz_plan_device_bytes", _I32, [_VP, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ), ctypes.POINTER(_SZ)]),
    ("bz_plan_bind", _I32, [_VP, _VP, _VP, _SZ, _VP]),
    ("bz_plan_destroy", _I32, [_VP]),
    ("bz_plan_capacity", _I32, [_VP, ctypes.POINTER(_I32)]),
    ("bz_plan_transform", _I32, [_VP, ctypes.POINTER(_I32)]),
    ("bz_set_tune_table", _I32, [ctypes.c_char_p]),
    ("bz_plan_strategy", _I32, [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("bz_plan_get_rule", _I32, [_VP, _c_double_p, _c_double_p]),
    ("bz_plan_get_multipliers", _I32, [_VP, _I32, _c_double_p]),
    ("bz_plan_rule_degree", _I32, [_VP, ctypes.POINTER(_I32)]),
    ("bz_collide_batch", _I32, [_VP, _VP, _I32, _VP, _I32, _VP, _VP, _I32, _VP]),
    ("bz_collide_batch_noalloc", _I32, [_VP, _VP, _I32, _VP, _I32, _VP, _VP, _I32, _VP]),
    ("bz_plan_sync", _I32, [_VP, _VP]),
    ("bz_plan_set_timing", _I32, [_VP, _I32]),
    ("bz_cell_moments", _I32, [_I32, ctypes.c_double, _VP, _I32, _VP, _I32, _VP, ctypes.POINTER(BzMomentsOut),
                               _I32, _VP]),
    ("bz_imex_euler", _I32, [_VP, ctypes.POINTER(BzImexDesc), _VP, _VP, _VP, _I32, _VP, _VP, _I32, _VP]),
    ("bz_pr222_stage1", _I32, [_VP, ctypes.POINTER(BzImexDesc), _VP, _VP, _I32, _VP, _VP, _VP]),
    ("bz_pr222_stage2", _I32, [_VP, ctypes.POINTER(BzImexDesc), _VP, _VP, _VP, _VP, _I32, _VP, _VP, _VP, _VP]),
    ("bz_pr222_finish", _I32, [_VP, ctypes.POINTER(BzImexDesc), _VP, _VP, _VP, _VP, _I32, _VP, _VP, _VP]),
    ("bz_esbgk_pr222_stage1", _I32, [ctypes.POINTER(BzEsbgkDesc), ctypes.POINTER(BzImexDesc), _VP, _VP, _I32, _VP,
                                     _VP, _VP]),
    ("bz_esbgk_pr222_stage2", _I32, [ctypes.POINTER(BzEsbgkDesc), ctypes.POINTER(BzImexDesc), _VP, _VP, _VP, _VP,
                                     _I32, _VP, _VP, _VP, _VP]),
    ("bz_esbgk_pr222_finish", _I32, [ctypes.POINTER(BzEsbgkDesc), ctypes.POINTER(BzImexDesc), _VP, _VP, _VP, _VP,
                                     _I32, _VP, _VP, _VP]),
    ("bz_esbgk_collide", _I32, [ctypes.POINTER(BzEsbgkDesc), _VP, _VP, _I32, _VP, _VP, _I32, _VP]),
    ("bz_esbgk_imex_euler", _I32, [ctypes.POINTER(BzEsbgkDesc), ctypes.POINTER(BzImexDesc), _VP, _VP, _VP, _I32,
                                   _VP, _VP, _I32, _VP]),
    ("bz_plan_last_times", _I32, [_VP, ctypes.POINTER(ctypes.c_float), _I32]),
    ("bz_realizability_mask", _I32, [ctypes.POINTER(BzMaskDesc), _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                     _VP, _VP, _VP, _VP, _VP, _VP]),
    ("bz_server_create", _I32, [ctypes.POINTER(BzServerDesc), ctypes.POINTER(_VP)]),
    ("bz_serve_submit", _I32, [_VP, ctypes.POINTER(BzRequest), ctypes.POINTER(ctypes.c_uint64)]),
    ("bz_serve_poll", _I32, [_VP, ctypes.c_uint64, ctypes.POINTER(BzResult)]),
    ("bz_server_stats", _I32, [_VP, _c_double_p, _c_double_p, _c_double_p]),
    ("bz_server_stats_ex", _I32, [_VP, ctypes.POINTER(BzServerStats)]),
    ("bz_mask_sync", _I32, [_VP, _VP]),
    ("bz_server_destroy", _I32, [_VP]),
    ("bz_step_create", _I32, [_VP, ctypes.POINTER(BzMaskDesc), ctypes.POINTER(BzStepBuffers), ctypes.POINTER(_VP)]),
    ("bz_step_launch", _I32, [_VP, _VP]),
    ("bz_step_destroy", _I32, [_VP]),
]


def lib():
    """Load libbz.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.bz_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {L.bz_abi_version()}, the binding expects {ABI_VERSION}: "
                               "rebuild it with __graft_entry__.build()")
        _LIB = L
    return _LIB


def _check(code: int) -> int:
    if code < 0:
        raise BzError(code, lib().bz_last_error().decode())
    return code


# ---------------------------------------------------------------- C ABI, same names
def bz_abi_version() -> int:
    return lib().bz_abi_version()


def bz_last_error() -> str:
    return lib().bz_last_error().decode()


def make_plan2d_desc(n: int, L: float = 8.0, R: float = 0.0, kernel_c: float = 1.0, m: int = 32,
                     precision: int = BZ_FP32, project: int = 1, max_cells: int = 1) -> BzPlanDesc:
    """Descriptor of the two-velocity-dimension Maxwell-molecule operator
    (gamma = 0, angles theta_p = pi p/m); kernel_c = 1 is the paper's Btilde = 1."""
    return make_plan_desc(n=n, L=L, R=R, gamma=0.0, kernel_c=kernel_c, m=m, dir_kind=BZ_DIRS_CIRCLE,
                          precision=precision, project=project, max_cells=max_cells, dim=2)


def make_plan_desc(n: int, L: float = 8.0, R: float = 0.0, gamma: float = 1.0, kernel_c: float = 4.0,
                   m: int = 6, dir_kind: int = BZ_DIRS_ICOSA6, dirs=None, weights=None, a1: int = 0,
                   a2: int = 0, precision: int = BZ_FP32, transform: int = BZ_XF_AUTO, project: int = 1,
                   max_cells: int = 1, chunks: int = 0, slices: int = 0, dealias: int = 0,
                   dim: int = 3) -> BzPlanDesc:
    d = BzPlanDesc()
    d.n, d.L, d.R, d.gamma, d.kernel_c = n, L, R, gamma, kernel_c
    d.m, d.dir_kind, d.a1, d.a2 = m, dir_kind, a1, a2
    d.precision, d.transform, d.project, d.max_cells, d.chunks = precision, transform, project, max_cells, chunks
    d.slices = slices
    d.dealias = dealias
    d.dim = dim
    d._keep = []
    if dirs is not None:
        import numpy as np
        da = np.ascontiguousarray(dirs, dtype=np.float64).ravel()
        wa = np.ascontiguousarray(weights, dtype=np.float64).ravel()
        d._keep = [da, wa]
        d.dirs = da.ctypes.data_as(_c_double_p)
        d.weights = wa.ctypes.data_as(_c_double_p)
        d.dir_kind = BZ_DIRS_EXPLICIT
        d.m = len(wa)
    return d


def bz_plan_create(desc: BzPlanDesc) -> int:
    out = _VP()
    _check(lib().bz_plan_create(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def bz_plan_device_bytes(plan: int):
    t, f, c = _SZ(), _SZ(), _SZ()
    _check(lib().bz_plan_device_bytes(plan, ctypes.byref(t), ctypes.byref(f), ctypes.byref(c)))
    return t.value, f.value, c.value


def bz_plan_bind(plan: int, tables_dev: int, ws_dev: int, ws_bytes: int, stream: int = 0) -> None:
    _check(lib().bz_plan_bind(plan, tables_dev, ws_dev, ws_bytes, stream))


def bz_plan_destroy(plan: int) -> None:
    _check(lib().bz_plan_destroy(plan))


def bz_plan_capacity(plan: int) -> int:
    c = _I32()
    _check(lib().bz_plan_capacity(plan, ctypes.byref(c)))
    return c.value


def bz_plan_transform(plan: int) -> int:
    c = _I32()
    _check(lib().bz_plan_transform(plan, ctypes.byref(c)))
    return c.value


def bz_set_tune_table(path) -> None:
    _check(lib().bz_set_tune_table(None if path is None else str(path).encode()))


def bz_plan_strategy(plan: int):
    t, c, s = _I32(), _I32(), _I32()
    _check(lib().bz_plan_strategy(plan, ctypes.byref(t), ctypes.byref(c), ctypes.byref(s)))
    return t.value, c.value, s.value


def bz_plan_get_rule(plan: int, m: int):
    import numpy as np
    d = np.zeros((m, 3))
    w = np.zeros(m)
    _check(lib().bz_plan_get_rule(plan, d.ctypes.data_as(_c_double_p), w.ctypes.data_as(_c_double_p)))
    return d, w


def bz_plan_rule_degree(plan: int) -> int:
    t = _I32()
    _check(lib().bz_plan_rule_degree(plan, ctypes.byref(t)))
    return t.value


def bz_plan_get_multipliers(plan: int, n: int, p: int, dim: int = 3):
    """FP64 host multipliers of pass p as ([k1][k2][k3] alpha, alpha'), or
    ([k1][k2] alpha, alpha') for a two-dimensional plan."""
    import numpy as np
    buf = np.zeros(n ** dim * 2)
    _check(lib().bz_plan_get_multipliers(plan, p, buf.ctypes.data_as(_c_double_p)))
    if dim == 2:
        t = buf.reshape(n, n, 2)  # [k2][k1]
        return t[..., 0].T.copy(), t[..., 1].T.copy()
    t = buf.reshape(n, n, n, 2)  # [k2][k3][k1]
    return t[..., 0].transpose(2, 0, 1).copy(), t[..., 1].transpose(2, 0, 1).copy()


def bz_collide_batch(plan: int, f: int, f_dtype: int, idx: int, ncells: int, ncells_dev: int,
                     q: int, flags: int = 0, stream: int = 0) -> None:
    _check(lib().bz_collide_batch(plan, f, f_dtype, idx, ncells, ncells_dev, q, flags, stream))


def bz_collide_batch_noalloc(plan: int, f: int, f_dtype: int, idx: int, ncells: int, ncells_dev: int,
                             q: int, flags: int, stream: int = 0) -> None:
    _check(lib().bz_collide_batch_noalloc(plan, f, f_dtype, idx, ncells, ncells_dev, q, flags, stream))


def bz_cell_moments(n: int, L: float, f: int, f_dtype: int, idx: int, ncells: int, ncells_dev: int,
                    out: BzMomentsOut, flags: int = 0, stream: int = 0) -> None:
    _check(lib().bz_cell_moments(n, L, f, f_dtype, idx, ncells, ncells_dev, ctypes.byref(out), flags, stream))


def bz_imex_euler(plan: int, desc: BzImexDesc, f: int, tr: int, idx: int, ncells: int, ncells_dev: int,
                  f_out: int, flags: int = 0, stream: int = 0) -> None:
    _check(lib().bz_imex_euler(plan, ctypes.byref(desc), f, tr, idx, ncells, ncells_dev, f_out, flags, stream))


def bz_pr222_stage1(plan: int, desc: BzImexDesc, y: int, idx: int, ncells: int, ncells_dev: int, y1: int,
                    stream: int = 0) -> None:
    _check(lib().bz_pr222_stage1(plan, ctypes.byref(desc), y, idx, ncells, ncells_dev, y1, stream))


def bz_pr222_stage2(plan: int, desc: BzImexDesc, y: int, y1: int, t1: int, idx: int, ncells: int,
                    ncells_dev: int, y2: int, a: int, stream: int = 0) -> None:
    _check(lib().bz_pr222_stage2(plan, ctypes.byref(desc), y, y1, t1, idx, ncells, ncells_dev, y2, a, stream))


def bz_pr222_finish(plan: int, desc: BzImexDesc, a: int, y2: int, t2: int, idx: int, ncells: int,
                    ncells_dev: int, y_out: int, stream: int = 0) -> None:
    _check(lib().bz_pr222_finish(plan, ctypes.byref(desc), a, y2, t2, idx, ncells, ncells_dev, y_out, stream))


def bz_esbgk_pr222_stage1(desc: BzEsbgkDesc, imex: BzImexDesc, y: int, idx: int, ncells: int, ncells_dev: int,
                          y1: int, stream: int = 0) -> None:
    _check(lib().bz_esbgk_pr222_stage1(ctypes.byref(desc), ctypes.byref(imex), y, idx, ncells, ncells_dev, y1, stream))


def bz_esbgk_pr222_stage2(desc: BzEsbgkDesc, imex: BzImexDesc, y: int, y1: int, t1: int, idx: int, ncells: int,
                          ncells_dev: int, y2: int, a: int, stream: int = 0) -> None:
    _check(lib().bz_esbgk_pr222_stage2(ctypes.byref(desc), ctypes.byref(imex), y, y1, t1, idx, ncells, ncells_dev,
                                       y2, a, stream))


def bz_esbgk_pr222_finish(desc: BzEsbgkDesc, imex: BzImexDesc, a: int, y2: int, t2: int, idx: int, ncells: int,
                          ncells_dev: int, y_out: int, stream: int = 0) -> None:
    _check(lib().bz_esbgk_pr222_finish(ctypes.byref(desc), ctypes.byref(imex), a, y2, t2, idx, ncells, ncells_dev,
                                       y_out, stream))


def bz_esbgk_collide(desc: BzEsbgkDesc, f: int, idx: int, ncells: int, ncells_dev: int, q: int,
                     flags: int = 0, stream: int = 0) -> None:
    _check(lib().bz_esbgk_collide(ctypes.byref(desc), f, idx, ncells, ncells_dev, q, flags, stream))


def bz_esbgk_imex_euler(desc: BzEsbgkDesc, imex: BzImexDesc, f: int, tr: int, idx: int, ncells: int,
                        ncells_dev: int, f_out: int, flags: int = 0, stream: int = 0) -> None:
    _check(lib().bz_esbgk_imex_euler(ctypes.byref(desc), ctypes.byref(imex), f, tr, idx, ncells, ncells_dev,
                                     f_out, flags, stream))


def bz_plan_sync(plan: int, stream: int = 0) -> None:
    _check(lib().bz_plan_sync(plan, stream))


def bz_plan_set_timing(plan: int, enable: bool) -> None:
    _check(lib().bz_plan_set_timing(plan, 1 if enable else 0))


def bz_plan_last_times(plan: int):
    ms = (ctypes.c_float * 5)()
    _check(lib().bz_plan_last_times(plan, ms, 5))
    return list(ms)


def bz_realizability_mask(desc: BzMaskDesc, rho: int, ux: int, uy: int, T: int, eps: int,
                          regime_in: int, l1dist: int, cell_flags: int, regime_out: int,
                          boltz_idx: int, counts: int, diag: int, stream: int = 0) -> None:
    _check(lib().bz_realizability_mask(ctypes.byref(desc), rho, ux, uy, T, eps, regime_in, l1dist,
                                       cell_flags, regime_out, boltz_idx, counts, diag, stream))


def bz_server_create(desc: BzServerDesc) -> int:
    out = _VP()
    _check(lib().bz_server_create(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def bz_serve_submit(server: int, req: BzRequest):
    """Returns the ticket, or None if the queue is full (BZ_AGAIN)."""
    t = ctypes.c_uint64()
    rc = _check(lib().bz_serve_submit(server, ctypes.byref(req), ctypes.byref(t)))
    return None if rc == BZ_AGAIN else t.value


def bz_serve_poll(server: int, ticket: int):
    """Returns (finished, BzResult)."""
    r = BzResult()
    rc = _check(lib().bz_serve_poll(server, ticket, ctypes.byref(r)))
    return rc == BZ_OK, r


def bz_server_stats(server: int):
    """(p50_ms, p99_ms, cells_per_s) of the completed requests."""
    v = [ctypes.c_double() for _ in range(3)]
    _check(lib().bz_server_stats(server, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def bz_server_stats_ex(server: int) -> BzServerStats:
    st = BzServerStats()
    _check(lib().bz_server_stats_ex(server, ctypes.byref(st)))
    return st


def bz_server_destroy(server: int) -> None:
    _check(lib().bz_server_destroy(server))


def bz_mask_sync(counts: int, stream: int = 0) -> None:
    """Raises BzError(BZ_ERR_NUMERIC) if the mask call that wrote `counts`
    found cells with invalid inputs."""
    _check(lib().bz_mask_sync(counts, stream))


def bz_step_create(plan: int, mask: BzMaskDesc, bufs: BzStepBuffers) -> int:
    out = _VP()
    _check(lib().bz_step_create(plan, ctypes.byref(mask), ctypes.byref(bufs), ctypes.byref(out)))
    return out.value


def bz_step_launch(step: int, stream: int = 0) -> None:
    _check(lib().bz_step_launch(step, stream))


def bz_step_destroy(step: int) -> None:
    _check(lib().bz_step_destroy(step))


# ---------------------------------------------------------------- torch-side helpers
def _torch():
    import torch
    return torch


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _out_rows(f, n_pts: int, ncells: int, scatter: bool) -> int:
    """Rows an output must have: with BZ_SCATTER cell c is written at row
    idx[c], which can be any row of f; otherwise rows 0..ncells."""
    return f.numel() // n_pts if scatter else ncells


def _output(out, f, n_pts: int, ncells: int, scatter: bool, dtype, cell_shape):
    """Allocate the output, or check a caller-supplied one (contiguous, on the
    GPU, of the right dtype, holding at least the rows the call writes)."""
    torch = _torch()
    rows = _out_rows(f, n_pts, ncells, scatter)
    if out is None:
        return torch.empty((rows,) + tuple(cell_shape), dtype=dtype, device=f.device)
    if out.dtype != dtype or not out.is_contiguous() or not out.is_cuda:
        raise ValueError(f"out must be a contiguous CUDA {dtype} tensor")
    if out.numel() < rows * n_pts:
        raise ValueError(f"out holds {out.numel() // n_pts} rows, the call writes up to row {rows - 1}")
    return out


def _stream(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Collider:
    """A bound plan whose tables and workspace are torch tensors on the GPU."""

    def __init__(self, n: int, max_cells: int, device="cuda", stream=None, **desc_kw):
        torch = _torch()
        self.desc = make_plan_desc(n=n, max_cells=max_cells, **desc_kw)
        self.n = n
        self.dim = 2 if self.desc.dim == 2 else 3
        self.plan = bz_plan_create(self.desc)
        tb, fixed, per = bz_plan_device_bytes(self.plan)
        self.tables = torch.empty(max(tb, 256), dtype=torch.uint8, device=device)
        self.ws_bytes = fixed + per * max_cells
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        bz_plan_bind(self.plan, _ptr(self.tables), _ptr(self.ws), self.ws_bytes, _stream(stream))
        self.capacity = bz_plan_capacity(self.plan)
        self.transform = bz_plan_transform(self.plan)
        self.out_dtype = torch.float64 if self.desc.project or self.desc.precision == BZ_FP64 else torch.float32

    def __call__(self, f, idx=None, ncells=None, ncells_dev=None, out=None, scatter=False, stream=None):
        torch = _torch()
        n3 = self.n ** self.dim
        if f.dtype not in (torch.float32, torch.float64) or not f.is_contiguous() or not f.is_cuda:
            raise ValueError("f must be a contiguous CUDA float32/float64 tensor")
        if ncells is None:
            ncells = idx.numel() if idx is not None else f.numel() // n3
        if idx is not None and (idx.dtype != torch.int32 or not idx.is_cuda):
            raise ValueError("idx must be a CUDA int32 tensor")
        out = _output(out, f, n3, ncells, scatter, self.out_dtype, (self.n,) * self.dim)
        fd = BZ_FP32 if f.dtype == torch.float32 else BZ_FP64
        bz_collide_batch(self.plan, _ptr(f), fd, _ptr(idx), ncells, _ptr(ncells_dev), _ptr(out),
                         BZ_SCATTER if scatter else 0, _stream(stream))
        return out

    def imex_euler(self, f, tr, dt: float, eps: float = 0.0, eps_cells=None, idx=None, ncells=None,
                   ncells_dev=None, out=None, scatter=False, stream=None):
        """One penalised IMEX step (bz_imex_euler) on FP64 CUDA tensors."""
        torch = _torch()
        for t in (f, tr):
            if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("f and tr must be contiguous CUDA float64 tensors")
        if ncells is None:
            ncells = idx.numel() if idx is not None else f.numel() // self.n ** 3
        out = _output(out, f, self.n ** 3, ncells, scatter, torch.float64, (self.n,) * 3)
        d = BzImexDesc(dt, eps, _ptr(eps_cells))
        bz_imex_euler(self.plan, d, _ptr(f), _ptr(tr), _ptr(idx), ncells, _ptr(ncells_dev), _ptr(out),
                      BZ_SCATTER if scatter else 0, _stream(stream))
        return out

    def pr222_step(self, y, transport, dt: float, eps: float = 0.0, eps_cells=None, idx=None, out=None,
                   stream=None):
        """One PR(2,2,2) step through bz_pr222_stage1/stage2/finish; `transport`
        maps a stage value (a tensor shaped like y) to v . grad_x of it and runs
        between the calls.  Stage buffers are allocated like y."""
        torch = _torch()
        if y.dtype != torch.float64 or not y.is_contiguous() or not y.is_cuda:
            raise ValueError("y must be a contiguous CUDA float64 tensor")
        ncells = idx.numel() if idx is not None else y.numel() // self.n ** 3
        d = BzImexDesc(dt, eps, _ptr(eps_cells))
        st = _stream(stream)
        y1, y2, a = torch.empty_like(y), torch.empty_like(y), torch.empty_like(y)
        out = torch.empty_like(y) if out is None else out
        bz_pr222_stage1(self.plan, d, _ptr(y), _ptr(idx), ncells, 0, _ptr(y1), st)
        t1 = transport(y1).contiguous()
        bz_pr222_stage2(self.plan, d, _ptr(y), _ptr(y1), _ptr(t1), _ptr(idx), ncells, 0, _ptr(y2), _ptr(a), st)
        t2 = transport(y2).contiguous()
        bz_pr222_finish(self.plan, d, _ptr(a), _ptr(y2), _ptr(t2), _ptr(idx), ncells, 0, _ptr(out), st)
        return out

    def close(self):
        if self.plan:
            bz_plan_destroy(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cell_moments(f, L: float, idx=None, ncells=None, ncells_dev=None, out=None, scatter=False,
                 l1=True, stream=None):
    """bz_cell_moments on a CUDA tensor [*][n][n][n]; returns a dict of FP64
    tensors rho, u1, u2, u3, T (and l1) indexed like the output rows."""
    torch = _torch()
    n = f.shape[-1]
    if ncells is None:
        ncells = idx.numel() if idx is not None else f.numel() // n ** 3
    if out is None:
        rows = f.numel() // n ** 3 if scatter else ncells
        keys = ("rho", "u1", "u2", "u3", "T") + (("l1",) if l1 else ())
        out = {k: torch.zeros(rows, dtype=torch.float64, device=f.device) for k in keys}
    o = BzMomentsOut(*[_ptr(out.get(k)) for k in ("rho", "u1", "u2", "u3", "T", "l1")])
    fd = BZ_FP32 if f.dtype == torch.float32 else BZ_FP64
    bz_cell_moments(n, L, _ptr(f), fd, _ptr(idx), ncells, _ptr(ncells_dev), o,
                    BZ_SCATTER if scatter else 0, _stream(stream))
    return out


def _f64_cells(f, idx, ncells):
    torch = _torch()
    if f.dtype != torch.float64 or not f.is_contiguous() or not f.is_cuda:
        raise ValueError("f must be a contiguous CUDA float64 tensor")
    n = f.shape[-1]
    if ncells is None:
        ncells = idx.numel() if idx is not None else f.numel() // n ** 3
    return n, ncells


def esbgk_collide(f, L: float, beta: float = -0.5, mu0: float = 1.0, idx=None, ncells=None, ncells_dev=None,
                  out=None, scatter=False, stream=None):
    """Q_ES(f) = nu (G[f] - f) for a batch of cells (bz_esbgk_collide)."""
    torch = _torch()
    n, ncells = _f64_cells(f, idx, ncells)
    out = _output(out, f, n ** 3, ncells, scatter, torch.float64, (n,) * 3)
    bz_esbgk_collide(BzEsbgkDesc(n, L, beta, mu0), _ptr(f), _ptr(idx), ncells, _ptr(ncells_dev), _ptr(out),
                     BZ_SCATTER if scatter else 0, _stream(stream))
    return out


def esbgk_imex_euler(f, tr, L: float, dt: float, eps: float = 0.0, eps_cells=None, beta: float = -0.5,
                     mu0: float = 1.0, idx=None, ncells=None, ncells_dev=None, out=None, scatter=False,
                     stream=None):
    """One first-order IMEX step of the ES-BGK layer (bz_esbgk_imex_euler)."""
    torch = _torch()
    n, ncells = _f64_cells(f, idx, ncells)
    out = _output(out, f, n ** 3, ncells, scatter, torch.float64, (n,) * 3)
    bz_esbgk_imex_euler(BzEsbgkDesc(n, L, beta, mu0), BzImexDesc(dt, eps, _ptr(eps_cells)), _ptr(f), _ptr(tr),
                        _ptr(idx), ncells, _ptr(ncells_dev), _ptr(out), BZ_SCATTER if scatter else 0,
                        _stream(stream))
    return out


def esbgk_pr222_step(y, transport, L: float, dt: float, eps: float = 0.0, eps_cells=None, beta: float = -0.5,
                     mu0: float = 1.0, idx=None, out=None, stream=None):
    """One PR(2,2,2) step of the ES-BGK layer through bz_esbgk_pr222_*;
    `transport` maps a stage value to v . grad_x of it between the calls."""
    torch = _torch()
    n, ncells = _f64_cells(y, idx, None)
    desc, im, st = BzEsbgkDesc(n, L, beta, mu0), BzImexDesc(dt, eps, _ptr(eps_cells)), _stream(stream)
    y1, y2, a = torch.empty_like(y), torch.empty_like(y), torch.empty_like(y)
    out = torch.empty_like(y) if out is None else out
    bz_esbgk_pr222_stage1(desc, im, _ptr(y), _ptr(idx), ncells, 0, _ptr(y1), st)
    t1 = transport(y1).contiguous()
    bz_esbgk_pr222_stage2(desc, im, _ptr(y), _ptr(y1), _ptr(t1), _ptr(idx), ncells, 0, _ptr(y2), _ptr(a), st)
    t2 = transport(y2).contiguous()
    bz_esbgk_pr222_finish(desc, im, _ptr(a), _ptr(y2), _ptr(t2), _ptr(idx), ncells, 0, _ptr(out), st)
    return out


class Server:
    """A serving runtime whose arena is one torch uint8 tensor."""

    def __init__(self, arena_bytes: int, max_inflight: int = 8, n_streams: int = 4, max_queue: int = 4096,
                 device="cuda", slice_cells: int = 0):
        torch = _torch()
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        d = BzServerDesc()
        d.arena_dev, d.arena_bytes = _ptr(self.arena), arena_bytes
        d.max_inflight, d.n_streams, d.max_queue = max_inflight, n_streams, max_queue
        d.slice_cells = slice_cells
        torch.cuda.synchronize()
        self.handle = bz_server_create(d)
        self._keep = {}

    def submit(self, f, q, plan: BzPlanDesc, idx=None, ncells=None, scatter=False, client_id=0):
        torch = _torch()
        n3 = plan.n ** (2 if plan.dim == 2 else 3)
        rows_f = f.numel() // n3
        k = ncells if ncells is not None else (idx.numel() if idx is not None else rows_f)
        # the server reads and writes exactly the rows the request names: check the buffers hold them
        if (idx is None and k > rows_f) or (idx is not None and (idx.numel() < k or idx.dtype != torch.int32)):
            raise ValueError(f"request names {k} cells, f holds {rows_f} rows and idx {None if idx is None else idx.numel()}")
        out_dtype = torch.float64 if plan.project or plan.precision == BZ_FP64 else torch.float32
        if q.dtype != out_dtype or not q.is_contiguous() or not f.is_contiguous():
            raise ValueError(f"f must be contiguous and q a contiguous {out_dtype} tensor")
        if q.numel() // n3 < (rows_f if scatter else k):
            raise ValueError(f"q holds {q.numel() // n3} rows, the request writes up to row {(rows_f if scatter else k) - 1}")
        r = BzRequest()
        r.plan = plan
        r.f = _ptr(f)
        r.f_dtype = BZ_FP32 if f.dtype == torch.float32 else BZ_FP64
        r.idx = _ptr(idx)
        r.ncells = k
        r.q = _ptr(q)
        r.flags = BZ_SCATTER if scatter else 0
        r.client_id = client_id
        # the request's kernels wait for the work queued so far on the current stream (the writes of f, idx)
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(f.device))
        r.ready_event = ev.cuda_event
        t = bz_serve_submit(self.handle, r)
        if t is not None:
            self._keep[t] = (f, q, idx, plan, ev)
        return t

    def poll(self, ticket):
        done, res = bz_serve_poll(self.handle, ticket)
        if done:
            self._keep.pop(ticket, None)
        return done, res

    def stats(self) -> BzServerStats:
        return bz_server_stats_ex(self.handle)

    def close(self):
        if self.handle:
            bz_server_destroy(self.handle)
            self.handle = 0
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def realizability_mask(desc: BzMaskDesc, rho, ux, uy, T, eps, regime_in, l1dist=None, cell_flags=None,
                       with_diag=False, stream=None):
    """Run bz_realizability_mask on torch CUDA tensors; returns (regime_out,
    boltz_idx, counts, diag)."""
    torch = _torch()
    dev = rho.device
    ncell = desc.nx * desc.ny
    rout = torch.empty_like(regime_in)
    idx = torch.empty(ncell, dtype=torch.int32, device=dev)
    counts = torch.empty(2, dtype=torch.int32, device=dev)
    diag = torch.empty((ncell, 4), dtype=torch.float64, device=dev) if with_diag else None
    bz_realizability_mask(desc, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(eps), _ptr(regime_in),
                          _ptr(l1dist), _ptr(cell_flags), _ptr(rout), _ptr(idx), _ptr(counts),
                          _ptr(diag), _stream(stream))
    return rout, idx, counts, diag


def mask_desc(nx, ny, dx, dy, mu0=1.0, kappa0=15.0 / 4.0, eta0=1e-3, eta1=1e-4, delta0=1e-4,
              laplacian_u_mode=0) -> BzMaskDesc:
    d = BzMaskDesc()
    d.nx, d.ny, d.dx, d.dy = nx, ny, dx, dy
    d.mu0, d.kappa0, d.eta0, d.eta1, d.delta0 = mu0, kappa0, eta0, eta1, delta0
    d.laplacian_u_mode = laplacian_u_mode
    return d


def default_R(L: float) -> float:
    return (math.sqrt(2.0) - 1.0) * L
