"""Thin Python binding of libftlm (include/ftlm.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels or its host C++. Device buffers are torch tensors on a HIP device;
streams default to torch's current stream. Names mirror the C entry points
without the ``ftlm_`` prefix (``hv`` is ``ftlm_hv``).

Importing this module raises ImportError when libftlm.so is missing; there
is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libftlm.so")

OK, E_INVALID, E_RANGE, E_NOSPACE, E_DEVICE, E_AGAIN, E_REJECTED, E_NUMERIC = 0, -1, -2, -3, -4, -5, -6, -7
CLT, CR, FULL, LIN = 0, 1, 2, 3
F32, F64 = 0, 1
PM1, GAUSS, UNIT = 0, 1, 2
NONE = (1 << 64) - 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libftlm.so not found at {LIB_PATH}: build it with paper_2605_26261_amd/build.py")

# torch ships its own HIP runtime. It has to be the one in the process before
# libftlm.so is loaded, so that the library binds to it: a system HIP runtime
# loaded first leaves one of the two without the device ("no ROCm-capable
# device") once torch starts its own.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_vp, _u64, _i32, _i64, _sz, _dbl = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64,
                                    ctypes.c_size_t, ctypes.c_double)


class SectorResult(ctypes.Structure):
    """ftlm_sector_result."""
    _fields_ = [("n_up", ctypes.c_int32), ("R", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("two_s", ctypes.c_int32), ("dim", ctypes.c_uint64), ("mult", ctypes.c_double),
                ("theta", _vp), ("weight", _vp), ("steps", _vp)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("ftlm_last_error", ctypes.c_char_p, [])
_sig("ftlm_version", _i32, [])
_sig("ftlm_graph_create", _i32, [_i32, _i32, _vp, _vp, _vp, ctypes.POINTER(_vp)])
_sig("ftlm_graph_destroy", None, [_vp])
_sig("ftlm_graph_n_sites", _i32, [_vp])
_sig("ftlm_graph_n_bonds", _i32, [_vp])
_sig("ftlm_sector_info", _i32, [_i32, _i32, ctypes.POINTER(_u64), ctypes.POINTER(_dbl)])
_sig("ftlm_sector_table_bytes", _i32, [_i32, _i32, _i32, ctypes.POINTER(_sz)])
_sig("ftlm_sector_create", _i32, [_i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)])
_sig("ftlm_sector_dim", _u64, [_vp])
_sig("ftlm_sector_mode", _i32, [_vp])
_sig("ftlm_sector_destroy", None, [_vp])
_sig("ftlm_sector_info_spin", _i32, [_i32, _i32, _i32, ctypes.POINTER(_u64), ctypes.POINTER(_dbl)])
_sig("ftlm_sector_table_bytes_spin", _i32, [_i32, _i32, _i32, _i32, ctypes.POINTER(_sz)])
_sig("ftlm_sector_create_spin", _i32, [_i32, _i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)])
_sig("ftlm_sector_two_s", _i32, [_vp])
_sig("ftlm_rank", _i32, [_vp, _vp, _vp, _u64, _vp])
_sig("ftlm_unrank", _i32, [_vp, _vp, _vp, _u64, _vp])
_sig("ftlm_clt_export", _i32, [_vp, _vp, _vp, _u64, _vp])
_sig("ftlm_neighbors", _i32, [_vp, _vp, _u64, _u64, _vp, _vp])
_sig("ftlm_hv", _i32, [_vp, _vp, _vp, _vp, _i32, _i32, _vp])
_sig("ftlm_hv_rows", _i32, [_vp, _vp, _vp, _vp, _i32, _i32, _u64, _u64, _vp])
_sig("ftlm_start_vectors", _i32, [_vp, _u64, _u64, _i32, _i32, _i32, _vp, _vp, _vp, _sz, _vp])
_sig("ftlm_lanczos_workspace_bytes", _i32, [_vp, _i32, _i32, ctypes.POINTER(_sz)])
_sig("ftlm_lanczos", _i32, [_vp, _vp, _u64, _u64, _i32, _i32, _i32, _i32, _vp, _sz, _vp, _vp, _vp, _vp])
_sig("ftlm_lanczos_noalloc", _i32, [_vp, _vp, _u64, _u64, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp])
_sig("ftlm_plan_workspace_bytes", _i32, [_vp, _i32, _vp, _i32, _i32, _i32, ctypes.POINTER(_sz)])
_sig("ftlm_plan_create", _i32, [_vp, _i32, _vp, _i32, _i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)])
_sig("ftlm_plan_run", _i32, [_vp, _u64, _u64, _i32, _i32, _vp, _vp, _vp, _vp])
_sig("ftlm_plan_tune", _i32, [_vp, _vp, _vp])
_sig("ftlm_plan_destroy", None, [_vp])
_sig("ftlm_ritz", _i32, [_i32, _vp, _vp, _vp, _vp])
_sig("ftlm_ritz_batch", _i32, [_i32, _i32, _vp, _vp, _vp, _vp, _vp])
_sig("ftlm_ghosts", _i32, [_i32, _vp, _vp, _dbl, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_dbl)])
_sig("ftlm_seed_spread", _i32, [_i32, _i32, _vp, _vp, _vp])
_sig("ftlm_thermo", _i32, [_i32, _i32, ctypes.POINTER(SectorResult), _i32, _vp, _dbl, _vp, _vp, _vp, _vp])
_sig("ftlm_stats_enable", _i32, [_i32])
_sig("ftlm_stats_reset", _i32, [])
_sig("ftlm_stats_read", _i32, [ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)])


class Tuning(ctypes.Structure):
    """ftlm_tuning."""
    _fields_ = [("batch", ctypes.c_int32), ("n_candidates", ctypes.c_int32), ("widths", ctypes.c_int32 * 12),
                ("ms", ctypes.c_double * 12), ("ms_per_step", ctypes.c_double), ("cached", ctypes.c_int32)]


_sig("ftlm_autotune", _i32, [_vp, _vp, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(Tuning)])


class PlanTuning(ctypes.Structure):
    """ftlm_plan_tuning."""
    _fields_ = [("n_candidates", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("max_width", ctypes.c_int32 * 8), ("n_launches", ctypes.c_int32 * 8),
                ("ms", ctypes.c_double * 8)]


class ServerOpts(ctypes.Structure):
    """ftlm_server_opts."""
    _fields_ = [("mode", ctypes.c_int32), ("dtype", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("batch_same_n", ctypes.c_int32), ("steps_per_round", ctypes.c_int32)]


class Request(ctypes.Structure):
    """ftlm_request."""
    _fields_ = [("n_sites", ctypes.c_int32), ("n_bonds", ctypes.c_int32), ("bi", _vp), ("bj", _vp), ("J", _vp),
                ("n_up", ctypes.c_int32), ("R", ctypes.c_int32), ("M", ctypes.c_int32), ("dist", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("nT", ctypes.c_int32), ("reserved", ctypes.c_int32), ("T", _vp),
                ("g", ctypes.c_double)]


class ResultInfo(ctypes.Structure):
    """ftlm_result_info."""
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("status", ctypes.c_int32), ("steps", ctypes.c_int32), ("dim", ctypes.c_uint64),
                ("footprint", ctypes.c_uint64)]


_sig("ftlm_server_request_bytes", _i32, [ctypes.POINTER(Request), _i32, _i32, ctypes.POINTER(_sz)])
_sig("ftlm_server_create", _i32, [_vp, _sz, ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)])
_sig("ftlm_server_submit", _i32, [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)])
_sig("ftlm_server_poll", _i32, [_vp, ctypes.c_uint64, _vp, _vp, _vp, _vp, ctypes.POINTER(ResultInfo)])
_sig("ftlm_server_clock", ctypes.c_double, [_vp])
_sig("ftlm_server_stats", _i32, [_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                 ctypes.POINTER(ctypes.c_int32)])
_sig("ftlm_server_destroy", None, [_vp])


class FtlmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libftlm error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise FtlmError(rc, _lib.ftlm_last_error().decode())
    return rc


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    """Device pointer of a torch tensor (contiguous, on a HIP device)."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _empty_device(nbytes, device="cuda"):
    import torch
    return torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device=device)


def version():
    return _lib.ftlm_version()


class Graph:
    """ftlm_graph: bonds [(i, j, J)] on n_sites sites."""

    def __init__(self, n_sites, bonds):
        bi = np.ascontiguousarray([b[0] for b in bonds], dtype=np.int32)
        bj = np.ascontiguousarray([b[1] for b in bonds], dtype=np.int32)
        J = np.ascontiguousarray([b[2] for b in bonds], dtype=np.float64)
        h = _vp()
        _check(_lib.ftlm_graph_create(n_sites, len(bonds), _hptr(bi), _hptr(bj), _hptr(J), ctypes.byref(h)))
        self.handle = h
        self.n_sites = n_sites

    @property
    def n_bonds(self):
        return _lib.ftlm_graph_n_bonds(self.handle)

    def __del__(self, _destroy=_lib.ftlm_graph_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


def sector_info(n_sites, n_up):
    """ftlm_sector_info: (D, multiplicity) of the sector n_up of n_sites sites."""
    d, m = _u64(), _dbl()
    _check(_lib.ftlm_sector_info(n_sites, n_up, ctypes.byref(d), ctypes.byref(m)))
    return int(d.value), float(m.value)


def sector_table_bytes(n_sites, n_up, mode):
    n = _sz()
    _check(_lib.ftlm_sector_table_bytes(n_sites, n_up, mode, ctypes.byref(n)))
    return n.value


def sector_info_spin(n_sites, two_s, a_tot):
    """ftlm_sector_info_spin: (D, multiplicity) of the sector with digit sum
    a_tot of N sites of spin two_s / 2."""
    d, m = _u64(), _dbl()
    _check(_lib.ftlm_sector_info_spin(n_sites, two_s, a_tot, ctypes.byref(d), ctypes.byref(m)))
    return int(d.value), float(m.value)


def sector_table_bytes_spin(n_sites, two_s, a_tot, mode):
    n = _sz()
    _check(_lib.ftlm_sector_table_bytes_spin(n_sites, two_s, a_tot, mode, ctypes.byref(n)))
    return n.value


class Sector:
    """ftlm_sector with its device table buffer (owned by this object).
    n_up is the sector's digit sum A (Eq. 17) when two_s = 2s > 1."""

    def __init__(self, n_sites, n_up, mode, device="cuda", stream=None, table=None, two_s=1):
        nbytes = sector_table_bytes_spin(n_sites, two_s, n_up, mode)
        self.table = table if table is not None else _empty_device(nbytes, device)
        if self.table.numel() < nbytes:
            raise ValueError(f"table holds {self.table.numel()} bytes, {nbytes} needed")
        h = _vp()
        _check(_lib.ftlm_sector_create_spin(n_sites, two_s, n_up, mode, _dptr(self.table), self.table.numel(),
                                            _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.n_sites, self.n_up, self.mode, self.two_s = n_sites, n_up, mode, two_s

    @property
    def dim(self):
        return int(_lib.ftlm_sector_dim(self.handle))

    def __del__(self, _destroy=_lib.ftlm_sector_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


def _need_u64(*ts):
    """The C ABI takes uint64 arrays: 8-byte integer tensors of one length."""
    import torch
    for t in ts:
        if t.dtype not in (torch.int64, torch.uint64):
            raise ValueError("labels and indices must be 8-byte integer tensors")
    if len({t.numel() for t in ts}) != 1:
        raise ValueError("labels and indices must have the same number of entries")


def rank(sector, labels, idx, stream=None):
    _need_u64(labels, idx)
    _check(_lib.ftlm_rank(sector.handle, _dptr(labels), _dptr(idx), labels.numel(), _stream(stream)))


def unrank(sector, idx, labels, stream=None):
    _need_u64(idx, labels)
    _check(_lib.ftlm_unrank(sector.handle, _dptr(idx), _dptr(labels), idx.numel(), _stream(stream)))


def clt_export(sector, nblocks, stream=None):
    mask = np.empty(nblocks, dtype=np.uint32)
    prefix = np.empty(nblocks, dtype=np.uint32)
    _check(_lib.ftlm_clt_export(sector.handle, _hptr(mask), _hptr(prefix), nblocks, _stream(stream)))
    return mask, prefix


def neighbors(sector, graph, t0, count, out, stream=None):
    import torch
    per_row = graph.n_bonds * (2 if getattr(sector, "two_s", 1) > 1 else 1)
    if out.dtype not in (torch.int64, torch.uint64) or out.numel() < count * per_row:
        raise ValueError("out must be an 8-byte integer tensor of at least count * n_bonds entries "
                         "(2 * n_bonds for general spin)")
    _check(_lib.ftlm_neighbors(sector.handle, graph.handle, t0, count, _dptr(out), _stream(stream)))


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise ValueError("vectors must be float32 or float64")


def _vector_block(x, rows, what="x"):
    """Number of columns of a [rows] or [rows, B] vector block."""
    if x.dim() not in (1, 2) or x.shape[0] != rows:
        raise ValueError(f"{what} must have shape [{rows}] or [{rows}, B], got {tuple(x.shape)}")
    return 1 if x.dim() == 1 else x.shape[1]


def _same_block(x, y):
    if y.dtype != x.dtype:
        raise ValueError(f"y has dtype {y.dtype}, x has {x.dtype}")


def hv(sector, graph, x, y, stream=None):
    """y = H x for x, y of shape [D] or [D, B]."""
    nvec = _vector_block(x, sector.dim)
    _same_block(x, y)
    if y.shape != x.shape:
        raise ValueError(f"y has shape {tuple(y.shape)}, x has {tuple(x.shape)}")
    _check(_lib.ftlm_hv(sector.handle, graph.handle, _dptr(x), _dptr(y), nvec, _dtype_code(x), _stream(stream)))


def hv_rows(sector, graph, x, y, row0, nrows, stream=None):
    nvec = _vector_block(x, sector.dim)
    _same_block(x, y)
    if y.dim() != x.dim() or y.shape[0] < nrows or y.shape[1:] != x.shape[1:]:
        raise ValueError(f"y must hold at least nrows = {nrows} rows of the columns of x")
    _check(_lib.ftlm_hv_rows(sector.handle, graph.handle, _dptr(x), _dptr(y), nvec, _dtype_code(x),
                             row0, nrows, _stream(stream)))


def lanczos_workspace_bytes(sector, R, dtype):
    n = _sz()
    _check(_lib.ftlm_lanczos_workspace_bytes(sector.handle, R, dtype, ctypes.byref(n)))
    return n.value


def start_vectors(sector, seed, r0, R, dist, q, work, stream=None):
    """Writes R start vectors into q [D, R]; returns their FP64 norms."""
    if _vector_block(q, sector.dim, "q") != R:
        raise ValueError(f"q must hold R = {R} columns")
    if work.numel() < lanczos_workspace_bytes(sector, R, _dtype_code(q)):
        raise ValueError("work is smaller than lanczos_workspace_bytes(sector, R, dtype)")
    norms = np.empty(R, dtype=np.float64)
    _check(_lib.ftlm_start_vectors(sector.handle, seed, r0, R, dist, _dtype_code(q), _dptr(q), _hptr(norms),
                                   _dptr(work), work.numel(), _stream(stream)))
    return norms


def lanczos(sector, graph, seed, r0, R, M, dist, dtype, work=None, stream=None):
    """R Lanczos chains; returns (alpha [R, M], beta [R, M], steps [R])."""
    if work is None:
        work = _empty_device(lanczos_workspace_bytes(sector, R, dtype), sector.table.device)
    alpha = np.zeros((R, M), dtype=np.float64)
    beta = np.zeros((R, M), dtype=np.float64)
    steps = np.zeros(R, dtype=np.int32)
    _check(_lib.ftlm_lanczos(sector.handle, graph.handle, seed, r0, R, M, dist, dtype, _dptr(work), work.numel(),
                             _hptr(alpha), _hptr(beta), _hptr(steps), _stream(stream)))
    return alpha, beta, steps


NOALLOC_SCRATCH_BYTES = 32 << 20  # FTLM_NOALLOC_SCRATCH_BYTES


def lanczos_noalloc(sector, graph, seed, r0, R, M, dist, dtype, stream=None):
    """ftlm_lanczos_noalloc: lanczos() with the workspace in the library's
    per-device array (no device allocation); returns (alpha, beta, steps)."""
    alpha = np.zeros((R, M), dtype=np.float64)
    beta = np.zeros((R, M), dtype=np.float64)
    steps = np.zeros(R, dtype=np.int32)
    _check(_lib.ftlm_lanczos_noalloc(sector.handle, graph.handle, seed, r0, R, M, dist, dtype, _hptr(alpha),
                                     _hptr(beta), _hptr(steps), _stream(stream)))
    return alpha, beta, steps


def autotune(sector, graph, R, dtype, work=None, stream=None):
    """Batch width for R chains of this sector (ftlm_autotune); returns a dict."""
    if work is None:
        work = _empty_device(lanczos_workspace_bytes(sector, R, dtype), sector.table.device)
    t = Tuning()
    _check(_lib.ftlm_autotune(sector.handle, graph.handle, R, dtype, _dptr(work), work.numel(), _stream(stream),
                              ctypes.byref(t)))
    return {"batch": t.batch, "ms_per_step": t.ms_per_step, "cached": bool(t.cached),
            "candidates": {t.widths[i]: t.ms[i] for i in range(t.n_candidates)}}


def plan_workspace_bytes(graph, n_ups, mode, R, dtype):
    nu = np.ascontiguousarray(n_ups, dtype=np.int32)
    n = _sz()
    _check(_lib.ftlm_plan_workspace_bytes(graph.handle, len(nu), _hptr(nu), mode, R, dtype, ctypes.byref(n)))
    return n.value


class Plan:
    """ftlm_plan: R chains in each listed sector, one launch per kernel per
    Lanczos step over all sectors; owns its device arena."""

    def __init__(self, graph, n_ups, mode, R, M, dtype, device="cuda", stream=None):
        self.n_ups = [int(v) for v in n_ups]
        nu = np.ascontiguousarray(self.n_ups, dtype=np.int32)
        self.arena = _empty_device(plan_workspace_bytes(graph, nu, mode, R, dtype), device)
        h = _vp()
        _check(_lib.ftlm_plan_create(graph.handle, len(nu), _hptr(nu), mode, R, M, dtype, _dptr(self.arena),
                                     self.arena.numel(), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.R, self.M = R, M

    def run(self, seed, dist, r0=0, use_graph=True, stream=None):
        """Returns alpha, beta [S, R, M] and steps [S, R]."""
        S = len(self.n_ups)
        alpha = np.zeros((S, self.R, self.M))
        beta = np.zeros((S, self.R, self.M))
        steps = np.zeros((S, self.R), dtype=np.int32)
        _check(_lib.ftlm_plan_run(self.handle, seed, r0, dist, 1 if use_graph else 0, _hptr(alpha), _hptr(beta),
                                  _hptr(steps), _stream(stream)))
        return alpha, beta, steps

    def tune(self, stream=None):
        """ftlm_plan_tune: keeps the fastest split of the R columns into
        launches; returns the candidates {max_width: (launches, ms)} and the
        chosen max_width."""
        t = PlanTuning()
        _check(_lib.ftlm_plan_tune(self.handle, _stream(stream), ctypes.byref(t)))
        cands = {int(t.max_width[i]): (int(t.n_launches[i]), float(t.ms[i])) for i in range(t.n_candidates)}
        return {"candidates": cands, "max_width": int(t.max_width[t.chosen])}

    def __del__(self, _destroy=_lib.ftlm_plan_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


def _request(n_sites, bonds, n_up, R, M, seed, dist, temps, g):
    """ftlm_request plus the arrays it points to (kept alive by the caller)."""
    bi = np.ascontiguousarray([b[0] for b in bonds], dtype=np.int32)
    bj = np.ascontiguousarray([b[1] for b in bonds], dtype=np.int32)
    J = np.ascontiguousarray([b[2] for b in bonds], dtype=np.float64)
    T = np.ascontiguousarray(temps, dtype=np.float64)
    q = Request(n_sites, len(bonds), bi.ctypes.data, bj.ctypes.data, J.ctypes.data, n_up, R, M, dist, seed,
                len(T), 0, T.ctypes.data, g)
    return q, (bi, bj, J, T)


def server_request_bytes(n_sites, bonds, n_up, R, M, mode, dtype, temps=(1.0,)):
    q, keep = _request(n_sites, bonds, n_up, R, M, 0, PM1, temps, 1.0)
    n = _sz()
    _check(_lib.ftlm_server_request_bytes(ctypes.byref(q), mode, dtype, ctypes.byref(n)))
    return n.value


class Server:
    """ftlm_server: continuous-batching FTLM request server over a device arena."""

    def __init__(self, arena_bytes, mode=CR, dtype=F32, max_active=0, batch_same_n=True, device="cuda",
                 steps_per_round=0):
        self.arena = _empty_device(arena_bytes, device)
        opts = ServerOpts(mode, dtype, max_active, 1 if batch_same_n else 0, steps_per_round)
        h = _vp()
        _check(_lib.ftlm_server_create(_dptr(self.arena), self.arena.numel(), ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h
        self.nT = {}

    def submit(self, n_sites, bonds, n_up, R, M, seed, dist, temps, g=1.0):
        q, keep = _request(n_sites, bonds, n_up, R, M, seed, dist, temps, g)
        rid = ctypes.c_uint64()
        _check(_lib.ftlm_server_submit(self.handle, ctypes.byref(q), ctypes.byref(rid)))
        self.nT[rid.value] = len(keep[3])
        return rid.value

    def poll(self, rid):
        """None while pending; else dict E, C, chi, lnZ, t_submit, t_admit, t_done, steps, dim."""
        n = self.nT[rid]
        out = {k: np.empty(n) for k in ("E", "C", "chi", "lnZ")}
        info = ResultInfo()
        rc = _lib.ftlm_server_poll(self.handle, rid, _hptr(out["E"]), _hptr(out["C"]), _hptr(out["chi"]),
                                   _hptr(out["lnZ"]), ctypes.byref(info))
        if rc == E_AGAIN:
            return None
        del self.nT[rid]
        _check(rc)
        out.update(t_submit=info.t_submit, t_admit=info.t_admit, t_done=info.t_done, steps=info.steps,
                   dim=info.dim, footprint=info.footprint)
        return out

    def clock(self):
        return _lib.ftlm_server_clock(self.handle)

    def stats(self):
        peak, rounds, active = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int32()
        _check(_lib.ftlm_server_stats(self.handle, ctypes.byref(peak), ctypes.byref(rounds), ctypes.byref(active)))
        return {"peak_bytes": peak.value, "rounds": rounds.value, "active": active.value}

    def close(self, _destroy=_lib.ftlm_server_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def ritz(alpha, beta, m=None):
    """Ritz values and weights of the m x m tridiagonal matrix (host FP64)."""
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    m = len(alpha) if m is None else m
    theta = np.empty(m, dtype=np.float64)
    weight = np.empty(m, dtype=np.float64)
    _check(_lib.ftlm_ritz(m, _hptr(alpha), _hptr(beta), _hptr(theta), _hptr(weight)))
    return theta, weight


def ghosts(alpha, beta, m=None, c_tau=1.0):
    """ftlm_ghosts: Cullum-Willoughby ghost test (Eq. 25) and Ritz clusters of
    one chain; returns a dict of theta, weight, ell, ghost (bool), cluster,
    cluster_weight (per cluster) and tau."""
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    m = len(alpha) if m is None else m
    if m < 1 or m > len(alpha) or (m > 1 and len(beta) < m - 1):
        raise ValueError("alpha needs m entries and beta m - 1")
    theta, weight, ell, cw = (np.empty(m, dtype=np.float64) for _ in range(4))
    ghost, cluster = np.empty(m, dtype=np.int32), np.empty(m, dtype=np.int32)
    nc, tau = _i32(), _dbl()
    _check(_lib.ftlm_ghosts(m, _hptr(alpha), _hptr(beta), c_tau, _hptr(theta), _hptr(weight), _hptr(ell),
                            _hptr(ghost), _hptr(cluster), _hptr(cw), ctypes.byref(nc), ctypes.byref(tau)))
    return {"theta": theta, "weight": weight, "ell": ell, "ghost": ghost.astype(bool), "cluster": cluster,
            "cluster_weight": cw[:nc.value].copy(), "tau": tau.value}


def seed_spread(estimates):
    """ftlm_seed_spread: (mean, sigma_emp) over the rows of [N_s][n] (Eq. 22)."""
    v = np.ascontiguousarray(estimates, dtype=np.float64)
    if v.ndim < 1 or v.shape[0] < 1:
        raise ValueError("estimates need at least one seed (one row)")
    shape = v.shape[1:]
    v = v.reshape(v.shape[0], -1)
    mean = np.empty(v.shape[1], dtype=np.float64)
    sigma = np.empty(v.shape[1], dtype=np.float64)
    _check(_lib.ftlm_seed_spread(v.shape[0], v.shape[1], _hptr(v), _hptr(mean), _hptr(sigma)))
    return mean.reshape(shape), sigma.reshape(shape)


def ritz_batch(alpha, beta, steps):
    """ftlm_ritz_batch: Ritz values and weights of every chain of [R][M]
    alpha/beta rows, chain r over its first steps[r] entries; returns [R][M]
    theta and weight (zeros past steps[r])."""
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    R, M = alpha.shape
    if beta.shape != (R, M) or steps.shape != (R,):
        raise ValueError("alpha and beta must be [R][M] and steps [R]")
    theta = np.empty((R, M), dtype=np.float64)
    weight = np.empty((R, M), dtype=np.float64)
    _check(_lib.ftlm_ritz_batch(R, M, _hptr(steps), _hptr(alpha), _hptr(beta), _hptr(theta), _hptr(weight)))
    return theta, weight


def thermo(n_sites, sectors, temps, g=1.0):
    """sectors: list of dicts n_up, dim, mult, theta [R, S], weight [R, S], steps [R]."""
    keep = []
    recs = (SectorResult * len(sectors))()
    for i, s in enumerate(sectors):
        th = np.ascontiguousarray(s["theta"], dtype=np.float64)
        w = np.ascontiguousarray(s["weight"], dtype=np.float64)
        st = np.ascontiguousarray(s["steps"], dtype=np.int32)
        keep += [th, w, st]
        recs[i] = SectorResult(s["n_up"], th.shape[0], th.shape[1], int(s.get("two_s", 1)), s["dim"], s["mult"],
                               th.ctypes.data, w.ctypes.data, st.ctypes.data)
    temps = np.ascontiguousarray(temps, dtype=np.float64)
    out = {k: np.empty(len(temps)) for k in ("E", "C", "chi", "lnZ")}
    _check(_lib.ftlm_thermo(n_sites, len(sectors), recs, len(temps), _hptr(temps), g, _hptr(out["E"]),
                            _hptr(out["C"]), _hptr(out["chi"]), _hptr(out["lnZ"])))
    return out


def stats_enable(on=True):
    _check(_lib.ftlm_stats_enable(1 if on else 0))


def stats_reset():
    _check(_lib.ftlm_stats_reset())


def stats_read():
    n = _i64()
    ms = ctypes.c_double()
    _check(_lib.ftlm_stats_read(ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def exported_symbols():
    """Names of the C entry points this binding loads."""
    return [n for n in dir(_lib) if n.startswith("ftlm_")]
