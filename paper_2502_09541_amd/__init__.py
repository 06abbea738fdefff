"""Python binding of the vx C ABI (include/vx.h): argument marshalling only.

Every step of the join / aggregate / partition path runs in the HIP library
``libvx.so`` built from ``csrc/`` by :func:`paper_2502_09541_amd.build.build`.
PyTorch provides the device arena (a uint8 CUDA tensor) and the compute
stream; pinned host columns come from :class:`HostBuffer` (vx_host_alloc) or
any page-locked numpy/torch buffer.

Importing this module does not load the library; the first call does, and it
raises if the library was not built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvx.so")
_lib = None

VX_OK, VX_EINVAL, VX_EBUDGET, VX_ENOMEM, VX_EHIP, VX_ENOTPINNED, VX_ECAPACITY, VX_EUNSUPPORTED, \
    VX_EDUPKEY = range(9)
STATUS_NAMES = ["VX_OK", "VX_EINVAL", "VX_EBUDGET", "VX_ENOMEM", "VX_EHIP", "VX_ENOTPINNED",
                "VX_ECAPACITY", "VX_EUNSUPPORTED", "VX_EDUPKEY"]
VX_I32, VX_I64 = 1, 2
VX_UNIQUE, VX_PREAGG, VX_HASHED = 1, 2, 4
VX_LATE_AUTO, VX_LATE_SDMA, VX_LATE_ZC, VX_LATE_PAPER = -1, 0, 1, 2
VX_PROBE_COUNT_ZC = 1
VX_JOIN_PLAIN, VX_JOIN_STAR, VX_JOIN_BATCH, VX_JOIN_PARTITIONED, VX_JOIN_RADIX = 1, 2, 3, 4, 5
(VX_PART_AUTO, VX_PART_RADIX_HASH, VX_PART_RADIX_BITS, VX_PART_LEARNED, VX_PART_QUANTILE,
 VX_PART_UNTRAINED, VX_PART_RANGE) = range(7)
PART_METHODS = {"auto": 0, "radix_hash": 1, "radix_bits": 2, "learned": 3, "quantile": 4,
                "untrained": 5, "range": 6}


class VxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


# ----------------------------------------------------------------------------- ABI structs

class Col(C.Structure):
    _fields_ = [("data", C.c_void_p), ("type", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("rows", C.c_uint64), ("chunks", C.c_uint64), ("chunk_rows", C.c_uint64),
                ("sdma_bytes", C.c_uint64), ("zc_bytes", C.c_uint64), ("zc_mask", C.c_uint32),
                ("n_buffers", C.c_uint32), ("build_ms", C.c_double), ("probe_ms", C.c_double),
                ("total_ms", C.c_double), ("kernel_ms", C.c_double), ("kernel_launches", C.c_uint64),
                ("table_bytes", C.c_uint64), ("n_parts", C.c_uint64), ("imbalance", C.c_double),
                ("part_ms", C.c_double), ("train_ms", C.c_double), ("singleton_rows", C.c_uint64),
                ("survivors", C.c_uint64), ("imbalance_tables", C.c_double),
                ("imbalance_distinct", C.c_double), ("zc_counted", C.c_uint32), ("reserved", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LinkCalib(C.Structure):
    _fields_ = [("h2d_gbs", C.c_double), ("zc_read_gbs", C.c_double), ("hbm_read_gbs", C.c_double),
                ("zc_granule", C.c_uint32), ("zc_stride_bytes", C.c_uint32 * 8),
                ("zc_stride_gelems", C.c_double * 8), ("d2h_gbs", C.c_double), ("duplex_sdma_gbs", C.c_double),
                ("zc_write_gbs", C.c_double), ("duplex_zcw_gbs", C.c_double), ("duplex_zcr_gbs", C.c_double)]


class JoinRows(C.Structure):
    _fields_ = [("row", C.c_void_p), ("build_pay", C.c_void_p * 4), ("probe_pay", C.c_void_p * 4),
                ("cap", C.c_uint64), ("n_out", C.c_uint64)]


class BuildDesc(C.Structure):
    _fields_ = [("key", Col), ("pay", C.POINTER(Col)), ("n_pay", C.c_uint32), ("flags", C.c_uint32),
                ("n", C.c_uint64), ("load_factor", C.c_float), ("reserved", C.c_uint32)]


class Agg(C.Structure):
    _fields_ = [("match_count", C.c_uint64), ("sum", C.c_uint64 * 8)]

    def to_list(self, nsums):
        return [int(self.match_count)] + [int(self.sum[i]) for i in range(nsums)]


class ProbeDesc(C.Structure):
    _fields_ = [("key", Col), ("pay", C.POINTER(Col)), ("n_pay", C.c_uint32), ("late_mat", C.c_int32),
                ("n", C.c_uint64), ("chunk_rows", C.c_uint64), ("n_buffers", C.c_uint32),
                ("flags", C.c_uint32), ("chunk_aggs", C.POINTER(Agg)), ("chunk_aggs_cap", C.c_uint64)]


class StarDim(C.Structure):
    _fields_ = [("key", Col), ("n", C.c_uint64), ("filter", Col), ("lo", C.c_int64), ("hi", C.c_int64),
                ("group", Col)]


class GroupRow(C.Structure):
    _fields_ = [("g0", C.c_int32), ("g1", C.c_int32), ("count", C.c_uint64), ("sum", C.c_uint64 * 4)]


class StarJoin(C.Structure):
    _fields_ = [("n_dims", C.c_uint32), ("n_measures", C.c_uint32), ("dims", StarDim * 4),
                ("fact_fk", Col * 4), ("measure", Col * 4), ("n_fact", C.c_uint64),
                ("chunk_rows", C.c_uint64), ("late_mat", C.c_int32), ("flags", C.c_uint32),
                ("groups", C.POINTER(GroupRow)), ("groups_cap", C.c_uint64)]


class BatchJoin(C.Structure):
    _fields_ = [("n_jobs", C.c_uint32), ("mode", C.c_int32), ("build_key", C.POINTER(Col)),
                ("build_pay", C.POINTER(Col)), ("n_build", C.POINTER(C.c_uint64)),
                ("probe_key", C.POINTER(Col)), ("n_probe", C.POINTER(C.c_uint64)),
                ("out", C.POINTER(Agg)), ("tile_rows", C.c_uint32), ("block", C.c_uint32),
                ("load_factor", C.c_float), ("flags", C.c_uint32)]


class PartOpts(C.Structure):
    _fields_ = [("method", C.c_uint32), ("n_parts", C.c_uint32), ("shift", C.c_uint32),
                ("train_steps", C.c_uint32), ("sample_frac", C.c_float), ("lr", C.c_float),
                ("seed", C.c_uint64), ("splitters", C.POINTER(C.c_int64)), ("n_splitters", C.c_uint32),
                ("reserved", C.c_uint32)]


class SortDesc(C.Structure):
    _fields_ = [("key", Col), ("n", C.c_uint64), ("chunk_rows", C.c_uint64), ("n_buffers", C.c_uint32),
                ("reserved", C.c_uint32)]


class PartitionedJoin(C.Structure):
    _fields_ = [("build", BuildDesc), ("probe", ProbeDesc), ("part", PartOpts)]


class RadixJoin(C.Structure):
    _fields_ = [("a", BuildDesc), ("b", ProbeDesc), ("n_parts", C.c_uint32), ("shift", C.c_uint32),
                ("hash", C.c_uint32), ("placement", C.c_int32)]


class _PlainJoin(C.Structure):
    _fields_ = [("build", BuildDesc), ("probe", ProbeDesc)]


class _JoinUnion(C.Union):
    _fields_ = [("plain", _PlainJoin), ("star", StarJoin), ("batch", BatchJoin),
                ("part", PartitionedJoin), ("radix", RadixJoin)]


class JoinDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("u", _JoinUnion)]


class JoinOut(C.Structure):
    _fields_ = [("agg", Agg), ("n_groups", C.c_uint64), ("part_method_used", C.c_uint32),
                ("reserved", C.c_uint32), ("stats", Stats)]


class PartitionDesc(C.Structure):
    _fields_ = [("key", Col), ("pay", C.POINTER(Col)), ("n_pay", C.c_uint32), ("reserved", C.c_uint32),
                ("n", C.c_uint64), ("opts", PartOpts), ("out_key", C.c_void_p),
                ("out_pay", C.POINTER(C.c_void_p))]


class PartitionOut(C.Structure):
    _fields_ = [("method_used", C.c_uint32), ("n_parts", C.c_uint32), ("hist", C.POINTER(C.c_uint64)),
                ("boundary", C.POINTER(C.c_uint64)), ("splitters", C.POINTER(C.c_int64)),
                ("n_parts_cap", C.c_uint32), ("n_splitters", C.c_uint32), ("imbalance", C.c_double),
                ("est_imbalance_radix", C.c_double), ("est_imbalance_range", C.c_double),
                ("final_loss", C.c_double), ("model", C.POINTER(C.c_float))]


EXPORTS = ["vx_ctx_create", "vx_ctx_destroy", "vx_last_error", "vx_ctx_arena_used", "vx_host_alloc",
           "vx_host_free", "vx_build", "vx_table_destroy", "vx_probe_stream", "vx_join_agg",
           "vx_partition", "vx_cdf_loss_grad", "vx_cdf_forward", "vx_cdf_train", "vx_calibrate",
           "vx_probe_rows", "vx_sort", "vx_merge_cuts", "vx_join_plain_noalloc"]
N_MODEL_PARAMS = 193


def lib():
    """Load libvx.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    L.vx_ctx_create.argtypes = [C.c_int, vp, C.c_uint64, vp, C.POINTER(vp)]
    L.vx_ctx_destroy.argtypes = [vp]
    L.vx_last_error.restype = C.c_char_p
    L.vx_ctx_arena_used.argtypes = [vp]
    L.vx_ctx_arena_used.restype = C.c_uint64
    L.vx_host_alloc.argtypes = [C.c_uint64, C.POINTER(vp)]
    L.vx_host_free.argtypes = [vp]
    L.vx_build.argtypes = [vp, C.POINTER(BuildDesc), C.POINTER(vp)]
    L.vx_table_destroy.argtypes = [vp]
    L.vx_probe_stream.argtypes = [vp, vp, C.POINTER(ProbeDesc), C.POINTER(Agg), C.POINTER(Stats)]
    L.vx_probe_rows.argtypes = [vp, vp, C.POINTER(ProbeDesc), C.POINTER(JoinRows), C.POINTER(Agg), C.POINTER(Stats)]
    L.vx_join_agg.argtypes = [vp, C.POINTER(JoinDesc), C.POINTER(JoinOut)]
    L.vx_partition.argtypes = [vp, C.POINTER(PartitionDesc), C.POINTER(PartitionOut)]
    fp = C.POINTER(C.c_float)
    L.vx_cdf_loss_grad.argtypes = [vp, vp, vp, C.c_uint64, fp, fp, C.POINTER(C.c_double)]
    L.vx_cdf_forward.argtypes = [vp, vp, C.c_uint64, fp, fp]
    L.vx_cdf_train.argtypes = [vp, vp, vp, C.c_uint64, fp, C.c_uint32, C.c_float, C.POINTER(C.c_double)]
    L.vx_calibrate.argtypes = [vp, vp, C.c_uint64, C.POINTER(LinkCalib)]
    L.vx_sort.argtypes = [vp, C.POINTER(SortDesc), C.POINTER(Stats)]
    L.vx_merge_cuts.argtypes = [C.POINTER(C.POINTER(C.c_int64)), C.POINTER(C.c_uint64), C.c_uint32, C.c_uint64,
                                C.POINTER(C.c_uint64)]
    L.vx_join_plain_noalloc.argtypes = [C.POINTER(BuildDesc), C.POINTER(ProbeDesc), vp, vp]
    for name in ("vx_join_plain_noalloc", "vx_ctx_create", "vx_ctx_destroy", "vx_host_alloc", "vx_host_free", "vx_build",
                 "vx_table_destroy", "vx_probe_stream", "vx_join_agg", "vx_partition",
                 "vx_cdf_loss_grad", "vx_cdf_forward", "vx_cdf_train", "vx_calibrate", "vx_sort",
                 "vx_merge_cuts", "vx_probe_rows"):
        getattr(L, name).restype = st
    _lib = L
    return L


def _check(status):
    if status != VX_OK:
        raise VxError(status, lib().vx_last_error().decode())


# ----------------------------------------------------------------------------- memory

class HostBuffer:
    """Pinned, device-mapped host memory from vx_host_alloc, viewed as a numpy array."""

    def __init__(self, n, dtype):
        self.dtype = np.dtype(dtype)
        self.n = int(n)
        p = C.c_void_p()
        _check(lib().vx_host_alloc(max(1, self.n * self.dtype.itemsize), C.byref(p)))
        self.ptr = p.value
        buf = (C.c_byte * max(1, self.n * self.dtype.itemsize)).from_address(self.ptr)
        self.array = np.frombuffer(buf, dtype=self.dtype, count=self.n)

    def free(self):
        if self.ptr:
            self.array = None
            lib().vx_host_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


_TORCH_TYPES = None


def _torch_types():
    global _TORCH_TYPES
    if _TORCH_TYPES is None:
        import torch
        _TORCH_TYPES = {torch.int32: VX_I32, torch.int64: VX_I64}
    return _TORCH_TYPES


def col(x):
    """A vx_col for a CUDA tensor, a numpy array (pinned host memory) or a HostBuffer."""
    if isinstance(x, HostBuffer):
        x = x.array
    if isinstance(x, np.ndarray):
        if not x.flags.c_contiguous:
            raise ValueError("columns must be contiguous")
        t = {np.dtype(np.int32): VX_I32, np.dtype(np.int64): VX_I64}.get(x.dtype)
        if t is None:
            raise TypeError(f"column dtype {x.dtype} is not int32/int64")
        return Col(x.ctypes.data if x.size else None, t, 0)
    import torch
    if isinstance(x, torch.Tensor):
        if not x.is_contiguous():
            raise ValueError("columns must be contiguous")
        t = _torch_types().get(x.dtype)
        if t is None:
            raise TypeError(f"column dtype {x.dtype} is not int32/int64")
        return Col(x.data_ptr() if x.numel() else None, t, 0)
    raise TypeError(f"unsupported column object {type(x)}")


_COL_NP = np.dtype([("data", "<u8"), ("type", "<i4"), ("reserved", "<i4")])


def _col_array(xs, none_ok=False):
    """A vx_col array and a uint64 length array for a list of columns (None entries allowed with
    none_ok: a null int32 column of length 0).  Contiguous int32/int64 tensors take a short path;
    anything else goes through col()."""
    J = len(xs)
    arr = (Col * max(1, J))()
    lens = (C.c_uint64 * max(1, J))()
    if not J:
        return arr, lens
    import torch
    types, tensor = _torch_types(), torch.Tensor
    ptr, typ, ln = [0] * J, [VX_I32] * J, [0] * J
    for i, x in enumerate(xs):
        if x is None and none_ok:
            continue
        t = types.get(x.dtype) if isinstance(x, tensor) else None
        if t is not None and x.dim() == 1 and x.is_contiguous():
            n = x.numel()
            ptr[i], typ[i], ln[i] = x.data_ptr() if n else 0, t, n
        else:
            c = col(x)
            ptr[i], typ[i], ln[i] = c.data or 0, c.type, _len(x)
    v = np.frombuffer(arr, dtype=_COL_NP, count=J)
    v["data"] = ptr
    v["type"] = typ
    np.frombuffer(lens, dtype=np.uint64, count=J)[:] = ln
    return arr, lens


def _cols(xs):
    xs = list(xs or [])
    arr = (Col * max(1, len(xs)))(*[col(x) for x in xs])
    return arr, len(xs)


# ----------------------------------------------------------------------------- context

class Context:
    """A vx_ctx over a torch-allocated device arena of `budget_bytes`."""

    def __init__(self, budget_bytes, device=0, stream=None):
        import torch
        self.device = device
        self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = C.c_void_p()
        _check(lib().vx_ctx_create(device, self.arena.data_ptr(), int(budget_bytes),
                                   C.c_void_p(s.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().vx_ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def calibrate(self, nbytes=1 << 30):
        """vx_calibrate over a fresh pinned buffer; returns a dict of the measured rates."""
        hb = HostBuffer(nbytes // 8, np.int64)
        hb.array[:] = 1
        c = LinkCalib()
        try:
            _check(lib().vx_calibrate(self.h, hb.ptr, nbytes, C.byref(c)))
        finally:
            hb.free()
        return {"h2d_gbs": c.h2d_gbs, "zc_read_gbs": c.zc_read_gbs, "hbm_read_gbs": c.hbm_read_gbs,
                "zc_granule": c.zc_granule, "d2h_gbs": c.d2h_gbs, "duplex_sdma_gbs": c.duplex_sdma_gbs,
                "zc_write_gbs": c.zc_write_gbs, "duplex_zcw_gbs": c.duplex_zcw_gbs,
                "duplex_zcr_gbs": c.duplex_zcr_gbs,
                "zc_stride": {int(c.zc_stride_bytes[i]): c.zc_stride_gelems[i] for i in range(8)}}

    def arena_used(self):
        return int(lib().vx_ctx_arena_used(self.h))

    # ------------------------------------------------------------------ build / probe
    def build(self, key, pays=(), unique=True, load_factor=0.0, hashed=False):
        pa, npay = _cols(pays)
        d = BuildDesc(col(key), pa, npay, (VX_UNIQUE if unique else VX_PREAGG) | (VX_HASHED if hashed else 0),
                      _len(key), float(load_factor), 0)
        h = C.c_void_p()
        _check(lib().vx_build(self.h, C.byref(d), C.byref(h)))
        return Table(self, h, npay, (pa, key, pays))

    def join_plain(self, bkey, bpays, pkey, ppays=(), unique=True, late_mat=VX_LATE_AUTO,
                   chunk_rows=0, n_buffers=0, load_factor=0.0, hashed=False, count_zc=False):
        """One-shot build + probe. Returns ([count, sums...], stats dict)."""
        bp, nbp = _cols(bpays)
        pp, npp = _cols(ppays)
        d = JoinDesc()
        d.kind = VX_JOIN_PLAIN
        d.u.plain.build = BuildDesc(col(bkey), bp, nbp,
                                    (VX_UNIQUE if unique else VX_PREAGG) | (VX_HASHED if hashed else 0),
                                    _len(bkey), float(load_factor), 0)
        d.u.plain.probe = ProbeDesc(col(pkey), pp, npp, late_mat, _len(pkey), int(chunk_rows),
                                    int(n_buffers), VX_PROBE_COUNT_ZC if count_zc else 0, None, 0)
        out = JoinOut()
        _check(lib().vx_join_agg(self.h, C.byref(d), C.byref(out)))
        return out.agg.to_list(nbp + npp), out.stats.as_dict()

    # ------------------------------------------------------------------ partitioning
    def partition(self, key, pays=(), method="radix_hash", n_parts=0, shift=0, splitters=None,
                  sample_frac=0.0, seed=0, train_steps=0, lr=0.0, out_key=None, out_pays=None,
                  n_parts_cap=4096):
        """vx_partition. Returns a dict: method_used, n_parts, hist, boundary, splitters,
        imbalance, est_imbalance_radix, est_imbalance_range, final_loss, model."""
        pa, npay = _cols(pays)
        spl = None
        if splitters is not None:
            spl = np.ascontiguousarray(splitters, dtype=np.int64)
        opts = PartOpts(PART_METHODS[method] if isinstance(method, str) else int(method), int(n_parts),
                        int(shift), int(train_steps), float(sample_frac), float(lr), int(seed),
                        spl.ctypes.data_as(C.POINTER(C.c_int64)) if spl is not None and len(spl) else None,
                        0 if spl is None else len(spl), 0)
        outp = None
        okey = None
        if out_key is not None:
            okey = col(out_key).data
            if out_pays:
                outp = (C.c_void_p * len(out_pays))(*[col(o).data for o in out_pays])
        d = PartitionDesc(col(key), pa, npay, 0, _len(key), opts, okey, outp)
        hist = np.zeros(n_parts_cap, np.uint64)
        bnd = np.zeros(n_parts_cap + 1, np.uint64)
        sp = np.zeros(n_parts_cap, np.int64)
        model = np.zeros(N_MODEL_PARAMS, np.float32)
        o = PartitionOut()
        o.hist = hist.ctypes.data_as(C.POINTER(C.c_uint64))
        o.boundary = bnd.ctypes.data_as(C.POINTER(C.c_uint64))
        o.splitters = sp.ctypes.data_as(C.POINTER(C.c_int64))
        o.n_parts_cap = n_parts_cap
        o.model = model.ctypes.data_as(C.POINTER(C.c_float))
        _check(lib().vx_partition(self.h, C.byref(d), C.byref(o)))
        P = int(o.n_parts)
        return dict(method_used=int(o.method_used), n_parts=P, hist=hist[:P].copy(),
                    boundary=bnd[:P + 1].copy(), splitters=sp[:int(o.n_splitters)].copy(),
                    imbalance=o.imbalance, est_imbalance_radix=o.est_imbalance_radix,
                    est_imbalance_range=o.est_imbalance_range, final_loss=o.final_loss, model=model)

    # ------------------------------------------------------------------ CDF model kernels
    def cdf_loss_grad(self, x, t, params):
        p = np.ascontiguousarray(params, np.float32)
        g = np.zeros(N_MODEL_PARAMS, np.float32)
        loss = C.c_double()
        _check(lib().vx_cdf_loss_grad(self.h, _fptr(x), _fptr(t), _len(x), p.ctypes.data_as(C.POINTER(C.c_float)),
                                      g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)))
        return loss.value, g

    def cdf_forward(self, x, params):
        p = np.ascontiguousarray(params, np.float32)
        y = np.zeros(_len(x), np.float32)
        _check(lib().vx_cdf_forward(self.h, _fptr(x), _len(x), p.ctypes.data_as(C.POINTER(C.c_float)),
                                    y.ctypes.data_as(C.POINTER(C.c_float))))
        return y

    def cdf_train(self, x, t, params, steps, lr=0.0):
        p = np.array(params, np.float32)
        loss = C.c_double()
        _check(lib().vx_cdf_train(self.h, _fptr(x), _fptr(t), _len(x), p.ctypes.data_as(C.POINTER(C.c_float)),
                                  int(steps), float(lr), C.byref(loss)))
        return p, loss.value

    def join_partitioned(self, bkey, bpays, pkey, method="auto", n_parts=0, seed=0, sample_frac=0.0,
                         train_steps=0, lr=0.0, splitters=None, per_partition=False):
        """Partitioned join (pre-aggregated build). Returns ([count, sums...], stats, method_used
        [, per-partition aggregate lists])."""
        bp, nbp = _cols(bpays)
        d = JoinDesc()
        d.kind = VX_JOIN_PARTITIONED
        pj = d.u.part
        pj.build = BuildDesc(col(bkey), bp, nbp, VX_PREAGG, _len(bkey), 0.0, 0)
        cap = 4096 if per_partition else 0
        pa = (Agg * cap)() if cap else None
        pj.probe = ProbeDesc(col(pkey), None, 0, VX_LATE_AUTO, _len(pkey), 0, 0, 0, pa, cap)
        spl = None if splitters is None else np.ascontiguousarray(splitters, np.int64)
        pj.part = PartOpts(PART_METHODS[method] if isinstance(method, str) else int(method), int(n_parts), 0,
                           int(train_steps), float(sample_frac), float(lr), int(seed),
                           spl.ctypes.data_as(C.POINTER(C.c_int64)) if spl is not None and len(spl) else None,
                           0 if spl is None else len(spl), 0)
        out = JoinOut()
        _check(lib().vx_join_agg(self.h, C.byref(d), C.byref(out)))
        res = (out.agg.to_list(nbp), out.stats.as_dict(), int(out.part_method_used))
        if per_partition:
            P = int(out.stats.n_parts)
            return res + ([pa[i].to_list(nbp) for i in range(P)],)
        return res

    def join_radix(self, akey, apays, bkey, bpays, n_parts=0, shift=0, hash=False, placement=0,
                   per_partition=False):
        """Two-table radix-partitioned join.  Returns ([count, A sums..., B sums...], stats
        [, per-partition aggregate lists])."""
        ap, nap = _cols(apays)
        bp, nbp = _cols(bpays)
        d = JoinDesc()
        d.kind = VX_JOIN_RADIX
        rj = d.u.radix
        rj.a = BuildDesc(col(akey), ap, nap, 0, _len(akey), 0.0, 0)
        cap = 1024 if per_partition else 0
        pa = (Agg * cap)() if cap else None
        rj.b = ProbeDesc(col(bkey), bp, nbp, VX_LATE_AUTO, _len(bkey), 0, 0, 0, pa, cap)
        rj.n_parts, rj.shift, rj.hash, rj.placement = int(n_parts), int(shift), int(bool(hash)), int(placement)
        out = JoinOut()
        _check(lib().vx_join_agg(self.h, C.byref(d), C.byref(out)))
        res = (out.agg.to_list(nap + nbp), out.stats.as_dict())
        if per_partition:
            P = int(out.stats.n_parts)
            return res + ([pa[i].to_list(nap + nbp) for i in range(P)],)
        return res

    def sort(self, key, chunk_rows=0, n_buffers=0):
        """Out-of-core sort of a key column in place.  Returns the stats dict."""
        d = SortDesc(col(key), _len(key), int(chunk_rows), int(n_buffers), 0)
        st = Stats()
        _check(lib().vx_sort(self.h, C.byref(d), C.byref(st)))
        return st.as_dict()

    def join_batch(self, bkeys, bpays, pkeys, mode=0, tile_rows=0, block=0, load_factor=0.0, hashed=False):
        """Batched joins (device-resident). bpays entries may be None. Returns
        ([[count, sum] per job], stats)."""
        J = len(bkeys)
        bk, nb = _col_array(bkeys)
        bp, _ = _col_array(bpays, none_ok=True)
        pk, npr = _col_array(pkeys)
        outs = (Agg * max(1, J))()
        d = JoinDesc()
        d.kind = VX_JOIN_BATCH
        d.u.batch = BatchJoin(J, int(mode), bk, bp, nb, pk, npr, outs, int(tile_rows), int(block),
                              float(load_factor), VX_HASHED if hashed else 0)
        out = JoinOut()
        self._keep_batch = (bk, bp, pk, nb, npr, outs, list(bkeys), list(bpays), list(pkeys))
        _check(lib().vx_join_agg(self.h, C.byref(d), C.byref(out)))
        res = np.frombuffer(outs, dtype=np.uint64).reshape(-1, 9)[:J, :2].tolist()
        return res, out.stats.as_dict()

    def join_star(self, dims, fks, meas, groups_cap=4096, late_mat=VX_LATE_AUTO, chunk_rows=0, count_zc=False):
        """Star join + GROUP BY. dims: list of {key, filt, lo, hi, group (or None)}.
        Returns (g [n,2] int64, count [n] uint64, sums [n, nmeas] uint64, stats), sorted by (g0, g1)."""
        return _star_call(self, dims, fks, meas, groups_cap, late_mat, chunk_rows, count_zc)


def _star_call(ctx, dims, fks, meas, groups_cap, late_mat, chunk_rows, count_zc=False):
    d = JoinDesc()
    d.kind = VX_JOIN_STAR
    sj = d.u.star
    sj.n_dims = len(dims)
    sj.n_measures = len(meas)
    for i, dm in enumerate(dims):
        grp = dm.get("group")
        sj.dims[i] = StarDim(col(dm["key"]), _len(dm["key"]), col(dm["filt"]), int(dm["lo"]), int(dm["hi"]),
                             col(grp) if grp is not None else Col(None, VX_I32, 0))
        sj.fact_fk[i] = col(fks[i])
    for i, m in enumerate(meas):
        sj.measure[i] = col(m)
    sj.n_fact = _len(fks[0])
    sj.chunk_rows = int(chunk_rows)
    sj.late_mat = int(late_mat)
    sj.flags = VX_PROBE_COUNT_ZC if count_zc else 0
    rows = (GroupRow * max(1, groups_cap))()
    sj.groups = rows
    sj.groups_cap = groups_cap
    out = JoinOut()
    _check(lib().vx_join_agg(ctx.h, C.byref(d), C.byref(out)))
    n = int(out.n_groups)
    g = np.array([[rows[i].g0, rows[i].g1] for i in range(n)], dtype=np.int64).reshape(n, 2)
    cnt = np.array([rows[i].count for i in range(n)], dtype=np.uint64)
    sums = np.array([[rows[i].sum[c] for c in range(len(meas))] for i in range(n)],
                    dtype=np.uint64).reshape(n, len(meas))
    return g, cnt, sums, out.stats.as_dict()


def _fptr(x):
    """Device address of a float32 CUDA tensor, or of a pinned float32 HostBuffer."""
    if isinstance(x, HostBuffer):
        return x.ptr
    import torch
    if isinstance(x, torch.Tensor) and x.dtype == torch.float32 and x.is_contiguous():
        return x.data_ptr()
    raise TypeError("float inputs must be contiguous float32 CUDA tensors or HostBuffers")


def _len(x):
    if isinstance(x, HostBuffer):
        return x.n
    return int(x.shape[0]) if hasattr(x, "shape") else len(x)


class Table:
    def __init__(self, ctx, h, n_pay, keep):
        self.ctx, self.h, self.n_pay, self._keep = ctx, h, n_pay, keep

    def probe(self, key, pays=(), late_mat=VX_LATE_AUTO, chunk_rows=0, n_buffers=0, chunk_aggs=False, count_zc=False):
        """Probe and aggregate. Returns ([count, sums...], stats dict[, per-chunk lists])."""
        pa, npay = _cols(pays)
        n = _len(key)
        ca, cap = None, 0
        if chunk_aggs:
            cr = chunk_rows or n or 1
            cap = max(1, (n + cr - 1) // cr)
            ca = (Agg * cap)()
        d = ProbeDesc(col(key), pa, npay, late_mat, n, int(chunk_rows), int(n_buffers),
                      VX_PROBE_COUNT_ZC if count_zc else 0, ca, cap)
        out, st = Agg(), Stats()
        _check(lib().vx_probe_stream(self.ctx.h, self.h, C.byref(d), C.byref(out), C.byref(st)))
        res = out.to_list(self.n_pay + npay)
        if chunk_aggs:
            return res, st.as_dict(), [ca[i].to_list(self.n_pay + npay) for i in range(cap)]
        return res, st.as_dict()

    def probe_rows(self, key, pays=(), cap=None, out=None, late_mat=VX_LATE_AUTO, chunk_rows=0, n_buffers=0,
                   count_zc=False):
        """Probe, aggregate and write the join's rows.  `out` = (row, [build pay cols], [probe pay cols])
        of uint64 / int64 arrays (pinned host: HostBuffer.array, or CUDA tensors), each of `cap` rows;
        allocated as pinned HostBuffers of `cap` (default: probe rows) when None.  Returns
        ([count, sums...], stats, n_out, (row, build cols, probe cols))."""
        pa, npay = _cols(pays)
        n = _len(key)
        keep = []
        if out is None:
            cap = n if cap is None else cap
            hb = [HostBuffer(max(cap, 1), np.uint64)] + [HostBuffer(max(cap, 1), np.int64)
                                                          for _ in range(self.n_pay + npay)]
            keep = hb
            out = (hb[0].array, [h.array for h in hb[1:1 + self.n_pay]], [h.array for h in hb[1 + self.n_pay:]])
        row, bcols, pcols = out
        cap = _len(row) if cap is None else cap

        def ptr(a):
            return None if a is None else (a.data_ptr() if hasattr(a, "data_ptr") else a.ctypes.data)
        r = JoinRows()
        r.row = ptr(row)
        for c, a in enumerate(bcols):
            r.build_pay[c] = ptr(a)
        for c, a in enumerate(pcols):
            r.probe_pay[c] = ptr(a)
        r.cap = int(cap)
        d = ProbeDesc(col(key), pa, npay, late_mat, n, int(chunk_rows), int(n_buffers),
                      VX_PROBE_COUNT_ZC if count_zc else 0, None, 0)
        agg, st = Agg(), Stats()
        status = lib().vx_probe_rows(self.ctx.h, self.h, C.byref(d), C.byref(r), C.byref(agg), C.byref(st))
        self._keep_rows = keep
        if status == VX_ECAPACITY:
            raise VxError(status, lib().vx_last_error().decode() + f" (n_out {r.n_out})")
        _check(status)
        return agg.to_list(self.n_pay + npay), st.as_dict(), int(r.n_out), (row, bcols, pcols)

    def destroy(self):
        if self.h:
            lib().vx_table_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def merge_cuts(runs, rank):
    """vx_merge_cuts over sorted int64 numpy runs: the per-run cut at a global rank."""
    runs = [np.ascontiguousarray(r, np.int64) for r in runs]
    ptrs = (C.POINTER(C.c_int64) * max(1, len(runs)))(*[r.ctypes.data_as(C.POINTER(C.c_int64)) for r in runs])
    lens = (C.c_uint64 * max(1, len(runs)))(*[len(r) for r in runs])
    cut = (C.c_uint64 * max(1, len(runs)))()
    _check(lib().vx_merge_cuts(ptrs, lens, len(runs), int(rank), cut))
    return np.array([cut[i] for i in range(len(runs))], np.uint64)


def join_plain_noalloc(bkey, bpays, pkey, ppays, out, unique=True, load_factor=0.0, stream=None):
    """vx_join_plain_noalloc: the plain join of device-resident columns with its table in the
    library's fixed device array; nothing is allocated.  `out` is a caller-owned CUDA tensor of at
    least 10 int64 (count, 8 sums, error flags), written in the order of `stream` (default: torch's
    current stream); the call does not wait."""
    import torch
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.int64 and out.numel() >= 10
            and out.is_contiguous()):
        raise ValueError("out must be a contiguous CUDA int64 tensor of at least 10 elements")
    bp, nbp = _cols(bpays)
    pp, npp = _cols(ppays)
    b = BuildDesc(col(bkey), bp, nbp, VX_UNIQUE if unique else VX_PREAGG, _len(bkey), float(load_factor), 0)
    p = ProbeDesc(col(pkey), pp, npp, VX_LATE_AUTO, _len(pkey), 0, 0, 0, None, 0)
    s = torch.cuda.current_stream().cuda_stream if stream is None else int(stream)
    _check(lib().vx_join_plain_noalloc(C.byref(b), C.byref(p), C.c_void_p(s), C.c_void_p(out.data_ptr())))
