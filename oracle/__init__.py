"""CPU oracle for the streamed join / aggregate / partition path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the GPU library never calls it.

A thin ctypes binding over ``oracle.cpp`` (plain single-threaded C++), built
into ``liboracle.so`` next to this file by :func:`build`.  Every function
takes numpy arrays and returns numpy arrays / Python ints; all integer sums
are modulo 2^64 and returned as Python ``int`` in [0, 2^64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile oracle.cpp with g++ into liboracle.so (always recompiles)."""
    src = os.path.join(_HERE, "oracle.cpp")
    tmp = _SO + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, src])
    os.replace(tmp, _SO)
    return _SO


class _Col(C.Structure):
    _fields_ = [("p", C.c_void_p), ("elsize", C.c_int32), ("pad_", C.c_int32)]


class _Dim(C.Structure):
    _fields_ = [("key", _Col), ("n", C.c_uint64), ("filt", _Col), ("lo", C.c_int64),
                ("hi", C.c_int64), ("group", _Col)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise RuntimeError(f"oracle library not built: {_SO} (run oracle.build())")
    lib = C.CDLL(_SO)
    u64p = C.POINTER(C.c_uint64)
    lib.or_join_agg_hash.argtypes = [_Col, C.POINTER(_Col), C.c_uint32, C.c_uint64, _Col,
                                     C.POINTER(_Col), C.c_uint32, C.c_uint64, u64p]
    lib.or_join_agg_sortmerge.argtypes = lib.or_join_agg_hash.argtypes
    lib.or_join_rows.argtypes = [_Col, C.POINTER(_Col), C.c_uint32, C.c_uint64, _Col, C.POINTER(_Col),
                                 C.c_uint32, C.c_uint64, C.c_uint64, C.POINTER(C.c_uint64),
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.or_join_rows.restype = C.c_uint64
    lib.or_build_create.argtypes = [_Col, C.POINTER(_Col), C.c_uint32, C.c_uint64]
    lib.or_build_create.restype = C.c_void_p
    lib.or_build_free.argtypes = [C.c_void_p]
    lib.or_build_probe.argtypes = [C.c_void_p, _Col, C.POINTER(_Col), C.c_uint32, C.c_uint64, u64p]
    lib.or_build_distinct.argtypes = [C.c_void_p]
    lib.or_build_distinct.restype = C.c_uint64
    lib.or_star_groupby.argtypes = [C.POINTER(_Dim), C.c_uint32, C.POINTER(_Col), C.POINTER(_Col),
                                    C.c_uint32, C.c_uint64, C.POINTER(C.c_int64), u64p, u64p,
                                    C.c_uint64, u64p]
    u32p = C.POINTER(C.c_uint32)
    lib.or_part_ids_bits.argtypes = [_Col, C.c_uint64, C.c_uint32, C.c_uint32, u32p]
    lib.or_part_ids_hash.argtypes = [_Col, C.c_uint64, C.c_uint32, u32p]
    lib.or_hash64.argtypes = [_Col, C.c_uint64, u64p]
    lib.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64, u64p]
    lib.or_part_ids_range.argtypes = [_Col, C.c_uint64, C.POINTER(C.c_int64), C.c_uint32, u32p]
    lib.or_histogram.argtypes = [u32p, C.c_uint64, C.c_uint32, u64p]
    lib.or_cluster_boundary.argtypes = [u32p, C.c_uint64, C.c_uint32, u64p, u64p]
    lib.or_late_mat_threshold.argtypes = [C.c_double, C.c_double, C.c_double]
    lib.or_late_mat_threshold.restype = C.c_double
    f32p = C.POINTER(C.c_float)
    f64p = C.POINTER(C.c_double)
    lib.or_cdf_feature.argtypes = [C.c_int64, C.c_int64, C.c_float]
    lib.or_cdf_feature.restype = C.c_float
    lib.or_cdf_targets.argtypes = [C.POINTER(C.c_int64), C.c_uint64, f32p]
    lib.or_mlp_loss_grad.argtypes = [f32p, C.c_uint32, f32p, f32p, C.c_uint64, f64p]
    lib.or_mlp_loss_grad.restype = C.c_double
    lib.or_mlp_forward.argtypes = [f32p, C.c_uint32, f32p, C.c_uint64, f64p]
    lib.or_adam_step.argtypes = [f32p, f32p, f32p, f32p, C.c_uint32, C.c_uint32, C.c_double,
                                 C.c_double, C.c_double, C.c_double]
    lib.or_splitters_from_cdf.argtypes = [C.POINTER(C.c_int64), f64p, C.c_uint64, C.c_uint32,
                                          C.POINTER(C.c_int64)]
    lib.or_splitters_from_cdf.restype = C.c_uint32
    lib.or_sample_bernoulli.argtypes = [_Col, C.c_uint64, C.c_uint64, C.c_double, C.POINTER(C.c_int64)]
    lib.or_sample_bernoulli.restype = C.c_uint64
    lib.or_sort.argtypes = [_Col, C.c_uint64, C.POINTER(C.c_int64)]
    lib.or_merge_cuts.argtypes = [C.POINTER(C.POINTER(C.c_int64)), u64p, C.c_uint32, C.c_uint64, u64p]
    _lib = lib
    return lib


def _col(a: np.ndarray) -> _Col:
    if a.dtype not in (np.int32, np.int64):
        raise TypeError(f"oracle columns must be int32 or int64, got {a.dtype}")
    if not a.flags.c_contiguous:
        raise ValueError("oracle columns must be contiguous")
    return _Col(a.ctypes.data, a.dtype.itemsize, 0)


def _cols(arrs):
    arrs = list(arrs or [])
    t = (_Col * max(1, len(arrs)))(*[_col(a) for a in arrs])
    return t, len(arrs)


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def join_agg(bkey, bpays, pkey, ppays, method: str = "hash"):
    """Join aggregates [count, SUM(build pays)..., SUM(probe pays)...] mod 2^64."""
    lib = _load()
    bp, nbp = _cols(bpays)
    pp, npp = _cols(ppays)
    out = np.zeros(1 + nbp + npp, dtype=np.uint64)
    fn = lib.or_join_agg_hash if method == "hash" else lib.or_join_agg_sortmerge
    fn(_col(bkey), bp, nbp, len(bkey), _col(pkey), pp, npp, len(pkey), _ptr(out, C.c_uint64))
    return [int(v) for v in out]


def join_rows(bkey, bpays, pkey, ppays):
    """The join's output rows in probe order (then build order): (probe row indices,
    [build payload columns], [probe payload columns]), payloads as int64."""
    lib = _load()
    bp, nbp = _cols(bpays)
    pp, npp = _cols(ppays)
    n = join_agg(bkey, [], pkey, [])[0]
    cap = max(int(n), 1)
    rows = np.zeros(cap, np.uint64)
    ob = np.zeros((max(nbp, 1), cap), np.int64)
    op = np.zeros((max(npp, 1), cap), np.int64)
    got = lib.or_join_rows(_col(bkey), bp, nbp, len(bkey), _col(pkey), pp, npp, len(pkey), cap,
                           _ptr(rows, C.c_uint64), _ptr(ob, C.c_int64), _ptr(op, C.c_int64))
    assert got == n
    return rows[:n], [ob[c, :n] for c in range(nbp)], [op[c, :n] for c in range(npp)]


class PreparedBuild:
    """A build side held by the oracle so several probe slices can be checked."""

    def __init__(self, bkey, bpays):
        lib = _load()
        self._keep = (bkey, list(bpays or []))
        bp, self.nbp = _cols(bpays)
        self._h = lib.or_build_create(_col(bkey), bp, self.nbp, len(bkey))

    def probe(self, pkey, ppays):
        lib = _load()
        pp, npp = _cols(ppays)
        out = np.zeros(1 + self.nbp + npp, dtype=np.uint64)
        lib.or_build_probe(self._h, _col(pkey), pp, npp, len(pkey), _ptr(out, C.c_uint64))
        return [int(v) for v in out]

    def distinct(self) -> int:
        return int(_load().or_build_distinct(self._h))

    def close(self):
        if self._h:
            _load().or_build_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def star_groupby(dims, fks, meas, cap: int = 1 << 16):
    """dims: list of dicts {key, filt, lo, hi, group (array or None)}.

    Returns (g, count, sums): g int64 [n,2], count uint64 [n], sums uint64 [n, nmeas],
    sorted ascending by (g0, g1), only groups with count > 0.
    """
    lib = _load()
    D = (_Dim * len(dims))()
    keep = []
    for i, d in enumerate(dims):
        grp = d.get("group")
        D[i] = _Dim(_col(d["key"]), len(d["key"]), _col(d["filt"]), int(d["lo"]), int(d["hi"]),
                    _col(grp) if grp is not None else _Col(None, 4, 0))
        keep.append(d)
    fk, _ = _cols(fks)
    ms, nm = _cols(meas)
    nfact = len(fks[0]) if fks else 0
    g = np.zeros((cap, 2), dtype=np.int64)
    cnt = np.zeros(cap, dtype=np.uint64)
    sums = np.zeros((cap, max(1, nm)), dtype=np.uint64)
    ng = C.c_uint64(0)
    rc = lib.or_star_groupby(D, len(dims), fk, ms, nm, nfact, _ptr(g, C.c_int64),
                             _ptr(cnt, C.c_uint64), _ptr(sums, C.c_uint64), cap, C.byref(ng))
    if rc == 1:
        raise ValueError("duplicate dimension key")
    if rc == 2:
        raise ValueError(f"more than {cap} groups ({ng.value})")
    n = ng.value
    return g[:n].copy(), cnt[:n].copy(), sums[:n, :nm].copy()


def part_ids_bits(keys, shift, log2p):
    ids = np.zeros(len(keys), dtype=np.uint32)
    _load().or_part_ids_bits(_col(keys), len(keys), shift, log2p, _ptr(ids, C.c_uint32))
    return ids


def part_ids_hash(keys, log2p):
    ids = np.zeros(len(keys), dtype=np.uint32)
    _load().or_part_ids_hash(_col(keys), len(keys), log2p, _ptr(ids, C.c_uint32))
    return ids


def hash64(keys):
    """The full 64-bit MurmurHash3 finalizer of each key (radix-hash ids are its top bits)."""
    out = np.zeros(len(keys), dtype=np.uint64)
    _load().or_hash64(_col(keys), len(keys), _ptr(out, C.c_uint64))
    return out


def splitmix64(seed, n):
    """The first n outputs of SplitMix64 started from state `seed` (the sampler's stream)."""
    out = np.zeros(max(1, n), dtype=np.uint64)
    _load().or_splitmix64(int(seed), n, _ptr(out, C.c_uint64))
    return out[:n]


def part_ids_range(keys, splitters):
    s = np.ascontiguousarray(splitters, dtype=np.int64)
    ids = np.zeros(len(keys), dtype=np.uint32)
    _load().or_part_ids_range(_col(keys), len(keys), _ptr(s, C.c_int64), len(s),
                              _ptr(ids, C.c_uint32))
    return ids


def histogram(ids, nparts):
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    h = np.zeros(nparts, dtype=np.uint64)
    _load().or_histogram(_ptr(ids, C.c_uint32), len(ids), nparts, _ptr(h, C.c_uint64))
    return h


def cluster_boundary(ids, nparts):
    """(order, boundary): stable clustering order and the find_boundary array."""
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    order = np.zeros(len(ids), dtype=np.uint64)
    b = np.zeros(nparts + 1, dtype=np.uint64)
    _load().or_cluster_boundary(_ptr(ids, C.c_uint32), len(ids), nparts, _ptr(order, C.c_uint64),
                                _ptr(b, C.c_uint64))
    return order, b


def late_mat_threshold(elem_bytes, line_bytes, n_exchange):
    return float(_load().or_late_mat_threshold(elem_bytes, line_bytes, n_exchange))


def cdf_feature(keys, kmin, scale):
    lib = _load()
    sc = np.float32(scale)
    return np.array([lib.or_cdf_feature(int(k), int(kmin), float(sc)) for k in keys],
                    dtype=np.float32)


def cdf_targets(sorted_keys):
    s = np.ascontiguousarray(sorted_keys, dtype=np.int64)
    t = np.zeros(len(s), dtype=np.float32)
    _load().or_cdf_targets(_ptr(s, C.c_int64), len(s), _ptr(t, C.c_float))
    return t


def mlp_loss_grad(params, x, t):
    p = np.ascontiguousarray(params, dtype=np.float32)
    H = (len(p) - 1) // 3
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    g = np.zeros(len(p), dtype=np.float64)
    loss = _load().or_mlp_loss_grad(_ptr(p, C.c_float), H, _ptr(x, C.c_float), _ptr(t, C.c_float),
                                    len(x), _ptr(g, C.c_double))
    return float(loss), g


def mlp_forward(params, x):
    p = np.ascontiguousarray(params, dtype=np.float32)
    H = (len(p) - 1) // 3
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.zeros(len(x), dtype=np.float64)
    _load().or_mlp_forward(_ptr(p, C.c_float), H, _ptr(x, C.c_float), len(x), _ptr(y, C.c_double))
    return y


def adam_step(params, m, v, grad, t, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float32 arrays params, m, v with float32 grad."""
    g = np.ascontiguousarray(grad, dtype=np.float32)
    _load().or_adam_step(_ptr(params, C.c_float), _ptr(m, C.c_float), _ptr(v, C.c_float),
                         _ptr(g, C.c_float), len(params), t, lr, b1, b2, eps)


def splitters_from_cdf(sorted_keys, y, nparts):
    s = np.ascontiguousarray(sorted_keys, dtype=np.int64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(max(1, 2 * nparts), dtype=np.int64)
    n = _load().or_splitters_from_cdf(_ptr(s, C.c_int64), _ptr(y, C.c_double), len(s), nparts,
                                      _ptr(out, C.c_int64))
    return out[:n].copy()


def sample_bernoulli(keys, seed, frac):
    """Keys of the rows kept by the SplitMix64 Bernoulli draw, in row order."""
    out = np.zeros(max(1, len(keys)), dtype=np.int64)
    m = _load().or_sample_bernoulli(_col(keys), len(keys), int(seed), float(frac), _ptr(out, C.c_int64))
    return out[:m].copy()


def feature_scale(kmin, kmax):
    """FP32 scale 1 / (L * 2^23) with L = floor(log2(min(kmax - kmin, 2^63 - 1) + 1)) + 1."""
    r = min((int(kmax) - int(kmin)), (1 << 63) - 1)
    L = (r + 1).bit_length()
    return np.float32(1.0 / (L * 8388608.0))


def sort(keys):
    """The keys in ascending signed order, as int64."""
    out = np.zeros(len(keys), np.int64)
    _load().or_sort(_col(keys), len(keys), _ptr(out, C.c_int64))
    return out


def merge_cuts(runs, rank):
    """Per-run cut of sorted int64 runs at a global rank: the rank smallest elements of their
    union, ties from lower-numbered runs first."""
    runs = [np.ascontiguousarray(r, np.int64) for r in runs]
    ptrs = (C.POINTER(C.c_int64) * max(1, len(runs)))(*[_ptr(r, C.c_int64) for r in runs])
    lens = np.array([len(r) for r in runs] or [0], np.uint64)
    cut = np.zeros(max(1, len(runs)), np.uint64)
    _load().or_merge_cuts(ptrs, _ptr(lens, C.c_uint64), len(runs), int(rank), _ptr(cut, C.c_uint64))
    return cut[:len(runs)]
