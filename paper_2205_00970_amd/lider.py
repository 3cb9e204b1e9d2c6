"""Python binding of the gfx950 LIDER library (include/lider.h).

Argument marshalling only: every step of build and search runs in the HIP
library.  torch supplies device memory (tensors) and streams.  If the library
is not built, every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libliderhip.so")

OK, EINVAL, ENOMEM, EDEVICE, ERANGE, EBUSY, EIO = 0, -1, -2, -3, -4, -5, -6
F32, BF16, FP8E4M3 = 0, 1, 2
MAX_K, MAX_C, MAX_M = 1024, 128, 16

EXPORTS = {
    "centroids": (0, np.float32), "assign": (1, np.int32), "offsets": (2, np.int64),
    "perm": (3, np.int64), "keys": (4, np.uint64), "digits": (5, np.int32),
    "l1_order": (6, np.int64), "l1_keys": (7, np.uint64), "l1_digits": (8, np.int32),
    "model_int": (9, np.int64), "model_box": (10, np.int32), "model_key": (11, np.uint64),
    "model_dbl": (12, np.float64), "leaves": (13, np.float64), "leaf_err": (14, np.int32),
    "reordered": (15, np.float32),
}


class LiderError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lider status {status}: {msg}")
        self.status = status


class BuildParams(C.Structure):
    _fields_ = [("n_clusters", C.c_int32), ("m", C.c_int32), ("rmi_fanout", C.c_int32),
                ("rmi_fanout_l1", C.c_int32), ("w", C.c_double), ("lsh_a_host", C.c_void_p),
                ("lsh_b_host", C.c_void_p), ("assignment_dev", C.c_void_p),
                ("kmeans_init_host", C.c_void_p), ("kmeans_iters", C.c_int32),
                ("storage", C.c_int32), ("centroid_storage", C.c_int32),
                ("kmeans_seeding", C.c_int32), ("hash_kind", C.c_int32),
                ("n_arrays", C.c_int32), ("seed", C.c_uint64)]


class SearchOpts(C.Structure):
    _fields_ = [("r1", C.c_int32), ("precision", C.c_int32), ("shortlist_mult", C.c_int32),
                ("persistent", C.c_int32), ("tile_rows", C.c_int32), ("l1_dense", C.c_int32),
                ("grid_mult", C.c_int32), ("pass_pairs", C.c_int32), ("expand_bits", C.c_int32),
                ("reserved", C.c_int32 * 7)]


class SearchDebug(C.Structure):
    _fields_ = [("qdigits_dev", C.c_void_p), ("l1_dev", C.c_void_p), ("routed_dev", C.c_void_p),
                ("pairs_dev", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("n_clusters", C.c_int32), ("m", C.c_int32),
                ("rmi_fanout", C.c_int32), ("rmi_fanout_l1", C.c_int32),
                ("kmeans_iters_run", C.c_int32), ("max_cluster", C.c_int64), ("w", C.c_double),
                ("storage", C.c_int32), ("centroid_storage", C.c_int32),
                ("n_arrays", C.c_int32), ("hash_kind", C.c_int32)]


SYMBOLS = ["lider_build", "lider_free", "lider_last_error", "lider_search_workspace",
           "lider_search", "lider_search_ex", "lider_get_info", "lider_export_bytes",
           "lider_export", "lider_hash", "lider_kmeans_assign", "lider_profile_begin",
           "lider_profile_end", "lider_debug_fail_next", "lider_save", "lider_load",
           "lider_draw_params", "lider_search_noalloc", "lider_noalloc_scratch_bytes"]
NSTAGES = 5
STAGES = ["hash", "route", "worklist", "rerank", "select"]

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        p, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.lider_build.argtypes = [p, i64, i32, C.POINTER(BuildParams), p, C.POINTER(p)]
        L.lider_free.argtypes = [p]
        L.lider_free.restype = None
        L.lider_last_error.restype = C.c_char_p
        L.lider_search_workspace.argtypes = [p, i64, i32, i32, i32, C.POINTER(SearchOpts)]
        L.lider_search_workspace.restype = sz
        L.lider_search.argtypes = [p, p, i64, i32, i32, i32, p, p, p, sz, p]
        L.lider_search_ex.argtypes = [p, p, i64, i32, i32, i32, p, p, p, sz, p,
                                      C.POINTER(SearchOpts), C.POINTER(SearchDebug)]
        L.lider_get_info.argtypes = [p, C.POINTER(Info)]
        L.lider_export_bytes.argtypes = [p, i32]
        L.lider_export_bytes.restype = sz
        L.lider_export.argtypes = [p, i32, p, sz]
        L.lider_hash.argtypes = [p, i64, i32, p, p, i32, C.c_double, p, p]
        L.lider_kmeans_assign.argtypes = [p, i64, i32, p, i32, p, p]
        L.lider_profile_begin.argtypes = [i32]
        L.lider_profile_end.argtypes = [C.POINTER(C.c_double), C.POINTER(i32)]
        L.lider_debug_fail_next.argtypes = [i32]
        L.lider_debug_fail_next.restype = None
        L.lider_save.argtypes = [p, C.c_char_p]
        L.lider_load.argtypes = [C.c_char_p, p, C.POINTER(p)]
        L.lider_draw_params.argtypes = [C.c_uint64, i32, i32, i32, C.c_double, i32, p, p, i64,
                                        i32, p]
        L.lider_search_noalloc.argtypes = [p, p, i64, i32, i32, i32, p, p, p,
                                           C.POINTER(SearchOpts)]
        L.lider_noalloc_scratch_bytes.argtypes = []
        L.lider_noalloc_scratch_bytes.restype = sz
        _lib = L
    return _lib


def _check(st):
    if st != OK:
        raise LiderError(st, lib().lider_last_error().decode(errors="replace"))


def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype, ndim=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _np_ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


_STORAGE = {"f32": F32, "bf16": BF16}
_CSTORAGE = {"f32": F32, "fp8": FP8E4M3}
_PREC = {"f32": F32, "bf16": BF16}


class Index:
    """A LIDER index resident in device memory (lider_build / lider_free)."""

    def __init__(self, corpus, n_clusters, m, w, rmi_fanout, lsh=None, rmi_fanout_l1=0,
                 kmeans_init=None, kmeans_iters=20, assignment=None, storage="f32",
                 centroid_storage="f32", seeding="given", hash_kind="e2lsh", stream=None,
                 n_arrays=1, seed=0):
        """hash_kind "e2lsh": integer digits floor((a.x + b) / w); "sign": the
        cosine variant (bits [a.x >= 0], key = Decimal(bits); w and b unused).
        n_arrays = H hashkey arrays per core model: lsh = (A [2Hm, d], b [2Hm]),
        rows h*m.. array h of layer 1, rows H*m + h*m.. array h of layer 2.
        lsh None / kmeans_init None: the library draws them from `seed`."""
        torch = _torch()
        cp = _dev_ptr(corpus, torch.float32, 2, "corpus")
        n, d = corpus.shape
        kind = {"e2lsh": 0, "sign": 1}[hash_kind]
        H = int(n_arrays)
        A = b = None
        if lsh is not None:
            A = np.ascontiguousarray(lsh[0], dtype=np.float32)
            b = np.ascontiguousarray(lsh[1] if lsh[1] is not None else np.zeros(2 * H * m),
                                     dtype=np.float32)
            if A.shape != (2 * H * m, d) or b.shape != (2 * H * m,):
                raise ValueError("lsh must be (A [2Hm, d], b [2Hm])")
        ini = None if kmeans_init is None else np.ascontiguousarray(kmeans_init, dtype=np.int64)
        seed_mode = {"given": 0, "farthest": 1}[seeding]
        if assignment is None and ini is not None and \
                ini.shape[0] < (1 if seed_mode else n_clusters):
            raise ValueError("kmeans_init needs n_clusters row ids (1 with farthest-first)")
        P = BuildParams(int(n_clusters), int(m), int(rmi_fanout), int(rmi_fanout_l1), float(w),
                        _np_ptr(A), _np_ptr(b),
                        None if assignment is None else _dev_ptr(assignment, torch.int32, 1,
                                                                 "assignment"),
                        _np_ptr(ini), int(kmeans_iters), _STORAGE[storage],
                        _CSTORAGE[centroid_storage], seed_mode, kind, H,
                        int(seed) & (2**64 - 1))
        h = C.c_void_p()
        _check(lib().lider_build(cp, n, d, C.byref(P), _stream(stream), C.byref(h)))
        self._h = h
        self._ws = None
        self._set_info()
        self.hash_kind = hash_kind

    def save(self, path):
        """Write the index to `path` (lider_save)."""
        _check(lib().lider_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path, stream=None):
        """Read an index written by save() onto the current device (lider_load)."""
        h = C.c_void_p()
        _check(lib().lider_load(os.fsencode(path), _stream(stream), C.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self._ws = None
        self._set_info()
        self.hash_kind = "sign" if self._hash_kind_code == 1 else "e2lsh"
        return self

    def _set_info(self):
        info = self.info()
        self.n, self.d = int(info.n), int(info.d)
        self.C, self.m = info.n_clusters, info.m
        self.F2, self.F1 = info.rmi_fanout, info.rmi_fanout_l1
        self.max_cluster = info.max_cluster
        self.iters_run = info.kmeans_iters_run
        self.H = info.n_arrays
        self._hash_kind_code = info.hash_kind

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lider_free(self._h)
            self._h = C.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        out = Info()
        _check(lib().lider_get_info(self._h, C.byref(out)))
        return out

    def export(self, what):
        code, dt = EXPORTS[what]
        nb = lib().lider_export_bytes(self._h, code)
        out = np.empty(nb // np.dtype(dt).itemsize, dtype=dt)
        _check(lib().lider_export(self._h, code, _np_ptr(out), nb))
        return out

    def workspace_bytes(self, nq, k, c, r, **opt):
        o = self._opts(**opt)
        return int(lib().lider_search_workspace(self._h, nq, k, c, r, C.byref(o)))

    @staticmethod
    def _opts(r1=0, precision="f32", shortlist_mult=0, persistent=False, tile_rows=0,
              grid_mult=0, l1_dense=True, pass_pairs=0, expand_bits=0):
        o = SearchOpts()
        o.r1, o.precision, o.shortlist_mult = int(r1), _PREC[precision], int(shortlist_mult)
        o.persistent, o.tile_rows, o.grid_mult = int(persistent), int(tile_rows), int(grid_mult)
        # True: automatic dense layer 1; False: window kernel; or the raw code
        o.l1_dense = 0 if l1_dense is True else -1 if l1_dense is False else int(l1_dense)
        o.pass_pairs = int(pass_pairs)
        o.expand_bits = int(expand_bits)
        return o

    def search(self, queries, k, c, r, r1=0, precision="f32", shortlist_mult=0,
               persistent=False, tile_rows=0, grid_mult=0, debug=False, stream=None, ws=None,
               out=None, l1_dense=True, pass_pairs=0, expand_bits=0):
        """Batched search; returns (ids int64 [nq,k], scores f32 [nq,k][, debug])."""
        torch = _torch()
        qp = _dev_ptr(queries, torch.float32, 2, "queries")
        nq = queries.shape[0]
        o = self._opts(r1, precision, shortlist_mult, persistent, tile_rows, grid_mult, l1_dense,
                       pass_pairs, expand_bits)
        need = int(lib().lider_search_workspace(self._h, nq, k, c, r, C.byref(o)))
        if need == 0 and nq > 0:
            # invalid arguments: let lider_search_ex report which
            _check(lib().lider_search_ex(self._h, qp, nq, k, c, r, None, None, None, 0,
                                         _stream(stream), C.byref(o), None))
        cur = torch.cuda.current_stream(queries.device)
        st_obj = stream if stream is not None else cur
        if ws is None:
            # one cached workspace per stream: searches on different streams
            # never share one, and a buffer replaced by a larger one is not
            # reused by the allocator while its stream may still read it
            key = int(st_obj.cuda_stream)
            if self._ws is None:
                self._ws = {}
            wsb = self._ws.get(key)
            if wsb is None or wsb.numel() < need:
                wsb = torch.empty(max(need, 256), dtype=torch.uint8, device=queries.device)
                if st_obj != cur:
                    wsb.record_stream(st_obj)
                self._ws[key] = wsb
            ws = wsb
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=queries.device)
            sc = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
            if st_obj != cur:
                ids.record_stream(st_obj)
                sc.record_stream(st_obj)
        else:
            ids, sc = out
        dbg = None
        dstruct = None
        H = self.H
        if debug:
            dev = queries.device
            dbg = dict(qdigits=torch.empty((nq, 2 * H * self.m), dtype=torch.int32, device=dev),
                       l1=torch.empty((nq, H, 3), dtype=torch.int64, device=dev),
                       routed=torch.empty((nq, c), dtype=torch.int32, device=dev),
                       pairs=torch.empty((nq, c, H, 3), dtype=torch.int64, device=dev))
            dstruct = SearchDebug(dbg["qdigits"].data_ptr(), dbg["l1"].data_ptr(),
                                  dbg["routed"].data_ptr(), dbg["pairs"].data_ptr())
        _check(lib().lider_search_ex(self._h, qp, nq, k, c, r, C.c_void_p(ids.data_ptr()),
                                     C.c_void_p(sc.data_ptr()), C.c_void_p(ws.data_ptr()),
                                     ws.numel(), _stream(stream), C.byref(o),
                                     C.byref(dstruct) if dstruct is not None else None))
        if debug and H == 1:  # one array: l1 [nq, 3], pairs [nq, c, 3]
            dbg["l1"] = dbg["l1"][:, 0]
            dbg["pairs"] = dbg["pairs"][:, :, 0]
        return (ids, sc, dbg) if debug else (ids, sc)


def draw_params(seed, m, d, w, n_arrays=1, hash_kind="e2lsh", n=0, n_rows=0):
    """The library's seeded draws (lider_draw_params, host only): returns
    (A [2Hm, d] f32, b [2Hm] f32, rows [n_rows] int64 or None)."""
    H = max(1, int(n_arrays))
    A = np.empty((2 * H * m, d), np.float32)
    b = np.empty(2 * H * m, np.float32)
    rows = np.empty(n_rows, np.int64) if n else None
    _check(lib().lider_draw_params(int(seed) & (2**64 - 1), int(n_arrays), int(m), int(d),
                                   float(w), {"e2lsh": 0, "sign": 1}[hash_kind], _np_ptr(A),
                                   _np_ptr(b), int(n), int(n_rows), _np_ptr(rows)))
    return A, b, rows


def noalloc_scratch_bytes():
    """Size of lider_search_noalloc's fixed workspace."""
    return int(lib().lider_noalloc_scratch_bytes())


def search_noalloc(index, queries, k, c, r, out, stream=None, **opts):
    """lider_search_noalloc: the search with the library's fixed workspace
    (no allocation).  `out` = (ids int64 [nq,k], scores f32 [nq,k]) tensors."""
    torch = _torch()
    qp = _dev_ptr(queries, torch.float32, 2, "queries")
    ids, sc = out
    o = Index._opts(**opts)
    _check(lib().lider_search_noalloc(index._h, qp, queries.shape[0], k, c, r,
                                      _dev_ptr(ids, torch.int64, 2, "ids"),
                                      _dev_ptr(sc, torch.float32, 2, "scores"), _stream(stream),
                                      C.byref(o)))


def hash(X, A, b, w, stream=None):
    """E2LSH digits floor((A.x + b)/w) of X's rows (lider_hash)."""
    torch = _torch()
    xp = _dev_ptr(X, torch.float32, 2, "X")
    ap = _dev_ptr(A, torch.float32, 2, "A")
    bp = _dev_ptr(b, torch.float32, 1, "b")
    out = torch.empty((X.shape[0], A.shape[0]), dtype=torch.int32, device=X.device)
    _check(lib().lider_hash(xp, X.shape[0], X.shape[1], ap, bp, A.shape[0], float(w),
                            C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def kmeans_assign(X, cent, stream=None):
    """One k-means assignment step, decided in FP64 (lider_kmeans_assign)."""
    torch = _torch()
    xp = _dev_ptr(X, torch.float32, 2, "X")
    cp = _dev_ptr(cent, torch.float32, 2, "cent")
    out = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    _check(lib().lider_kmeans_assign(xp, X.shape[0], X.shape[1], cp, cent.shape[0],
                                     C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def profile_begin(max_calls):
    """Time the stages of this thread's next max_calls searches (HIP events)."""
    _check(lib().lider_profile_begin(int(max_calls)))


def profile_end():
    """Return ({stage: summed ms}, timed calls) of the profiled searches."""
    ms = (C.c_double * NSTAGES)()
    calls = C.c_int32(0)
    _check(lib().lider_profile_end(ms, C.byref(calls)))
    return {STAGES[i]: float(ms[i]) for i in range(NSTAGES)}, int(calls.value)


def fail_next(status):
    """Test hook: make the next search on this thread fail with `status`."""
    lib().lider_debug_fail_next(int(status))
