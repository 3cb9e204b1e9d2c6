"""Plain FP64 CPU oracle of LIDER (arXiv 2205.00970) -- test infrastructure only.

The arithmetic lives in ``lider_oracle.c`` (sequential FP64, no FMA contraction);
this module only builds it with gcc and marshals numpy arrays through ctypes.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It imports nothing from the HIP package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "lider_oracle.c")
_LIB = os.path.join(_DIR, "liblider_oracle.so")

OK, EINVAL, ENOMEM, ERANGE = 0, -1, -2, -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP over rows)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        p = C.c_void_p
        i32, i64, u64, f64 = C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.or_digits.argtypes = [p, i64, i32, p, p, i32, f64, p]
        L.or_digits_sign.argtypes = [p, i64, i32, p, i32, p]
        L.or_dist_e.argtypes = [u64, u64, i32, i32]
        L.or_dist_e.restype = i64
        L.or_window_expand_pub.argtypes = [p, i64, i64, i64, u64, i32, i32, p, p]
        L.or_kmeans_assign.argtypes = [p, i64, i32, p, i32, p]
        L.or_kmeans_update.argtypes = [p, i64, i32, p, i32, p, p]
        L.or_kmeans.argtypes = [p, i64, i32, i32, p, i32, p, p, p]
        L.or_kmeans_seed_farthest.argtypes = [p, i64, i32, i32, i64, p]
        L.or_rmi_train.argtypes = [p, i64, i32, p, p, p, p]
        L.or_rmi_predict.argtypes = [p, p, i32, i64, f64]
        L.or_rmi_predict.restype = i64
        L.or_rmi_leaf.argtypes = [p, i32, i64, f64]
        L.or_rmi_leaf.restype = i32
        L.or_encode_box.argtypes = [p, i32, p, p, i32, p]
        L.or_encode_box.restype = u64
        L.or_window_pub.argtypes = [i64, i64, i64, p, p]
        L.or_build.argtypes = [p, i64, i32, i32, p, p, i32, p, p, i32, i32, f64, i32, i32, i32, p]
        L.or_build.restype = p
        L.or_free.argtypes = [p]
        L.or_search.argtypes = [p, p, i64, i32, i32, i32, i32, i32, p, p, p, p, p, p]
        L.or_bruteforce.argtypes = [p, i64, i32, p, i64, i32, p, p]
        L.or_pair_scores.argtypes = [p, p, i32, p, p, i64, p]
        L.or_iters_run.argtypes = [p]
        L.or_iters_run.restype = i32
        for name in ("or_get_centroids", "or_get_assign", "or_get_offsets", "or_get_perm",
                     "or_get_keys", "or_get_digits"):
            getattr(L, name).argtypes = [p, p]
        L.or_get_l1.argtypes = [p, p, p, p]
        L.or_get_model.argtypes = [p, i32, p, p, p, p, p, p, p, p]
        L.or_core.argtypes = [i64, i32, i32, p, i32, p, p, p, p, p, p, p, p, p, p]
        L.or_core_query.argtypes = [i64, i32, i32, i32, p, p, p, p, p, p, p, p]
        L.or_core_query.restype = i64
        L.or_splitmix64.argtypes = [u64, i64, p]
        L.or_splitmix64.restype = None
        L.or_seeded_lsh.argtypes = [u64, i32, i32, f64, i32, p, p]
        L.or_seeded_rows.argtypes = [u64, i64, i32, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _check(st: int, what: str):
    if st != OK:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def splitmix64(state, count):
    """`count` consecutive SplitMix64 outputs from `state` (uint64 array)."""
    out = np.empty(count, np.uint64)
    lib().or_splitmix64(int(state) & (2**64 - 1), count, _ptr(out))
    return out


def seeded_params(seed, m, d, w, n_arrays=1, hash_kind="e2lsh"):
    """The seeded hash draws (A [2Hm, d], b [2Hm]) of a build from `seed`."""
    nh = 2 * int(n_arrays) * int(m)
    A = np.empty((nh, d), np.float32)
    b = np.empty(nh, np.float32)
    _check(lib().or_seeded_lsh(int(seed) & (2**64 - 1), nh, d, float(w),
                               int(hash_kind == "sign"), _ptr(A), _ptr(b)), "seeded_lsh")
    return A, b


def seeded_rows(seed, n, count):
    """The seeded k-means rows: the first `count` ids of a seeded shuffle."""
    out = np.empty(count, np.int64)
    _check(lib().or_seeded_rows(int(seed) & (2**64 - 1), int(n), int(count), _ptr(out)),
           "seeded_rows")
    return out


def digits(X, A, b, w):
    X, A, b = _f32(X), _f32(A), _f32(b)
    out = np.empty((X.shape[0], A.shape[0]), np.int32)
    _check(lib().or_digits(_ptr(X), X.shape[0], X.shape[1], _ptr(A), _ptr(b), A.shape[0],
                           float(w), _ptr(out)), "digits")
    return out


def digits_sign(X, A):
    """Random-hyperplane bits: out[r, i] = 1 if A[i] . X[r] >= 0 else 0."""
    X, A = _f32(X), _f32(A)
    out = np.empty((X.shape[0], A.shape[0]), np.int32)
    _check(lib().or_digits_sign(_ptr(X), X.shape[0], X.shape[1], _ptr(A), A.shape[0],
                                _ptr(out)), "digits_sign")
    return out


def dist_e(K1, K2, m, B):
    """2^B * dist_e of two m-bit hashkeys (an exact integer)."""
    return int(lib().or_dist_e(int(K1), int(K2), int(m), int(B)))


def window_expand(keys, pos, r, Kq, m, B):
    """(start, length) of the dist_e-guided expansion around `pos`."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    st = np.zeros(1, np.int64)
    ln = np.zeros(1, np.int64)
    lib().or_window_expand_pub(_ptr(keys), keys.shape[0], int(pos), int(r), int(Kq), int(m),
                               int(B), _ptr(st), _ptr(ln))
    return int(st[0]), int(ln[0])


def kmeans_assign(X, cent):
    X, cent = _f32(X), _f32(cent)
    out = np.empty(X.shape[0], np.int32)
    _check(lib().or_kmeans_assign(_ptr(X), X.shape[0], X.shape[1], _ptr(cent), cent.shape[0],
                                  _ptr(out)), "kmeans_assign")
    return out


def kmeans_update(X, assign, cent):
    X = _f32(X)
    cent = np.array(cent, dtype=np.float32, copy=True)
    assign = np.ascontiguousarray(assign, dtype=np.int32)
    counts = np.empty(cent.shape[0], np.int64)
    _check(lib().or_kmeans_update(_ptr(X), X.shape[0], X.shape[1], _ptr(assign),
                                  cent.shape[0], _ptr(cent), _ptr(counts)), "kmeans_update")
    return cent, counts


def kmeans_seed_farthest(X, C, first):
    """Farthest-first traversal from row `first`: C initial centre row ids."""
    X = _f32(X)
    ids = np.empty(C, np.int64)
    _check(lib().or_kmeans_seed_farthest(_ptr(X), X.shape[0], X.shape[1], C, int(first),
                                         _ptr(ids)), "kmeans_seed_farthest")
    return ids


def kmeans(X, C, init_ids, iters):
    X = _f32(X)
    init_ids = np.ascontiguousarray(init_ids, dtype=np.int64)
    cent = np.empty((C, X.shape[1]), np.float32)
    assign = np.empty(X.shape[0], np.int32)
    it = np.zeros(1, np.int32)
    _check(lib().or_kmeans(_ptr(X), X.shape[0], X.shape[1], C, _ptr(init_ids), iters,
                           _ptr(cent), _ptr(assign), _ptr(it)), "kmeans")
    return cent, assign, int(it[0])


def rmi_train(x, F):
    x = np.ascontiguousarray(x, dtype=np.float64)
    root = np.zeros(2)
    leaf = np.zeros(2 * F)
    elo = np.zeros(F, np.int32)
    ehi = np.zeros(F, np.int32)
    _check(lib().or_rmi_train(_ptr(x), x.shape[0], F, _ptr(root), _ptr(leaf), _ptr(elo),
                              _ptr(ehi)), "rmi_train")
    return root, leaf, elo, ehi


def rmi_predict(root, leaf, F, L, x):
    root = np.ascontiguousarray(root, dtype=np.float64)
    leaf = np.ascontiguousarray(leaf, dtype=np.float64)
    return int(lib().or_rmi_predict(_ptr(root), _ptr(leaf), F, L, float(x)))


def rmi_leaf(root, F, L, x):
    root = np.ascontiguousarray(root, dtype=np.float64)
    return int(lib().or_rmi_leaf(_ptr(root), F, L, float(x)))


def encode(h, mins, maxs, query=False):
    h = np.ascontiguousarray(h, dtype=np.int32)
    mins = np.ascontiguousarray(mins, dtype=np.int32)
    maxs = np.ascontiguousarray(maxs, dtype=np.int32)
    me = np.zeros(1, np.int32)
    K = lib().or_encode_box(_ptr(h), h.shape[0], _ptr(mins), _ptr(maxs), int(query), _ptr(me))
    return int(K), int(me[0])


def window(pos, r, L):
    s = np.zeros(1, np.int64)
    n = np.zeros(1, np.int64)
    lib().or_window_pub(pos, r, L, _ptr(s), _ptr(n))
    return int(s[0]), int(n[0])


def bruteforce(X, Q, k):
    X, Q = _f32(X), _f32(Q)
    ids = np.empty((Q.shape[0], k), np.int64)
    sc = np.empty((Q.shape[0], k), np.float64)
    _check(lib().or_bruteforce(_ptr(X), X.shape[0], X.shape[1], _ptr(Q), Q.shape[0], k,
                               _ptr(ids), _ptr(sc)), "bruteforce")
    return ids, sc


def pair_scores(X, Q, qi, xi):
    X, Q = _f32(X), _f32(Q)
    qi = np.ascontiguousarray(qi, dtype=np.int64)
    xi = np.ascontiguousarray(xi, dtype=np.int64)
    out = np.empty(qi.shape[0], np.float64)
    lib().or_pair_scores(_ptr(X), _ptr(Q), X.shape[1], _ptr(qi), _ptr(xi), qi.shape[0],
                         _ptr(out))
    return out


def core(digits, F, binary=False):
    """Build one stand-alone core model over items given in ascending id order
    (binary: bit hashkeys with the fixed [0, 1] box, key = Decimal(bits))."""
    dg = np.ascontiguousarray(digits, dtype=np.int32)
    L, m = dg.shape
    order = np.empty(L, np.int64)
    keys = np.empty(L, np.uint64)
    me = np.zeros(1, np.int32)
    mins = np.zeros(m, np.int32)
    maxs = np.zeros(m, np.int32)
    kk = np.zeros(2, np.uint64)
    dbl = np.zeros(3)
    leaf = np.zeros(2 * F)
    elo = np.zeros(F, np.int32)
    ehi = np.zeros(F, np.int32)
    _check(lib().or_core(L, m, F, _ptr(dg), int(bool(binary)), _ptr(order), _ptr(keys), _ptr(me),
                         _ptr(mins),
                         _ptr(maxs), _ptr(kk), _ptr(dbl), _ptr(leaf), _ptr(elo), _ptr(ehi)),
           "core")
    model = Model(L, int(me[0]), F, mins, maxs, int(kk[0]), int(kk[1]), float(dbl[0]),
                  dbl[1:3].copy(), leaf, elo, ehi)
    return order, keys, model


def core_query(model, qdigits):
    """(key, re-scaled key, predicted location) of query digits in a core model."""
    q = np.ascontiguousarray(qdigits, dtype=np.int32)
    m = q.shape[0]
    K = np.zeros(1, np.uint64)
    x = np.zeros(1)
    kk = np.array([model.kmin, model.kmax], np.uint64)
    dbl = np.array([model.scale, model.root[0], model.root[1]])
    leaf = np.ascontiguousarray(model.leaf, dtype=np.float64)
    pos = lib().or_core_query(model.L, m, model.F, model.m_eff,
                              _ptr(np.ascontiguousarray(model.mins, np.int32)),
                              _ptr(np.ascontiguousarray(model.maxs, np.int32)), _ptr(kk),
                              _ptr(dbl), _ptr(leaf), _ptr(q), _ptr(K), _ptr(x))
    return int(K[0]), float(x[0]), int(pos)


class Model:
    """One core model's parameters as copied out of the oracle index."""

    def __init__(self, L, m_eff, F, mins, maxs, kmin, kmax, scale, root, leaf, elo, ehi):
        self.L, self.m_eff, self.F = L, m_eff, F
        self.mins, self.maxs = mins, maxs
        self.kmin, self.kmax, self.scale = kmin, kmax, scale
        self.root, self.leaf, self.elo, self.ehi = root, leaf, elo, ehi


class Index:
    """Oracle LIDER index (Sections 3.2-3.3).  Keeps a reference to X.

    n_arrays = H hashkey arrays per core model (Section 3.3.1): A is
    [2 H m, d] -- rows h*m.. hash array h of the centroids retriever, rows
    H*m + h*m.. array h of every in-cluster retriever -- and b is [2 H m]."""

    def __init__(self, X, n_clusters, A, b, m, w, rmi_fanout, rmi_fanout_l1=None,
                 assignment=None, init_ids=None, kmeans_iters=20, seeding="given",
                 hash_kind="e2lsh", n_arrays=1):
        self.X = _f32(X)
        self.n, self.d = self.X.shape
        self.C, self.m, self.w = int(n_clusters), int(m), float(w)
        self.kind = {"e2lsh": 0, "sign": 1}[hash_kind]
        self.F2 = int(rmi_fanout)
        self.F1 = int(rmi_fanout_l1 if rmi_fanout_l1 is not None else rmi_fanout)
        self.H = int(n_arrays)
        self.A, self.b = _f32(A), _f32(b)
        nh = 2 * self.H * self.m
        assert self.A.shape == (nh, self.d) and self.b.shape == (nh,)
        asg = None if assignment is None else np.ascontiguousarray(assignment, dtype=np.int32)
        ini = None if init_ids is None else np.ascontiguousarray(init_ids, dtype=np.int64)
        if asg is None and ini is not None and seeding == "farthest":
            ini = kmeans_seed_farthest(self.X, self.C, int(ini[0]))
        self.seeds = ini
        if asg is None and ini is None:
            raise ValueError("need an assignment or k-means initial ids")
        st = C.c_int(0)
        h = lib().or_build(_ptr(self.X), self.n, self.d, self.C, _ptr(asg), _ptr(ini),
                           int(kmeans_iters), _ptr(self.A), _ptr(self.b), self.m, self.H, self.w,
                           self.F2, self.F1, self.kind, C.byref(st))
        _check(st.value, "build")
        self._h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_free(h)
            self._h = None

    # -- exported state ------------------------------------------------------
    def centroids(self):
        out = np.empty((self.C, self.d), np.float32)
        lib().or_get_centroids(self._h, _ptr(out))
        return out

    def assignment(self):
        out = np.empty(self.n, np.int32)
        lib().or_get_assign(self._h, _ptr(out))
        return out

    def iters_run(self):
        return int(lib().or_iters_run(self._h))

    def offsets(self):
        out = np.empty(self.C + 1, np.int64)
        lib().or_get_offsets(self._h, _ptr(out))
        return out

    def perm(self, array=0):
        """Sorted position -> original id in hashkey array `array`."""
        out = np.empty((self.H, self.n), np.int64)
        lib().or_get_perm(self._h, _ptr(out))
        return out[array].copy()

    def keys(self, array=0):
        out = np.empty((self.H, self.n), np.uint64)
        lib().or_get_keys(self._h, _ptr(out))
        return out[array].copy()

    def digits(self, array=0):
        out = np.empty((self.H, self.n, self.m), np.int32)
        lib().or_get_digits(self._h, _ptr(out))
        return out[array].copy()

    def layer1(self, array=0):
        order = np.empty((self.H, self.C), np.int64)
        keys = np.empty((self.H, self.C), np.uint64)
        dig = np.empty((self.H, self.C, self.m), np.int32)
        lib().or_get_l1(self._h, _ptr(order), _ptr(keys), _ptr(dig))
        return order[array].copy(), keys[array].copy(), dig[array].copy()

    def model(self, j, array=0):
        """Core model j of hashkey array `array` (j = C: the centroids retriever)."""
        F = self.F1 if j == self.C else self.F2
        j = array * (self.C + 1) + j
        ints = np.zeros(3, np.int64)
        mins = np.zeros(self.m, np.int32)
        maxs = np.zeros(self.m, np.int32)
        kk = np.zeros(2, np.uint64)
        dbl = np.zeros(3)
        leaf = np.zeros(2 * F)
        elo = np.zeros(F, np.int32)
        ehi = np.zeros(F, np.int32)
        lib().or_get_model(self._h, j, _ptr(ints), _ptr(mins), _ptr(maxs), _ptr(kk), _ptr(dbl),
                           _ptr(leaf), _ptr(elo), _ptr(ehi))
        return Model(int(ints[0]), int(ints[1]), int(ints[2]), mins, maxs, int(kk[0]),
                     int(kk[1]), float(dbl[0]), dbl[1:3].copy(), leaf, elo, ehi)

    # -- search ----------------------------------------------------------------
    def search(self, Q, k, c, r, r1=None, debug=False, expand_bits=0):
        Q = _f32(Q)
        nq = Q.shape[0]
        r1 = r if r1 is None else r1
        ids = np.empty((nq, k), np.int64)
        sc = np.empty((nq, k), np.float64)
        dbg = None
        H = self.H
        if debug:
            dbg = dict(qdigits=np.empty((nq, 2 * H * self.m), np.int32),
                       l1=np.empty((nq, H, 3), np.int64),
                       routed=np.empty((nq, c), np.int32),
                       pairs=np.empty((nq, c, H, 3), np.int64))
        _check(lib().or_search(self._h, _ptr(Q), nq, k, c, r, r1, int(expand_bits), _ptr(ids),
                               _ptr(sc),
                               _ptr(dbg["qdigits"]) if dbg else None,
                               _ptr(dbg["l1"]) if dbg else None,
                               _ptr(dbg["routed"]) if dbg else None,
                               _ptr(dbg["pairs"]) if dbg else None), "search")
        if debug and H == 1:  # one array: l1 [nq, 3], pairs [nq, c, 3]
            dbg["l1"] = dbg["l1"][:, 0]
            dbg["pairs"] = dbg["pairs"][:, :, 0]
        return (ids, sc, dbg) if debug else (ids, sc)
