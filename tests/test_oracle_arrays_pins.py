"""Pins of the oracle's multi-array core models (H hashkey arrays per core
model, Section 3.3.1): each array of an H-array index is the single-array
index built with that array's hash functions; a search scans every array's
window and keeps the union.  The single-array oracle is pinned elsewhere
against the paper; here the H-array oracle is pinned against it through the
paper's description of a multi-array core model -- the same process on every
array in parallel, then a merge of the results -- and against brute force."""
import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen


def _setup(H, n=3000, d=24, C=12, m=4, w=2.0, seed=0, kind="e2lsh"):
    X, lab, Q, _ = datagen.tiny(n=n, d=d, ncomp=C, nq=40, seed=seed)
    if kind == "sign":
        X = datagen.normalize_rows(X)
        Q = datagen.normalize_rows(Q)
    A, b = datagen.lsh_params(m, d, w, seed=seed + 5, n_arrays=H)
    return X, lab, Q, A, b, m, w, C


def _single(X, lab, A, b, m, w, C, H, h, F=4, kind="e2lsh"):
    Ah, bh = datagen.array_params(A, b, m, H, h)
    return oracle.Index(X, C, Ah, bh, m, w, F, assignment=lab, hash_kind=kind)


def _merge(lists, k):
    """Top k of the union of (id, score) lists by (score desc, id asc), each id once."""
    best = {}
    for ids, sc in lists:
        for i, s in zip(ids, sc):
            if i >= 0:
                best[int(i)] = float(s)
    order = sorted(best.items(), key=lambda t: (-t[1], t[0]))[:k]
    return [i for i, _ in order], [s for _, s in order]


@pytest.mark.parametrize("kind", ["e2lsh", "sign"])
def test_each_array_is_the_single_array_index(kind):
    H = 3
    X, lab, Q, A, b, m, w, C = _setup(H, kind=kind)
    oi = oracle.Index(X, C, A, b, m, w, 4, assignment=lab, n_arrays=H, hash_kind=kind)
    for h in range(H):
        si = _single(X, lab, A, b, m, w, C, H, h, kind=kind)
        assert np.array_equal(oi.perm(h), si.perm())
        assert np.array_equal(oi.keys(h), si.keys())
        assert np.array_equal(oi.digits(h), si.digits())
        for a, e in zip(oi.layer1(h), si.layer1()):
            assert np.array_equal(a, e)
        for j in (0, 5, C):
            Ma, Me = oi.model(j, array=h), si.model(j)
            assert (Ma.L, Ma.m_eff, Ma.kmin, Ma.kmax, Ma.scale) == \
                (Me.L, Me.m_eff, Me.kmin, Me.kmax, Me.scale)
            assert np.array_equal(Ma.leaf, Me.leaf) and np.array_equal(Ma.root, Me.root)
    assert np.array_equal(oi.offsets(), si.offsets())


@pytest.mark.parametrize("r1", [3, 5])
def test_routing_is_the_merge_of_the_arrays_routings(r1):
    """Layer 1: the routed clusters are the top c of the union of the H
    windows = the merge of the H single-array routings."""
    H, c = 3, 3
    X, lab, Q, A, b, m, w, C = _setup(H)
    oi = oracle.Index(X, C, A, b, m, w, 4, assignment=lab, n_arrays=H)
    _, _, dbg = oi.search(Q, 5, c, 50, r1=r1, debug=True)
    cent = oi.centroids().astype(np.float64)
    per = []
    for h in range(H):
        si = _single(X, lab, A, b, m, w, C, H, h)
        _, _, dh = si.search(Q, 5, c, 50, r1=r1, debug=True)
        per.append(dh)
        assert np.array_equal(dbg["l1"][:, h], dh["l1"])
    for q in range(Q.shape[0]):
        lists = []
        for dh in per:
            rt = dh["routed"][q]
            lists.append((rt, [float(Q[q].astype(np.float64) @ cent[j]) if j >= 0 else 0
                               for j in rt]))
        want, _ = _merge(lists, c)
        got = [int(j) for j in dbg["routed"][q] if j >= 0]
        assert got == want, q


@pytest.mark.parametrize("kind,eb", [("e2lsh", 0), ("sign", 0), ("sign", 2)])
def test_results_are_the_merge_of_the_arrays_results(kind, eb):
    """With every centroid in the layer-1 window the routing does not depend on
    the hashes, so the H-array top k is the merge of the H single-array top k
    lists (each id once)."""
    H, c, k, r = 4, 2, 10, 40
    X, lab, Q, A, b, m, w, C = _setup(H, kind=kind)
    oi = oracle.Index(X, C, A, b, m, w, 4, assignment=lab, n_arrays=H, hash_kind=kind)
    ids, sc, dbg = oi.search(Q, k, c, r, r1=C, debug=True, expand_bits=eb)
    res = []
    for h in range(H):
        si = _single(X, lab, A, b, m, w, C, H, h, kind=kind)
        ih, sh, dh = si.search(Q, k, c, r, r1=C, debug=True, expand_bits=eb)
        assert np.array_equal(dh["routed"], dbg["routed"])
        assert np.array_equal(dh["pairs"], dbg["pairs"][:, :, h])
        res.append((ih, sh))
    for q in range(Q.shape[0]):
        want_i, want_s = _merge([(ih[q], sh[q]) for ih, sh in res], k)
        nv = len(want_i)
        assert ids[q, :nv].tolist() == want_i and np.array_equal(sc[q, :nv], want_s), q
        assert (ids[q, nv:] == -1).all()
    # the union is larger than any single window: some query gains candidates
    assert any(len(set(ids[q]) - set(res[0][0][q])) > 0 for q in range(Q.shape[0]))


def test_repeated_array_changes_nothing():
    """Two arrays with the same hash functions index the same order: the union
    of their windows is one window, so results equal the single-array index."""
    X, lab, Q, A1, b1, m, w, C = _setup(1)
    A = np.vstack([A1[:m], A1[:m], A1[m:], A1[m:]])
    b = np.concatenate([b1[:m], b1[:m], b1[m:], b1[m:]])
    o2 = oracle.Index(X, C, A, b, m, w, 4, assignment=lab, n_arrays=2)
    o1 = oracle.Index(X, C, A1, b1, m, w, 4, assignment=lab)
    for r1 in (4, C):
        i2, s2 = o2.search(Q, 10, 3, 30, r1=r1)
        i1, s1 = o1.search(Q, 10, 3, 30, r1=r1)
        assert np.array_equal(i1, i2) and np.array_equal(s1, s2)
        for row in i2:  # no id twice
            v = row[row >= 0]
            assert len(set(v.tolist())) == len(v)


def test_whole_windows_give_exact_search():
    H = 3
    X, lab, Q, A, b, m, w, C = _setup(H)
    oi = oracle.Index(X, C, A, b, m, w, 4, assignment=lab, n_arrays=H)
    ids, sc = oi.search(Q, 7, C, X.shape[0], r1=C)
    bi, bs = oracle.bruteforce(X, Q, 7)
    assert np.array_equal(ids, bi) and np.allclose(sc, bs, rtol=0, atol=1e-12)


def test_union_windows_cover_more_than_one():
    """Small windows: the union of H windows holds up to H*r rows per cluster
    and never repeats a row; recall grows with H (Table 3's trend)."""
    X, lab, Q, A, b, m, w, C = _setup(8, n=4000, C=8)
    bi, _ = oracle.bruteforce(X, Q, 10)
    rec = []
    for H in (1, 2, 4, 8):
        AH = np.vstack([A[:H * m], A[8 * m:8 * m + H * m]])
        bH = np.concatenate([b[:H * m], b[8 * m:8 * m + H * m]])
        oi = oracle.Index(X, C, AH, bH, m, w, 4, assignment=lab, n_arrays=H)
        ids, _ = oi.search(Q, 10, 2, 20, r1=C)
        rec.append(np.mean([len(set(a) & set(t)) / 10 for a, t in zip(ids, bi)]))
    assert all(b2 >= a2 for a2, b2 in zip(rec, rec[1:])), rec
    assert rec[-1] > rec[0]
