"""Pins of the FP64 oracle against things other than itself: hand-computed
cases (tests/golden/hand_cases.json), closed forms, library routines (numpy
least squares, FP64 matmul, lexicographic tuple sort) and brute force.
CPU only."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


# --------------------------------------------------------------------------- hashes
@pytest.mark.parametrize("case", GOLD["hash"]["cases"])
def test_hand_hashes(case):
    X = np.array([case["x"]], np.float32)
    A = np.array([case["a"]], np.float32)
    b = np.array([case["b"]], np.float32)
    h = oracle.digits(X, A, b, case["w"])
    assert h[0, 0] == case["h"]


def test_digits_match_fp64_matmul_away_from_edges():
    g = np.random.default_rng(11)
    X = g.standard_normal((500, 96)).astype(np.float32) * 3
    A = g.standard_normal((12, 96)).astype(np.float32)
    b = (g.random(12) * 2.0).astype(np.float32)
    h = oracle.digits(X, A, b, 2.0)
    t = (X.astype(np.float64) @ A.T.astype(np.float64) + b.astype(np.float64)) / 2.0
    ok = np.abs(t - np.round(t)) > 1e-9
    assert ok.mean() > 0.99
    assert np.array_equal(h[ok], np.floor(t[ok]).astype(np.int32))


def test_digit_range_error():
    X = np.array([[3e9]], np.float32)
    with pytest.raises(RuntimeError):
        oracle.digits(X, np.ones((1, 1), np.float32), np.zeros(1, np.float32), 1.0)


# --------------------------------------------------------------------------- keys
def test_hand_keys_and_ranks():
    kc = GOLD["key"]
    mem = np.array(kc["members"], np.int32)
    mins, maxs = np.array(kc["box_min"]), np.array(kc["box_max"])
    for t, K in zip(mem, kc["keys"]):
        assert oracle.encode(t, mins, maxs)[0] == K
    order, keys, model = oracle.core(mem, 1)
    assert list(order) == kc["sorted_order"]
    assert list(keys) == kc["sorted_keys"]
    assert list(model.mins) == kc["box_min"] and list(model.maxs) == kc["box_max"]
    for qc in kc["queries"]:
        K, _ = oracle.encode(np.array(qc["h"]), mins, maxs, query=True)
        assert K == qc["K"]
        assert int(np.searchsorted(keys.astype(np.int64), K, side="left")) == qc["rank"]


@pytest.mark.parametrize("seed", range(5))
def test_key_order_is_lexicographic_and_query_rank_exact(seed):
    """Data keys sort exactly like the digit tuples (Section 4.2 element-wise
    order), and a saturated query key's rank among data keys equals the number
    of data tuples lexicographically smaller than the query tuple."""
    g = np.random.default_rng(seed)
    m = int(g.integers(1, 5))
    L = int(g.integers(1, 60))
    dig = g.integers(-4, 5, size=(L, m)).astype(np.int32)
    order, keys, model = oracle.core(dig, 3)
    tuples = [tuple(r) for r in dig]
    ref = sorted(range(L), key=lambda i: (tuples[i], i))
    assert list(order) == ref
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    for q in g.integers(-7, 8, size=(40, m)).astype(np.int32):
        K, x, pos = oracle.core_query(model, q)
        rank = sum(1 for t in tuples if t < tuple(q))
        assert int(np.searchsorted(keys.astype(np.int64), K, side="left")) == rank


def test_key_prefix_when_radix_product_exceeds_2_53():
    mins = np.zeros(4, np.int32)
    maxs = np.array([2 ** 20, 2 ** 20, 2 ** 20, 5], np.int32)
    K, m_eff = oracle.encode(np.array([1, 2, 3, 4], np.int32), mins, maxs)
    assert m_eff == 2  # (2^20+1)^3 > 2^53, (2^20+1)^2 fits
    assert K == 1 * (2 ** 20 + 1) + 2


# --------------------------------------------------------------------------- RMI
def test_hand_rmi():
    rc, kc = GOLD["rmi"], GOLD["key"]
    order, keys, model = oracle.core(np.array(kc["members"], np.int32), rc["F"])
    assert model.scale == float(Fraction(rc["scale_num"], rc["scale_den"]))
    assert abs(model.root[0] - rc["slope_num"] / rc["slope_den"]) < 1e-15
    assert abs(model.root[1] - rc["icpt_num"] / rc["icpt_den"]) < 1e-15
    assert model.elo[0] == rc["elo"] and model.ehi[0] == rc["ehi"]
    for p, K in enumerate(keys):
        x = (int(K) - model.kmin) * model.scale
        assert abs(x - rc["x"][p]) < 1e-15
        assert oracle.rmi_predict(model.root, model.leaf, 1, 3, x) == rc["positions"][p]
    for qc in rc["queries"]:
        K, x, pos = oracle.core_query(model, np.array(qc["h"], np.int32))
        assert K == qc["K"]
        assert abs(x - qc["x_num"] / qc["x_den"]) < 1e-15
        assert pos == qc["pos"]


@pytest.mark.parametrize("F", [2, 4])
def test_hand_rmi_leaf_routing(F):
    """Two-stage RMI with F >= 2 worked out by hand (golden "rmi_leaves"):
    the root line, which leaf owns each key, each leaf's least-squares line
    (an empty leaf copies the root), the error bounds, and the leaf and
    location of query keys on both sides of every leaf boundary, beyond
    both ends of the location range, and NaN."""
    gc = GOLD["rmi_leaves"]
    fc = gc[f"F{F}"]
    L = gc["L"]
    x = np.array(gc["x"])
    root, leaf, elo, ehi = oracle.rmi_train(x, F)
    rs = Fraction(gc["root_slope_num"], gc["root_slope_den"])
    ri = Fraction(gc["root_icpt_num"], gc["root_icpt_den"])
    assert root[0] == float(rs)  # 42 / 49.875, both exact: one correctly rounded division
    assert abs(root[1] - float(ri)) <= 2e-16 * 4
    for j, want in enumerate(fc["leaves"]):
        if want == "root":
            assert (leaf[2 * j], leaf[2 * j + 1]) == (root[0], root[1])
        else:  # collinear members with dyadic coordinates: the fit is exact
            assert (leaf[2 * j], leaf[2 * j + 1]) == tuple(want)
    assert list(elo) == fc["elo"] and list(ehi) == fc["ehi"]
    for i in range(L):
        assert oracle.rmi_leaf(root, F, L, x[i]) == fc["leaf_of_key"][i]
        assert oracle.rmi_predict(root, leaf, F, L, x[i]) == i
    for qc in fc["queries"]:
        xq = float(qc["x"])
        if "p0" in qc:
            assert abs(root[0] * xq + root[1] - float(Fraction(qc["p0"]))) < 1e-12
        assert oracle.rmi_leaf(root, F, L, xq) == qc["leaf"], qc
        assert oracle.rmi_predict(root, leaf, F, L, xq) == qc["pos"], qc
    # the same model built from one-digit keys, and queried through the key path
    order, keys, model = oracle.core(np.array(gc["keys"], np.int32)[:, None], F)
    assert list(order) == list(range(L)) and [int(k) for k in keys] == gc["keys"]
    assert model.scale == 0.5
    assert np.array_equal(model.root, root) and np.array_equal(model.leaf, leaf)
    for qc in fc["key_queries"]:
        K, xq, pos = oracle.core_query(model, np.array([qc["digit"]], np.int32))
        assert K == qc["K"] and xq == K / 2
        assert oracle.rmi_leaf(model.root, F, L, xq) == qc["leaf"]
        assert pos == qc["pos"], qc


@pytest.mark.parametrize("seed", range(4))
def test_ols_matches_numpy_least_squares(seed):
    g = np.random.default_rng(seed)
    L = int(g.integers(50, 3000))
    x = np.sort(g.random(L) ** 2 * (L - 1))
    F = int(g.integers(1, 9))
    root, leaf, elo, ehi = oracle.rmi_train(x, F)
    y = np.arange(L, dtype=np.float64)
    s, c = np.polyfit(x, y, 1)
    assert abs(root[0] - s) <= 1e-9 * max(1, abs(s)) and abs(root[1] - c) <= 1e-7 * max(1, L)
    leafs = np.array([oracle.rmi_leaf(root, F, L, v) for v in x])
    assert np.all(np.diff(leafs) >= 0)  # routing is monotone: leaves own position ranges
    for j in range(F):
        sel = leafs == j
        if sel.sum() >= 2 and np.ptp(x[sel]) > 0:
            s, c = np.polyfit(x[sel], y[sel], 1)
            assert abs(leaf[2 * j] - s) <= 1e-7 * max(1, abs(s))
            assert abs(leaf[2 * j + 1] - c) <= 1e-6 * max(1, L)
        elif sel.sum() == 0:
            assert leaf[2 * j] == root[0] and leaf[2 * j + 1] == root[1]
        # residual conditions of least squares
        if sel.sum() >= 2 and np.ptp(x[sel]) > 0:
            res = y[sel] - (leaf[2 * j] * x[sel] + leaf[2 * j + 1])
            assert abs(res.sum()) < 1e-6 * L
            assert abs((res * (x[sel] - x[sel].mean())).sum()) < 1e-6 * L * L
        # error bounds contain every true position
        for i in np.where(sel)[0]:
            p = oracle.rmi_predict(root, leaf, F, L, x[i])
            assert elo[j] <= i - p <= ehi[j]


def test_exactly_linear_keys_have_zero_error():
    L = 1000
    dig = np.arange(L, dtype=np.int32)[:, None] * 3  # keys 0,3,6,... -> x = i exactly
    order, keys, model = oracle.core(dig, 8)
    assert model.scale == (L - 1) / (3 * (L - 1))
    assert np.all(model.elo == 0) and np.all(model.ehi == 0)


def test_rmi_clamps_out_of_range():
    root, leaf, elo, ehi = oracle.rmi_train(np.arange(10.0), 2)
    assert oracle.rmi_predict(root, leaf, 2, 10, -100.0) == 0
    assert oracle.rmi_predict(root, leaf, 2, 10, 1e6) == 9
    assert oracle.rmi_predict(root, leaf, 2, 10, float("nan")) == 0


@pytest.mark.parametrize("case", GOLD["window"]["cases"])
def test_window(case):
    assert oracle.window(case["pos"], case["r"], case["L"]) == (case["start"], case["len"])


# --------------------------------------------------------------------------- k-means
def test_kmeans_assign_matches_numpy_argmin():
    g = np.random.default_rng(5)
    X = g.standard_normal((700, 40)).astype(np.float32)
    cent = g.standard_normal((13, 40)).astype(np.float32)
    a = oracle.kmeans_assign(X, cent)
    d = ((X.astype(np.float64)[:, None, :] - cent.astype(np.float64)[None]) ** 2).sum(-1)
    srt = np.sort(d, axis=1)
    clear = srt[:, 1] - srt[:, 0] > 1e-9
    assert np.array_equal(a[clear], d.argmin(1)[clear])


def test_kmeans_assign_tie_goes_to_smaller_index():
    X = np.array([[0.0, 0.0]], np.float32)
    cent = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]], np.float32)
    assert oracle.kmeans_assign(X, cent)[0] == 0


def test_kmeans_update_is_member_mean():
    g = np.random.default_rng(6)
    X = g.standard_normal((1000, 24)).astype(np.float32)
    asg = g.integers(0, 9, 1000).astype(np.int32)
    asg[asg == 4] = 5  # cluster 4 empty
    prev = np.full((9, 24), 7.0, np.float32)
    cent, counts = oracle.kmeans_update(X, asg, prev)
    assert counts[4] == 0 and np.all(cent[4] == 7.0)
    for j in range(9):
        if counts[j]:
            mem = X[asg == j].astype(np.float64)
            exact = mem.sum(0) / counts[j]
            assert np.all(np.abs(cent[j] - exact) <= np.spacing(np.abs(exact).astype(np.float32)))


def test_kmeans_recovers_separated_blobs():
    g = np.random.default_rng(7)
    centers = g.standard_normal((6, 16)) * 50
    lab = np.repeat(np.arange(6), 40)
    X = (centers[lab] + g.standard_normal((240, 16))).astype(np.float32)
    init = np.array([0, 40, 80, 120, 160, 200])
    cent, asg, it = oracle.kmeans(X, 6, init, 20)
    assert np.array_equal(asg, lab)
    assert it == 2  # second assignment finds no change
    for j in range(6):
        assert np.allclose(cent[j], X[lab == j].astype(np.float64).mean(0), atol=1e-5)


def test_farthest_first_seeds_match_numpy_maximin():
    g = np.random.default_rng(16)
    X = (g.standard_normal((700, 12)) * g.uniform(0.5, 3, (700, 1))).astype(np.float32)
    ids = oracle.kmeans_seed_farthest(X, 9, 5)
    Xd = X.astype(np.float64)
    ref = [5]
    D = np.full(700, np.inf)
    for t in range(1, 9):
        D = np.minimum(D, ((Xd - Xd[ref[-1]]) ** 2).sum(1))
        ref.append(int(np.argmax(D)))  # first maximum = smallest id
    assert list(ids) == ref
    # every chosen row maximises the distance to its nearest earlier centre
    for t in range(1, 9):
        dmin = ((Xd[:, None, :] - Xd[ids[:t]][None]) ** 2).sum(-1).min(1)
        assert dmin[ids[t]] == dmin.max()


def test_farthest_first_seeds_every_blob():
    g = np.random.default_rng(17)
    centers = g.standard_normal((7, 20)) * 30
    lab = np.repeat(np.arange(7), 50)
    X = (centers[lab] + g.standard_normal((350, 20))).astype(np.float32)
    ids = oracle.kmeans_seed_farthest(X, 7, 0)
    assert sorted(lab[ids].tolist()) == list(range(7))


def test_kmeans_objective_never_increases():
    X, lab, _, _ = datagen.tiny(n=3000, d=32)
    init = datagen.kmeans_init(3000, 16)
    prev = np.inf
    for iters in range(1, 6):
        cent, asg, it = oracle.kmeans(X, 16, init, iters)
        obj = ((X.astype(np.float64) - cent[asg].astype(np.float64)) ** 2).sum()
        assert obj <= prev * (1 + 1e-12)
        prev = obj


# --------------------------------------------------------------------------- index + search
def _tiny_index(n=4000, d=32, C=8, m=4, w=1.0, F=4, assignment=None):
    X, lab, Q, src = datagen.tiny(n=n, d=d, ncomp=C, nq=50)
    A, b = datagen.lsh_params(m, d, w)
    ix = oracle.Index(X, C, A, b, m, w, F, assignment=assignment,
                      init_ids=datagen.kmeans_init(n, C), kmeans_iters=10)
    return ix, X, Q


def test_index_invariants():
    ix, X, Q = _tiny_index()
    off, perm, keys = ix.offsets(), ix.perm(), ix.keys()
    asg, dig = ix.assignment(), ix.digits()
    assert off[0] == 0 and off[-1] == ix.n
    assert np.array_equal(np.sort(perm), np.arange(ix.n))
    cent = ix.centroids()
    for j in range(ix.C):
        ids = perm[off[j]:off[j + 1]]
        assert np.all(asg[ids] == j)
        model = ix.model(j)
        assert model.L == len(ids)
        kj = keys[off[j]:off[j + 1]].astype(np.int64)
        assert np.all(np.diff(kj) >= 0)  # sorted array is monotone
        tup = [tuple(dig[i]) + (i,) for i in ids]
        assert tup == sorted(tup)  # key order = lexicographic digit order, ties by id
        if model.L:
            assert np.array_equal(model.mins, dig[ids].min(0))
            assert np.array_equal(model.maxs, dig[ids].max(0))
            x = (kj - model.kmin) * model.scale
            assert x[0] == 0.0 and abs(x[-1] - (model.L - 1)) <= 4 * np.spacing(model.L)
            assert np.all(x >= 0) and np.all(x <= model.L - 1 + 1e-9)  # Eq. (8) range
            for p, xv in enumerate(x):
                lf = oracle.rmi_leaf(model.root, model.F, model.L, xv)
                pos = oracle.rmi_predict(model.root, model.leaf, model.F, model.L, xv)
                assert model.elo[lf] <= p - pos <= model.ehi[lf]
            np.testing.assert_allclose(cent[j], X[ids].astype(np.float64).mean(0), atol=1e-5)
    order, k1, d1 = ix.layer1()
    assert np.array_equal(np.sort(order), np.arange(ix.C))
    assert np.array_equal(d1, oracle.digits(cent, ix.A[:ix.m], ix.b[:ix.m], ix.w))


def test_search_degenerates_to_flat_search():
    """c = all clusters, r >= largest cluster, r1 >= clusters: LIDER scans the
    whole corpus, so it must return exactly the Flat (brute-force) top-k."""
    ix, X, Q = _tiny_index()
    L = np.diff(ix.offsets()).max()
    ids, sc = ix.search(Q, 10, ix.C, int(L), ix.C)
    bi, bs = oracle.bruteforce(X, Q, 10)
    assert np.array_equal(ids, bi) and np.array_equal(sc, bs)


def test_bruteforce_matches_numpy():
    g = np.random.default_rng(9)
    X = g.standard_normal((800, 20)).astype(np.float32)
    Q = g.standard_normal((30, 20)).astype(np.float32)
    ids, sc = oracle.bruteforce(X, Q, 7)
    S = Q.astype(np.float64) @ X.astype(np.float64).T
    for q in range(30):
        ref = np.lexsort((np.arange(800), -S[q]))[:7]
        assert np.array_equal(ids[q], ref)
        np.testing.assert_allclose(sc[q], S[q, ref], rtol=1e-12)


def test_search_debug_consistency():
    ix, X, Q = _tiny_index(C=8)
    k, c, r, r1 = 5, 3, 40, 6
    ids, sc, dbg = ix.search(Q, k, c, r, r1, debug=True)
    cent = ix.centroids()
    order, _, _ = ix.layer1()
    qd = oracle.digits(Q, ix.A, ix.b, ix.w)
    assert np.array_equal(dbg["qdigits"], qd)
    off, perm = ix.offsets(), ix.perm()
    for q in range(Q.shape[0]):
        pos1, s1, len1 = dbg["l1"][q]
        assert (s1, len1) == oracle.window(pos1, r1, ix.C)
        win = order[s1:s1 + len1]
        sc1 = cent[win].astype(np.float64) @ Q[q].astype(np.float64)
        ref = win[np.lexsort((win, -sc1))][:c]
        assert np.array_equal(dbg["routed"][q][:len(ref)], ref)
        cand = []
        for t, j in enumerate(dbg["routed"][q]):
            pos, s, ln = dbg["pairs"][q, t]
            model = ix.model(j)
            K, x, p2 = oracle.core_query(model, qd[q, ix.m:])
            assert p2 == pos and (s, ln) == oracle.window(pos, r, model.L)
            cand.extend(perm[off[j] + s: off[j] + s + ln])
        cand = np.array(cand)
        s2 = X[cand].astype(np.float64) @ Q[q].astype(np.float64)
        top = cand[np.lexsort((cand, -s2))][:k]
        assert np.array_equal(ids[q][:len(top)], top)
        assert np.all(ids[q][len(top):] == -1)


def test_search_pads_when_fewer_than_k_candidates():
    ix, X, Q = _tiny_index(C=8)
    ids, sc = ix.search(Q[:3], 50, 1, 7, 8)
    assert np.all(ids[:, 7:] == -1) and np.all(np.isneginf(sc[:, 7:]))
    assert np.all(ids[:, :7] >= 0)


def test_given_assignment_build():
    X, lab, Q, src = datagen.tiny(n=2000, d=16, ncomp=5, nq=10)
    A, b = datagen.lsh_params(3, 16, 1.0)
    ix = oracle.Index(X, 6, A, b, 3, 1.0, 4, assignment=lab)  # cluster 5 is empty
    assert np.array_equal(ix.assignment(), lab)
    assert ix.model(5).L == 0 and np.all(ix.centroids()[5] == 0)
    ids, sc = ix.search(Q, 5, 6, 10000, 6)
    bi, bs = oracle.bruteforce(X, Q, 5)
    assert np.array_equal(ids, bi)
