"""Pins of the oracle's cosine variant (Section 4.1: random-hyperplane bits,
key = Decimal(bits)) and of the dist_e-guided bi-directional expansion
(Section 4.2), against hand-computed values, the paper's worked example, the
closed forms of Eq. (2) and Eq. (3) by Monte Carlo, Lemmas 2-3 by brute force,
and an independent sort-based formulation of the expansion."""
import math

import numpy as np
import pytest

import oracle


def test_sign_bits_hand():
    A = np.array([[1.0, -2.0, 0.5], [1.0, -1.0, 0.0]], np.float32)
    X = np.array([[1.5, 0.25, -1.0], [-1.0, 0.5, 2.0], [2.0, 2.0, 7.0]], np.float32)
    # row 0: a0.x = 0.5 -> 1, a1.x = 1.25 -> 1; row 1: -1.0 -> 0, -1.5 -> 0;
    # row 2: a0.x = 2 - 4 + 3.5 = 1.5 -> 1, a1.x = 0 exactly -> 1 (zero counts as >= 0)
    assert oracle.digits_sign(X, A).tolist() == [[1, 1], [0, 0], [1, 1]]


def test_sign_collision_probability_eq2():
    """P[h(p1) = h(p2)] = 1 - theta / pi for random hyperplanes (Eq. (2))."""
    rng = np.random.default_rng(1)
    d, nh = 16, 40000
    A = rng.standard_normal((nh, d)).astype(np.float32)
    for theta in (0.3, 1.0, 2.2):
        p1 = np.zeros(d, np.float32)
        p2 = np.zeros(d, np.float32)
        p1[0] = 1.0
        p2[0], p2[1] = math.cos(theta), math.sin(theta)
        h = oracle.digits_sign(np.stack([p1, p2]), A)
        frac = float(np.mean(h[0] == h[1]))
        p = 1.0 - theta / math.pi
        assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / nh), (theta, frac, p)


def test_prefix_probability_eq3():
    """P[KL(G(p1), G(p2)) <= m - l] = p(theta)^l (Lemma 1, Eq. (3)); KL is the
    integer part of dist_e."""
    rng = np.random.default_rng(2)
    d, m, trials, theta = 8, 6, 6000, 0.9
    p1 = np.zeros(d, np.float32)
    p2 = np.zeros(d, np.float32)
    p1[0] = 1.0
    p2[0], p2[1] = math.cos(theta), math.sin(theta)
    A = rng.standard_normal((trials * m, d)).astype(np.float32)
    h = oracle.digits_sign(np.stack([p1, p2]), A).reshape(2, trials, m)
    w = 1 << np.arange(m - 1, -1, -1)
    K1, K2 = (h[0] * w).sum(1), (h[1] * w).sum(1)
    B = 3
    KL = np.array([oracle.dist_e(a, b, m, B) >> B for a, b in zip(K1, K2)])
    p = 1.0 - theta / math.pi
    for l in range(0, m + 1):
        frac = float(np.mean(KL <= m - l))
        want = p ** l
        assert abs(frac - want) < 5 * math.sqrt(max(want * (1 - want), 1e-4) / trials) + 1e-9


def test_dist_e_worked_example():
    """Section 4.2's example: K_q = 000000, K_1 = 111111, K_2 = 100000, B = 3:
    dist_e(K_q, K_1) = 6 + 7/C, dist_e(K_q, K_2) = 6 + 4/C with C = 2^3."""
    Kq, K1, K2 = 0b000000, 0b111111, 0b100000
    assert oracle.dist_e(Kq, K1, 6, 3) == 6 * 8 + 7
    assert oracle.dist_e(Kq, K2, 6, 3) == 6 * 8 + 4
    # symmetric; identical keys are at distance 0
    assert oracle.dist_e(K1, Kq, 6, 3) == 6 * 8 + 7
    assert oracle.dist_e(K2, K2, 6, 3) == 0
    # common prefix '10' (l = 2): KL = 4, next 3 bits 110 vs 001 -> 5
    assert oracle.dist_e(0b101100, 0b100011, 6, 3) == 4 * 8 + 5
    # common prefix '0' (l = 1): KL = 5, next 3 bits 011 vs 100 -> 1
    assert oracle.dist_e(0b001100, 0b010000, 6, 3) == 5 * 8 + 1
    # fewer than B bits after the prefix: the remaining bits only
    assert oracle.dist_e(0b111110, 0b111111, 6, 3) == 1 * 8 + 1


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_dist_e_linear_order_lemmas(seed):
    """Lemmas 2 and 3: in a sorted array, distances to a key never decrease
    moving away from it on either side."""
    rng = np.random.default_rng(seed)
    m, B = 7, 3
    keys = np.sort(rng.integers(0, 1 << m, 60))
    for t in range(len(keys)):
        D = [oracle.dist_e(int(k), int(keys[t]), m, B) for k in keys]
        for i in range(t):  # left of t: farther left is not closer
            assert all(D[i2] >= D[i] for i2 in range(i)), (t, i)
        for j in range(t + 1, len(keys)):  # right of t
            assert all(D[j2] >= D[j] for j2 in range(j + 1, len(keys))), (t, j)


def test_expand_hand_case():
    keys = [0b0000, 0b0011, 0b0100, 0b1000, 0b1100]
    # Kq = 0101, pos 2 taken first; left 0011: prefix '0', KL 3, '01' vs '10' -> 13;
    # right 1000: KL 4, '10' vs '01' -> 17 -> left; then 0000: KL 3, '00' vs '10' -> 14
    # < 17 -> left: window [0, 3)
    assert oracle.window_expand(keys, 2, 3, 0b0101, 4, 2) == (0, 3)
    assert oracle.window_expand(keys, 2, 1, 0b0101, 4, 2) == (2, 1)
    assert oracle.window_expand(keys, 0, 3, 0b0101, 4, 2) == (0, 3)   # left end
    assert oracle.window_expand(keys, 4, 2, 0b0000, 4, 2) == (3, 2)   # right end
    assert oracle.window_expand(keys, 1, 9, 0b0101, 4, 2) == (0, 5)   # r > L
    assert oracle.window_expand([], 0, 4, 0, 4, 2) == (0, 0)


@pytest.mark.parametrize("seed", [6, 7, 8, 9])
def test_expand_matches_sorted_selection(seed):
    """From the query's own position the greedy expansion takes candidates in
    non-decreasing dist_e (Lemmas 2-3), left first on ties: the same set as
    sorting all candidates by (dist_e, left before right, distance)."""
    rng = np.random.default_rng(seed)
    m, B = 8, 3
    for _ in range(40):
        L = int(rng.integers(1, 50))
        keys = np.sort(rng.integers(0, 1 << m, L)).astype(np.uint64)
        Kq = int(rng.integers(0, 1 << m))
        pos = min(int(np.searchsorted(keys, Kq, side="left")), L - 1)
        r = int(rng.integers(1, L + 3))
        s, ln = oracle.window_expand(keys, pos, r, Kq, m, B)
        take = min(r, L)
        cand = [(oracle.dist_e(int(keys[p]), Kq, m, B), 0 if p < pos else 1, abs(p - pos), p)
                for p in range(L) if p != pos]
        chosen = {pos} | {c[3] for c in sorted(cand)[:take - 1]}
        assert ln == take and set(range(s, s + ln)) == chosen, (keys, Kq, pos, r)


def test_binary_core_key_is_decimal():
    """Binary hashkeys use the fixed box [0, 1]: the key is Decimal(bits) even
    where a bit is constant over the items."""
    bits = np.array([[1, 0, 1, 1], [0, 0, 1, 0], [1, 0, 0, 1], [0, 0, 1, 1]], np.int32)
    order, keys, model = oracle.core(bits, 1, binary=True)
    dec = [int("".join(map(str, b)), 2) for b in bits]
    assert sorted(dec) == keys.tolist()
    assert [dec[i] for i in order] == keys.tolist()
    assert model.mins.tolist() == [0] * 4 and model.maxs.tolist() == [1] * 4
    K, x, pos = oracle.core_query(model, np.array([1, 1, 1, 1], np.int32))
    assert K == 15  # a query bit string is never outside the box


def test_cosine_index_flat_special_case_and_expand():
    """Sign hashes with every cluster, whole clusters and the whole layer 1 give
    exact search; the expansion with r >= cluster size returns the same."""
    rng = np.random.default_rng(10)
    n, d, C, m = 1500, 24, 6, 5
    X = rng.standard_normal((n, d)).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Q = X[rng.choice(n, 20, replace=False)] + 0.05 * rng.standard_normal((20, d)).astype(np.float32)
    A = rng.standard_normal((2 * m, d)).astype(np.float32)
    b = np.zeros(2 * m, np.float32)
    lab = rng.integers(0, C, n).astype(np.int32)
    oi = oracle.Index(X, C, A, b, m, 1.0, 4, assignment=lab, hash_kind="sign")
    assert set(np.unique(oi.digits())) <= {0, 1}
    bi, bs = oracle.bruteforce(X, Q, 7)
    for eb in (0, 3):
        ids, sc = oi.search(Q, 7, C, n, C, expand_bits=eb)
        assert np.array_equal(ids, bi) and np.allclose(sc, bs, rtol=0, atol=1e-12)
    # keys are Decimal(bits) of the layer-2 digits in sorted order
    w = 1 << np.arange(m - 1, -1, -1)
    dg = oi.digits()[oi.perm()]
    assert np.array_equal(oi.keys(), (dg * w).sum(1).astype(np.uint64))
    with pytest.raises(RuntimeError):  # expansion needs binary hashkeys
        oracle.Index(X, C, A, b, m, 1.0, 4, assignment=lab).search(Q, 7, 2, 50, expand_bits=3)
