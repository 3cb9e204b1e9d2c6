"""Pins of the oracle's seeded draws (the E2LSH parameters a_i ~ N(0, I),
b_i ~ U[0, w) of Section 4 and the k-means seed rows) against published
SplitMix64 output values, the polar form of the Box-Muller transform, the
uniform and normal distributions, and the uniformity of the shuffle.  CPU only."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle


def test_splitmix64_published_outputs():
    # the first outputs from state 1234567 and from state 0, as published with
    # the generator's reference implementation and its ports
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [int(v) for v in oracle.splitmix64(1234567, 5)] == want
    assert int(oracle.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


def _stream_state(seed, s):
    # stream s starts at seed xor the (s+1)-th output of the generator from state 0
    return (int(seed) ^ int(oracle.splitmix64(0, s + 1)[s])) & (2**64 - 1)


def _uniforms(seed, s, count):
    x = oracle.splitmix64(_stream_state(seed, s), count)
    return (x >> np.uint64(11)).astype(np.float64) * 2.0**-53


@pytest.mark.parametrize("seed,m,d,H", [(0, 4, 129, 1), (12345, 8, 768, 1), (2**63 + 5, 3, 40, 2)])
def test_seeded_projections_are_box_muller_pairs(seed, m, d, H):
    A, b = oracle.seeded_params(seed, m, d, 2.0, n_arrays=H)
    nh = 2 * H * m
    a = A.reshape(-1).astype(np.float64)
    npair = (a.size + 1) // 2
    u = _uniforms(seed, 0, 2 * npair + nh)
    u1, u2 = u[0:2 * npair:2], u[1:2 * npair:2]
    z0 = a[0::2]
    z1 = a[1::2]
    # radius: z0^2 + z1^2 = -2 ln(1 - u1) (up to the fp32 rounding of z0, z1)
    full = z1.size
    r2 = z0[:full] ** 2 + z1 ** 2
    want = -2.0 * np.log1p(-u1[:full])
    assert np.all(np.abs(r2 - want) <= 3e-7 * want + 1e-30)
    # angle: atan2(z1, z0) = 2 pi u2 modulo 2 pi
    ang = np.mod(np.arctan2(z1, z0[:full]), 2 * np.pi)
    dif = np.abs(ang - 2 * np.pi * u2[:full])
    dif = np.minimum(dif, 2 * np.pi - dif)
    big = want > 1e-6
    assert np.all(dif[big] <= 1e-6 / np.sqrt(want[big]) + 1e-9)
    if a.size % 2:  # odd count: the last value is the cosine half of its pair
        assert abs(z0[-1] - math.sqrt(-2 * math.log1p(-u1[-1])) * math.cos(2 * math.pi * u2[-1])) \
            <= 1e-6 * max(1.0, abs(z0[-1]))
    # offsets: the uniforms after the normals, times w, rounded to fp32
    ub = u[2 * npair:]
    assert np.array_equal(b, (ub * 2.0).astype(np.float32))
    assert np.all((b >= 0) & (b <= 2.0))


def test_seeded_projections_are_standard_normal():
    A, _ = oracle.seeded_params(99, 16, 768, 1.0, n_arrays=2)
    a = A.reshape(-1).astype(np.float64)
    assert stats.kstest(a, "norm").pvalue > 1e-4
    assert abs(a.mean()) < 5 / math.sqrt(a.size)
    assert abs(a.var() - 1) < 5 * math.sqrt(2 / a.size)


def test_seeded_offsets_are_uniform_and_sign_hash_has_none():
    _, b = oracle.seeded_params(5, 16, 8, 3.0, n_arrays=16)
    assert stats.kstest(b / 3.0, "uniform").pvalue > 1e-4
    A1, b1 = oracle.seeded_params(5, 16, 8, 3.0, n_arrays=16, hash_kind="sign")
    A2, _ = oracle.seeded_params(5, 16, 8, 3.0, n_arrays=16)
    assert np.array_equal(A1, A2) and not b1.any()


def test_seeded_rows_are_a_shuffle_prefix():
    n = 1000
    full = oracle.seeded_rows(42, n, n)
    assert np.array_equal(np.sort(full), np.arange(n))
    for cnt in (0, 1, 7, 999):
        assert np.array_equal(oracle.seeded_rows(42, n, cnt), full[:cnt])
    # the first id is the high half of x * n for the first output x of stream 1
    x = int(oracle.splitmix64(_stream_state(42, 1), 1)[0])
    assert full[0] == (x * n) >> 64
    # large n: in range and distinct
    big = oracle.seeded_rows(7, 3_000_000_000 // 1000, 64)
    assert len(set(big.tolist())) == 64 and big.min() >= 0 and big.max() < 3_000_000


def test_seeded_shuffle_is_uniform():
    # all 24 orders of 4 ids over 2,400 seeds: chi-square against uniform
    counts = {}
    for seed in range(2400):
        key = tuple(oracle.seeded_rows(seed, 4, 4).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 24
    assert stats.chisquare(list(counts.values())).pvalue > 1e-4
