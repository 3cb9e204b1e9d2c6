"""GPU parity of multi-array core models (H hashkey arrays per core model,
Section 3.3.1): every array's digits, sorted order, keys and RMI bit-exact
against the oracle; searches scan one window per array in both layers and
score the union -- query digits, every array's windows and the routed sets
identical, ids and scores within the fp32 tolerance."""
import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen

from parity_util import build_pair, compare_debug, compare_index, compare_topk

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _run(fx, k, c, r, r1, **kw):
    torch = _torch()
    X, Q, gi, oi = fx["X"], fx["Q"], fx["gi"], fx["oi"]
    eb = kw.get("expand_bits", 0)
    ids, sc, dbg = gi.search(torch.from_numpy(Q).cuda(), k, c, r, r1=r1, debug=True, **kw)
    torch.cuda.synchronize()
    oids, osc, odbg = oi.search(Q, k, c, r, r1 or None, debug=True, expand_bits=eb)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    return ids, sc


@pytest.fixture(scope="module")
def tiny3():
    """Tiny mixture (N=20,000, d=128, 16 given clusters, m=4, w=1), H=3."""
    _torch()
    X, lab, Q, _ = datagen.tiny()
    A, b = datagen.lsh_params(4, 128, 1.0, seed=21, n_arrays=3)
    gi, oi, _ = build_pair(X, 16, 4, 1.0, 8, A, b, assignment=lab, n_arrays=3)
    return dict(X=X, Q=Q, gi=gi, oi=oi)


def test_tiny3_build_bit_exact(tiny3):
    compare_index(tiny3["gi"], tiny3["oi"])


@pytest.mark.parametrize("k,c,r,r1", [(10, 4, 64, 3), (10, 2, 200, 16), (100, 4, 64, 5),
                                       (7, 3, 33, 1), (1, 1, 1, 0), (10, 16, 5000, 16),
                                       (200, 2, 40, 2),
                                       # 64 < k <= 128 over at most 2,048 hull rows per
                                       # query: the wave selection with dropped rows
                                       (100, 1, 64, 5), (70, 1, 300, 3)])
def test_tiny3_search(tiny3, k, c, r, r1):
    _run(tiny3, k, c, r, r1)


@pytest.fixture(scope="module")
def mid10():
    """768-d mixture at 60,000 rows, 64 given clusters (cluster 63 empty),
    m=8, w=2, fanout 16 / 4, and the paper's H = 10 arrays."""
    torch = _torch()
    X, lab = datagen.mixture(60000, 768, ncomp=63, seed=5, device="cpu")
    X, lab = X.numpy(), lab.numpy()
    Qt, _ = datagen.queries_from(torch.from_numpy(X), 200, 0.1, seed=6)
    A, b = datagen.lsh_params(8, 768, 2.0, seed=23, n_arrays=10)
    gi, oi, _ = build_pair(X, 64, 8, 2.0, 16, A, b, assignment=lab, F1=4, n_arrays=10,
                           storage="bf16")
    return dict(X=X, Q=Qt.numpy(), gi=gi, oi=oi, A=A, b=b, lab=lab)


def test_mid10_build_bit_exact(mid10):
    compare_index(mid10["gi"], mid10["oi"])


@pytest.mark.parametrize("k,c,r,r1", [(10, 8, 256, 32), (100, 8, 256, 32), (10, 4, 64, 64),
                                       (1000, 16, 100, 20), (3, 1, 17, 1), (10, 2, 2000, 6),
                                       (100, 2, 256, 32)])
def test_mid10_search(mid10, k, c, r, r1):
    _run(mid10, k, c, r, r1)


def test_mid10_schedules_identical(mid10):
    """Persistent / plain / workgroup rerank, all tile sizes, routing paths:
    bitwise equal."""
    torch = _torch()
    Qd = torch.from_numpy(mid10["Q"]).cuda()
    gi = mid10["gi"]
    ref = gi.search(Qd, 10, 8, 256, r1=32)
    for kw in [dict(persistent=True), dict(tile_rows=32), dict(tile_rows=64),
               dict(persistent=2), dict(tile_rows=32, persistent=2, grid_mult=1),
               dict(pass_pairs=16), dict(pass_pairs=32), dict(pass_pairs=64),
               dict(tile_rows=32, pass_pairs=128), dict(tile_rows=128),
               dict(tile_rows=128, pass_pairs=128), dict(tile_rows=128, pass_pairs=16)]:
        got = gi.search(Qd, 10, 8, 256, r1=32, **kw)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), kw
    sub = gi.search(Qd[11:50].contiguous(), 10, 8, 256, r1=32)
    assert torch.equal(sub[0], ref[0][11:50]) and torch.equal(sub[1], ref[1][11:50])
    # whole layer 1: bf16-candidate routing and the fp32 dense product agree
    a = gi.search(Qd, 10, 4, 128, r1=64)
    b = gi.search(Qd, 10, 4, 128, r1=64, l1_dense=1)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_mid10_recall_grows_with_arrays(mid10):
    """Same windows, more arrays: the candidate union grows, so recall@10
    against exact search does not fall (Table 3's trend), and H = 10 beats
    H = 1 on these small windows."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    X, Q, A, b, lab = mid10["X"], mid10["Q"], mid10["A"], mid10["b"], mid10["lab"]
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    exact, _ = oracle.bruteforce(X, Q, 10)
    rec = []
    for H in (1, 2, 5, 10):
        AH = np.vstack([A[:H * 8], A[80:80 + H * 8]])
        bH = np.concatenate([b[:H * 8], b[80:80 + H * 8]])
        gi = lider.Index(Xd, 64, 8, 2.0, 16, (AH, bH), rmi_fanout_l1=4,
                         assignment=torch.from_numpy(lab).cuda(), n_arrays=H)
        ids, _ = gi.search(Qd, 10, 4, 64, r1=64)
        ids = ids.cpu().numpy()
        rec.append(np.mean([len(set(a) & set(t)) / 10 for a, t in zip(ids, exact)]))
        gi.close()
    assert all(y >= x for x, y in zip(rec, rec[1:])), rec
    assert rec[-1] > rec[0] + 0.05, rec


def test_mid10_precision_form(mid10):
    """Ten arrays, bf16 union windows + certified shortlist + fp32 rerank: ids
    and scores equal the oracle's within the fp32 tolerance for every query."""
    torch = _torch()
    X, Q, gi, oi = mid10["X"], mid10["Q"], mid10["gi"], mid10["oi"]
    Qd = torch.from_numpy(Q).cuda()
    for k in (10, 100):
        ids, sc, dbg = gi.search(Qd, k, 8, 256, r1=32, precision="bf16", debug=True)
        torch.cuda.synchronize()
        oids, osc, odbg = oi.search(Q, k, 8, 256, 32, debug=True)
        compare_debug(dbg, odbg)
        compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


@pytest.fixture(scope="module")
def cos4():
    """Cosine variant: normalised tiny mixture, sign bits, m=10, H=4."""
    _torch()
    X, lab, Q, _ = datagen.tiny(n=20000, d=128, ncomp=16)
    X, Q = datagen.normalize_rows(X), datagen.normalize_rows(Q)
    A, b = datagen.lsh_params(10, 128, 1.0, seed=25, n_arrays=4)
    gi, oi, _ = build_pair(X, 16, 10, 1.0, 8, A, b, assignment=lab, n_arrays=4,
                           hash_kind="sign")
    return dict(X=X, Q=Q, gi=gi, oi=oi)


def test_cos4_build_bit_exact(cos4):
    compare_index(cos4["gi"], cos4["oi"])


@pytest.mark.parametrize("k,c,r,r1,eb", [(10, 4, 64, 3, 0), (10, 4, 64, 3, 3), (10, 2, 100, 16, 2),
                                          (50, 3, 40, 5, 5)])
def test_cos4_search(cos4, k, c, r, r1, eb):
    _run(cos4, k, c, r, r1, expand_bits=eb)


@pytest.mark.parametrize("C", [3, 2])
def test_large_clusters_union_masks(C):
    """Two arrays over clusters of about 8,700 rows (C = 3) and 13,000 rows
    (C = 2): the pair masks' LDS bitmap takes four copies, then one (the
    clusters of the other fixtures take eight); masks, windows and results
    equal the oracle."""
    _torch()
    X, lab, Q, _ = datagen.tiny(n=26000, d=32, ncomp=C, nq=64, seed=50, qseed=51)
    asg = (np.arange(X.shape[0]) % C).astype(np.int32)
    A, b = datagen.lsh_params(3, 32, 1.0, seed=52, n_arrays=2)
    fx = {}
    fx["gi"], fx["oi"], _ = build_pair(X, C, 3, 1.0, 4, A, b, assignment=asg, n_arrays=2)
    fx["X"], fx["Q"] = X, Q
    compare_index(fx["gi"], fx["oi"])
    assert int(fx["gi"].max_cluster) > (6144 if C == 3 else 12288)
    for k, c, r in ((10, 1, 300), (10, 2, 2000)):
        _run(fx, k, c, r, C)


def test_max_arrays_and_limits():
    """H = 16 (the maximum) on a small index; H = 17 and clusters above 65,536
    rows with several arrays are rejected."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    X, lab, Q, _ = datagen.tiny(n=6000, d=32, ncomp=8, nq=30)
    A, b = datagen.lsh_params(3, 32, 1.0, seed=27, n_arrays=16)
    fx = {}
    fx["gi"], fx["oi"], _ = build_pair(X, 8, 3, 1.0, 4, A, b, assignment=lab, n_arrays=16)
    fx["X"], fx["Q"] = X, Q
    compare_index(fx["gi"], fx["oi"])
    _run(fx, 10, 3, 20, 2)
    A17, b17 = datagen.lsh_params(3, 32, 1.0, seed=27, n_arrays=17)
    with pytest.raises(lider.LiderError):
        lider.Index(torch.from_numpy(X).cuda(), 8, 3, 1.0, 4, (A17, b17),
                    assignment=torch.from_numpy(lab).cuda(), n_arrays=17)
    Xb = np.random.default_rng(3).standard_normal((70000, 8)).astype(np.float32)
    A2, b2 = datagen.lsh_params(2, 8, 1.0, seed=28, n_arrays=2)
    with pytest.raises(lider.LiderError):
        lider.Index(torch.from_numpy(Xb).cuda(), 1, 2, 1.0, 4, (A2, b2),
                    assignment=torch.zeros(70000, dtype=torch.int32).cuda(), n_arrays=2)
