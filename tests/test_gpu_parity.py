"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.  Integer results (digits, keys, orders, positions,
routing sets, RMI parameters as bits) must be identical; ids and scores within
the fp32 tolerance |d score| <= 1e-4 |q| |x|."""
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


@pytest.fixture(scope="module")
def tiny():
    """The tiny mixture workload: N=20,000, d=128, 16 clusters, m=4, w=1,
    RMI fanout 8, 100 queries; k-means from seeded initial ids."""
    _torch()
    X, lab, Q, src = datagen.tiny()
    A, b = datagen.lsh_params(4, 128, 1.0)
    init = datagen.kmeans_init(X.shape[0], 16)
    gi, oi, Xd = build_pair(X, 16, 4, 1.0, 8, A, b, init_ids=init, iters=20)
    return dict(X=X, Q=Q, gi=gi, oi=oi)


def test_tiny_build_bit_exact(tiny):
    compare_index(tiny["gi"], tiny["oi"])


@pytest.mark.parametrize("k,c,r,r1", [(10, 4, 64, 0), (1, 1, 1, 0), (100, 4, 64, 8),
                                       (10, 16, 5000, 16), (7, 3, 33, 5),
                                       # up to 4096 / 6144 candidates per query: the
                                       # 64- and 96-register selections
                                       (10, 4, 1000, 0), (10, 5, 1100, 16)])
def test_tiny_search(tiny, k, c, r, r1):
    torch = _torch()
    X, Q, gi, oi = tiny["X"], tiny["Q"], tiny["gi"], tiny["oi"]
    Qd = torch.from_numpy(Q).cuda()
    ids, sc, dbg = gi.search(Qd, k, c, r, r1=r1, debug=True)
    torch.cuda.synchronize()
    oids, osc, odbg = oi.search(Q, k, c, r, r1 or None, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


def test_tiny_queries_outside_the_digit_box(tiny):
    """Queries scaled far out (and mirrored): their digits leave the models'
    digit boxes below and above, so the keys saturate (Sec. 5.1); keys,
    positions, windows, routing and results still equal the oracle's."""
    torch = _torch()
    X, Q, gi, oi = tiny["X"], tiny["Q"], tiny["gi"], tiny["oi"]
    Qo = np.concatenate([Q[:30] * 25.0, -Q[30:60] * 25.0, Q[60:] + 40.0]).astype(np.float32)
    ids, sc, dbg = gi.search(torch.from_numpy(Qo).cuda(), 10, 3, 64, r1=8, debug=True)
    torch.cuda.synchronize()
    oids, osc, odbg = oi.search(Qo, 10, 3, 64, 8, debug=True)
    # the case is exercised: layer-1 digit vectors below and above the box
    m, C = 4, 16
    box = gi.export("model_box").reshape(1, C + 1, 2 * m)[0, C]
    qd = odbg["qdigits"][:, :m]
    first_out = [next((i for i in range(m) if not box[i] <= v[i] <= box[m + i]), None) for v in qd]
    below = sum(1 for v, i in zip(qd, first_out) if i is not None and v[i] < box[i])
    above = sum(1 for v, i in zip(qd, first_out) if i is not None and v[i] > box[m + i])
    assert below > 0 and above > 0, (below, above)
    compare_debug(dbg, odbg)
    compare_topk(X, Qo, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


def test_tiny_flat_special_case(tiny):
    """All clusters, whole clusters, whole layer 1: exact (Flat) search."""
    torch = _torch()
    X, Q, gi = tiny["X"], tiny["Q"], tiny["gi"]
    ids, sc = gi.search(torch.from_numpy(Q).cuda(), 10, 16, int(gi.max_cluster), r1=16)
    bi, bs = oracle.bruteforce(X, Q, 10)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), bi, bs)


@pytest.fixture(scope="module")
def mid():
    """768-d mixture of the 1M family at 60,000 rows, 64 clusters given by the
    generator's labels (cluster 63 left empty), m=8, w=2, fanout 16 / 4."""
    torch = _torch()
    X, lab = datagen.mixture(60000, 768, ncomp=63, seed=5, device="cpu")
    X = X.numpy()
    lab = lab.numpy()
    Qt, _ = datagen.queries_from(torch.from_numpy(X), 300, 0.1, seed=6)
    Q = Qt.numpy()
    A, b = datagen.lsh_params(8, 768, 2.0, seed=7)
    gi, oi, Xd = build_pair(X, 64, 8, 2.0, 16, A, b, assignment=lab, F1=4)
    return dict(X=X, Q=Q, gi=gi, oi=oi)


def test_mid_build_bit_exact(mid):
    compare_index(mid["gi"], mid["oi"])
    assert mid["gi"].export("model_int").reshape(-1, 3)[63, 0] == 0  # the empty cluster


@pytest.mark.parametrize("k,c,r,r1", [(10, 8, 256, 32), (100, 8, 256, 32), (10, 2, 2000, 64),
                                       (1000, 16, 100, 20), (3, 1, 17, 1)])
def test_mid_search(mid, k, c, r, r1):
    torch = _torch()
    X, Q, gi, oi = mid["X"], mid["Q"], mid["gi"], mid["oi"]
    ids, sc, dbg = gi.search(torch.from_numpy(Q).cuda(), k, c, r, r1=r1, debug=True)
    oids, osc, odbg = oi.search(Q, k, c, r, r1, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


def test_mid_schedules_identical(mid):
    """Persistent and plain rerank, all tile sizes, sub-batches: bitwise equal."""
    torch = _torch()
    Qd = torch.from_numpy(mid["Q"]).cuda()
    gi = mid["gi"]
    ref = gi.search(Qd, 10, 8, 256, r1=32)
    for kw in [dict(persistent=True), dict(tile_rows=32), dict(tile_rows=128),
               dict(tile_rows=128, persistent=True, grid_mult=1), dict(persistent=2),
               dict(tile_rows=32, persistent=2, grid_mult=1),
               dict(tile_rows=128, persistent=2, grid_mult=8), dict(pass_pairs=16),
               dict(pass_pairs=64), dict(pass_pairs=128), dict(tile_rows=32, pass_pairs=64),
               dict(tile_rows=32, pass_pairs=128), dict(tile_rows=128, pass_pairs=128),
               dict(tile_rows=32, pass_pairs=128, persistent=2), dict()]:
        got = gi.search(Qd, 10, 8, 256, r1=32, **kw)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), kw
    sub = gi.search(Qd[37:90].contiguous(), 10, 8, 256, r1=32)
    assert torch.equal(sub[0], ref[0][37:90]) and torch.equal(sub[1], ref[1][37:90])


@pytest.mark.parametrize("k,c,r", [(1, 16, 256), (10, 16, 256), (10, 16, 100), (15, 16, 256),
                                   (64, 16, 256), (10, 16, 1200), (10, 20, 1200)])
def test_mid_block_selection(mid, k, c, r):
    """More than 2,048 candidates per query and k < 16: the rerank writes the
    smallest key of every 32-row block of every window and the selection
    reads only the blocks that can hold the k + 1 best (windows of 100 rows
    start inside blocks; k = 15 reads up to 16 blocks; k = 64 takes the
    register selection instead; 20 whole clusters of about 950 rows span
    more than 512 blocks and take the re-reading selection).  Results equal
    the oracle's, and every rerank schedule (each writes the block keys its
    own way) returns the same bits."""
    torch = _torch()
    X, Q, gi, oi = mid["X"], mid["Q"], mid["gi"], mid["oi"]
    Qd = torch.from_numpy(Q).cuda()
    ids, sc, dbg = gi.search(Qd, k, c, r, r1=32, debug=True)
    torch.cuda.synchronize()
    oids, osc, odbg = oi.search(Q, k, c, r, 32, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    for kw in [dict(tile_rows=32), dict(tile_rows=64), dict(tile_rows=128, pass_pairs=16),
               dict(persistent=True), dict(tile_rows=32, persistent=2, grid_mult=1)]:
        got = gi.search(Qd, k, c, r, r1=32, **kw)
        assert torch.equal(got[0], ids) and torch.equal(got[1], sc), kw


def test_workspace_monotone_in_k(mid):
    """The workspace never shrinks as k grows (the block keys' room is taken
    whatever k is): one sized for the largest k serves every smaller k."""
    torch = _torch()
    gi, Q = mid["gi"], mid["Q"]
    for c, r in [(16, 256), (8, 256), (2, 1200), (1, 17)]:
        sizes = [gi.workspace_bytes(len(Q), k, c, r, r1=32) for k in (1, 10, 15, 16, 64, 65, 100, 128, 1000)]
        assert sizes == sorted(sizes), (c, r, sizes)
    Qd = torch.from_numpy(Q).cuda()
    ws = torch.empty(gi.workspace_bytes(len(Q), 100, 16, 256, r1=32), dtype=torch.uint8, device="cuda")
    ref = gi.search(Qd, 10, 16, 256, r1=32)
    got = gi.search(Qd, 10, 16, 256, r1=32, ws=ws)
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])


def test_mid_many_pairs_per_tile(mid):
    """Every tile overlapped by hundreds of pairs (3,000 queries, c = 8, whole
    clusters): the listed pairs of a tile carry over between passes for every
    pass width and tile size; results are bitwise equal across them and equal
    the oracle's on a sample."""
    torch = _torch()
    X, Q, gi, oi = mid["X"], mid["Q"], mid["gi"], mid["oi"]
    g = np.random.default_rng(11)
    Qm = np.concatenate([Q + 0.01 * g.standard_normal(Q.shape) for _ in range(10)]).astype(np.float32)
    Qd = torch.from_numpy(Qm).cuda()
    L = int(gi.max_cluster)
    ref = gi.search(Qd, 10, 8, L, r1=64, pass_pairs=16, tile_rows=32)
    for tr in (32, 64, 128):
        for pp in (16, 32, 64, 128):
            got = gi.search(Qd, 10, 8, L, r1=64, pass_pairs=pp, tile_rows=tr)
            assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), (tr, pp)
    got = gi.search(Qd, 10, 8, L, r1=64, pass_pairs=128, tile_rows=32, persistent=1)
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    sel = np.arange(0, Qm.shape[0], 10)
    oids, osc = oi.search(Qm[sel], 10, 8, L, 64)
    compare_topk(X, Qm[sel], ref[0].cpu().numpy()[sel], ref[1].cpu().numpy()[sel], oids, osc)


def test_mid_two_streams_identical(mid):
    """Consecutive searches alternating over two streams, each with its own
    workspace and outputs and no synchronisation between them (the batches
    overlap on the device): every result equals the one-stream search."""
    torch = _torch()
    Qd = torch.from_numpy(mid["Q"]).cuda()
    gi = mid["gi"]
    ref = gi.search(Qd, 10, 2, 4000, r1=64)
    need = gi.workspace_bytes(Qd.shape[0], 10, 2, 4000, r1=64)
    streams = [torch.cuda.Stream() for _ in range(2)]
    wss = [torch.empty(need, dtype=torch.uint8, device="cuda") for _ in range(2)]
    outs = [[(torch.empty_like(ref[0]), torch.empty_like(ref[1])) for _ in range(3)] for _ in range(2)]
    torch.cuda.synchronize()
    for it in range(3):
        for j in range(2):
            gi.search(Qd, 10, 2, 4000, r1=64, stream=streams[j], ws=wss[j], out=outs[j][it])
    torch.cuda.synchronize()
    for j in range(2):
        for it in range(3):
            assert torch.equal(outs[j][it][0], ref[0]) and torch.equal(outs[j][it][1], ref[1]), (j, it)


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_mid_dense_layer1_identical(mid, precision):
    """r1 = C: the bf16-candidate routing (split by default at c > 1, plain
    and split forced), the fp32 dense GEMM and the window kernel route
    identically (the window kernel on an index with fp8 centroids scores
    those, approximately, in the precision form: not compared here)."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    X, Q = mid["X"], mid["Q"]
    gi = mid["gi"]
    if precision == "bf16":
        A, b = datagen.lsh_params(8, 768, 2.0, seed=7)
        gi = lider.Index(torch.from_numpy(X).cuda(), 64, 8, 2.0, 16, (A, b), rmi_fanout_l1=4,
                         assignment=torch.from_numpy(mid["oi"].assignment()).cuda(),
                         storage="bf16", centroid_storage="fp8")
    Qd = torch.from_numpy(Q).cuda()
    for sl in (slice(None), slice(5, 6), slice(17, 300)):
        q = Qd[sl].contiguous()
        a = gi.search(q, 10, 3, 500, r1=64, precision=precision, debug=True)
        for mode in ((False, 1, 2, 3) if precision == "f32" else (1, 2, 3)):
            # window kernel; dense fp32 without bf16 candidates
            b = gi.search(q, 10, 3, 500, r1=64, precision=precision, debug=True, l1_dense=mode)
            # the routed sets agree (their listing order is not part of the result)
            assert torch.equal(a[2]["routed"].sort(dim=1)[0], b[2]["routed"].sort(dim=1)[0])
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("l1_dense", [0, 2, 3])
def test_mid_routing_near_ties(mid, l1_dense):
    """Queries with many equal or nearly equal centroid scores (zero vectors,
    midpoints of two centroids, tiny perturbations of them): the bf16-candidate
    routing (automatic, plain bf16, split bf16) still returns the FP64 routed
    sets of the oracle."""
    torch = _torch()
    X, gi, oi = mid["X"], mid["gi"], mid["oi"]
    cent = oi.centroids()
    rng = np.random.default_rng(12)
    rows = [np.zeros(768, np.float32)]
    for _ in range(40):
        a, b = rng.choice(63, 2, replace=False)
        mpt = 0.5 * (cent[a] + cent[b])
        rows.append(mpt)
        rows.append(mpt + 1e-6 * rng.standard_normal(768))
    Q = np.ascontiguousarray(np.stack(rows).astype(np.float32))
    for c in (1, 2, 5, 40):
        ids, sc, dbg = gi.search(torch.from_numpy(Q).cuda(), 10, c, 300, r1=64, debug=True,
                                 l1_dense=l1_dense)
        oids, osc, odbg = oi.search(Q, 10, c, 300, 64, debug=True)
        compare_debug(dbg, odbg)
        compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


@pytest.mark.parametrize("n,C,d", [(20000, 16, 128), (30000, 48, 768)])
def test_farthest_first_kmeans_bit_exact(n, C, d):
    """Farthest-first seeding + Lloyd: every integer decision in FP64."""
    torch = _torch()
    if d == 128:
        X, lab, Q, src = datagen.tiny(n=n, d=d, ncomp=C, seed=30, qseed=31)
    else:
        Xt, lab = datagen.mixture(n, d, ncomp=C, seed=32, device="cpu")
        X = Xt.numpy()
        Q = datagen.queries_from(Xt, 64, 0.1, seed=33)[0].numpy()
    A, b = datagen.lsh_params(6, d, 2.0, seed=34)
    init = datagen.kmeans_init(n, C, seed=35)
    gi, oi, _ = build_pair(X, C, 6, 2.0, 8, A, b, init_ids=init, iters=15, seeding="farthest")
    compare_index(gi, oi)
    ids, sc, dbg = gi.search(torch.from_numpy(Q).cuda(), 10, 2, 4000, r1=C, debug=True)
    oids, osc, odbg = oi.search(Q, 10, 2, 4000, C, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


@pytest.mark.parametrize("d", [100, 130])
def test_odd_dimensions(d):
    """d not a multiple of 16 (MFMA tail) and not a multiple of 4 (scalar path)."""
    torch = _torch()
    X, lab, Q, src = datagen.tiny(n=3000, d=d, ncomp=6, nq=40, seed=8, qseed=9)
    A, b = datagen.lsh_params(3, d, 1.5, seed=10)
    init = datagen.kmeans_init(3000, 6, seed=11)
    gi, oi, _ = build_pair(X, 6, 3, 1.5, 4, A, b, init_ids=init, iters=10)
    compare_index(gi, oi)
    for r1 in (3, 6):  # window kernel, then the dense layer-1 product (r1 = C)
        ids, sc, dbg = gi.search(torch.from_numpy(Q).cuda(), 5, 2, 40, r1=r1, debug=True)
        oids, osc, odbg = oi.search(Q, 5, 2, 40, r1, debug=True)
        compare_debug(dbg, odbg)
        compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


@pytest.mark.parametrize("d", [64, 192])
def test_lds_product_ragged_tiles(d):
    """The LDS-staged layer-1 product at the smallest dimensions it takes (two
    and six K chunks of 32 in the split form, one and three of 64 in the plain
    one), 200 centroids (a ragged second centroid tile) and 300 queries (a
    ragged third query tile): plain and split bf16 routing equal the oracle's
    FP64 routed sets and results, and each other."""
    torch = _torch()
    X, lab, Q, src = datagen.tiny(n=20000, d=d, ncomp=40, nq=300, seed=60, qseed=61)
    C = 200
    asg = (np.arange(X.shape[0]) % C).astype(np.int32)
    A, b = datagen.lsh_params(4, d, 1.5, seed=62)
    gi, oi, _ = build_pair(X, C, 4, 1.5, 8, A, b, assignment=asg)
    Qd = torch.from_numpy(Q).cuda()
    for c in (1, 4):
        oids, osc, odbg = oi.search(Q, 10, c, 60, C, debug=True)
        res = []
        for mode in (2, 3):
            ids, sc, dbg = gi.search(Qd, 10, c, 60, r1=C, debug=True, l1_dense=mode)
            compare_debug(dbg, odbg)
            compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
            res.append((ids, sc))
        assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])


def test_routing_window_past_candidate_room():
    """400 centroids and queries whose scores all tie (the zero vector) or
    nearly tie (a centroid midpoint): more candidates than the rescoring's
    room of 256, so the whole window is decided by the sequential FP64 pass;
    routed sets and results equal the oracle's."""
    torch = _torch()
    X, lab, Q, src = datagen.tiny(n=24000, d=64, ncomp=40, nq=20, seed=70, qseed=71)
    C = 400
    asg = (np.arange(X.shape[0]) % C).astype(np.int32)
    A, b = datagen.lsh_params(4, 64, 1.5, seed=72)
    gi, oi, _ = build_pair(X, C, 4, 1.5, 8, A, b, assignment=asg)
    cent = oi.centroids()
    rows = [np.zeros(64, np.float32), 0.5 * (cent[3] + cent[7])]
    Qm = np.ascontiguousarray(np.concatenate([np.stack(rows), Q]).astype(np.float32))
    for c in (1, 3):
        ids, sc, dbg = gi.search(torch.from_numpy(Qm).cuda(), 10, c, 60, r1=C, debug=True)
        oids, osc, odbg = oi.search(Qm, 10, c, 60, C, debug=True)
        compare_debug(dbg, odbg)
        compare_topk(X, Qm, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


@pytest.mark.parametrize("c,r1", [(1, 64), (5, 64), (5, 32)])
def test_mid_non_finite_queries(mid, c, r1):
    """Queries holding a NaN, an infinity or a value whose products overflow
    fp32, in one coordinate or all of them, inside a batch of ordinary ones:
    the search returns, their ids are -1 or corpus rows, and the ordinary
    queries still equal the oracle (a routing window whose scores are not
    finite is decided by the sequential FP64 pass)."""
    torch = _torch()
    X, Q, gi, oi = mid["X"], mid["Q"], mid["gi"], mid["oi"]
    bad = Q[40:47].copy()
    bad[0, 5] = np.nan
    bad[1, :] = np.nan
    bad[2, 7] = np.inf
    bad[3, 100] = -np.inf
    bad[4, :] = np.inf
    bad[5, 3] = 3e38
    bad[6, :] = -3e38
    Qm = np.ascontiguousarray(np.concatenate([Q[:20], bad, Q[20:40]]))
    ids, sc = gi.search(torch.from_numpy(Qm).cuda(), 10, c, 300, r1=r1)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    assert ((ids >= -1) & (ids < X.shape[0])).all()
    fin = np.r_[0:20, 27:47]
    oids, osc = oi.search(Q[:40], 10, c, 300, r1)[:2]
    compare_topk(X, Q[:40], ids[fin], sc[fin], oids, osc)


@pytest.mark.parametrize("nrep", [1, 12])
def test_many_clusters_unfused_work_list(nrep):
    """More than 8,192 clusters: the cluster-count scan and the pair scatter run
    as two launches (the fused launch keeps the counts in LDS); build and
    search still equal the oracle.  nrep = 12: 768 queries, 4,608 pairs, so
    every copy of the per-cluster counters holds pairs and clusters take pairs
    in several copies."""
    torch = _torch()
    X, lab, Q, src = datagen.tiny(n=30000, d=32, ncomp=16, nq=64, seed=40, qseed=41)
    if nrep > 1:
        g = np.random.default_rng(43)
        Q = np.concatenate([Q] + [Q + 0.05 * g.standard_normal(Q.shape) for _ in range(nrep - 1)])
        Q = np.ascontiguousarray(Q.astype(np.float32))
    C = 9000
    asg = (np.arange(X.shape[0]) % C).astype(np.int32)
    A, b = datagen.lsh_params(4, 32, 1.0, seed=42)
    gi, oi, _ = build_pair(X, C, 4, 1.0, 8, A, b, assignment=asg)
    compare_index(gi, oi)
    ids, sc, dbg = gi.search(torch.from_numpy(Q).cuda(), 10, 6, 4, r1=64, debug=True)
    oids, osc, odbg = oi.search(Q, 10, 6, 4, 64, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


def test_hash_near_bucket_edges():
    """Projections placed within 1e-7 of bucket edges take the FP64 path and
    still equal the FP64 definition."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    g = np.random.default_rng(12)
    d, nh, w = 768, 16, 2.0
    A = g.standard_normal((nh, d)).astype(np.float32)
    b = (g.random(nh) * w).astype(np.float32)
    X = g.standard_normal((4096, d)).astype(np.float32)
    # shift each row along A[0] so that a_0.x + b_0 lands near an edge
    t = (X.astype(np.float64) @ A[0].astype(np.float64) + b[0]) / w
    a0 = A[0].astype(np.float64)
    X = (X + np.outer((np.round(t) - t) * w + 1e-7 * (g.random(4096) - 0.5), a0 / (a0 @ a0))
         ).astype(np.float32)
    got = lider.hash(torch.from_numpy(X).cuda(), torch.from_numpy(A).cuda(),
                     torch.from_numpy(b).cuda(), w).cpu().numpy()
    ref = oracle.digits(X, A, b, w)
    assert np.array_equal(got, ref)


def test_hash_exact_bucket_edges():
    """Integer data and projections: every a.x + b is an exact multiple of w
    (and zero rows give exactly b), so every projection sits on a bucket edge
    and is decided by the sequential FP64 sum of the definition; the digits
    still equal it."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    g = np.random.default_rng(21)
    d, nh, w = 768, 32, 1.0
    A = g.integers(-3, 4, (nh, d)).astype(np.float32)
    b = g.integers(-2, 3, nh).astype(np.float32)
    X = g.integers(-3, 4, (1000, d)).astype(np.float32)
    X[:7] = 0.0
    got = lider.hash(torch.from_numpy(X).cuda(), torch.from_numpy(A).cuda(),
                     torch.from_numpy(b).cuda(), w).cpu().numpy()
    ref = oracle.digits(X, A, b, w)
    assert np.array_equal(got, ref)
    exact = (X.astype(np.float64) @ A.T.astype(np.float64) + b) / w
    assert np.array_equal(ref, np.floor(exact).astype(np.int64))


def test_kmeans_assign_step():
    """One assignment step on 768-d data with 1,000 centroids (FP64 decision)."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    Xt, lab = datagen.mixture(120000, 768, ncomp=1000, seed=13, device="cuda")
    init = datagen.kmeans_init(120000, 1000, seed=14)
    cent = Xt[torch.from_numpy(init).cuda()].contiguous()
    got = lider.kmeans_assign(Xt, cent).cpu().numpy()
    sample = np.random.default_rng(15).choice(120000, 3000, replace=False)
    X = Xt.cpu().numpy()
    ref = oracle.kmeans_assign(X[sample], cent.cpu().numpy())
    assert np.array_equal(got[sample], ref)


def test_errors_and_edge_cases(tiny):
    torch = _torch()
    from paper_2205_00970_amd import lider
    gi = tiny["gi"]
    Qd = torch.from_numpy(tiny["Q"]).cuda()
    for bad in [dict(k=0, c=4, r=64), dict(k=10, c=17, r=64), dict(k=10, c=4, r=0),
                dict(k=2000, c=4, r=64)]:
        with pytest.raises(lider.LiderError) as e:
            gi.search(Qd, **bad)
        assert e.value.status == lider.EINVAL
    ids, sc = gi.search(Qd[:0], 10, 4, 64)
    assert ids.shape == (0, 10)
    lider.fail_next(lider.EDEVICE)
    with pytest.raises(lider.LiderError) as e:
        gi.search(Qd, 10, 4, 64)
    assert e.value.status == lider.EDEVICE
    ids2, _ = gi.search(Qd, 10, 4, 64)  # the index is untouched
    ids1, _ = gi.search(Qd, 10, 4, 64)
    assert torch.equal(ids1, ids2)
    with pytest.raises(lider.LiderError):
        gi.search(Qd, 10, 4, 64, precision="bf16")  # index has no bf16 copy


@pytest.mark.parametrize("k,l1_dense", [(10, True), (100, True), (10, False), (100, False)])
def test_precision_form(mid, k, l1_dense):
    """Precision form with the certified shortlist (bf16 windows, every
    candidate within the bf16 error margin of the k-th best reranked in fp32),
    routed exactly from bf16 dense scores or from fp8 window scores: routed
    sets and windows equal the oracle's, and the ids and scores equal the
    oracle's top k within the fp32 tolerance for every query."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    X, Q, oi = mid["X"], mid["Q"], mid["oi"]
    A, b = datagen.lsh_params(8, 768, 2.0, seed=7)
    lab = oi.assignment()
    gi = lider.Index(torch.from_numpy(X).cuda(), 64, 8, 2.0, 16, (A, b), rmi_fanout_l1=4,
                     assignment=torch.from_numpy(lab).cuda(), storage="bf16",
                     centroid_storage="fp8")
    Qd = torch.from_numpy(Q).cuda()
    ids, sc, dbg = gi.search(Qd, k, 4, 4000, r1=64, precision="bf16", l1_dense=l1_dense,
                             debug=True)
    torch.cuda.synchronize()
    oids, osc, odbg = oi.search(Q, k, 4, 4000, 64, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    # window shorter than the clusters: windows, routing and results again
    ids, sc, dbg = gi.search(Qd, k, 8, 256, r1=32, precision="bf16", l1_dense=l1_dense,
                             debug=True)
    oids, osc, odbg = oi.search(Q, k, 8, 256, 32, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    # the bf16 windows through the workgroup rerank (128-row tiles): the same
    # scores bit for bit, so the same results
    for kw in (dict(tile_rows=128), dict(tile_rows=128, pass_pairs=64)):
        got = gi.search(Qd, k, 8, 256, r1=32, precision="bf16", l1_dense=l1_dense, **kw)
        assert torch.equal(got[0], ids) and torch.equal(got[1], sc), kw
    gi.close()


@pytest.mark.parametrize("mult", [1, 4])
def test_precision_form_fixed_shortlist(mid, mult):
    """The fixed-length shortlist (the mult * k best bf16 scores, reranked in
    fp32) is approximate: every returned score is its id's exact score within
    tolerance, ids are unique candidates sorted by score, and no returned
    score exceeds the oracle's score at the same rank (it can only miss)."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    X, Q, oi = mid["X"], mid["Q"], mid["oi"]
    A, b = datagen.lsh_params(8, 768, 2.0, seed=7)
    gi = lider.Index(torch.from_numpy(X).cuda(), 64, 8, 2.0, 16, (A, b), rmi_fanout_l1=4,
                     assignment=torch.from_numpy(oi.assignment()).cuda(), storage="bf16")
    k = 10
    ids, sc = gi.search(torch.from_numpy(Q).cuda(), k, 4, 4000, r1=64, precision="bf16",
                        shortlist_mult=mult)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy().astype(np.float64)
    oids, osc = oi.search(Q, k, 4, 4000, 64)
    qn = np.linalg.norm(Q.astype(np.float64), axis=1)
    xn = np.linalg.norm(X.astype(np.float64), axis=1)
    hits = 0
    for q in range(Q.shape[0]):
        g = ids[q][ids[q] >= 0]
        assert len(g) == int((oids[q] >= 0).sum()) and len(set(g.tolist())) == len(g)
        s64 = oracle.pair_scores(X, Q, np.full(len(g), q), g)
        tol = 1e-4 * qn[q] * xn[g]
        assert np.all(np.abs(sc[q][:len(g)] - s64) <= tol)
        assert np.all(np.diff(sc[q][:len(g)]) <= 0)
        assert np.all(s64 <= osc[q][:len(g)] + 1e-4 * qn[q] * np.maximum(xn[g], xn[oids[q][:len(g)]]))
        hits += len(set(g.tolist()) & set(oids[q][oids[q] >= 0].tolist()))
    print(f"fixed shortlist {mult}k: {hits} of {(oids >= 0).sum()} oracle ids returned")
    gi.close()
