"""GPU parity at the full 1M x 768 size, in the launch configuration the
benchmark times (the whole 10,000-query batch in one call).

The corpus is the 1,000-component Gaussian mixture (component norms U[8,12],
sigma 0.5), queries are perturbed corpus points (sigma 0.1), m=8, w=2, RMI
fanout 64.  With the generator's labels as the clustering, the oracle builds
the same index in seconds, so the whole build is compared bit for bit and every
query's layer-1 window, routed set and per-cluster windows are compared
exactly; top-k lists are compared on a sample within the fp32 tolerance.  The
k-means build at this size (farthest-first seeding + Lloyd) is checked through
properties that hold at any size: every centroid is the FP64 mean of its
members, and on convergence every point's cluster is its FP64 argmin."""
import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen

from parity_util import compare_debug, compare_index, compare_topk

pytestmark = pytest.mark.gpu

N, D, C, M, W, F = 1_000_000, 768, 1000, 8, 2.0, 64
NQ = 10_000


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def full():
    torch = _torch()
    from paper_2205_00970_amd import lider
    print(f"[fullsize] generating {N}x{D}", flush=True)
    Xd, labd = datagen.mixture(N, D, ncomp=C, seed=0, device="cuda")
    Qd, _ = datagen.queries_from(Xd, NQ, 0.1, seed=1)
    A, b = datagen.lsh_params(M, D, W, seed=2)
    X, lab, Q = Xd.cpu().numpy(), labd.cpu().numpy().astype(np.int32), Qd.cpu().numpy()
    print("[fullsize] building GPU index (generator labels)", flush=True)
    gi = lider.Index(Xd, C, M, W, F, (A, b), assignment=labd.to(torch.int32), storage="bf16",
                     centroid_storage="fp8")
    torch.cuda.synchronize()
    print("[fullsize] building oracle index", flush=True)
    oi = oracle.Index(X, C, A, b, M, W, F, assignment=lab)
    return dict(X=X, Q=Q, Xd=Xd, Qd=Qd, A=A, b=b, gi=gi, oi=oi)


def test_full_build_bit_exact(full):
    compare_index(full["gi"], full["oi"])


@pytest.mark.parametrize("k,c,r,r1", [(10, 8, 256, 256), (100, 8, 256, 256), (10, 1, 0, 1000)])
def test_full_search(full, k, c, r, r1):
    """The whole batch on the GPU; every query's integer path exactly, a
    sample of 1,000 top-k lists within tolerance."""
    torch = _torch()
    gi, oi, X, Q = full["gi"], full["oi"], full["X"], full["Q"]
    r = r or int(gi.max_cluster)
    print(f"[fullsize] search k={k} c={c} r={r} r1={r1}", flush=True)
    ids, sc, dbg = gi.search(full["Qd"], k, c, r, r1=r1, debug=True)
    torch.cuda.synchronize()
    oids, osc, odbg = oi.search(Q, k, c, r, r1, debug=True)
    compare_debug(dbg, odbg)
    sel = np.arange(0, NQ, NQ // 1000)
    compare_topk(X, Q[sel], ids.cpu().numpy()[sel], sc.cpu().numpy()[sel], oids[sel], osc[sel])


def test_full_schedules_identical(full):
    """Every rerank schedule returns bit-identical results on the full batch."""
    torch = _torch()
    gi, Qd = full["gi"], full["Qd"]
    ref = gi.search(Qd, 10, 8, 256, r1=256)
    for kw in [dict(tile_rows=32), dict(tile_rows=128), dict(persistent=1, grid_mult=4),
               dict(persistent=2, grid_mult=4), dict(tile_rows=128, persistent=2, grid_mult=8),
               dict(pass_pairs=64), dict(tile_rows=32, pass_pairs=128),
               dict(tile_rows=128, pass_pairs=64)]:
        got = gi.search(Qd, 10, 8, 256, r1=256, **kw)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), kw


@pytest.mark.parametrize("k,c,r,r1", [(10, 8, 256, 256), (100, 8, 256, 256), (10, 1, 0, 1000)])
def test_full_precision_form(full, k, c, r, r1):
    """Precision form (bf16 windows, certified shortlist, fp32 rerank) on the
    full batch in one call: routing and windows of every query equal the
    oracle's, and 1,000 sampled top-k lists equal the oracle's within the
    fp32 tolerance."""
    torch = _torch()
    gi, oi, X, Q = full["gi"], full["oi"], full["X"], full["Q"]
    r = r or int(gi.max_cluster)
    ids, sc, dbg = gi.search(full["Qd"], k, c, r, r1=r1, precision="bf16", debug=True)
    torch.cuda.synchronize()
    sel = np.arange(0, NQ, NQ // 1000)
    oids, osc, odbg = oi.search(Q[sel], k, c, r, r1, debug=True)
    tsel = torch.from_numpy(sel).cuda()
    compare_debug({kk: v[tsel] for kk, v in dbg.items()}, odbg)
    compare_topk(X, Q[sel], ids.cpu().numpy()[sel], sc.cpu().numpy()[sel], oids, osc)


def test_full_kmeans_properties(full):
    """The benchmark's build: farthest-first seeding + Lloyd at 1M x 768."""
    torch = _torch()
    from paper_2205_00970_amd import lider
    X = full["X"]
    init = datagen.kmeans_init(N, C, seed=3)
    print("[fullsize] k-means build", flush=True)
    gi = lider.Index(full["Xd"], C, M, W, F, (full["A"], full["b"]), kmeans_init=init,
                     kmeans_iters=20, seeding="farthest")
    torch.cuda.synchronize()
    asg = gi.export("assign")
    cent = gi.export("centroids").reshape(C, D)
    assert asg.min() >= 0 and asg.max() < C
    # every centroid is the FP64 mean (rounded to fp32) of its final members
    upd, counts = oracle.kmeans_update(X, asg, cent)
    assert np.array_equal(upd.view(np.uint32), cent.view(np.uint32))
    assert counts.sum() == N and np.array_equal(counts, np.bincount(asg, minlength=C))
    # offsets are the cluster sizes' prefix sums
    assert np.array_equal(np.diff(gi.export("offsets")), counts)
    if gi.iters_run < 20:  # converged: the assignment is a fixed point
        sel = np.random.default_rng(0).choice(N, 4000, replace=False)
        assert np.array_equal(oracle.kmeans_assign(X[sel], cent), asg[sel])
