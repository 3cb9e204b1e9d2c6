"""Batching form at the shape of the uneven-cluster workload, scaled to fit
the oracle: 400,000 x 768 rows in 512 clusters with Zipf(1.1) sizes from 50
to 40,000 rows (the generator's components as the clustering), c = 16,
r = r1 = 512, k = 100.  Hot clusters receive thousands of (query, cluster)
pairs and hold hundreds of row tiles, so every rerank schedule runs many
ballot rounds and passes per tile.  The whole build is compared bit for bit
with the oracle, the search of a 512-query batch element by element, every
schedule candidate of the autotuner and every batch size from 1 to 4,096
bitwise against that search, and the precision form against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen

from parity_util import compare_debug, compare_index, compare_topk

pytestmark = pytest.mark.gpu

N, D, C, M, W, F = 400_000, 768, 512, 8, 2.0, 64
K, CC, R = 100, 16, 512


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def zipf():
    torch = _torch()
    from paper_2205_00970_amd import lider
    sizes = datagen.zipf_sizes(N, C, 1.1, 50, 40_000)
    Xd, labd = datagen.mixture(N, D, ncomp=C, seed=50, device="cuda", sizes=sizes)
    Qd, _ = datagen.queries_from(Xd, 4096, 0.1, seed=51)
    A, b = datagen.lsh_params(M, D, W, seed=52)
    print(f"[batching] building, cluster sizes {sizes.min()}..{sizes.max()}", flush=True)
    gi = lider.Index(Xd, C, M, W, F, (A, b), assignment=labd, storage="bf16",
                     centroid_storage="fp8")
    X, lab, Q = Xd.cpu().numpy(), labd.cpu().numpy(), Qd.cpu().numpy()
    oi = oracle.Index(X, C, A, b, M, W, F, assignment=lab)
    return dict(X=X, Q=Q, Qd=Qd, gi=gi, oi=oi, sizes=sizes)


def test_zipf_build_bit_exact(zipf):
    compare_index(zipf["gi"], zipf["oi"])
    assert int(zipf["gi"].max_cluster) == int(zipf["sizes"].max())


def test_zipf_search_schedules_and_batch_sizes(zipf):
    torch = _torch()
    from paper_2205_00970_amd import autotune
    gi, oi, X, Q, Qd = zipf["gi"], zipf["oi"], zipf["X"], zipf["Q"], zipf["Qd"]
    q512 = Qd[:512].contiguous()
    ids, sc, dbg = gi.search(q512, K, CC, R, r1=R, debug=True)
    torch.cuda.synchronize()
    oids, osc, odbg = oi.search(Q[:512], K, CC, R, R, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q[:512], ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    # pairs per cluster: several ballot rounds in the hot clusters
    routed = dbg["routed"].cpu().numpy()
    assert np.bincount(routed[routed >= 0], minlength=C).max() > 64
    for cand in autotune.CANDIDATES:
        got = gi.search(q512, K, CC, R, r1=R, **cand)
        assert torch.equal(got[0], ids) and torch.equal(got[1], sc), cand
    # the 4,096-query batch, then sub-batches of every size class, are the
    # same rows of the same results
    full_i, full_s = gi.search(Qd, K, CC, R, r1=R)
    assert torch.equal(full_i[:512], ids) and torch.equal(full_s[:512], sc)
    a = 0
    for bsz in (1, 3, 64, 200, 1000, 2828):
        for kw in (dict(), dict(persistent=1), dict(persistent=2, tile_rows=32, pass_pairs=64)):
            bi, bs = gi.search(Qd[a:a + bsz].contiguous(), K, CC, R, r1=R, **kw)
            assert torch.equal(bi, full_i[a:a + bsz]) and torch.equal(bs, full_s[a:a + bsz]), (bsz, kw)
        a += bsz
    assert a == 4096


def test_zipf_precision_form(zipf):
    torch = _torch()
    gi, oi, X, Q, Qd = zipf["gi"], zipf["oi"], zipf["X"], zipf["Q"], zipf["Qd"]
    sel = np.arange(0, 4096, 8)
    ids, sc, dbg = gi.search(Qd[torch.from_numpy(sel).cuda()].contiguous(), K, CC, R, r1=R,
                             precision="bf16", debug=True)
    torch.cuda.synchronize()
    oids, osc, odbg = oi.search(Q[sel], K, CC, R, R, debug=True)
    compare_debug(dbg, odbg)
    compare_topk(X, Q[sel], ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
