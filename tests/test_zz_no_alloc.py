"""lider_search_noalloc (the search with the library's fixed workspace, for
callers that cannot allocate) against lider_search_ex with a caller
workspace: bitwise equal results on consecutive calls, the second with a
smaller batch (the fixed array keeps the previous call's contents), and the
size limit enforced before anything is enqueued."""
import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen

from parity_util import compare_topk

pytestmark = pytest.mark.gpu


def test_noalloc_matches_workspace_search():
    import torch
    from paper_2205_00970_amd import lider
    assert torch.cuda.is_available()
    X, lab, Q, src = datagen.tiny(n=20000, d=128, ncomp=16, nq=400, seed=41, qseed=42)
    Xd = torch.from_numpy(X).cuda()
    gi = lider.Index(Xd, 16, 4, 1.0, 8, seed=43, kmeans_iters=20)
    Qd = torch.from_numpy(Q).cuda()
    assert lider.noalloc_scratch_bytes() == 64 << 20
    cases = [(Qd, 10, 4, 64, dict(r1=8)),                       # 400 queries
             (Qd[:37].contiguous(), 100, 3, 200, dict(r1=6)),   # then fewer, larger k
             (Qd[5:9].contiguous(), 10, 16, int(gi.max_cluster), dict(r1=16, pass_pairs=128,
                                                                       tile_rows=32))]
    for Qc, k, c, r, kw in cases:
        ref = gi.search(Qc, k, c, r, **kw)
        ids = torch.full((Qc.shape[0], k), -7, dtype=torch.int64, device="cuda")
        sc = torch.full((Qc.shape[0], k), 7.0, dtype=torch.float32, device="cuda")
        lider.search_noalloc(gi, Qc, k, c, r, (ids, sc), **kw)
        torch.cuda.synchronize()
        assert torch.equal(ids, ref[0]) and torch.equal(sc, ref[1]), (k, c, r)
    # the last call (whole clusters, every cluster) is exact search
    ids = torch.empty((4, 10), dtype=torch.int64, device="cuda")
    sc = torch.empty((4, 10), dtype=torch.float32, device="cuda")
    lider.search_noalloc(gi, Qd[5:9].contiguous(), 10, 16, int(gi.max_cluster), (ids, sc), r1=16)
    torch.cuda.synchronize()
    bi, bs = oracle.bruteforce(X, Q[5:9], 10)
    compare_topk(X, Q[5:9], ids.cpu().numpy(), sc.cpu().numpy(), bi, bs)
    # a batch whose workspace exceeds the fixed array is rejected, nothing written
    big = torch.from_numpy(np.repeat(Q, 60, axis=0)).cuda()  # 24,000 queries
    need = gi.workspace_bytes(big.shape[0], 1000, 16, int(gi.max_cluster), r1=16)
    assert need > lider.noalloc_scratch_bytes()
    ids = torch.full((big.shape[0], 1000), -7, dtype=torch.int64, device="cuda")
    sc = torch.zeros((big.shape[0], 1000), dtype=torch.float32, device="cuda")
    with pytest.raises(lider.LiderError) as e:
        lider.search_noalloc(gi, big, 1000, 16, int(gi.max_cluster), (ids, sc), r1=16)
    assert e.value.status == lider.EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert int((ids != -7).sum()) == 0
    gi.close()
