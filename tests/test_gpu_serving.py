"""Serving form on the GPU: requests served by continuous batching over
several HIP streams give bit-identical results to the same requests searched
alone, and every served request equals the FP64 oracle's answer within the
fp32 tolerance."""
import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen

from parity_util import compare_topk

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_results_identical_alone_and_in_the_mix(precision):
    import torch
    from paper_2205_00970_amd import lider, serving
    X, lab, Q, src = datagen.tiny(n=20000, d=128, ncomp=16, nq=2000, seed=40, qseed=41)
    A, b = datagen.lsh_params(4, 128, 1.0, seed=42)
    gi = lider.Index(torch.from_numpy(X).cuda(), 16, 4, 1.0, 8, (A, b),
                     assignment=torch.from_numpy(lab).cuda(), storage="bf16",
                     centroid_storage="fp8")
    Qd = torch.from_numpy(Q).cuda()
    c, r, r1 = 2, 600, 16
    ex = serving.GpuExecutor(gi, Qd, c, r, r1, precision=precision, slots=3, max_batch=1024)
    reqs = serving.make_requests(400000, 6000, pool_rows=2000, seed=43, bmax=64)
    sch = serving.Scheduler(ex, slots=3, max_batch=1024)
    out = sch.run(reqs)
    assert all(q.status == "done" for q in out)
    assert max(len(bt.reqs) for bt in sch.batches) > 1  # requests were merged
    oi = oracle.Index(X, 16, A, b, 4, 1.0, 8, assignment=lab)
    ores = {kk: oi.search(Q, kk, c, r, r1) for kk in sorted({q.k for q in out})}
    for q in out:
        oids, osc = ores[q.k]
        compare_topk(X, Q[q.rows], q.ids, q.scores, oids[q.rows], osc[q.rows])
    for q in out:
        rows = torch.from_numpy(q.rows).cuda()
        ids, sc = gi.search(Qd[rows].contiguous(), q.k, c, r, r1=r1, precision=precision)
        assert np.array_equal(q.ids, ids.cpu().numpy()), q.rid
        assert np.array_equal(q.scores.view(np.uint32), sc.cpu().numpy().view(np.uint32)), q.rid
