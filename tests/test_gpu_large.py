"""Corpus element offsets beyond 2^31: 3,000,000 x 768 fp32 rows (2.3e9
elements, 9.2 GB) in 300 clusters of about 10,000 rows (the generator's
labels).  The build is compared bit for bit with the oracle, and queries
drawn from the last clusters -- whose rows sit past element 2^31 of every
corpus copy -- are searched with the fp32 path and the precision form and
compared with the oracle."""
import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen

from parity_util import compare_debug, compare_index, compare_topk

pytestmark = pytest.mark.gpu

N, D, C, M, W, F = 3_000_000, 768, 300, 8, 2.0, 64


def test_past_2_to_31_elements():
    import torch
    from paper_2205_00970_amd import lider
    assert torch.cuda.is_available()
    print("[large] generating", flush=True)
    Xd, labd = datagen.mixture(N, D, ncomp=C, seed=60, device="cuda")
    A, b = datagen.lsh_params(M, D, W, seed=61)
    print("[large] building GPU index", flush=True)
    gi = lider.Index(Xd, C, M, W, F, (A, b), assignment=labd, storage="bf16")
    torch.cuda.synchronize()
    X, lab = Xd.cpu().numpy(), labd.cpu().numpy()
    # queries near rows of the last clusters: sorted positions past 2^31 / d
    g = np.random.default_rng(62)
    tail = np.where(lab >= C - 12)[0]
    src = g.choice(tail, 200, replace=False)
    Q = (X[src] + 0.1 * g.standard_normal((200, D))).astype(np.float32)
    Qd = torch.from_numpy(Q).cuda()
    del Xd
    torch.cuda.empty_cache()
    print("[large] building oracle index", flush=True)
    oi = oracle.Index(X, C, A, b, M, W, F, assignment=lab)
    compare_index(gi, oi)
    off = gi.export("offsets")
    assert off[C - 12] * D > 2**31
    for prec in ("f32", "bf16"):
        print(f"[large] search {prec}", flush=True)
        ids, sc, dbg = gi.search(Qd, 10, 4, 512, r1=C, precision=prec, debug=True)
        torch.cuda.synchronize()
        oids, osc, odbg = oi.search(Q, 10, 4, 512, C, debug=True)
        compare_debug(dbg, odbg)
        compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
        pr = dbg["pairs"].cpu().numpy()
        routed = dbg["routed"].cpu().numpy()
        # the windows read past element 2^31 (the routed set is listed in no
        # particular order: some window of each query)
        rows = off[routed] + pr[:, :, 1]
        assert (rows * D > 2**31).any(axis=1).mean() > 0.9
    gi.close()
