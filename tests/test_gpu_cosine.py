"""GPU parity of the cosine variant (random-hyperplane bits, key =
Decimal(bits)) and of the dist_e-guided expansion windows against the FP64
oracle: bit-exact build, query bits, windows and routed sets; ids and scores
within the fp32 tolerance."""
import numpy as np
import pytest

import oracle
from paper_2205_00970_amd import datagen

from parity_util import compare_debug, compare_index, compare_topk

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _pair(X, C, m, F, A, assignment=None, init=None, iters=20, F1=0, seeding="given"):
    torch = _torch()
    from paper_2205_00970_amd import lider
    b = np.zeros(2 * m, np.float32)
    asg = None if assignment is None else torch.from_numpy(assignment.astype(np.int32)).cuda()
    gi = lider.Index(torch.from_numpy(X).cuda(), C, m, 1.0, F, (A, None), rmi_fanout_l1=F1,
                     kmeans_init=init, kmeans_iters=iters, assignment=asg, seeding=seeding,
                     hash_kind="sign")
    oi = oracle.Index(X, C, A, b, m, 1.0, F, rmi_fanout_l1=(F1 or None), assignment=assignment,
                      init_ids=init, kmeans_iters=iters, seeding=seeding, hash_kind="sign")
    return gi, oi


@pytest.fixture(scope="module")
def tiny_cos():
    X, lab, Q, src = datagen.tiny()
    X, Q = datagen.normalize_rows(X), datagen.normalize_rows(Q)
    A, _ = datagen.lsh_params(6, 128, 1.0, seed=40)
    gi, oi = _pair(X, 16, 6, 8, A, init=datagen.kmeans_init(X.shape[0], 16), iters=20)
    return dict(X=X, Q=Q, gi=gi, oi=oi)


def test_tiny_cos_build_bit_exact(tiny_cos):
    compare_index(tiny_cos["gi"], tiny_cos["oi"])
    assert set(np.unique(tiny_cos["gi"].export("digits"))) <= {0, 1}


@pytest.mark.parametrize("k,c,r,r1,B", [(10, 4, 64, 8, 0), (10, 4, 64, 8, 3), (5, 2, 33, 5, 1),
                                         (10, 16, 5000, 16, 4), (1, 1, 1, 1, 3)])
def test_tiny_cos_search(tiny_cos, k, c, r, r1, B):
    torch = _torch()
    X, Q, gi, oi = tiny_cos["X"], tiny_cos["Q"], tiny_cos["gi"], tiny_cos["oi"]
    ids, sc, dbg = gi.search(torch.from_numpy(Q).cuda(), k, c, r, r1=r1, debug=True,
                             expand_bits=B)
    oids, osc, odbg = oi.search(Q, k, c, r, r1, debug=True, expand_bits=B)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


@pytest.fixture(scope="module")
def mid_cos():
    torch = _torch()
    Xt, lab = datagen.mixture(60000, 768, ncomp=63, seed=41, device="cpu")
    X = datagen.normalize_rows(Xt.numpy())
    Qt, _ = datagen.queries_from(torch.from_numpy(X), 300, 0.02, seed=42)
    Q = datagen.normalize_rows(Qt.numpy())
    A, _ = datagen.lsh_params(10, 768, 1.0, seed=43)
    gi, oi = _pair(X, 64, 10, 16, A, assignment=lab.numpy(), F1=4)
    return dict(X=X, Q=Q, gi=gi, oi=oi)


def test_mid_cos_build_bit_exact(mid_cos):
    compare_index(mid_cos["gi"], mid_cos["oi"])


@pytest.mark.parametrize("k,c,r,r1,B", [(10, 8, 256, 32, 0), (10, 8, 256, 32, 3),
                                         (100, 4, 300, 64, 5), (10, 2, 2000, 20, 2)])
def test_mid_cos_search(mid_cos, k, c, r, r1, B):
    torch = _torch()
    X, Q, gi, oi = mid_cos["X"], mid_cos["Q"], mid_cos["gi"], mid_cos["oi"]
    ids, sc, dbg = gi.search(torch.from_numpy(Q).cuda(), k, c, r, r1=r1, debug=True,
                             expand_bits=B)
    oids, osc, odbg = oi.search(Q, k, c, r, r1, debug=True, expand_bits=B)
    compare_debug(dbg, odbg)
    compare_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)


def test_expand_needs_sign_index(mid_cos):
    torch = _torch()
    from paper_2205_00970_amd import lider
    X = mid_cos["X"][:5000]
    A, b = datagen.lsh_params(4, 768, 2.0, seed=44)
    lab = (np.arange(5000) % 8).astype(np.int32)
    gi = lider.Index(torch.from_numpy(X).cuda(), 8, 4, 2.0, 4, (A, b),
                     assignment=torch.from_numpy(lab).cuda())
    with pytest.raises(lider.LiderError):
        gi.search(torch.from_numpy(mid_cos["Q"][:10]).cuda(), 10, 2, 64, expand_bits=3)
