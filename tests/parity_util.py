"""Shared helpers of the GPU parity tests: build both sides from the same
seeded inputs and compare the GPU index / search against the FP64 oracle."""
import numpy as np

import oracle

SCORE_TOL = 1e-4  # |score difference| <= SCORE_TOL * |q| * |x| (fp32 vs FP64)


def build_pair(X, n_clusters, m, w, F, A, b, assignment=None, init_ids=None, iters=20, F1=0,
               storage="f32", centroid_storage="f32", seeding="given"):
    """GPU index and oracle index over the same host data."""
    import torch
    from paper_2205_00970_amd import lider
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    asg_d = None if assignment is None else torch.from_numpy(
        np.ascontiguousarray(assignment, dtype=np.int32)).cuda()
    gi = lider.Index(Xd, n_clusters, m, w, F, (A, b), rmi_fanout_l1=F1, kmeans_init=init_ids,
                     kmeans_iters=iters, assignment=asg_d, storage=storage,
                     centroid_storage=centroid_storage, seeding=seeding)
    oi = oracle.Index(X, n_clusters, A, b, m, w, F, rmi_fanout_l1=(F1 or None),
                      assignment=assignment, init_ids=init_ids, kmeans_iters=iters,
                      seeding=seeding)
    return gi, oi, Xd


def compare_index(gi, oi):
    """Everything the build produces must match bit for bit."""
    C, m = oi.C, oi.m
    assert gi.iters_run == oi.iters_run()
    assert np.array_equal(gi.export("assign"), oi.assignment())
    assert np.array_equal(gi.export("centroids").view(np.uint32),
                          oi.centroids().reshape(-1).view(np.uint32))
    assert np.array_equal(gi.export("digits"), oi.digits().reshape(-1))
    assert np.array_equal(gi.export("offsets"), oi.offsets())
    assert np.array_equal(gi.export("perm"), oi.perm())
    assert np.array_equal(gi.export("keys"), oi.keys())
    order, keys1, dig1 = oi.layer1()
    assert np.array_equal(gi.export("l1_order"), order)
    assert np.array_equal(gi.export("l1_keys"), keys1)
    assert np.array_equal(gi.export("l1_digits"), dig1.reshape(-1))
    mi = gi.export("model_int").reshape(C + 1, 3)
    mb = gi.export("model_box").reshape(C + 1, 2 * m)
    mk = gi.export("model_key").reshape(C + 1, 2)
    md = gi.export("model_dbl").reshape(C + 1, 3)
    lv = gi.export("leaves").reshape(-1, 2)
    le = gi.export("leaf_err").reshape(-1, 2)
    for j in range(C + 1):
        om = oi.model(j)
        assert (mi[j, 0], mi[j, 1], mi[j, 2]) == (om.L, om.m_eff, om.F), j
        assert np.array_equal(mb[j, :m], om.mins) and np.array_equal(mb[j, m:], om.maxs), j
        assert (int(mk[j, 0]), int(mk[j, 1])) == (om.kmin, om.kmax), j
        got = md[j].view(np.uint64)
        ref = np.array([om.scale, om.root[0], om.root[1]]).view(np.uint64)
        assert np.array_equal(got, ref), (j, md[j], om.scale, om.root)
        base = j * oi.F2
        F = om.F
        assert np.array_equal(lv[base:base + F].reshape(-1).view(np.uint64),
                              om.leaf.view(np.uint64)), j
        assert np.array_equal(le[base:base + F, 0], om.elo), j
        assert np.array_equal(le[base:base + F, 1], om.ehi), j


def compare_debug(gdbg, odbg):
    """Query digits, layer-1 windows, routed sets and per-cluster windows."""
    assert np.array_equal(gdbg["qdigits"].cpu().numpy(), odbg["qdigits"])
    assert np.array_equal(gdbg["l1"].cpu().numpy(), odbg["l1"])
    gr = gdbg["routed"].cpu().numpy()
    gp = gdbg["pairs"].cpu().numpy()
    orr, op = odbg["routed"], odbg["pairs"]
    for q in range(gr.shape[0]):
        gmap = {int(j): tuple(gp[q, t]) for t, j in enumerate(gr[q]) if j >= 0}
        omap = {int(j): tuple(op[q, t]) for t, j in enumerate(orr[q]) if j >= 0}
        assert gmap == omap, (q, gmap, omap)


def compare_topk(X, Q, gids, gsc, oids, osc, tol=SCORE_TOL):
    """Ids equal wherever FP64 score gaps exceed the tolerance; returned fp32
    scores within tolerance of the FP64 scores of the returned ids."""
    gids = np.asarray(gids)
    gsc = np.asarray(gsc, dtype=np.float64)
    nq, k = gids.shape
    xn = np.linalg.norm(X.astype(np.float64), axis=1)
    qn = np.linalg.norm(Q.astype(np.float64), axis=1)
    mism = 0
    for q in range(nq):
        gv, ov = gids[q] >= 0, oids[q] >= 0
        assert np.array_equal(gv, ov), (q, gids[q], oids[q])
        g, o = gids[q][gv], oids[q][ov]
        assert len(set(g.tolist())) == len(g)
        if len(g) == 0:
            continue
        s64 = oracle.pair_scores(X, Q, np.full(len(g), q), g)
        t = tol * qn[q] * np.maximum(xn[g], xn[o])
        assert np.all(np.abs(gsc[q][gv] - s64) <= tol * qn[q] * xn[g]), q
        assert np.all(np.abs(s64 - osc[q][ov]) <= t), (q, s64, osc[q][ov])
        mism += int(np.sum(g != o))
        assert np.all(np.isneginf(gsc[q][~gv]))
    return mism
