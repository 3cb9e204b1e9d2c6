"""Shared helpers of the GPU parity tests: build both sides from the same
seeded inputs and compare the GPU index / search against the FP64 oracle."""
import numpy as np

import oracle

SCORE_TOL = 1e-4  # |score difference| <= SCORE_TOL * |q| * |x| (fp32 vs FP64)


def build_pair(X, n_clusters, m, w, F, A, b, assignment=None, init_ids=None, iters=20, F1=0,
               storage="f32", centroid_storage="f32", seeding="given", n_arrays=1,
               hash_kind="e2lsh"):
    """GPU index and oracle index over the same host data."""
    import torch
    from paper_2205_00970_amd import lider
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    asg_d = None if assignment is None else torch.from_numpy(
        np.ascontiguousarray(assignment, dtype=np.int32)).cuda()
    gi = lider.Index(Xd, n_clusters, m, w, F, (A, b), rmi_fanout_l1=F1, kmeans_init=init_ids,
                     kmeans_iters=iters, assignment=asg_d, storage=storage,
                     centroid_storage=centroid_storage, seeding=seeding, n_arrays=n_arrays,
                     hash_kind=hash_kind)
    oi = oracle.Index(X, n_clusters, A, b, m, w, F, rmi_fanout_l1=(F1 or None),
                      assignment=assignment, init_ids=init_ids, kmeans_iters=iters,
                      seeding=seeding, n_arrays=n_arrays, hash_kind=hash_kind)
    return gi, oi, Xd


def compare_index(gi, oi):
    """Everything the build produces must match bit for bit (every array)."""
    C, m, H = oi.C, oi.m, oi.H
    n = oi.n
    assert gi.H == H
    assert gi.iters_run == oi.iters_run()
    assert np.array_equal(gi.export("assign"), oi.assignment())
    assert np.array_equal(gi.export("centroids").view(np.uint32),
                          oi.centroids().reshape(-1).view(np.uint32))
    assert np.array_equal(gi.export("offsets"), oi.offsets())
    dg = gi.export("digits").reshape(H, n * m)
    pm = gi.export("perm").reshape(H, n)
    ky = gi.export("keys").reshape(H, n)
    lo = gi.export("l1_order").reshape(H, C)
    lk = gi.export("l1_keys").reshape(H, C)
    ld = gi.export("l1_digits").reshape(H, C * m)
    mi = gi.export("model_int").reshape(H, C + 1, 3)
    mb = gi.export("model_box").reshape(H, C + 1, 2 * m)
    mk = gi.export("model_key").reshape(H, C + 1, 2)
    md = gi.export("model_dbl").reshape(H, C + 1, 3)
    lv = gi.export("leaves").reshape(H, -1, 2)
    le = gi.export("leaf_err").reshape(H, -1, 2)
    for h in range(H):
        assert np.array_equal(dg[h], oi.digits(h).reshape(-1)), h
        assert np.array_equal(pm[h], oi.perm(h)), h
        assert np.array_equal(ky[h], oi.keys(h)), h
        order, keys1, dig1 = oi.layer1(h)
        assert np.array_equal(lo[h], order), h
        assert np.array_equal(lk[h], keys1), h
        assert np.array_equal(ld[h], dig1.reshape(-1)), h
        _compare_models(oi, h, mi[h], mb[h], mk[h], md[h], lv[h], le[h])


def _compare_models(oi, h, mi, mb, mk, md, lv, le):
    C, m = oi.C, oi.m
    for j in range(C + 1):
        om = oi.model(j, array=h)
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
        gmap = {int(j): tuple(gp[q, t].reshape(-1)) for t, j in enumerate(gr[q]) if j >= 0}
        omap = {int(j): tuple(op[q, t].reshape(-1)) for t, j in enumerate(orr[q]) if j >= 0}
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
