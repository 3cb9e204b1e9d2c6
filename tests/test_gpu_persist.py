"""GPU checks of index save / load (lider_save / lider_load): a loaded index
holds the same arrays and searches bit-identically to the one that was saved,
for one and several hashkey arrays, both hash families, bf16 and fp8 copies;
damaged files are rejected."""
import os

import numpy as np
import pytest

from paper_2205_00970_amd import datagen, lider

pytestmark = pytest.mark.gpu

EXPORTS = ["centroids", "assign", "offsets", "perm", "keys", "digits", "l1_order", "l1_keys",
           "l1_digits", "model_int", "model_box", "model_key", "model_dbl", "leaves", "leaf_err",
           "reordered"]


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("H,kind,storage,cstorage", [(1, "e2lsh", "bf16", "fp8"),
                                                     (3, "e2lsh", "f32", "f32"),
                                                     (2, "sign", "bf16", "f32")])
def test_save_load_round_trip(tmp_path, H, kind, storage, cstorage):
    torch = _torch()
    X, lab, Q, _ = datagen.tiny(n=12000, d=64, ncomp=12, nq=80)
    if kind == "sign":
        X, Q = datagen.normalize_rows(X), datagen.normalize_rows(Q)
    A, b = datagen.lsh_params(6, 64, 1.0, seed=41, n_arrays=H)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    gi = lider.Index(Xd, 12, 6, 1.0, 8, (A, b), kmeans_init=datagen.kmeans_init(12000, 12),
                     kmeans_iters=5, storage=storage, centroid_storage=cstorage, hash_kind=kind,
                     n_arrays=H)
    path = str(tmp_path / "index.lider")
    gi.save(path)
    assert os.path.getsize(path) > X.nbytes
    li = lider.Index.load(path)
    assert (li.n, li.d, li.C, li.m, li.H, li.max_cluster, li.iters_run, li.hash_kind) == \
        (gi.n, gi.d, gi.C, gi.m, gi.H, gi.max_cluster, gi.iters_run, kind)
    for e in EXPORTS:
        assert np.array_equal(gi.export(e).view(np.uint8), li.export(e).view(np.uint8)), e
    runs = [dict(k=10, c=3, r=40, r1=4), dict(k=100, c=12, r=5000, r1=12),
            dict(k=10, c=2, r=64, r1=12, persistent=2)]
    if storage == "bf16":
        runs.append(dict(k=10, c=3, r=40, r1=4, precision="bf16"))
    if kind == "sign":
        runs.append(dict(k=10, c=3, r=40, r1=4, expand_bits=3))
    for kw in runs:
        a = gi.search(Qd, **kw)
        bb = li.search(Qd, **kw)
        assert torch.equal(a[0], bb[0]) and torch.equal(a[1], bb[1]), kw
    # the saved index is still usable and the loaded one survives it being freed
    gi.close()
    again = li.search(Qd, k=10, c=3, r=40, r1=4)
    assert again[0].shape == (80, 10)
    li.close()


def test_damaged_files_are_rejected(tmp_path):
    torch = _torch()
    X, lab, Q, _ = datagen.tiny(n=3000, d=32, ncomp=4, nq=10)
    A, b = datagen.lsh_params(3, 32, 1.0, seed=43)
    gi = lider.Index(torch.from_numpy(X).cuda(), 4, 3, 1.0, 4, (A, b),
                     assignment=torch.from_numpy(lab).cuda())
    path = tmp_path / "ok.lider"
    gi.save(str(path))
    data = path.read_bytes()
    cut = tmp_path / "cut.lider"
    cut.write_bytes(data[: len(data) // 2])
    longer = tmp_path / "long.lider"
    longer.write_bytes(data + b"\0")
    badver = tmp_path / "ver.lider"
    badver.write_bytes(data[:8] + b"\x07" + data[9:])
    for p in (cut, longer, badver, tmp_path / "none.lider"):
        with pytest.raises(lider.LiderError) as ei:
            lider.Index.load(str(p))
        assert ei.value.status == lider.EIO, p
    li = lider.Index.load(str(path))  # the intact file still loads
    Qd = torch.from_numpy(Q).cuda()
    assert torch.equal(li.search(Qd, 5, 2, 100)[0], gi.search(Qd, 5, 2, 100)[0])
