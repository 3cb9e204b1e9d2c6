"""Seeded synthetic inputs shaped like the paper's passage-embedding corpora.

This module draws random numbers and nothing else: it holds none of LIDER's
arithmetic, so both the HIP path and the FP64 oracle can be fed from it.  The
random draws LIDER itself needs (LSH projections and offsets, k-means initial
ids) are also produced here and handed to both sides as inputs.

Workload families (the paper's corpora are 768-d passage embeddings of
100k-21M passages, Section 7.1.1; these Gaussian mixtures stand in for them):
  * tiny:    N=20,000, d=128, 16 components with means ~ N(0, I), sigma 0.3;
             queries = corpus points + N(0, 0.05^2) noise.
  * mixture: N rows, d=768, components with means rho*g/|g|, rho ~ U[8, 12],
             isotropic sigma 0.5; queries = corpus points + N(0, 0.1^2) noise.
             Generated chunk-wise with per-chunk seeds on any torch device.
"""
from __future__ import annotations

import numpy as np

CHUNK = 65536


def tiny(n=20000, d=128, ncomp=16, sigma=0.3, nq=100, qnoise=0.05, seed=0, qseed=1):
    """Tiny mixture: returns X [n,d] f32, labels [n] i32, Q [nq,d] f32, qsrc [nq] i64."""
    g = np.random.default_rng(seed)
    mu = g.standard_normal((ncomp, d))
    lab = g.integers(0, ncomp, size=n).astype(np.int32)
    X = (mu[lab] + sigma * g.standard_normal((n, d))).astype(np.float32)
    gq = np.random.default_rng(qseed)
    src = gq.choice(n, size=nq, replace=False).astype(np.int64)
    Q = (X[src].astype(np.float64) + qnoise * gq.standard_normal((nq, d))).astype(np.float32)
    return X, lab, Q, src


def lsh_params(m, d, w, seed=2, n_arrays=1):
    """E2LSH draws for both layers and H = n_arrays hashkey arrays:
    A [2Hm, d] ~ N(0,1), b [2Hm] ~ U[0, w).  Rows h*m.. are array h of the
    centroids retriever, rows H*m + h*m.. array h of the in-cluster retrievers
    (one set per array shared by every cluster)."""
    g = np.random.default_rng(seed)
    A = g.standard_normal((2 * n_arrays * m, d)).astype(np.float32)
    b = (g.random(2 * n_arrays * m) * w).astype(np.float32)
    return A, b


def array_params(A, b, m, n_arrays, h):
    """The single-array hash set [2m, d] of array h of a stacked [2Hm, d] set."""
    H = n_arrays
    rows = np.r_[h * m:(h + 1) * m, H * m + h * m:H * m + (h + 1) * m]
    return A[rows].copy(), b[rows].copy()


def kmeans_init(n, n_clusters, seed=3):
    """k-means initial centroids: the first n_clusters ids of a random permutation."""
    g = np.random.default_rng(seed)
    return g.permutation(n)[:n_clusters].astype(np.int64)


def _torch():
    import torch
    return torch


def mixture(n, d=768, ncomp=1000, sigma=0.5, rho=(8.0, 12.0), seed=0, device="cpu",
            dtype=None, sizes=None):
    """Gaussian mixture on a torch device, chunk-seeded.

    Component means are rho_j * g_j / |g_j|.  Labels are uniform over the
    components unless `sizes` (rows per component, summing to n) is given, in
    which case rows are laid out component by component and then shuffled.
    Returns (X [n, d], labels [n] int32) as torch tensors on `device`."""
    torch = _torch()
    dtype = dtype or torch.float32
    gm = torch.Generator(device="cpu").manual_seed(int(seed) * 7919 + 17)
    gdir = torch.randn(ncomp, d, generator=gm, dtype=torch.float64)
    rr = rho[0] + (rho[1] - rho[0]) * torch.rand(ncomp, generator=gm, dtype=torch.float64)
    mu = (gdir / gdir.norm(dim=1, keepdim=True) * rr[:, None]).to(torch.float32).to(device)
    if sizes is None:
        lab = torch.randint(0, ncomp, (n,), generator=gm, dtype=torch.int64)
    else:
        sizes = np.asarray(sizes, dtype=np.int64)
        assert sizes.sum() == n and sizes.shape[0] == ncomp
        lab = torch.repeat_interleave(torch.arange(ncomp), torch.from_numpy(sizes))
        lab = lab[torch.randperm(n, generator=gm)]
    lab = lab.to(device)
    X = torch.empty((n, d), dtype=dtype, device=device)
    for c0 in range(0, n, CHUNK):
        c1 = min(n, c0 + CHUNK)
        gc = torch.Generator(device=device).manual_seed(int(seed) * 1000003 + c0 // CHUNK)
        z = torch.randn((c1 - c0, d), generator=gc, device=device, dtype=torch.float32)
        X[c0:c1] = (mu[lab[c0:c1]] + sigma * z).to(dtype)
    return X, lab.to(torch.int32)


def queries_from(X, nq, noise, seed=1):
    """nq distinct corpus rows plus isotropic N(0, noise^2) perturbation."""
    torch = _torch()
    n, d = X.shape
    g = torch.Generator(device="cpu").manual_seed(int(seed) * 7919 + 29)
    src = torch.randperm(n, generator=g)[:nq].to(X.device)
    gz = torch.Generator(device=X.device).manual_seed(int(seed) * 1000003 + 5)
    z = torch.randn((nq, d), generator=gz, device=X.device, dtype=torch.float32)
    Q = X[src].to(torch.float32) + noise * z
    return Q.contiguous(), src


def normalize_rows(X):
    """Rows scaled to unit L2 norm (embeddings for the cosine variant); works on
    numpy arrays and torch tensors."""
    if isinstance(X, np.ndarray):
        nrm = np.linalg.norm(X.astype(np.float64), axis=1, keepdims=True)
        return (X / np.maximum(nrm, 1e-30)).astype(np.float32)
    nrm = X.double().norm(dim=1, keepdim=True).clamp_min(1e-30)
    return (X.double() / nrm).float()


def zipf_sizes(n, ncomp, s=1.1, lo=50, hi=200000):
    """Component sizes proportional to i^-s, clipped to [lo, hi] and
    water-filled to sum exactly n (remainder to the largest unclipped)."""
    w = np.arange(1, ncomp + 1, dtype=np.float64) ** (-s)
    lam_lo, lam_hi = 0.0, float(n) / w.min() * 4
    for _ in range(200):
        lam = 0.5 * (lam_lo + lam_hi)
        tot = np.clip(np.floor(lam * w), lo, hi).sum()
        if tot > n:
            lam_hi = lam
        else:
            lam_lo = lam
    sz = np.clip(np.floor(lam_lo * w), lo, hi).astype(np.int64)
    rem = n - int(sz.sum())
    free = np.where(sz < hi)[0]
    i = 0
    while rem != 0 and free.size:
        j = free[i % free.size]
        step = 1 if rem > 0 else -1
        if lo <= sz[j] + step <= hi:
            sz[j] += step
            rem -= step
        i += 1
    assert sz.sum() == n
    return sz


def poisson_arrivals(rate_qps, n_queries, mean_batch=128.5, bmin=1, bmax=256, seed=4):
    """Open-loop request stream: batch sizes U[bmin, bmax], exponential
    inter-arrival times at rate rate_qps/mean_batch requests per second.
    Returns (arrival times in s, batch sizes, k per request in {10, 100})."""
    g = np.random.default_rng(seed)
    sizes, times, ks = [], [], []
    t, tot = 0.0, 0
    lam = rate_qps / mean_batch
    while tot < n_queries:
        t += g.exponential(1.0 / lam)
        b = int(g.integers(bmin, bmax + 1))
        sizes.append(b)
        times.append(t)
        ks.append(10 if g.random() < 0.5 else 100)
        tot += b
    return np.array(times), np.array(sizes, np.int64), np.array(ks, np.int32)
