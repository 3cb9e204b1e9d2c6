"""Schedule autotuner for the rerank kernel (batching form).

For one shape bucket -- (index shape, precision, k, c, r, r1, batch-size
bucket) -- it times every candidate schedule of the window-scoring kernel
(rows per wave tile 32 / 64 / 128; 16, 32, 64 or 128 pairs per MFMA pass;
the library's own default shape; one wave per tile of the whole index, a persistent grid of 1 / 2 / 4 workgroups per CU pulling
tiles in chunks from per-XCD counters, or the same grid dealt only the tiles
some window overlaps from a list built on the device) on a representative
batch, checks that every candidate returns bit-identical ids and scores, and
keeps the fastest.  Results are cached in memory and, optionally, in a JSON
file.
"""
from __future__ import annotations

import json
import os

KEYS = ("tile_rows", "persistent", "grid_mult", "pass_pairs")
CANDIDATES = ([dict(tile_rows=0, persistent=0, grid_mult=0, pass_pairs=0)]
              + [dict(tile_rows=t, persistent=0, grid_mult=0, pass_pairs=pp)
                 for t in (32, 64, 128) for pp in (16, 32)]
              + [dict(tile_rows=t, persistent=0, grid_mult=0, pass_pairs=pp)
                 for t in (32, 64) for pp in (64, 128) if t * pp <= 4096]
              + [dict(tile_rows=t, persistent=p, grid_mult=g, pass_pairs=pp)
                 for p in (1, 2) for t in (32, 64) for g in (1, 2, 4) for pp in (0, 64)])


def bucket(nq):
    """Power-of-two batch-size bucket."""
    b = 1
    while b < nq:
        b <<= 1
    return b


class Autotuner:
    def __init__(self, index, path=None, reps=5):
        self.index = index
        self.path = path
        self.reps = reps
        self.cache = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    def key(self, nq, k, c, r, r1, precision):
        ix = self.index
        return (f"n{ix.n}-d{ix.d}-C{ix.C}-{precision}-k{k}-c{c}-r{r}-r1{r1}-b{bucket(nq)}")

    def tune(self, queries, k, c, r, r1=0, precision="f32"):
        """Best schedule for this bucket (tuning on `queries` if not cached)."""
        import torch
        from . import lider
        key = self.key(queries.shape[0], k, c, r, r1, precision)
        if key in self.cache:
            return self.cache[key]
        ref = None
        best = None
        timings = []
        for cand in CANDIDATES:
            out = self.index.search(queries, k, c, r, r1=r1, precision=precision, **cand)
            torch.cuda.synchronize()
            if ref is None:
                ref = out
            elif not (torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])):
                raise RuntimeError(f"schedule {cand} changed the results")
            lider.profile_begin(self.reps)
            for _ in range(self.reps):
                self.index.search(queries, k, c, r, r1=r1, precision=precision, **cand)
            torch.cuda.synchronize()
            stages, calls = lider.profile_end()
            ms = stages["rerank"] / calls
            timings.append(dict(cand, rerank_ms=round(ms, 4)))
            if best is None or ms < best[0]:
                best = (ms, cand)
        res = dict(best[1], rerank_ms=round(best[0], 4), candidates=timings)
        self.cache[key] = res
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return res

    def schedule(self, nq, k, c, r, r1=0, precision="f32"):
        """Cached schedule for a bucket (defaults if the bucket was never tuned)."""
        res = self.cache.get(self.key(nq, k, c, r, r1, precision))
        if res is None:
            return dict(tile_rows=0, persistent=0, grid_mult=0, pass_pairs=0)
        return {k2: res[k2] for k2 in KEYS}
