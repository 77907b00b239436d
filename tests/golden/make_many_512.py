"""Write tests/golden/many_512_subset.npz from the CPU oracle only.

Workload: the 512 independent tensors of workloads/synth.many_tensors (I, J
uniform in 500..5000, K in 20..200, 10k-200k nonzeros with Zipf(1.2) degrees,
uniform(0,1] values), mode 0, s_b = ceil(5% of tensor b's non-empty fibers),
Philox seed 0, tensor b drawing with counter word b (the batched CTD-S form),
eps = 1e-6.  The oracle decomposes a subset of 16 tensors whose nonzero
counts span the range (every 34th of the 512 sorted by nonzero count, plus the
largest).  Stored per tensor: index b, s_b, draws, unique fibers and
multiplicities, kept fibers, err2, norm2.
Run: python tests/golden/make_many_512.py  (about 15 minutes on 8 cores).
"""
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ctd  # noqa: E402
from workloads import synth  # noqa: E402

SEED = 0
N_PICK = 16


def pick(nnz):
    order = np.argsort(nnz, kind="stable")
    ranks = np.unique(np.concatenate([np.arange(0, len(nnz), len(nnz) // (N_PICK - 1))[:N_PICK - 1],
                                      [len(nnz) - 1]]))
    return np.sort(order[ranks])


def run_one(args):
    b, t = args
    t0 = time.time()
    s = max(1, math.ceil(0.05 * synth.count_nonempty_fibers(t, 0)))
    o = ctd.ctd_s(t.dims, t.idx, t.val, 0, s, SEED, tensor=b)
    print(b, t.dims, t.nnz, s, len(o.uniq), len(o.accepted), f"{time.time() - t0:.0f}s", flush=True)
    return dict(b=b, s=s, draws=o.draws.astype(np.uint64), unique=o.uniq.astype(np.uint64),
                counts=o.counts.astype(np.int32), accepted=o.accepted.astype(np.uint64),
                err2=o.err2, norm2=o.norm2)


def main():
    ts = synth.many_tensors()
    sel = pick(np.array([t.nnz for t in ts]))
    with mp.get_context("fork").Pool(4) as pool:
        res = pool.map(run_one, [(int(b), ts[b]) for b in sel], chunksize=1)
    out = dict(tensors=np.array([r["b"] for r in res], dtype=np.int64),
               s=np.array([r["s"] for r in res], dtype=np.int64),
               err2=np.array([r["err2"] for r in res]), norm2=np.array([r["norm2"] for r in res]))
    for key in ("draws", "unique", "counts", "accepted"):
        out[key] = np.concatenate([r[key] for r in res])
        out[key + "_len"] = np.array([len(r[key]) for r in res], dtype=np.int64)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "many_512_subset.npz")
    np.savez_compressed(path, **out)
    print(path)


if __name__ == "__main__":
    main()
