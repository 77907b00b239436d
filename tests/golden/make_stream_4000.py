"""Write tests/golden/stream_4000_s800_d8.npz from the CPU oracle only.

Workload: the CTD-D traffic stream of workloads/synth.traffic_stream with its
defaults: initial 4,000 x 4,000 x 200 tensor (1M nonzeros, Zipf(1.1) sources
and destinations, lognormal(0,1) values), then 200 one-step slices of
2,000-50,000 nonzeros, slices 5, 81 and 196 (0-based) carrying a dense
50 x 50 burst.  Mode 0, s = 800 for the initial CTD-S, d = 8 per slice,
Philox seed 0, eps = 1e-6.

The oracle runs the initial decomposition and all slices (Algorithm 2)
without carrying the block update of C (keep_C=False); the error of each step
follows from the frozen-history identity.  Stored per step: draws, unique
fibers, kept fibers, the error and the norm.  At the end, columns of C_(alpha)
from their closed form R^T P_tau x (Dynamic.core_columns): 64 seeded columns
over the whole stream plus 16 seeded columns of each burst slice.
Run: python tests/golden/make_stream_4000.py  (several minutes on 8 cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ctd  # noqa: E402
from workloads import synth  # noqa: E402

S, D, SEED = 800, 8, 0


def main():
    st = synth.traffic_stream()
    X = st.initial
    t0 = time.time()
    o = ctd.Dynamic(X.dims, X.idx, X.val, 0, S, SEED, keep_C=False)
    out = dict(init_draws=o.static.draws.astype(np.uint64),
               init_unique=o.static.uniq.astype(np.uint64),
               init_accepted=o.static.accepted.astype(np.uint64),
               init_err2=np.float64(o.static.err2), init_norm2=np.float64(o.static.norm2))
    draws, uniq, acc, err2, norm2, dt, ncols = [], [], [], [], [], [], []
    n_slices = len(st.slices)
    for t in range(n_slices):
        sl = st.slices[t]
        info = o.update(sl.dims, sl.idx, sl.val, D)
        draws.append(np.asarray(info["draws"], dtype=np.uint64))
        uniq.append(np.asarray(info["uniq"], dtype=np.uint64))
        acc.append(np.asarray(o.accepted[len(o.accepted) - info["added"]:], dtype=np.uint64))
        err2.append(info["err2"])
        norm2.append(info["norm2"])
        dt.append(info["d_tilde"])
        ncols.append(o.col_fids.shape[0])
        print(t, sl.nnz, info["added"], info["d_tilde"], info["err2"] / info["norm2"],
              f"{time.time() - t0:.0f}s", flush=True)
    n_cols = o.col_fids.shape[0]
    rng = np.random.Generator(np.random.Philox(7))
    cols = [rng.choice(n_cols, size=64, replace=False)]
    for b in st.anomaly_steps:
        lo = ncols[b - 1] if b else o.inputs[0][1].n_f
        cols.append(lo + rng.choice(ncols[b] - lo, size=16, replace=False))
    cols = np.unique(np.concatenate(cols))
    C_sample = o.core_columns(cols)
    out.update(n_slices=np.int64(n_slices),
               draws=np.concatenate(draws), draws_len=np.array([len(x) for x in draws]),
               unique=np.concatenate(uniq), unique_len=np.array([len(x) for x in uniq]),
               accepted=np.concatenate(acc), accepted_len=np.array([len(x) for x in acc]),
               err2=np.array(err2), norm2=np.array(norm2), d_tilde=np.array(dt),
               n_cols=np.array(ncols, dtype=np.int64),
               anomaly_steps=np.array(st.anomaly_steps, dtype=np.int64),
               all_accepted=np.asarray(o.accepted, dtype=np.uint64),
               C_cols=cols.astype(np.int64), C_fids=o.col_fids[cols].astype(np.uint64),
               C_sample=np.ascontiguousarray(C_sample))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stream_4000_s800_d8.npz")
    np.savez_compressed(path, **out)
    print(path, o.rel_err, len(o.accepted), n_cols, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
