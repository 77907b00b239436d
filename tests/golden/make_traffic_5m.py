"""Write tests/golden/traffic_5m_s2000_seed0.npz from the CPU oracle only.

Workload: 10,000 x 10,000 x 1,000 traffic tensor, 5M nonzeros, Zipf(1.2)
sources and destinations, uniform time, lognormal(0,1) values (workloads/
synth.traffic_5m), mode 0, s = 2000 draws, Philox seed 0, eps = 1e-6.
Stores the draws, unique fibers, multiplicities, kept fibers, the error and
a seeded sample of per-fiber residuals ||x_f||^2 - ||P x_f||^2.
Run: python tests/golden/make_traffic_5m.py  (about a minute on 8 cores).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ctd  # noqa: E402
from workloads import synth  # noqa: E402


def main():
    X = synth.traffic_5m()
    r = ctd.ctd_s(X.dims, X.idx, X.val, 0, 2000, 0)
    u = r.unfolding
    col_norm2 = np.asarray(u.mat.multiply(u.mat).sum(axis=0)).ravel()
    resid = col_norm2 - r.proj
    acc_pos = np.searchsorted(u.fids, r.accepted)
    resid[acc_pos] = 0.0
    rng = np.random.Generator(np.random.Philox(99))
    sample = np.sort(rng.choice(u.n_f, size=4000, replace=False))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "traffic_5m_s2000_seed0.npz")
    np.savez_compressed(out, draws=r.draws.astype(np.uint64), unique=r.uniq.astype(np.uint64),
                        counts=r.counts.astype(np.int32), prob=r.p, scale=r.omega,
                        accepted=r.accepted.astype(np.uint64), rho=r.rho,
                        err2=np.float64(r.err2), norm2=np.float64(r.norm2),
                        rel_err=np.float64(r.rel_err), n_f=np.int64(u.n_f),
                        sample_pos=sample.astype(np.int64),
                        sample_fid=u.fids[sample].astype(np.uint64),
                        sample_resid=resid[sample])
    print(out, r.rel_err, len(r.uniq), len(r.accepted))


if __name__ == "__main__":
    main()
