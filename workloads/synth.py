"""Seeded synthetic sparse tensors shaped like the paper's network-traffic workloads.

This module only draws inputs.  It contains none of the decomposition's
arithmetic, so both the CPU oracle and the GPU path may take their inputs
from here without sharing any part of the method.

The paper's own data (Section 4.1, Table 3: KONECT contact networks and a
CAIDA-derived traffic tensor, source x destination x time) is not available,
so these generators stand in for it: same mode semantics, power-law source
and destination degrees, uniform time, heavy-tailed positive values.

Conventions shared by every generator:
  * coordinates are 0-based, distinct, and returned in a random (unordered)
    order, matching the sparse-unordered storage the paper assumes (Section 2.1);
  * values are drawn in float64 and rounded to float32, so the float64 and the
    float32 paths see bit-identical inputs after widening;
  * the data RNG is numpy's Philox bit generator seeded with the config seed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class CooTensor:
    dims: tuple            # mode lengths (I_1, ..., I_N)
    idx: np.ndarray        # int32 [N, nnz], 0-based
    val: np.ndarray        # float64 [nnz], every value exactly representable in float32

    @property
    def order(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])

    def val32(self) -> np.ndarray:
        return self.val.astype(np.float32)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed)))


def _zipf_indices(rng, n_items: int, a: float, size: int, perm: np.ndarray) -> np.ndarray:
    """Truncated Zipf(a) over ranks 1..n_items, ranks mapped to ids by `perm`."""
    k = np.arange(1, n_items + 1, dtype=np.float64)
    pmf = k ** (-a)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    u = rng.random(size)
    rank = np.searchsorted(cdf, u, side="right")
    rank = np.minimum(rank, n_items - 1)
    return perm[rank]


def _linear(coords, dims):
    """Row-major linear cell id, used only to enforce distinct coordinates."""
    lin = np.zeros(coords[0].shape[0], dtype=np.int64)
    for m, d in enumerate(dims):
        lin = lin * int(d) + coords[m].astype(np.int64)
    return lin


def _distinct(draw, dims, nnz, rng):
    """Draw batches of coordinates until exactly `nnz` distinct cells are held.

    `draw(m)` returns a tuple of N int arrays of length m.  Earlier draws win
    over later ones; the final order is shuffled.
    """
    kept = np.zeros(0, dtype=np.int64)
    coords_kept = [np.zeros(0, dtype=np.int64) for _ in dims]
    need = nnz
    while need > 0:
        m = max(1024, int(need * 1.3) + 64)
        c = draw(m)
        lin = _linear(c, dims)
        allc = np.concatenate([kept, lin])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        # keep cells in order of first appearance
        new_pos = first[first >= kept.shape[0]] - kept.shape[0]
        take = new_pos[:need]
        kept = np.concatenate([kept, lin[take]])
        coords_kept = [np.concatenate([coords_kept[i], c[i][take].astype(np.int64)])
                       for i in range(len(dims))]
        need = nnz - kept.shape[0]
    order = rng.permutation(nnz)
    return np.stack([ck[order] for ck in coords_kept]).astype(np.int32)


def _f32(x: np.ndarray) -> np.ndarray:
    return x.astype(np.float32).astype(np.float64)


def uniform_tensor(dims, nnz, seed, low_open=True) -> CooTensor:
    """Distinct uniform coordinates, values uniform on (0, 1]."""
    rng = _rng(seed)
    dims = tuple(int(d) for d in dims)

    def draw(m):
        return tuple(rng.integers(0, d, size=m) for d in dims)

    idx = _distinct(draw, dims, nnz, rng)
    v = 1.0 - rng.random(nnz)          # (0, 1]
    v = _f32(v)
    v[v == 0.0] = 1.0
    return CooTensor(dims, idx, v)


def power_law_tensor(dims, nnz, seed, zipf_a=1.2, values="lognormal") -> CooTensor:
    """Source x destination x time traffic tensor.

    Sources and destinations follow a truncated Zipf(zipf_a) law with a
    seeded rank-to-id permutation (hot hosts are scattered), time is uniform.
    Values are lognormal(0, 1) or uniform (0, 1].
    """
    rng = _rng(seed)
    dims = tuple(int(d) for d in dims)
    perms = [rng.permutation(d) for d in dims[:2]]

    def draw(m):
        src = _zipf_indices(rng, dims[0], zipf_a, m, perms[0])
        dst = _zipf_indices(rng, dims[1], zipf_a, m, perms[1])
        rest = [rng.integers(0, d, size=m) for d in dims[2:]]
        return (src, dst, *rest)

    idx = _distinct(draw, dims, nnz, rng)
    if values == "lognormal":
        v = rng.lognormal(0.0, 1.0, nnz)
    else:
        v = 1.0 - rng.random(nnz)
    v = _f32(v)
    v[v == 0.0] = np.float64(np.float32(1e-30))
    return CooTensor(dims, idx, v)


def planted_low_rank(dims=(5000, 5000, 500), rank=20, seed=3, noise_frac=0.01,
                     noise_rel=0.01, factor_nnz=(100, 100, 10)) -> tuple:
    """Sum of `rank` sparse nonnegative rank-1 terms plus additive sparse noise.

    Factor entries are dyadic k/16, k in 1..16, so every product and every sum
    of up to a few thousand terms is exact in float32 and float64; the
    noise-free tensor therefore has mode-1 rank exactly `rank` (for generic
    supports).  Returns (noisy tensor, noise-free tensor).
    """
    rng = _rng(seed)
    dims = tuple(int(d) for d in dims)
    cells = {}
    acc = {}
    for _q in range(rank):
        fac_idx = []
        fac_val = []
        for m in range(3):
            ids = np.sort(rng.choice(dims[m], size=factor_nnz[m], replace=False))
            vals = rng.integers(1, 17, size=factor_nnz[m]).astype(np.float64) / 16.0
            fac_idx.append(ids)
            fac_val.append(vals)
        I, J, K = np.meshgrid(fac_idx[0], fac_idx[1], fac_idx[2], indexing="ij")
        V = (fac_val[0][:, None, None] * fac_val[1][None, :, None]) * fac_val[2][None, None, :]
        lin = ((I.astype(np.int64) * dims[1] + J) * dims[2] + K).ravel()
        for key, val in ((lin, V.ravel()),):
            acc.setdefault("k", []).append(key)
            acc.setdefault("v", []).append(val)
    keys = np.concatenate(acc["k"])
    vals = np.concatenate(acc["v"])
    uk, inv = np.unique(keys, return_inverse=True)
    sv = np.zeros(uk.shape[0], dtype=np.float64)
    np.add.at(sv, inv, vals)
    del cells
    clean_keys = uk
    clean_vals = sv
    # additive sparse noise: noise_frac of nnz at uniform coordinates
    n_noise = int(round(noise_frac * clean_keys.shape[0]))
    total = dims[0] * dims[1] * dims[2]
    nk = np.unique(rng.integers(0, total, size=int(n_noise * 1.05) + 16))
    nk = rng.permutation(nk)[:n_noise]
    nv = rng.standard_normal(nk.shape[0])
    s_norm = math.sqrt(float(np.sum(clean_vals ** 2)))
    nv *= noise_rel * s_norm / max(1e-300, math.sqrt(float(np.sum(nv ** 2))))
    all_k = np.concatenate([clean_keys, nk])
    all_v = np.concatenate([clean_vals, nv])
    uk2, inv2 = np.unique(all_k, return_inverse=True)
    v2 = np.zeros(uk2.shape[0], dtype=np.float64)
    np.add.at(v2, inv2, all_v)
    v2 = _f32(v2)
    keep = v2 != 0.0
    uk2, v2 = uk2[keep], v2[keep]

    def unlin(k):
        K = k % dims[2]
        J = (k // dims[2]) % dims[1]
        I = k // (dims[1] * dims[2])
        return np.stack([I, J, K]).astype(np.int32)

    p1 = rng.permutation(uk2.shape[0])
    noisy = CooTensor(dims, unlin(uk2[p1]), v2[p1])
    p2 = rng.permutation(clean_keys.shape[0])
    clean = CooTensor(dims, unlin(clean_keys[p2]), _f32(clean_vals[p2]))
    return noisy, clean


@dataclasses.dataclass
class Stream:
    initial: CooTensor          # I x J x T0
    slices: list                # list of CooTensor, each I x J x 1
    anomaly_steps: list         # slice numbers (0-based) carrying an injected block
    anomaly_blocks: list        # (sources, destinations) of each block


def traffic_stream(dims=(4000, 4000, 200), nnz0=1_000_000, n_slices=200,
                   slice_nnz=(2000, 50000), zipf_a=1.1, n_anomalies=3,
                   block=50, seed=4) -> Stream:
    """Initial traffic tensor plus a stream of one-step time slices.

    Slices follow the initial tensor's law with a uniformly drawn nnz count;
    `n_anomalies` slices get a dense block x block burst (random sources x
    random destinations) of lognormal(ln 20, 0.25) values overwriting any
    traffic already in those cells.
    """
    I, J, T0 = (int(d) for d in dims)
    initial = power_law_tensor((I, J, T0), nnz0, seed, zipf_a=zipf_a)
    rng = _rng(seed + 1000)
    perms = [rng.permutation(I), rng.permutation(J)]
    steps = sorted(rng.choice(n_slices, size=n_anomalies, replace=False).tolist()) if n_anomalies else []
    blocks = []
    slices = []
    for t in range(n_slices):
        n = int(rng.integers(slice_nnz[0], slice_nnz[1] + 1))

        def draw(m):
            return (_zipf_indices(rng, I, zipf_a, m, perms[0]),
                    _zipf_indices(rng, J, zipf_a, m, perms[1]),
                    np.zeros(m, dtype=np.int64))

        idx = _distinct(draw, (I, J, 1), n, rng)
        v = _f32(rng.lognormal(0.0, 1.0, n))
        if t in steps:
            srcs = np.sort(rng.choice(I, size=block, replace=False))
            dsts = np.sort(rng.choice(J, size=block, replace=False))
            blocks.append((srcs, dsts))
            S, D = np.meshgrid(srcs, dsts, indexing="ij")
            bk = (S.astype(np.int64) * J + D).ravel()
            bv = _f32(rng.lognormal(math.log(20.0), 0.25, bk.shape[0]))
            old = idx[0].astype(np.int64) * J + idx[1]
            keep = ~np.isin(old, bk)
            idx = np.concatenate([idx[:, keep],
                                  np.stack([S.ravel(), D.ravel(), np.zeros(bk.shape[0], np.int64)]).astype(np.int32)],
                                 axis=1)
            v = np.concatenate([v[keep], bv])
            p = rng.permutation(v.shape[0])
            idx, v = idx[:, p], v[p]
        slices.append(CooTensor((I, J, 1), idx.astype(np.int32), v))
    return Stream(initial, slices, steps, blocks)


@dataclasses.dataclass
class AttackStream:
    initial: CooTensor          # I x J x T0 normal traffic
    slices: list                # list of CooTensor, each I x J x 1
    attacks: list               # (slice number, victim destination, attacking sources)


def attack_stream(dims=(300, 400, 10), nnz0=20_000, n_slices=20, slice_nnz=(500, 2000),
                  zipf_a=1.1, n_attacks=3, attacker_frac=0.2, seed=8) -> AttackStream:
    """Traffic with injected DDoS attacks (the setting of the paper's application
    section): normal source x destination traffic under Zipf(zipf_a) degrees, and
    `n_attacks` slices in which a randomly chosen `attacker_frac` of all sources
    each send lognormal(ln 20, 0.25) traffic to one victim destination.  The
    victims are destinations that normal traffic never reaches, so that each
    attack is a new activity in R.
    """
    I, J, T0 = (int(d) for d in dims)
    rng = _rng(seed)
    perm_src = rng.permutation(I)
    perm_dst = rng.permutation(J)
    victims_all = perm_dst[J - n_attacks:]          # reserved for the attacks
    normal_dst = perm_dst[:J - n_attacks]

    def normal(n, t_len):
        def draw(m):
            return (_zipf_indices(rng, I, zipf_a, m, perm_src),
                    _zipf_indices(rng, J - n_attacks, zipf_a, m, normal_dst),
                    rng.integers(0, t_len, m))
        idx = _distinct(draw, (I, J, t_len), n, rng)
        return idx, _f32(rng.lognormal(0.0, 1.0, n))

    idx0, v0 = normal(nnz0, T0)
    initial = CooTensor((I, J, T0), idx0.astype(np.int32), v0)
    steps = sorted(rng.choice(n_slices, size=n_attacks, replace=False).tolist())
    attacks = []
    slices = []
    for t in range(n_slices):
        idx, v = normal(int(rng.integers(slice_nnz[0], slice_nnz[1] + 1)), 1)
        if t in steps:
            victim = int(victims_all[len(attacks)])
            srcs = np.sort(rng.choice(I, size=max(1, int(round(attacker_frac * I))), replace=False))
            attacks.append((t, victim, srcs))
            add_idx = np.stack([srcs, np.full(srcs.shape[0], victim), np.zeros(srcs.shape[0], np.int64)])
            idx = np.concatenate([idx, add_idx.astype(idx.dtype)], axis=1)
            v = np.concatenate([v, _f32(rng.lognormal(math.log(20.0), 0.25, srcs.shape[0]))])
            p = rng.permutation(v.shape[0])
            idx, v = idx[:, p], v[p]
        slices.append(CooTensor((I, J, 1), idx.astype(np.int32), v))
    return AttackStream(initial, slices, attacks)


def many_tensors(n_tensors=512, seed=5, ij=(500, 5000), k=(20, 200),
                 nnz=(10_000, 200_000), zipf_a=1.2) -> list:
    """Independent tensors of uneven shape and size (uniform(0,1] values)."""
    rng = _rng(seed)
    out = []
    for b in range(n_tensors):
        I = int(rng.integers(ij[0], ij[1] + 1))
        J = int(rng.integers(ij[0], ij[1] + 1))
        K = int(rng.integers(k[0], k[1] + 1))
        n = int(rng.integers(nnz[0], nnz[1] + 1))
        n = min(n, I * J * K // 4)
        out.append(power_law_tensor((I, J, K), n, seed * 100003 + b, zipf_a=zipf_a,
                                    values="uniform"))
    return out


def count_nonempty_fibers(t: CooTensor, mode: int) -> int:
    """Number of distinct index tuples over the modes other than `mode`."""
    rest = [m for m in range(t.order) if m != mode]
    lin = _linear([t.idx[m] for m in rest], [t.dims[m] for m in rest])
    return int(np.unique(lin).shape[0])


# The workloads, by name, with their sizes.
def tiny_uniform(seed=1):
    """200 x 200 x 50, 20,000 uniform nonzeros, values uniform (0,1]."""
    return uniform_tensor((200, 200, 50), 20_000, seed)


def traffic_5m(seed=2):
    """10,000 x 10,000 x 1,000, 5M nonzeros, Zipf(1.2) src/dst, lognormal(0,1)."""
    return power_law_tensor((10_000, 10_000, 1_000), 5_000_000, seed, zipf_a=1.2)


def small_shapes(seed=11):
    """Tensors shaped like the paper's Table 3 datasets (shapes and nnz only)."""
    shapes = [((112, 113, 5246), 20818), ((77, 274, 1567), 27972),
              ((167, 166, 2615), 70523), ((407, 410, 1392), 17298),
              ((189, 189, 1000), 20511)]
    return [power_law_tensor(d, n, seed + i, zipf_a=1.2) for i, (d, n) in enumerate(shapes)]
