"""Seeded synthetic inputs for the spatial-index hot path.

This module only produces inputs (points, query points, boxes, delete-id
batches). It contains none of the index arithmetic: no space-filling-curve
code, no sorting by key, no distances. Both the CPU oracle and the GPU path
take their inputs from here, so the two sides always see identical arrays.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw i of stream s is mix64(s + (i + 1) * GAMMA). Every purpose
(data, inserts, deletes, queries, boxes) gets its own stream derived from
(seed, purpose), so arrays can be regenerated independently and in any order.

Workloads stand in for the paper's synthetic sets (Sec. 5.1 "Setup"):
  * uniform  -- every coordinate uniform over the domain;
  * varden   -- clustered random walks (the paper's Varden workload, which
               walks through space and rarely restarts).  Here: 1000 walks
               whose sizes follow a Zipf law (s = 1.1), each walk with its own
               step scale, log-uniform over 2^4..2^20.
The paper's real-world datasets are not available and are not reproduced.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream purposes
P_DATA, P_INSERT, P_DELETE, P_QUERY, P_BOX, P_AUX = 0, 1, 2, 3, 4, 5


def _mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, purpose: int) -> np.uint64:
    """Key of the stream for (seed, purpose)."""
    a = _mix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))
    with np.errstate(over="ignore"):
        b = _mix64(a + np.uint64((purpose * 0x632BE59BD9B4E019) & 0xFFFFFFFFFFFFFFFF))
    return b[0]


def draws(key: np.uint64, start: int, count: int) -> np.ndarray:
    """count u64 draws i = start .. start+count-1 of the stream `key`."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(key) + idx * GAMMA)


def unit(u: np.ndarray) -> np.ndarray:
    """u64 draws -> float64 in [0, 1) using the top 53 bits."""
    return (u >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _bounded(u: np.ndarray, bound) -> np.ndarray:
    """u64 draws -> integers in [0, bound) (bound <= 2^32) by multiply-shift."""
    hi = (u >> np.uint64(32))
    with np.errstate(over="ignore"):
        return ((hi * np.asarray(bound, dtype=np.uint64)) >> np.uint64(32))


# --------------------------------------------------------------------- points

def uniform(n: int, dim: int, bits: int, seed: int, purpose: int = P_DATA) -> np.ndarray:
    """n points, uint32 [n, dim], each coordinate = top `bits` bits of a draw.

    Draw order is x, then y (then z) for point 0, then point 1, ...
    """
    if n == 0:
        return np.zeros((0, dim), dtype=np.uint32)
    u = draws(stream_key(seed, purpose), 0, n * dim)
    return (u >> np.uint64(64 - bits)).astype(np.uint32).reshape(n, dim)


def zipf_sizes(n: int, clusters: int, s: float) -> np.ndarray:
    """Cluster sizes proportional to r^-s (r = 1..clusters), summing to n.

    Rounding is by largest remainder (ties to the smaller rank).
    """
    w = np.arange(1, clusters + 1, dtype=np.float64) ** (-s)
    ideal = n * w / w.sum()
    base = np.floor(ideal).astype(np.int64)
    rem = n - int(base.sum())
    frac = ideal - base
    order = np.lexsort((np.arange(clusters), -frac))
    base[order[:rem]] += 1
    return base


def _fold(v: np.ndarray, hi: int) -> np.ndarray:
    """Reflect integers into [0, hi] (a walk that bounces off the domain edges)."""
    period = 2 * hi
    r = np.mod(v, period)
    return np.where(r > hi, period - r, r)


def varden(n: int, dim: int, bits: int, seed: int, purpose: int = P_DATA,
           clusters: int = 1000, zipf_s: float = 1.1,
           step_lo: int = 4, step_hi: int = 20) -> np.ndarray:
    """Clustered random-walk points, uint32 [n, dim], shuffled.

    Walk c has size from `zipf_sizes`, starts at a uniform point, and has a
    step scale L_c = floor(2^(step_lo + (step_hi - step_lo) * u)). Every step
    moves each coordinate by a uniform integer in [-L_c, L_c]; positions are
    the running sums folded back into [0, 2^bits - 1] (mirror reflection at
    both edges). All visited positions are emitted, then the whole set is
    shuffled by sorting on fresh draws.
    """
    if n == 0:
        return np.zeros((0, dim), dtype=np.uint32)
    key = stream_key(seed, purpose)
    hi = (1 << bits) - 1
    sizes = zipf_sizes(n, clusters, zipf_s)
    c = clusters
    head = draws(key, 0, c * (dim + 1))
    starts = (head[: c * dim] >> np.uint64(64 - bits)).astype(np.int64).reshape(c, dim)
    scale = np.floor(2.0 ** (step_lo + (step_hi - step_lo) * unit(head[c * dim:]))).astype(np.int64)
    owner = np.repeat(np.arange(c), sizes)
    first = np.concatenate(([0], np.cumsum(sizes)[:-1]))
    out = np.empty((n, dim), dtype=np.uint32)
    for d in range(dim):
        u = draws(key, c * (dim + 1) + d * n, n)
        span = (2 * scale[owner] + 1).astype(np.uint64)
        step = _bounded(u, span).astype(np.int64) - scale[owner]
        cs = np.cumsum(step)
        # per-walk running sum: subtract the global prefix before each walk
        before = np.where(first > 0, cs[np.maximum(first - 1, 0)], 0)
        cs -= np.repeat(np.where(sizes > 0, before, 0), sizes)
        pos = starts[owner, d] + cs
        out[:, d] = _fold(pos, hi).astype(np.uint32)
        del u, span, step, cs, pos
    perm = np.argsort(draws(key, c * (dim + 1) + dim * n, n), kind="stable")
    return out[perm]


def sweepline(n: int, dim: int, bits: int, seed: int, purpose: int = P_DATA) -> np.ndarray:
    """The uniform points of `uniform(n, ...)` ordered by their first
    coordinate (stable: equal first coordinates keep their draw order), the
    skewed update order of the paper's Sweepline workload (Sec. 5.1): batches
    taken in this order are slabs of space."""
    u = uniform(n, dim, bits, seed, purpose)
    return u[np.argsort(u[:, 0], kind="stable")] if n else u


def points(dist: str, n: int, dim: int, bits: int, seed: int, purpose: int = P_DATA) -> np.ndarray:
    if dist == "uniform":
        return uniform(n, dim, bits, seed, purpose)
    if dist == "varden":
        return varden(n, dim, bits, seed, purpose)
    if dist == "sweepline":
        return sweepline(n, dim, bits, seed, purpose)
    raise ValueError(f"unknown distribution {dist!r}")


def workload(dist: str, dim: int, bits: int, seed: int, n: int, n_insert: int = 0,
             n_query: int = 0):
    """Data, insert batch and query points drawn from one distribution.

    For `varden` the three sets are slices of one generation, so inserts and
    queries follow the same clusters as the data. For `uniform` they are
    separate streams of the same law.
    """
    if dist == "varden":
        allp = varden(n + n_insert + n_query, dim, bits, seed)
        return allp[:n], allp[n:n + n_insert], allp[n + n_insert:]
    return (uniform(n, dim, bits, seed, P_DATA), uniform(n_insert, dim, bits, seed, P_INSERT),
            uniform(n_query, dim, bits, seed, P_QUERY))


# ---------------------------------------------------------------- other input

def delete_ids(live_ids: np.ndarray, m: int, seed: int) -> np.ndarray:
    """m distinct ids taken from `live_ids` by a seeded partial shuffle."""
    live = np.asarray(live_ids, dtype=np.uint32)
    m = min(m, live.size)
    if m == 0:
        return np.zeros(0, dtype=np.uint32)
    r = draws(stream_key(seed, P_DELETE), 0, live.size)
    pick = np.argpartition(r, m - 1)[:m] if m < live.size else np.arange(live.size)
    pick = pick[np.argsort(r[pick], kind="stable")]
    return live[pick].copy()


def boxes(centres: np.ndarray, bits: int, seed: int, side_lo: int = 8, side_hi: int = 18) -> np.ndarray:
    """Axis-aligned closed boxes, uint32 [nb, 2, dim] (row 0 = lo, row 1 = hi).

    Each side is floor(2^(side_lo + (side_hi - side_lo) * u)) drawn per box and
    per dimension; the box is centred on the given point and shifted to stay
    inside [0, 2^bits).
    """
    c = np.asarray(centres, dtype=np.int64)
    nb, dim = c.shape
    u = unit(draws(stream_key(seed, P_BOX), 0, nb * dim)).reshape(nb, dim)
    side = np.floor(2.0 ** (side_lo + (side_hi - side_lo) * u)).astype(np.int64)
    side = np.minimum(side, 1 << bits)
    lo = np.clip(c - side // 2, 0, (1 << bits) - side)
    hi = lo + side - 1
    out = np.empty((nb, 2, dim), dtype=np.uint32)
    out[:, 0, :] = lo
    out[:, 1, :] = hi
    return out


def sample_rows(n_total: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct row indices in [0, n_total), ascending (seeded)."""
    count = min(count, n_total)
    if count == 0:
        return np.zeros(0, dtype=np.int64)
    r = draws(stream_key(seed, P_AUX), 0, n_total)
    return np.sort(np.argpartition(r, count - 1)[:count]) if count < n_total else np.arange(n_total)


# ---------------------------------------------------------- request streams

def log_uniform_ints(key: np.uint64, start: int, count: int, lo: float, hi: float) -> np.ndarray:
    """`count` integers floor(10^(log10 lo + u (log10 hi - log10 lo))), >= 1."""
    u = unit(draws(key, start, count))
    return np.maximum(1, np.floor(10 ** (np.log10(lo) + u * (np.log10(hi) - np.log10(lo))))).astype(np.int64)


def request_stream(n_requests: int, n0: int, dim: int, bits: int, seed: int, rate_per_s: float,
                   mix=(0.4, 0.2, 0.3, 0.1), upd_size=(1e3, 1e6), knn_size=(1, 1e5), range_size=(1, 1e4),
                   dist: str = "uniform"):
    """A Poisson stream of mixed requests against an index built from `n0`
    points with ids 0..n0-1.

    Returns a list of dicts with keys kind ('insert'|'delete'|'knn'|'range'),
    arrival (seconds), and the payload: points (insert), ids (delete), queries
    (knn) or boxes (range). Delete requests name ids that are live when the
    request arrives, given that every earlier insert took the next ids in
    arrival order. Only bookkeeping here: no index arithmetic.
    """
    key = stream_key(seed, P_AUX + 10)
    gaps = -np.log1p(-unit(draws(key, 0, n_requests))) / rate_per_s
    arrivals = np.cumsum(gaps)
    kinds_u = unit(draws(key, n_requests, n_requests))
    edges = np.cumsum(mix)
    kinds = np.searchsorted(edges, kinds_u * edges[-1], side="right")
    sizes_upd = log_uniform_ints(key, 2 * n_requests, n_requests, *upd_size)
    sizes_knn = log_uniform_ints(key, 3 * n_requests, n_requests, *knn_size)
    sizes_rng = log_uniform_ints(key, 4 * n_requests, n_requests, *range_size)
    is_ins = kinds == 0
    cap = n0 + int(sizes_upd[is_ins].sum())
    live = np.zeros(cap, dtype=bool)
    live[:n0] = True
    n_live = n0
    next_id = n0
    out = []
    for r in range(n_requests):
        kind = ("insert", "delete", "knn", "range")[min(int(kinds[r]), 3)]
        req = {"kind": kind, "arrival": float(arrivals[r])}
        s = seed * 100_003 + r
        if kind == "insert":
            m = int(sizes_upd[r])
            req["points"] = points(dist, m, dim, bits, s, P_INSERT)
            live[next_id:next_id + m] = True
            next_id += m
            n_live += m
        elif kind == "delete":
            # uniform draws over [0, next_id), keeping live ids at their first
            # occurrence (rejection sampling; the live fraction stays high)
            want = min(int(sizes_upd[r]), n_live)
            dkey = stream_key(s, P_DELETE)
            got = np.zeros(0, dtype=np.int64)
            pos = 0
            while got.size < want:
                cnt = max(2 * (want - got.size), 64)
                cand = _bounded(draws(dkey, pos, cnt), next_id).astype(np.int64)
                pos += cnt
                cand = cand[live[cand]]
                allc = np.concatenate([got, cand])
                _, first = np.unique(allc, return_index=True)
                got = allc[np.sort(first)]
            ids = got[:want].astype(np.uint32)
            live[ids] = False
            n_live -= want
            req["ids"] = ids
        elif kind == "knn":
            req["queries"] = points(dist, int(sizes_knn[r]), dim, bits, s, P_QUERY)
            req["k"] = 10
        else:
            c = points(dist, int(sizes_rng[r]), dim, bits, s, P_QUERY)
            req["boxes"] = boxes(c, bits, s)
        out.append(req)
    return out
