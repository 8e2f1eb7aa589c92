"""Seeded synthetic workloads for BatMap pair-support counting.

This module only draws random inputs: tidlists (the vertical format of
Sec. I, "Set representations"), transactions (the horizontal format), the
three hash permutations pi_t that the layout of Sec. III-A asks for, batches
of instances and query streams.  It holds none of the method's arithmetic;
both the oracle and the HIP path consume what it produces.

Every item/transaction incidence is an independent Bernoulli draw, the
instance model of Sec. IV-A ("including each of the n distinct items with
probability p").  Per-item probabilities are either constant (Bernoulli
workloads) or a capped Zipf law over item ranks.  Tidlists are sampled per
item by geometric gaps, which is exactly a Bernoulli(p) process over the
transaction ids 0..m-1 and costs O(|S_i|) per item.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GEN_VERSION = 1


def _bernoulli_positions(rng: np.random.Generator, m: int, p: float) -> np.ndarray:
    """Sorted positions in [0, m) of an i.i.d. Bernoulli(p) process."""
    if m <= 0 or p <= 0.0:
        return np.zeros(0, dtype=np.uint32)
    if p >= 1.0:
        return np.arange(m, dtype=np.uint32)
    out = []
    last = -1
    mean = m * p
    while True:
        want = int(mean + 6.0 * math.sqrt(max(mean * (1.0 - p), 1.0)) + 64)
        gaps = rng.geometric(p, size=want).astype(np.int64)
        pos = last + np.cumsum(gaps)
        inside = pos[pos < m]
        out.append(inside)
        if inside.size < pos.size:
            break
        last = int(pos[-1])
    return np.concatenate(out).astype(np.uint32)


def sets_from_probs(m: int, probs, seed: int):
    """CSR tidlists (offsets u64[n+1], tids u32[nnz]) for per-item probabilities."""
    rng = np.random.default_rng(seed)
    lists = [_bernoulli_positions(rng, m, float(p)) for p in probs]
    sizes = np.array([a.size for a in lists], dtype=np.uint64)
    offsets = np.zeros(len(lists) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    tids = np.concatenate(lists).astype(np.uint32) if lists else np.zeros(0, np.uint32)
    return offsets, tids


def bernoulli_sets(m: int, n: int, p: float, seed: int):
    """Every item in every transaction with probability p."""
    return sets_from_probs(m, np.full(n, p), seed)


def zipf_probs(n: int, alpha: float, density: float, seed: int):
    """Capped Zipf item probabilities p_rank = min(1, c * rank^-alpha).

    c is found by bisection so that the mean probability equals `density`;
    ranks are assigned to item ids by a seeded shuffle.  Returns (probs by
    item id, c).
    """
    ranks = np.arange(1, n + 1, dtype=np.float64)
    base = ranks ** (-alpha)

    def mean_p(c):
        return np.minimum(1.0, c * base).mean()

    lo, hi = 0.0, 1.0
    while mean_p(hi) < density:
        hi *= 2.0
        if hi > 1e18:
            break
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_p(mid) < density:
            lo = mid
        else:
            hi = mid
    c = 0.5 * (lo + hi)
    p_rank = np.minimum(1.0, c * base)
    order = np.random.default_rng(seed ^ 0x5EED).permutation(n)
    probs = np.empty(n)
    probs[order] = p_rank
    return probs, c


def zipf_sets(m: int, n: int, alpha: float, density: float, seed: int):
    probs, _ = zipf_probs(n, alpha, density, seed)
    return sets_from_probs(m, probs, seed)


def sets_to_transactions(m: int, offsets, tids):
    """Horizontal form of the same incidences: CSR over transactions (items per row, ascending)."""
    offsets = np.asarray(offsets, dtype=np.uint64)
    tids = np.asarray(tids, dtype=np.uint32)
    n = offsets.size - 1
    sizes = np.diff(offsets).astype(np.int64)
    items = np.repeat(np.arange(n, dtype=np.uint32), sizes)
    order = np.argsort(tids, kind="stable")
    t_sorted = tids[order]
    rows = np.zeros(m + 1, dtype=np.uint64)
    np.cumsum(np.bincount(t_sorted, minlength=m).astype(np.uint64), out=rows[1:])
    return rows, items[order].astype(np.uint32)


def hash_permutations(m: int, seed: int):
    """Three independent uniformly random permutations of [0, m) (the pi_t of Sec. III-A)."""
    rng = np.random.default_rng([seed, 0x9E37])
    return [rng.permutation(m).astype(np.uint32) for _ in range(3)]


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the instance families the method is meant
# for: Bernoulli instances (Sec. IV-A), skewed Zipf item popularity, many
# uneven instances, a dense crossover sweep and a serving query stream.
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    kind: str          # "bernoulli" | "zipf"
    density: float
    alpha: float = 0.0
    seed: int = 0
    sigma: int = 0
    note: str = ""

    def sets(self):
        if self.kind == "bernoulli":
            return bernoulli_sets(self.m, self.n, self.density, self.seed)
        return zipf_sets(self.m, self.n, self.alpha, self.density, self.seed)

    def describe(self):
        d = dataclasses.asdict(self)
        d["gen_version"] = GEN_VERSION
        return d


TINY = Workload("tiny-bernoulli", m=10_000, n=200, kind="bernoulli", density=0.02, seed=1, sigma=50,
                note="all 19,900 pair supports; sigma=50")
LARGE = Workload("large-zipf", m=1_000_000, n=2_000, kind="zipf", alpha=1.0, density=0.02, seed=2,
                 sigma=1_000, note="capped Zipf(1.0) item popularity at 2% mean density")
PAPER_REPLICA = Workload("paper-replica", m=50_000, n=4_000, kind="bernoulli", density=0.05, seed=0,
                         note="n=4000, 1e7 incidences, p=5% (Sec. IV-A, throughput computation)")
DENSE = Workload("dense-crossover", m=1_048_576, n=8_192, kind="bernoulli", density=0.05, seed=4003)
SERVING = Workload("serving-resident", m=4_000_000, n=16_384, kind="zipf", alpha=1.1, density=0.01, seed=5)

DENSE_SWEEP = [0.0001, 0.0002, 0.0005, 0.001, 0.002, 0.005, 0.01, 0.02, 0.05, 0.10, 0.20]


def batch_instances(count: int = 64, seed: int = 3000, m_lo: float = 1e4, m_hi: float = 1e6,
                    n_lo: int = 100, n_hi: int = 4_000, d_lo: float = 0.01, d_hi: float = 0.10):
    """Uneven instances: m log-uniform, n uniform, density uniform; per-instance seeds."""
    out = []
    for q in range(count):
        rng = np.random.default_rng(seed + q)
        m = int(round(10 ** rng.uniform(math.log10(m_lo), math.log10(m_hi))))
        n = int(rng.integers(n_lo, n_hi + 1))
        d = float(rng.uniform(d_lo, d_hi))
        out.append(Workload(f"batch-{q}", m=m, n=n, kind="bernoulli", density=d, seed=seed + q))
    return out


def query_stream(n_items: int, count: int, seed: int, k_lo: int = 16, k_hi: int = 4_096,
                 rate_per_s: float = 100.0):
    """Poisson arrivals of subset queries; k log-uniform in [k_lo, k_hi], items distinct."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps)
    qs = []
    for a in arrivals:
        k = int(round(math.exp(rng.uniform(math.log(k_lo), math.log(k_hi)))))
        k = max(2, min(k, n_items))
        items = rng.choice(n_items, size=k, replace=False).astype(np.uint32)
        qs.append((float(a), items))
    return qs


def bernoulli_sets_device(m: int, n: int, p: float, seed: int, device="cuda:0", chunk_bytes: int = 1 << 30):
    """Bernoulli(p) tidlists drawn on the GPU with torch's seeded generator (for instances too large
    to draw on the host).  Returns (offsets int64[n+1], tids int32[nnz]) on `device`, sorted per item.
    Same model as bernoulli_sets; a different random stream."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    rows_per_chunk = max(1, chunk_bytes // (4 * max(m, 1)))
    sizes, parts = [], []
    for i0 in range(0, n, rows_per_chunk):
        i1 = min(n, i0 + rows_per_chunk)
        hit = torch.rand((i1 - i0, m), generator=g, device=device) < p
        sizes.append(hit.sum(dim=1))
        parts.append(torch.nonzero(hit, as_tuple=True)[1].to(torch.int32))   # row-major: sorted per item
        del hit
    sizes = torch.cat(sizes)
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(sizes, 0)
    tids = torch.cat(parts) if parts else torch.zeros(0, dtype=torch.int32, device=device)
    return offsets, tids
