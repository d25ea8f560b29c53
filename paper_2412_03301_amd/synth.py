"""Seeded synthetic vector-set workloads.

This module draws inputs only: it holds none of the search method's
arithmetic, and both the HIP path and the CPU oracle take its output as
plain arrays.  The recipe stands in for the paper's text and image
collections (Sec. 6.1.1): each database set belongs to one of a fixed
number of topics, every set has its own entity centre drawn around its
topic, and members scatter around the entity.

Recipe (all normal draws are standard normal per component):
  topic centre   t  ~ N(0, I_d)
  entity centre  e  = t + 0.5 * g
  member vector  v  = grid(normalise(e + 0.2 * g))
  grid(x)           = round-half-even(4096 * x) / 4096, stored as float32
Query sets (a database set with part of it dropped and a little noise):
  pick distinct source sets uniformly, keep m - floor(0.3 m) members
  (at least one) uniformly without replacement, and emit
  q = grid(normalise(v + (0.05 / sqrt(d)) * g)) for each kept member.
Fresh-entity queries (sizes log-uniform, used for uneven batches):
  m_q = floor(exp(U[0, ln(max+1)))) clipped to [1, max]; members are drawn
  around a new entity of a random topic exactly like database members.

Randomness is split into independent torch generators whose seeds come
from numpy's SeedSequence, and database sets are drawn in fixed chunks of
``CHUNK_SETS`` sets with one generator per chunk, so a chunk's content
does not depend on how many other chunks are drawn.  The same seed on
the same device type gives the same data; CPU and GPU streams differ.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

GRID = 4096.0
CHUNK_SETS = 8192


def _seed(seed: int, *path: int) -> int:
    ss = np.random.SeedSequence([int(seed), *[int(p) for p in path]])
    return int(ss.generate_state(1, dtype=np.uint64)[0] & ((1 << 63) - 1))


def _gen(device, seed: int, *path: int) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(_seed(seed, *path))
    return g


def to_grid(x: torch.Tensor) -> torch.Tensor:
    """Round to the 2^-12 grid (half to even) after L2-normalising rows."""
    x = x / torch.linalg.vector_norm(x, dim=-1, keepdim=True).clamp_min(1e-30)
    return torch.round(x * GRID) / GRID


@dataclass
class Database:
    vectors: torch.Tensor      # float32 [N, d], rows on the 2^-12 grid
    offsets: np.ndarray        # int64 [n + 1], offsets[0] = 0
    topic: np.ndarray          # int64 [n], topic of each set
    entity_seed: int

    @property
    def n_sets(self) -> int:
        return len(self.offsets) - 1


def set_sizes(n_sets: int, lo: int, hi: int, seed: int) -> np.ndarray:
    g = _gen("cpu", seed, 1)
    return torch.randint(lo, hi + 1, (n_sets,), generator=g).numpy().astype(np.int64)


def make_database(n_sets: int, size_lo: int, size_hi: int, dim: int,
                  n_topics: int, seed: int = 0, device="cpu",
                  out: torch.Tensor | None = None) -> Database:
    """Draw ``n_sets`` sets with sizes uniform in [size_lo, size_hi]."""
    device = torch.device(device)
    sizes = set_sizes(n_sets, size_lo, size_hi, seed)
    offsets = np.zeros(n_sets + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    topic = torch.randint(0, n_topics, (n_sets,), generator=_gen("cpu", seed, 2)).numpy()
    centres = torch.randn(n_topics, dim, generator=_gen(device, seed, 3), device=device)
    total = int(offsets[-1])
    if out is None:
        out = torch.empty(total, dim, dtype=torch.float32, device=device)
    for c0 in range(0, n_sets, CHUNK_SETS):
        c1 = min(n_sets, c0 + CHUNK_SETS)
        out[offsets[c0]:offsets[c1]] = _draw_chunk(c0, c1, sizes, topic, centres, dim, seed, device)
    return Database(out, offsets, topic, seed)


def _draw_chunk(c0, c1, sizes, topic, centres, dim, seed, device):
    g = _gen(device, seed, 4, c0 // CHUNK_SETS)
    m = torch.from_numpy(sizes[c0:c1]).to(device)
    t = torch.from_numpy(topic[c0:c1]).to(device)
    ent = centres[t] + 0.5 * torch.randn(c1 - c0, dim, generator=g, device=device)
    owner = torch.repeat_interleave(torch.arange(c1 - c0, device=device), m)
    v = ent[owner] + 0.2 * torch.randn(owner.numel(), dim, generator=g, device=device)
    return to_grid(v)


def redraw_sets(n_sets: int, size_lo: int, size_hi: int, dim: int, n_topics: int, set_ids,
                seed: int = 0, device="cpu") -> dict:
    """The vectors of the given sets of make_database(...) with the same
    arguments and device type, drawn again chunk by chunk (float32, host)."""
    device = torch.device(device)
    sizes = set_sizes(n_sets, size_lo, size_hi, seed)
    offsets = np.zeros(n_sets + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    topic = torch.randint(0, n_topics, (n_sets,), generator=_gen("cpu", seed, 2)).numpy()
    centres = torch.randn(n_topics, dim, generator=_gen(device, seed, 3), device=device)
    out = {}
    by_chunk = {}
    for j in sorted(set(int(x) for x in set_ids)):
        by_chunk.setdefault(j // CHUNK_SETS, []).append(j)
    for ch, js in by_chunk.items():
        c0 = ch * CHUNK_SETS
        c1 = min(n_sets, c0 + CHUNK_SETS)
        v = _draw_chunk(c0, c1, sizes, topic, centres, dim, seed, device)
        for j in js:
            out[j] = v[offsets[j] - offsets[c0]:offsets[j + 1] - offsets[c0]].cpu().numpy()
    return out


def make_subset_queries(db: Database, n_queries: int, seed: int = 0,
                        drop: float = 0.3, noise: float = 0.05):
    """Queries built from distinct database sets (drop 30 %, add noise).

    Returns (vectors float32 [Nq, d] on the database's device,
    offsets int64 [n_q + 1], source set id per query)."""
    n = db.n_sets
    dim = db.vectors.shape[1]
    device = db.vectors.device
    g = _gen("cpu", seed, 10)
    src = torch.randperm(n, generator=g)[:n_queries].numpy().astype(np.int64)
    rows = []
    for j in src:
        o0, o1 = int(db.offsets[j]), int(db.offsets[j + 1])
        m = o1 - o0
        keep = max(1, m - int(math.floor(drop * m)))
        pick = torch.randperm(m, generator=g)[:keep].numpy()
        rows.append(o0 + np.sort(pick))
    q_off = np.zeros(len(src) + 1, np.int64)
    np.cumsum([len(r) for r in rows], out=q_off[1:])
    rows_t = torch.from_numpy(np.concatenate(rows)).to(device)
    base = db.vectors[rows_t].to(torch.float32)
    gn = _gen(device, seed, 11)
    sigma = noise / math.sqrt(dim)
    q = to_grid(base + sigma * torch.randn(base.shape, generator=gn, device=device))
    return q, q_off, src


def make_fresh_queries(n_queries: int, max_size: int, dim: int, n_topics: int,
                       db_seed: int, seed: int = 0, device="cpu", sizes=None):
    """Queries around new entities, sizes log-uniform in [1, max_size]
    (or the given sizes)."""
    device = torch.device(device)
    g = _gen("cpu", seed, 20)
    u = torch.rand(n_queries, generator=g, dtype=torch.float64).numpy()
    if sizes is None:
        sizes = np.clip(np.floor(np.exp(u * math.log(max_size + 1))), 1, max_size).astype(np.int64)
    else:
        sizes = np.asarray(sizes, dtype=np.int64)
        assert sizes.shape == (n_queries,) and (sizes >= 1).all()
    topic = torch.randint(0, n_topics, (n_queries,), generator=g).numpy()
    centres = torch.randn(n_topics, dim, generator=_gen(device, db_seed, 3), device=device)
    gd = _gen(device, seed, 21)
    t = torch.from_numpy(topic).to(device)
    ent = centres[t] + 0.5 * torch.randn(n_queries, dim, generator=gd, device=device)
    owner = torch.repeat_interleave(torch.arange(n_queries, device=device),
                                    torch.from_numpy(sizes).to(device))
    v = ent[owner] + 0.2 * torch.randn(owner.numel(), dim, generator=gd, device=device)
    q_off = np.zeros(n_queries + 1, np.int64)
    np.cumsum(sizes, out=q_off[1:])
    return to_grid(v), q_off


# Workload presets: sizes and hashing parameters of the evaluated configurations.
WORKLOADS = {
    "tiny": dict(n_sets=5000, size_lo=8, size_hi=32, dim=128, n_topics=50,
                 code_bits=1024, fan_in=8, wta_k=32, n_queries=16, top_t=200, k=10),
    "scale": dict(n_sets=1_000_000, size_lo=5, size_hi=100, dim=384, n_topics=10_000,
                  code_bits=4096, fan_in=16, wta_k=64, n_queries=1024, top_t=1000, k=10),
    # the scale generator at d = 768, for the BF16 / FP8 re-rank
    "precision": dict(n_sets=1_000_000, size_lo=5, size_hi=100, dim=768, n_topics=10_000,
                      code_bits=4096, fan_in=16, wta_k=64, n_queries=1024, top_t=1000, k=10),
    # learned projection: trained on a separate 100k-set corpus (its own seed)
    # with triplets mined by brute force, evaluated on the precision database
    "learned": dict(n_sets=1_000_000, size_lo=5, size_hi=100, dim=768, n_topics=10_000,
                    code_bits=4096, fan_in=16, wta_k=64, n_queries=1024, top_t=1000, k=10,
                    hidden=1024, train_sets=100_000, train_seed=100, mine_queries=20_000, negatives=10),
    # the scale database searched by the full scan of Alg. 2, and by the
    # re-rank with other set measures
    "full": dict(n_sets=1_000_000, size_lo=5, size_hi=100, dim=384, n_topics=10_000,
                 code_bits=4096, fan_in=16, wta_k=64, n_queries=1024, top_t=1000, k=10),
    "metrics": dict(n_sets=1_000_000, size_lo=5, size_hi=100, dim=384, n_topics=10_000,
                    code_bits=4096, fan_in=16, wta_k=64, n_queries=1024, top_t=1000, k=10),
    # the parameter study: the scale database, fewer queries, many settings
    "trends": dict(n_sets=1_000_000, size_lo=5, size_hi=100, dim=384, n_topics=10_000,
                   code_bits=4096, fan_in=16, wta_k=64, n_queries=256, top_t=1000, k=10),
    # the scale database, searched by fresh-entity queries of 1-256 vectors
    "batched": dict(n_sets=1_000_000, size_lo=5, size_hi=100, dim=384, n_topics=10_000,
                    code_bits=4096, fan_in=16, wta_k=64, n_queries=4096, max_query=256, top_t=1000, k=10),
}
