"""Shared helpers of the GPU parity tests: one seeded workload, built both by
the oracle (CPU, float64) and by the HIP library, compared element by element."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from oracle import flyhash, prng, search
from paper_2412_03301_amd import synth


@dataclass
class Case:
    params: object          # bvs.Params
    db: synth.Database
    X: np.ndarray           # float64 copy of the database
    ix_oracle: search.Index
    ix_gpu: object          # bvs.Index
    q: torch.Tensor         # queries on the GPU
    q_np: np.ndarray
    q_off: np.ndarray

    def query(self, i):
        return self.q_np[self.q_off[i]:self.q_off[i + 1]]


def build_case(n_sets, size_lo, size_hi, dim, n_topics, code_bits, fan_in, wta_k, top_t,
               n_queries, A=3, M=1, seed=0, queries="subset"):
    from paper_2412_03301_amd import bvs
    db = synth.make_database(n_sets, size_lo, size_hi, dim, n_topics, seed=seed)
    X = db.vectors.numpy().astype(np.float64)
    p = bvs.Params.make(dim=dim, code_bits=code_bits, fan_in=fan_in, wta_k=wta_k, access_lists=A,
                        min_count=M, top_t=top_t, seed=seed)
    idx = prng.projection_rows(seed, dim, code_bits, fan_in)
    ix_o = search.build_index(X, db.offsets, idx, wta_k)
    ix_g = bvs.Index(p, db.vectors.cuda(), db.offsets)
    if queries == "subset":
        q, q_off, _ = synth.make_subset_queries(db, n_queries, seed=seed + 1)
    elif isinstance(queries, (list, tuple)):
        q, q_off = synth.make_fresh_queries(n_queries, max(queries), dim, n_topics, db_seed=seed, seed=seed + 1,
                                            sizes=queries)
    else:
        q, q_off = synth.make_fresh_queries(n_queries, queries, dim, n_topics, db_seed=seed, seed=seed + 1)
    q_np = q.numpy().astype(np.float64)
    return Case(p, db, X, ix_o, ix_g, q.cuda().contiguous(), q_np, q_off)


def oracle_query_codes(case: Case, i: int):
    return flyhash.codes(case.query(i), case.ix_oracle.idx, case.ix_oracle.wta_k)


def to_np(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()
