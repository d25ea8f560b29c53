"""Literal list-and-heap forms of the first and second filter.

These follow the data structures the paper names, step by step, and are
used only to cross-check the dense forms in `oracle.filter`:

  Def. 9 / Alg. 4  one list per position i of (set j, C^(j)[i]) pairs,
                   sorted by descending count
  Alg. 6           walk the lists of the positions in P and keep sets
                   whose count is at least M (first layer), then push
                   (Hamming distance, id) pairs through a max-heap of
                   capacity T that is replaced only on a strictly smaller
                   distance (second layer)
"""
from __future__ import annotations

import heapq

import numpy as np


def build_inverted_index(C: np.ndarray):
    n, L = C.shape
    lists = []
    for i in range(L):
        entries = [(j, int(C[j, i])) for j in range(n)]
        entries.sort(key=lambda e: -e[1])
        lists.append(entries)
    return lists


def first_filter_lists(lists, P, M: int) -> set:
    F1 = set()
    for p in P:
        for j, c in lists[int(p)]:
            if c >= M:
                F1.add(j)
    return F1


def second_filter_heap(F1_in_order, S_Q: np.ndarray, B: np.ndarray, T: int):
    """Max-heap on (d, i) kept with heapq over negated pairs."""
    heap: list[tuple[int, int]] = []
    for i in F1_in_order:
        d = int(np.count_nonzero(B[i] != S_Q))
        if len(heap) < T:
            heapq.heappush(heap, (-d, -i))
        elif d < -heap[0][0]:
            heapq.heappop(heap)
            heapq.heappush(heap, (-d, -i))
    return sorted((-nd, -ni) for nd, ni in heap)
