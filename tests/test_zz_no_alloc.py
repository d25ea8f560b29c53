"""bvs_search_noalloc (the search on the library's fixed device scratch, for
callers that cannot allocate) against bvs_search on the same queries: two
calls in a row, the second on a smaller batch, each equal to bvs_search
bit for bit (ids, distances, counts)."""
import numpy as np
import pytest
import torch

from paper_2412_03301_amd import synth

pytestmark = pytest.mark.gpu


def _subset(q, q_off, n):
    off = np.asarray(q_off[:n + 1], dtype=np.uint64)
    return q[:int(off[-1])].contiguous(), off


def test_noalloc_matches_search_twice():
    from paper_2412_03301_amd import bvs
    assert torch.cuda.is_available()
    db = synth.make_database(3000, 5, 60, 128, n_topics=30, seed=11)
    p = bvs.Params.make(dim=128, code_bits=1024, fan_in=8, wta_k=32, access_lists=3, min_count=1,
                        top_t=200, seed=11)
    ix = bvs.Index(p, db.vectors.cuda(), db.offsets)
    q, q_off, _ = synth.make_subset_queries(db, 24, seed=12)
    q = q.cuda().contiguous()
    assert bvs.lib().bvs_search_noalloc_max_bytes() == 64 << 20
    for n in (24, 7):   # the second call is smaller: leftovers of the first must not leak into it
        qs, off = _subset(q, q_off, n)
        ids_a, dist_a, cnt_a = ix.search(qs, off, 10)
        ids_b, dist_b, cnt_b = ix.search_noalloc(qs, off, 10)
        torch.cuda.synchronize()
        assert torch.equal(cnt_a, cnt_b)
        assert torch.equal(ids_a, ids_b)
        assert torch.equal(dist_a.view(torch.int32), dist_b.view(torch.int32))
        assert int(cnt_b.min()) == 10


def test_noalloc_rejects_batches_beyond_the_scratch():
    from paper_2412_03301_amd import bvs
    db = synth.make_database(300, 3, 20, 64, n_topics=8, seed=3)
    p = bvs.Params.make(dim=64, code_bits=512, fan_in=4, wta_k=16, top_t=60, seed=3)
    ix = bvs.Index(p, db.vectors.cuda(), db.offsets)
    # 40,000 one-vector queries need a workspace above 64 MiB
    n_q = 40000
    need = bvs._bytes(bvs.lib().bvs_search_workspace_bytes, ix._h, n_q, n_q)
    assert need > 64 << 20
    q = db.vectors[:1].repeat(n_q, 1).cuda().contiguous()
    off = np.arange(n_q + 1, dtype=np.uint64)
    with pytest.raises(bvs.BvsError) as e:
        ix.search_noalloc(q, off, 10)
    assert e.value.status == bvs.BVS_ENOSPC
