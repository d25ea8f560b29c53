"""Failure handling and concurrency on the GPU, forced from the host.

A stage made to fail by the test hook (BVS_TEST_FAIL=<stage>) returns
BVS_EDEVICE without launching it; the index stays valid, and the next call
returns the same results as before.  Two host threads searching on two
streams with their own workspaces get the results of one call each
(determinism as a race detector)."""
import os
import threading

import numpy as np
import pytest
import torch

from tests.gpu_util import build_case, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    print("[failure] workload", flush=True)
    return build_case(2000, 5, 40, 128, 30, 1024, 8, 32, 200, 12)


@pytest.mark.parametrize("stage", ["encode", "filter", "rerank", "topk"])
def test_forced_stage_failure_leaves_index_usable(case, stage):
    from paper_2412_03301_amd import bvs
    ix = case.ix_gpu
    ref = [to_np(t) for t in ix.search(case.q, case.q_off, 10)]
    os.environ["BVS_TEST_FAIL"] = stage
    try:
        with pytest.raises(bvs.BvsError) as e:
            ix.search(case.q, case.q_off, 10)
        assert e.value.status == bvs.BVS_EDEVICE
    finally:
        del os.environ["BVS_TEST_FAIL"]
    torch.cuda.synchronize()
    again = [to_np(t) for t in ix.search(case.q, case.q_off, 10)]
    for x, y in zip(ref, again):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


def test_two_streams_two_threads(case):
    ix = case.ix_gpu
    ref = [to_np(t) for t in ix.search(case.q, case.q_off, 10)]
    n_q = len(case.q_off) - 1
    NQ = int(case.q_off[-1])
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [ix.search_workspace(n_q, NQ) for _ in streams]
    outs = [ix._outs(n_q, 10) for _ in streams]
    errors = []

    def run(i):
        try:
            torch.cuda.set_device(case.q.device)
            for _ in range(20):
                ix.search(case.q, case.q_off, 10, ws=wss[i], out=outs[i], stream=streams[i])
        except Exception as ex:   # surfaced below
            errors.append(ex)

    th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for out in outs:
        for x, y in zip(ref, (to_np(t) for t in out)):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
