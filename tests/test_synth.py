"""The input generator: redrawing single sets reproduces the database."""
import numpy as np

from paper_2412_03301_amd import synth


def test_redraw_sets_matches_database():
    db = synth.make_database(20000, 5, 30, 16, 10, seed=3)
    ids = [0, 8191, 8192, 19999, 12345]
    r = synth.redraw_sets(20000, 5, 30, 16, 10, ids, seed=3)
    for j in ids:
        assert np.array_equal(r[j], db.vectors[db.offsets[j]:db.offsets[j + 1]].numpy())


def test_fixed_query_sizes():
    q, off = synth.make_fresh_queries(4, 256, 8, 3, db_seed=0, seed=1, sizes=[1, 256, 7, 16])
    assert np.diff(off).tolist() == [1, 256, 7, 16] and q.shape == (280, 8)
