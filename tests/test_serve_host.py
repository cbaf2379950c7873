"""Host-side logic of the serving loop (no GPU): which jobs share a launch,
and the footprint estimate used for admission."""
import numpy as np

from paper_2012_03550_amd import serve


def _job(dims, ranks, nnz=1000):
    idx = np.zeros((len(dims), nnz), np.int32)
    return serve.Job(0, 0.0, dims, ranks, idx, np.zeros(nnz, np.float32), epochs=1)


def test_jobs_share_a_launch_with_the_same_workgroups_order_class_and_dtype():
    a = _job((10, 20, 30), (8, 8, 8))
    b = _job((40, 50, 60), (8, 8, 8))
    c = _job((10, 20, 30, 40), (8, 8, 8, 8))
    d = _job((10, 20, 30), (4, 4, 4))
    e = _job((10, 20, 30), (5, 5, 5))
    f = _job((10, 20, 30), (4, 8, 4))
    g = _job((10, 20, 30, 40, 50), (4, 4, 4, 4, 4))
    assert a.key("f32") == b.key("f32") == d.key("f32") == e.key("f32") == f.key("f32")  # any ranks
    assert a.key("f32") != a.key("bf16")
    assert a.key("f32") != c.key("f32")  # three modes vs four
    assert c.key("f32") == g.key("f32")  # four and five modes share the general kernels
    h = serve.Job(1, 0.0, (10, 20, 30), (8, 8, 8), np.zeros((3, 10), np.int32), np.zeros(10, np.float32), epochs=1,
                  batch=512)
    assert h.key("f32") != a.key("f32")  # another minibatch size: another workgroup count


def test_footprint_grows_with_entries_and_rows():
    small = _job((100, 100, 100), (8, 8, 8), nnz=1000)
    more_entries = _job((100, 100, 100), (8, 8, 8), nnz=100000)
    more_rows = _job((100000, 100, 100), (8, 8, 8), nnz=1000)
    assert small.footprint("f32") < more_entries.footprint("f32")
    assert small.footprint("f32") < more_rows.footprint("f32")
    assert small.footprint("f32") < small.footprint("bf16")
    # at least the three COO copies of every entry
    assert more_entries.footprint("f32") >= 100000 * 16 * 3
