"""stdecomp_predict_noalloc (the entry point that allocates nothing) against
stdecomp_predict, through the C ABI: the same kernels, so the same values bit
for bit, on two calls in a row (the second smaller, so stale scratch contents
from the first would show), with host and with device buffers, for models of
two orders sharing the device's scratch array; and a request larger than the
array is refused with STD_E_INVAL."""
import numpy as np
import pytest

from paper_2012_03550_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_03550_amd import binding
    binding.load()
    return binding


def _queries(rng, dims, q):
    return np.stack([rng.integers(0, I, q) for I in dims]).astype(np.int32)


@pytest.mark.parametrize("dims,ranks", [((300, 200, 100), (4, 4, 4)), ((40, 30, 20, 10), (3, 4, 2, 5))])
def test_predict_noalloc_matches_predict(lib, dims, ranks):
    import torch
    rng = np.random.default_rng(17)
    idx, vals = synth.random_tiny(len(dims), dims, ranks, 4000, seed=18)
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=256, seed_sample=19, seed_init=20, chunk=32)
    h.epoch(1)
    for q in (70001, 1234):  # the second call is smaller
        say("noalloc", dims, "q", q)
        qi = _queries(rng, dims, q)
        want = h.predict(qi)
        got = h.predict_noalloc(qi)
        np.testing.assert_array_equal(got, want)
        qd = torch.from_numpy(qi).cuda()
        got_d = h.predict_noalloc(qd)
        np.testing.assert_array_equal(got_d.cpu().numpy(), want)
        np.testing.assert_array_equal(h.predict(qd).cpu().numpy(), want)
    # a bad index is refused before anything is written
    bad = _queries(rng, dims, 10)
    bad[0, 3] = dims[0]
    with pytest.raises(lib.StdecompError) as ei:
        h.predict_noalloc(bad)
    assert ei.value.code == lib.STD_E_INVAL
    h.close()


def test_predict_noalloc_refuses_oversize(lib):
    import torch
    dims, ranks = (50, 40, 30), (2, 2, 2)
    idx, vals = synth.random_tiny(3, dims, ranks, 1000, seed=21)
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=64)
    R, N = 4, 3
    scratch = 16 << 20
    pad = lambda x: (x + 255) // 256 * 256  # noqa: E731
    q_dev = scratch // (4 * R)
    assert pad(4 * q_dev * R) <= scratch
    rng = np.random.default_rng(22)
    qi = torch.from_numpy(_queries(rng, dims, q_dev + 1)).cuda()
    out = torch.full((q_dev + 1,), -7.0, device="cuda")
    with pytest.raises(lib.StdecompError) as ei:
        h.predict_noalloc(qi, out)
    assert ei.value.code == lib.STD_E_INVAL
    assert bool(torch.all(out == -7.0))  # nothing written
    got = h.predict_noalloc(qi[:, :q_dev].contiguous())  # the largest accepted request
    np.testing.assert_array_equal(got.cpu().numpy(), h.predict(qi[:, :q_dev].cpu().numpy()))
    h.close()
