"""The C ABI's options beyond the SGD step itself, through the binding on a
GPU: device memory from the caller's allocator (torch's caching allocator),
out-of-memory from that allocator at every point of set-up, the training
RMSE in the epoch statistics, and the sampler writing straight into device
memory on a given stream."""
import math

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


def _model(lib, dims, ranks, idx, vals, A0, G0, **kw):
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=256, lr_factor=0.02, lr_core=0.02, lam_factor=0.01,
                     lam_core=0.01, seed_sample=91, init="caller", chunk=32, **kw)
    h.set_params(A0, G0)
    return h


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_torch_allocator_bit_identical(lib, dtype):
    """A handle whose every device buffer comes from torch's caching
    allocator trains bit for bit as one using hipMalloc, and returns every
    block it took when it is freed."""
    dims, ranks = (300, 200, 100), (4, 4, 4)
    idx, vals = synth.random_tiny(3, dims, ranks, 12000, seed=81, skew=1.2)
    A0, G0 = synth.init_params(dims, ranks, seed=82)
    say("allocator", dtype)
    h = _model(lib, dims, ranks, idx, vals, A0, G0, dtype=dtype)
    h.epoch(2)
    ref = h.get_params()
    pred_ref = h.predict(idx[:, :500])
    h.close()
    al = lib.TorchAllocator()
    h = _model(lib, dims, ranks, idx, vals, A0, G0, dtype=dtype, allocator=al)
    assert al.allocs > 10 and al.live, (al.allocs, len(al.live))
    h.epoch(2)
    got = h.get_params()
    pred = h.predict(idx[:, :500])  # temporary buffers of a call come from the allocator too
    loss = h.loss(idx[:, :500], vals[:500])
    h.close()
    say("  allocs", al.allocs, "frees", al.frees)
    assert al.frees == al.allocs and not al.live
    for a, b in zip(ref[0], got[0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ref[1], got[1])
    np.testing.assert_array_equal(pred_ref, pred)
    assert math.isfinite(loss["rmse"])


def test_allocator_failure_is_nomem_and_frees_everything(lib):
    """When the caller's allocator fails at the k-th request of set-up (every
    k up to the last), stdecomp_init returns STD_E_NOMEM and gives back every
    block it had taken; a failure inside a call (predict's temporary buffers)
    returns STD_E_NOMEM and leaves the handle usable."""
    dims, ranks = (120, 90, 60), (4, 4, 4)
    idx, vals = synth.random_tiny(3, dims, ranks, 5000, seed=83)
    A0, G0 = synth.init_params(dims, ranks, seed=84)
    probe = lib.TorchAllocator()
    h = _model(lib, dims, ranks, idx, vals, A0, G0, allocator=probe)
    n_init = probe.allocs
    h.close()
    say("set-up takes", n_init, "blocks")
    assert n_init > 5
    for k in range(n_init):
        al = lib.TorchAllocator(fail_after=k)
        with pytest.raises(lib.StdecompError) as ei:
            lib.Stdecomp(dims, ranks, idx, vals, batch=256, seed_sample=91, chunk=32, allocator=al)
        assert ei.value.code == lib.STD_E_NOMEM, (k, ei.value)
        assert al.allocs == k and al.frees == k and not al.live, (k, al.allocs, al.frees)
    al = lib.TorchAllocator()
    h = _model(lib, dims, ranks, idx, vals, A0, G0, allocator=al)
    al.fail_after = al.allocs  # the next request fails
    with pytest.raises(lib.StdecompError) as ei:
        h.predict(idx[:, :100])
    assert ei.value.code == lib.STD_E_NOMEM
    al.fail_after = None
    h.epoch(1)
    assert np.all(np.isfinite(h.predict(idx[:, :100])))
    h.close()
    assert al.frees == al.allocs and not al.live


def test_train_rmse_in_epoch_stats(lib, oracle_mod):
    """With report_train_rmse, the epoch statistics carry the RMSE over the
    training set after the epoch (the loss kernel's FP64 sums), equal to the
    oracle's RMSE of the same parameters; without it the field is NaN."""
    dims, ranks = (200, 150, 100), (5, 5, 5)
    idx, vals = synth.random_tiny(3, dims, ranks, 8000, seed=85)
    A0, G0 = synth.init_params(dims, ranks, seed=86)
    h = _model(lib, dims, ranks, idx, vals, A0, G0, train_rmse=True)
    st = h.epoch(1)
    A, G = h.get_params()
    ref = oracle_mod.Model(dims, ranks, [a.astype(np.float64) for a in A], G.astype(np.float64))
    want = ref.loss(idx, vals)["rmse"]
    say("train RMSE", st["train_rmse"], "oracle", want)
    assert abs(st["train_rmse"] - want) <= 1e-5 * want
    assert st["train_rmse"] == h.loss()["rmse"]
    h.close()
    h = _model(lib, dims, ranks, idx, vals, A0, G0)
    assert math.isnan(h.epoch(1)["train_rmse"])
    h.close()


def test_sample_order_on_device_and_stream(lib, oracle_mod):
    """The sampler writes pi_e into device memory on a given stream (no
    allocation) and into host memory; both equal the oracle's order."""
    import torch
    T, seed, epoch = 100_003, 3001, 4
    want = oracle_mod.perm(T, seed, epoch)
    s = torch.cuda.Stream()
    got_dev = lib.sample_order(T, seed, epoch, device=True, stream=s.cuda_stream)
    np.testing.assert_array_equal(got_dev.cpu().numpy(), want)
    np.testing.assert_array_equal(lib.sample_order(T, seed, epoch), want)
    np.testing.assert_array_equal(lib.sample_order(T, seed, epoch, device=True).cpu().numpy(), want)


def test_predict_while_training(lib):
    """Predictions from one thread while another trains the same handle:
    they run on the handle's query stream (through the entry point that
    allocates nothing: a hipFree would wait for the training launch), return
    finite values, several of them complete while the epochs run, and the
    training ends bit for bit where it ends with no queries."""
    import threading
    dims, ranks = (3000, 2000, 1000), (8, 8, 8)
    idx, vals = synth.random_tiny(3, dims, ranks, 400000, seed=87, skew=1.1)
    A0, G0 = synth.init_params(dims, ranks, seed=88)
    ref = _model(lib, dims, ranks, idx, vals, A0, G0)
    ref.epoch(3)
    want = ref.get_params()
    ref.close()
    h = _model(lib, dims, ranks, idx, vals, A0, G0)
    done = threading.Event()
    err = []

    def train():
        try:
            h.epoch(3)
        except Exception as e:  # reported below
            err.append(e)
        done.set()

    th = threading.Thread(target=train)
    rng = np.random.default_rng(89)
    th.start()
    calls = 0
    while not done.is_set() or calls == 0:
        q = np.stack([rng.integers(0, I, 2000) for I in dims]).astype(np.int32)
        out = h.predict_noalloc(q)
        assert np.all(np.isfinite(out))
        calls += 1
    th.join()
    assert not err, err
    say("predictions during training:", calls, "calls")
    # the predictions ran beside the training launch, not after it
    assert calls >= 3, calls
    got = h.get_params()
    for a, b in zip(want[0], got[0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(want[1], got[1])
    h.close()
