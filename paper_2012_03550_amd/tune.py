"""Chain geometry picked by measurement.

tune_chunk: for one model shape, time the first minibatches of epoch 0 with
each candidate chunk (entries per workgroup and sub-step; the workgroup
count follows) on throwaway handles and keep the fastest.

tune_batch: for a batch of models trained together by the batched launch
(every chain must have the same workgroup count, so one chunk serves the
whole batch), time one batched epoch of every model with each candidate
chunk and keep the one with the most nonzero-updates per second.

Results are cached per shape: order, ranks, mode sizes, entry count, the
share of the most frequent row of each mode (the skew sets the run structure
the chain works through), minibatch size and dtype."""
import numpy as np

from . import binding

_cache = {}


def _signature(dims, ranks, idx):
    idx = np.asarray(idx)
    top = []
    for n in range(len(dims)):
        counts = np.bincount(np.asarray(idx[n], np.int64), minlength=1) if idx.shape[1] else np.zeros(1)
        top.append(round(float(counts.max()) / max(1, idx.shape[1]), 2))
    return (len(dims), tuple(int(r) for r in ranks), tuple(int(d) for d in dims), int(idx.shape[1]), tuple(top))


def tune_chunk(dims, ranks, idx, vals, batch, dtype="f32", candidates=(32, 64, 128, 256), minibatches=48):
    """Returns (best chunk, {chunk: seconds per minibatch}).  Candidates that
    do not fit (LDS, or more workgroups than compute units) are skipped."""
    key = ("one", _signature(dims, ranks, idx), int(batch), dtype)
    if key in _cache:
        return _cache[key]
    times = {}
    for c in candidates:
        if c > batch and times:
            continue
        try:
            h = binding.Stdecomp(dims, ranks, idx, vals, batch=batch, seed_sample=1, seed_init=2, chunk=c, dtype=dtype)
        except binding.StdecompError:
            continue
        try:
            nb = h.info()["minibatches"]
            k = min(minibatches, nb)
            h.run_minibatches(0, 0, min(2, k))  # first launch (code load, schedule)
            st = h.run_minibatches(0, 0, k)
            times[c] = st["chain_seconds"] / k
        finally:
            h.close()
    if not times:
        raise RuntimeError("no candidate chunk fits this model")
    best = min(times, key=times.get)
    _cache[key] = (best, times)
    return best, times


def tune_batch(models, batch, dtype="f32", candidates=(64, 128, 256), lr=0.01, lam=0.01):
    """models: list of (dims, ranks, idx, vals), all trained with minibatch
    `batch`.  Returns (best chunk, {chunk: nonzero-updates per second of one
    batched epoch}).  A candidate some model cannot take (LDS, workgroups) is
    skipped; the epochs run on throwaway handles from their own
    initialisation, so the caller's models are not touched."""
    key = ("batch", tuple(sorted(_signature(d, r, i) for d, r, i, _ in models)), int(batch), dtype)
    if key in _cache:
        return _cache[key]
    rates = {}
    for c in candidates:
        if c > batch:
            continue
        hs = []
        try:
            for d, r, i, v in models:
                hs.append(binding.Stdecomp(d, r, i, v, batch=batch, lr_factor=lr, lr_core=lr, lam_factor=lam,
                                           lam_core=lam, seed_sample=1, seed_init=2, chunk=c, dtype=dtype))
        except binding.StdecompError:
            for h in hs:
                h.close()
            continue
        try:
            binding.step_batched(hs, 2)  # first launch (code load, schedule)
            for h in hs:
                h.set_epoch(1)
            st = binding.epoch_batched(hs, 1)
            rates[c] = sum(s["updates"] for s in st) / max(st[0]["chain_seconds"], 1e-12)
        finally:
            for h in hs:
                h.close()
    if not rates:
        raise RuntimeError("no candidate chunk fits every model of the batch")
    best = max(rates, key=rates.get)
    _cache[key] = (best, rates)
    return best, rates
