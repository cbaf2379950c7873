"""Chain geometry picked by measurement: for a model shape, time the first
minibatches of epoch 0 with each candidate chunk (entries per workgroup and
sub-step; the workgroup count follows) on throwaway handles and keep the
fastest.  Results are cached per (order, ranks, minibatch size, dtype)."""
from . import binding

_cache = {}


def tune_chunk(dims, ranks, idx, vals, batch, dtype="f32", candidates=(32, 64, 128, 256), minibatches=48):
    """Returns (best chunk, {chunk: seconds per minibatch}).  Candidates that
    do not fit (LDS, or more workgroups than compute units) are skipped."""
    key = (len(dims), tuple(int(r) for r in ranks), int(batch), dtype)
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
