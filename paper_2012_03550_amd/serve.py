"""A continuous-batching host loop for many SGD_Tucker jobs and prediction
queries on one GPU.

Jobs (a tensor to decompose for a number of epochs) wait in arrival order and
are admitted while their estimated device footprint fits the budget and their
chain workgroups fit the device.  Every round advances each admitted job by
one epoch: jobs whose kernels match (equal ranks 4, 8 or 16, the same class of
order and dtype) share one batched launch (``binding.epoch_batched``), so a
job admitted while others train runs beside them on the device.  A job that
has run its epochs is retired and its memory freed, which admits the next.
Prediction queries are answered between rounds, batched per resident model.
Each job's result is the same as when it runs alone (the batched launch is
bit-identical to separate epochs).
"""
import numpy as np

from . import binding


class Job:
    def __init__(self, jid, arrival, dims, ranks, idx, vals, epochs, batch=1024, seed=0):
        self.jid = jid
        self.arrival = arrival
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(r) for r in ranks)
        self.idx = idx
        self.vals = vals
        self.epochs = epochs
        self.batch = batch
        self.seed = seed
        self.handle = None
        self.done_epochs = 0
        self.admitted = None
        self.finished = None

    def footprint(self, dtype):
        """Device bytes the handle will hold (COO copies, schedule, factors,
        core; an over-estimate)."""
        T, N = self.idx.shape[1], len(self.dims)
        rows = sum(I * ((J + 3) // 4 * 4) for I, J in zip(self.dims, self.ranks))
        return T * (12 * (N + 1) + 4 * (N + 1) + 2 * N + 8) + rows * (6 if dtype == "bf16" else 4) + (4 << 20)

    def key(self, dtype):
        """Jobs with the same key share a batched launch."""
        r = self.ranks
        if len(set(r)) == 1 and r[0] in (4, 8, 16):
            return (r[0], len(r) == 3, dtype)
        return ("alone", self.jid)


class Server:
    def __init__(self, hbm_budget, max_workgroups=256, chunk=128, dtype="f32", lr=0.01, lam=0.01, on_finish=None,
                 on_epoch=None):
        self.budget = hbm_budget
        self.on_finish = on_finish  # called with a finished job while its handle is still open
        self.on_epoch = on_epoch    # called with a job after each of its epochs (handle open)
        self.max_wgs = max_workgroups
        self.chunk = chunk
        self.dtype = dtype
        self.lr, self.lam = lr, lam
        self.pending = []
        self.active = []
        self.done = []
        self.used = 0
        self.updates = 0

    def submit(self, job):
        self.pending.append(job)

    def admit(self, now):
        while self.pending:
            job = self.pending[0]
            need = job.footprint(self.dtype)
            if self.active and self.used + need > self.budget:
                break
            job.handle = binding.Stdecomp(job.dims, job.ranks, job.idx, job.vals, batch=job.batch,
                                          lr_factor=self.lr, lr_core=self.lr, lam_factor=self.lam,
                                          lam_core=self.lam, seed_sample=job.seed, seed_init=job.seed + 1,
                                          chunk=self.chunk, dtype=self.dtype)
            job.admitted = now
            job.need = need
            self.used += need
            self.active.append(job)
            self.pending.pop(0)

    def round(self, clock, between=None):
        """One epoch of every admitted job; retires the jobs that finish.
        ``between()`` (if given) runs after each batched launch, so queries
        need not wait for the whole round."""
        groups = {}
        for job in self.active:
            groups.setdefault(job.key(self.dtype), []).append(job)
        for jobs in groups.values():
            batch, wgs = [], 0
            for job in jobs + [None]:
                w = job.handle.info()["workgroups"] if job is not None else 0
                if job is None or (batch and wgs + w > self.max_wgs):
                    if batch:
                        binding.epoch_batched([j.handle for j in batch], 1)
                        for j in batch:
                            j.done_epochs += 1
                            self.updates += j.idx.shape[1]
                            if self.on_epoch is not None:
                                self.on_epoch(j)
                        if between is not None:
                            between()
                    batch, wgs = [], 0
                if job is not None:
                    batch.append(job)
                    wgs += w
        now = clock()
        for job in list(self.active):
            if job.done_epochs >= job.epochs:
                job.finished = now
                job.rmse = job.handle.loss()["rmse"]
                if self.on_finish is not None:
                    self.on_finish(job)
                job.handle.close()
                job.handle = None
                self.used -= job.need
                self.active.remove(job)
                self.done.append(job)

    def answer(self, n, rng):
        """n queries, each a random index tuple of a uniformly chosen admitted
        model, answered in one predict call per model.  Returns the number
        answered (0 if no model is resident)."""
        if n <= 0 or not self.active:
            return 0
        target = rng.integers(0, len(self.active), size=n)
        for k, job in enumerate(self.active):
            q = int(np.sum(target == k))
            if q == 0:
                continue
            idx = np.stack([rng.integers(0, I, q) for I in job.dims]).astype(np.int32)
            job.handle.predict(idx)
        return n
