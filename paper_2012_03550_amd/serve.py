"""A continuous-batching loop for many SGD_Tucker jobs and prediction
queries on one GPU.

Jobs (a tensor to decompose for a number of epochs) wait in arrival order and
are admitted while their estimated device footprint fits the budget; a job
whose model the library cannot hold (its core and tables exceed one
workgroup's LDS) is rejected with the library's reason.  Every round advances
each admitted job by a window of minibatches of its current epoch: jobs with
the same chain workgroup count, class of order and dtype (any ranks) share
one batched launch (``binding.step_batched``), whose chains the library
spreads over slots of the device, so a job admitted while others train joins
them at the next window.  A job that
has run its epochs is retired and its memory freed, which admits the next.

Prediction queries go to the models resident at the time, on each handle's
query stream through the entry point that allocates nothing: ``run`` trains in a
background thread while ``answer`` serves queries from the caller's thread,
so queries run on the device beside the training launches instead of waiting
for them.  Each job's result is the same
as when it runs alone (the batched launch runs each chain exactly as alone,
and predictions write nothing the training reads).
"""
import threading
import time

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
        self.qlock = threading.Lock()  # held while a query uses the handle, and to close it
        self.done_epochs = 0
        self.admitted = None
        self.finished = None
        self.rejected = None
        self.need = 0
        self.workgroups = 0

    def footprint(self, dtype):
        """Device bytes the handle will hold (COO copies, schedule, factors,
        core; an over-estimate)."""
        T, N = self.idx.shape[1], len(self.dims)
        rows = sum(I * ((J + 3) // 4 * 4) for I, J in zip(self.dims, self.ranks))
        return T * (12 * (N + 1) + 4 * (N + 1) + 2 * N + 8) + rows * (6 if dtype == "bf16" else 4) + (4 << 20)

    def key(self, dtype):
        """Jobs with the same key share a batched launch: the same minibatch
        size and chain workgroup count, class of order (three modes or
        other) and dtype; ranks may differ."""
        return (self.batch, self.workgroups, len(self.dims) == 3, dtype)


class Server:
    def __init__(self, hbm_budget, chunk=128, dtype="f32", lr=0.01, lam=0.01, on_finish=None, on_epoch=None,
                 window=512):
        self.budget = hbm_budget
        self.window = window        # minibatches per job and round (continuous batching granularity)
        self.on_finish = on_finish  # called with a finished job while its handle is still open
        self.on_epoch = on_epoch    # called with a job after each of its epochs (handle open)
        self.chunk = chunk          # entries per chain workgroup (0: the library's automatic choice)
        self.dtype = dtype
        self.lr, self.lam = lr, lam
        self.lock = threading.Lock()  # pending / active / done / rejected lists
        self.pending = []
        self.active = []
        self.done = []
        self.rejected = []
        self.used = 0
        self.updates = 0
        self.rounds = 0

    def submit(self, job):
        with self.lock:
            self.pending.append(job)

    def admit(self, now):
        """Admit waiting jobs in arrival order while their footprint fits (a
        job is always admitted when nothing else is resident)."""
        while True:
            with self.lock:
                if not self.pending:
                    return
                job = self.pending[0]
                need = job.footprint(self.dtype)
                if self.active and self.used + need > self.budget:
                    return
                self.pending.pop(0)
            try:
                h = binding.Stdecomp(job.dims, job.ranks, job.idx, job.vals, batch=job.batch, lr_factor=self.lr,
                                     lr_core=self.lr, lam_factor=self.lam, lam_core=self.lam, seed_sample=job.seed,
                                     seed_init=job.seed + 1, chunk=self.chunk, dtype=self.dtype)
            except binding.StdecompError as e:
                job.rejected = str(e)
                with self.lock:
                    self.rejected.append(job)
                continue
            job.handle = h
            job.workgroups = h.info()["workgroups"]
            job.admitted = now
            job.need = need
            with self.lock:
                self.used += need
                self.active.append(job)

    def round(self, clock, between=None):
        """One window of every admitted job (up to ``window`` minibatches of
        its current epoch); retires the jobs that finish.  ``between()`` (if
        given) runs after each batched launch."""
        with self.lock:
            active = list(self.active)
        groups = {}
        for job in active:
            groups.setdefault(job.key(self.dtype), []).append(job)
        for batch in groups.values():
            stats = binding.step_batched([j.handle for j in batch], self.window)
            for j, st in zip(batch, stats):
                self.updates += st["updates"]
                for _ in range(st["epochs_run"]):
                    j.done_epochs += 1
                    if self.on_epoch is not None:
                        self.on_epoch(j)
            if between is not None:
                between()
        self.rounds += 1
        now = clock()
        for job in active:
            if job.done_epochs >= job.epochs:
                job.finished = now
                job.rmse = job.handle.loss()["rmse"]
                if self.on_finish is not None:
                    self.on_finish(job)
                with self.lock:
                    self.active.remove(job)
                    self.used -= job.need
                    self.done.append(job)
                with job.qlock:  # no query is using the handle
                    job.handle.close()
                    job.handle = None

    def busy(self):
        with self.lock:
            return bool(self.pending or self.active)

    def run(self, clock, stop):
        """Training loop for a background thread: admit, run rounds, retire,
        until ``stop`` is set and no job is waiting or resident."""
        while True:
            self.admit(clock())
            with self.lock:
                idle = not self.active
            if not idle:
                self.round(clock)
            elif stop.is_set() and not self.busy():
                return
            else:
                time.sleep(0.0005)

    def answer(self, n, rng):
        """n queries, each a random index tuple of a uniformly chosen resident
        model, answered in one predict call per model (on the handle's query
        stream, beside any training launch in flight).  Returns the number
        answered (0 if no model is resident; queries of a model retired
        meanwhile are not answered)."""
        if n <= 0:
            return 0
        with self.lock:
            models = list(self.active)
        if not models:
            return 0
        target = rng.integers(0, len(models), size=n)
        answered = 0
        for k, job in enumerate(models):
            q = int(np.sum(target == k))
            if q == 0:
                continue
            idx = np.stack([rng.integers(0, I, q) for I in job.dims]).astype(np.int32)
            with job.qlock:
                if job.handle is None:  # retired since the snapshot: these queries are not answered
                    continue
                # (the entry point that allocates nothing: a hipFree would wait for the training launch)
                job.handle.predict_noalloc(idx)
            answered += q
        return answered
