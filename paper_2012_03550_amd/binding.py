"""Thin ctypes binding of libstdecomp (C ABI in include/stdecomp.h).

Argument marshalling only: every step of the SGD_Tucker update runs in the
library's HIP kernels.  Host arrays are numpy; device arrays may be torch
tensors on a HIP device (their data pointers are passed with on_device=1).
The binding raises if the library has not been built -- there is no fallback.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstdecomp.so")

STD_OK, STD_E_INVAL, STD_E_NOMEM, STD_E_DEVICE, STD_E_STATE, STD_E_DIVERGED = 0, -1, -2, -3, -4, -5
DTYPES = {"f32": 0, "bf16": 1}
INITS = {"scaled": 0, "paper": 1, "caller": 2}
PLACEMENTS = {"auto": 0, "spread": 1, "one_xcc": 2}

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f32p = ctypes.POINTER(ctypes.c_float)


class Problem(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("dims", _i64p), ("ranks", _i32p), ("nnz", ctypes.c_int64),
                ("idx", ctypes.c_void_p), ("vals", ctypes.c_void_p)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int64), ("lr_factor", ctypes.c_float), ("lr_core", ctypes.c_float),
                ("lambda_factor", ctypes.c_float), ("lambda_core", ctypes.c_float),
                ("seed_sample", ctypes.c_uint64), ("seed_init", ctypes.c_uint64), ("init_kind", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("r_core", ctypes.c_int32), ("inputs_on_device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("chain_chunk", ctypes.c_int32), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_ctx", ctypes.c_void_p), ("report_train_rmse", ctypes.c_int32),
                ("momentum", ctypes.c_float), ("placement", ctypes.c_int32), ("reserved", ctypes.c_int32 * 9)]


class EpochStats(ctypes.Structure):
    _fields_ = [("epochs_run", ctypes.c_int64), ("updates", ctypes.c_int64), ("minibatches", ctypes.c_int64),
                ("device_seconds", ctypes.c_double), ("schedule_seconds", ctypes.c_double),
                ("chain_seconds", ctypes.c_double), ("chain_launches", ctypes.c_int64),
                ("bytes_alg", ctypes.c_double), ("flops_alg", ctypes.c_double), ("train_rmse", ctypes.c_double)]


class LossOut(ctypes.Structure):
    _fields_ = [("rmse", ctypes.c_double), ("mae", ctypes.c_double), ("sse", ctypes.c_double),
                ("objective", ctypes.c_double), ("count", ctypes.c_int64), ("nonfinite", ctypes.c_int64)]


class InfoOut(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_int32), ("chunk", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("lds_bytes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("minibatches", ctypes.c_int64), ("epoch", ctypes.c_int64), ("cursor", ctypes.c_int64),
                ("placement", ctypes.c_int32)]


# Every symbol the header declares, with its ctypes signature.
SIGNATURES = {
    "stdecomp_default_options": (ctypes.c_int, [ctypes.POINTER(Options)]),
    "stdecomp_init": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_void_p)]),
    "stdecomp_epoch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(EpochStats)]),
    "stdecomp_run_minibatches": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.POINTER(EpochStats)]),
    "stdecomp_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "stdecomp_predict_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_int32]),
    "stdecomp_loss": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.POINTER(LossOut)]),
    "stdecomp_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "stdecomp_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "stdecomp_set_epoch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "stdecomp_get_velocity": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "stdecomp_set_velocity": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "stdecomp_get_kruskal": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "stdecomp_set_kruskal": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "stdecomp_debug_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _i64p,
                                               _i32p, _i32p, _i32p, _i32p, _i32p]),
    "stdecomp_sample_order": (ctypes.c_int, [ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_int32, ctypes.c_void_p]),
    "stdecomp_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(InfoOut)]),
    "stdecomp_debug_barrier": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "stdecomp_debug_barrier_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "stdecomp_epoch_batched": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32,
                                              ctypes.POINTER(EpochStats)]),
    "stdecomp_step_batched": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int64,
                                             ctypes.POINTER(EpochStats)]),
    "stdecomp_free": (ctypes.c_int, [ctypes.c_void_p]),
    "stdecomp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "stdecomp_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
}

_lib = None


def load():
    """Load libstdecomp.so; raises if it was not built (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libstdecomp.so is not built: run `python -m paper_2012_03550_amd.build`")
        # torch first, so that the library binds to the HIP runtime torch has
        # loaded: two runtimes in one process do not share the device
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        # registered after torch's own exit hooks, so it runs before them
        atexit.register(_close_live_handles)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


# Handles still open.  They are released by an exit hook, before the
# interpreter tears down its modules (and with them torch's HIP runtime state),
# instead of by __del__ during that teardown in an unspecified order.
_live = weakref.WeakSet()


def _close_live_handles():
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass


class StdecompError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (load().stdecomp_strerror(code).decode(), code, msg))
        self.code = code


def _is_device(x):
    return hasattr(x, "is_cuda") and x.is_cuda


def _dev_coo(idx, vals=None):
    """Device COO in the library's layout: int32 [N][nnz] indices, float32 values."""
    import torch
    idx = idx.to(torch.int32).contiguous()
    if vals is not None:
        assert _is_device(vals) and vals.device == idx.device, "indices and values must be on the same device"
        vals = vals.to(torch.float32).contiguous()
    # the library reads them on its own stream
    torch.cuda.current_stream(idx.device).synchronize()
    return idx if vals is None else (idx, vals)


class TorchAllocator:
    """Device memory for a handle from torch's caching allocator (the
    library's dev_alloc / dev_free callbacks): blocks are taken on the
    handle's stream and returned to torch's cache when the handle frees them.
    Counts calls and failures (``fail_after``: the allocation with this
    0-based number and every later one fail, for tests of the library's
    out-of-memory path)."""

    def __init__(self, device=None, fail_after=None):
        import torch
        self.device = torch.cuda.current_device() if device is None else device
        self.fail_after = fail_after
        self.allocs = 0
        self.frees = 0
        self.failed = 0
        self.live = {}
        self._alloc = ALLOC_FN(self._alloc_cb)
        self._free = FREE_FN(self._free_cb)

    def _alloc_cb(self, ctx, nbytes, stream):
        import torch
        if self.fail_after is not None and self.allocs >= self.fail_after:
            self.failed += 1
            return None
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device, stream=int(stream or 0))
        except Exception:
            self.failed += 1
            return None
        self.allocs += 1
        self.live[p] = int(nbytes)
        return p

    def _free_cb(self, ctx, ptr, stream):
        import torch
        self.frees += 1
        self.live.pop(ptr, None)
        torch.cuda.caching_allocator_delete(ptr)


def _ptr(x):
    if _is_device(x):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(x.ctypes.data)


class Stdecomp:
    """One SGD_Tucker model on the GPU (a libstdecomp handle)."""

    def __init__(self, dims, ranks, idx, vals, batch=256, lr_factor=0.01, lr_core=0.01, lam_factor=0.01,
                 lam_core=0.01, seed_sample=0, seed_init=0, init="scaled", dtype="f32", chunk=0, stream=None,
                 allocator=None, train_rmse=False, r_core=0, momentum=0.0, placement="auto"):
        """allocator: None (the library calls hipMalloc) or a TorchAllocator
        (every device buffer of the handle from torch's caching allocator);
        train_rmse: epoch() also reports the RMSE over the training set;
        r_core: 0 for a dense core, R > 0 for the Kruskal core of rank R;
        momentum: heavy-ball factor mu in [0, 1) (0: the plain method);
        placement: "auto", "spread" or "one_xcc" (where the chain's workgroups run)."""
        L = load()
        self.N = len(dims)
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(r) for r in ranks)
        on_dev = _is_device(idx)
        if on_dev:
            idx_c, vals_c = _dev_coo(idx, vals)
            nnz = idx_c.shape[1]
        else:
            idx_c = np.ascontiguousarray(idx, np.int32)
            vals_c = np.ascontiguousarray(vals, np.float32)
            nnz = idx_c.shape[1]
        self._dims_a = np.asarray(self.dims, np.int64)
        self._ranks_a = np.asarray(self.ranks, np.int32)
        prob = Problem(self.N, self._dims_a.ctypes.data_as(_i64p), self._ranks_a.ctypes.data_as(_i32p), nnz,
                       _ptr(idx_c), _ptr(vals_c))
        opt = Options()
        L.stdecomp_default_options(ctypes.byref(opt))
        opt.batch = batch
        opt.lr_factor, opt.lr_core = lr_factor, lr_core
        opt.lambda_factor, opt.lambda_core = lam_factor, lam_core
        opt.seed_sample, opt.seed_init = seed_sample, seed_init
        opt.init_kind = INITS[init]
        opt.dtype = DTYPES[dtype]
        opt.inputs_on_device = 1 if on_dev else 0
        opt.chain_chunk = chunk
        opt.stream = ctypes.c_void_p(stream) if stream else None
        opt.report_train_rmse = 1 if train_rmse else 0
        opt.r_core = int(r_core)
        self.r_core = int(r_core)
        opt.momentum = float(momentum)
        opt.placement = PLACEMENTS[placement]
        self.allocator = allocator  # kept alive as long as the handle: the library calls it
        if allocator is not None:
            opt.dev_alloc = allocator._alloc
            opt.dev_free = allocator._free
        h = ctypes.c_void_p()
        rc = L.stdecomp_init(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(h))
        if rc != STD_OK:
            raise StdecompError(rc, "stdecomp_init failed: %s" % L.stdecomp_last_error(None).decode())
        self._h = h
        self.nnz = nnz
        self.batch = batch
        _live.add(self)

    def _check(self, rc, what):
        if rc != STD_OK:
            raise StdecompError(rc, "%s: %s" % (what, load().stdecomp_last_error(self._h).decode()))

    def close(self):
        if getattr(self, "_h", None):
            load().stdecomp_free(self._h)
            self._h = None
            _live.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def epoch(self, n=1):
        st = EpochStats()
        self._check(load().stdecomp_epoch(self._h, n, ctypes.byref(st)), "stdecomp_epoch")
        return {f: getattr(st, f) for f, _ in EpochStats._fields_}

    def run_minibatches(self, epoch, b_begin, b_end):
        st = EpochStats()
        self._check(load().stdecomp_run_minibatches(self._h, epoch, b_begin, b_end, ctypes.byref(st)),
                    "stdecomp_run_minibatches")
        return {f: getattr(st, f) for f, _ in EpochStats._fields_}

    def predict(self, idx):
        if _is_device(idx):
            import torch
            idx = _dev_coo(idx)
            out = torch.empty(idx.shape[1], dtype=torch.float32, device=idx.device)
            self._check(load().stdecomp_predict(self._h, idx.shape[1], _ptr(idx), _ptr(out), 1), "stdecomp_predict")
            return out
        idx = np.ascontiguousarray(idx, np.int32)
        out = np.empty(idx.shape[1], np.float32)
        self._check(load().stdecomp_predict(self._h, idx.shape[1], _ptr(idx), _ptr(out), 0), "stdecomp_predict")
        return out

    def predict_noalloc(self, idx, out=None):
        """predict() through the entry point that allocates nothing (the
        library's fixed scratch array).  Host numpy indices give a numpy
        result; device indices write into ``out`` (a float32 device tensor of
        q values, allocated here if not given)."""
        L = load()
        if _is_device(idx):
            import torch
            idx = _dev_coo(idx)
            if out is None:
                out = torch.empty(idx.shape[1], dtype=torch.float32, device=idx.device)
            self._check(L.stdecomp_predict_noalloc(self._h, idx.shape[1], _ptr(idx), _ptr(out), 1),
                        "stdecomp_predict_noalloc")
            return out
        idx = np.ascontiguousarray(idx, np.int32)
        res = np.empty(idx.shape[1], np.float32)
        self._check(L.stdecomp_predict_noalloc(self._h, idx.shape[1], _ptr(idx), _ptr(res), 0),
                    "stdecomp_predict_noalloc")
        return res

    def loss(self, idx=None, vals=None):
        out = LossOut()
        if idx is None:
            rc = load().stdecomp_loss(self._h, 0, None, None, 0, ctypes.byref(out))
        elif _is_device(idx):
            idx, vals = _dev_coo(idx, vals)
            rc = load().stdecomp_loss(self._h, idx.shape[1], _ptr(idx), _ptr(vals), 1, ctypes.byref(out))
        else:
            idx = np.ascontiguousarray(idx, np.int32)
            vals = np.ascontiguousarray(vals, np.float32)
            rc = load().stdecomp_loss(self._h, idx.shape[1], _ptr(idx), _ptr(vals), 0, ctypes.byref(out))
        res = {f: getattr(out, f) for f, _ in LossOut._fields_}
        if rc == STD_E_DIVERGED:
            res["diverged"] = True
            return res
        self._check(rc, "stdecomp_loss")
        return res

    def get_params(self):
        A = [np.empty((I, J), np.float32) for I, J in zip(self.dims, self.ranks)]
        G = np.empty(int(np.prod(self.ranks)), np.float32)
        ptrs = (ctypes.c_void_p * self.N)(*[a.ctypes.data for a in A])
        self._check(load().stdecomp_get_params(self._h, ptrs, _ptr(G)), "stdecomp_get_params")
        return A, G

    def set_params(self, A, G):
        A = [np.ascontiguousarray(a, np.float32) for a in A]
        G = np.ascontiguousarray(G, np.float32).reshape(-1)
        ptrs = (ctypes.c_void_p * self.N)(*[a.ctypes.data for a in A])
        self._check(load().stdecomp_set_params(self._h, ptrs, _ptr(G)), "stdecomp_set_params")

    def get_velocity(self):
        """Heavy-ball velocities (laid out as the parameters) of a handle with momentum."""
        VA = [np.empty((I, J), np.float32) for I, J in zip(self.dims, self.ranks)]
        VG = np.empty(int(np.prod(self.ranks)), np.float32)
        ptrs = (ctypes.c_void_p * self.N)(*[a.ctypes.data for a in VA])
        self._check(load().stdecomp_get_velocity(self._h, ptrs, _ptr(VG)), "stdecomp_get_velocity")
        return VA, VG

    def set_velocity(self, VA, VG):
        VA = [np.ascontiguousarray(a, np.float32) for a in VA]
        VG = np.ascontiguousarray(VG, np.float32).reshape(-1)
        ptrs = (ctypes.c_void_p * self.N)(*[a.ctypes.data for a in VA])
        self._check(load().stdecomp_set_velocity(self._h, ptrs, _ptr(VG)), "stdecomp_set_velocity")

    def get_kruskal(self):
        """The Kruskal factors B(n) (J_n x R each) of a handle with r_core > 0."""
        B = [np.empty((J, self.r_core), np.float32) for J in self.ranks]
        ptrs = (ctypes.c_void_p * self.N)(*[b.ctypes.data for b in B])
        self._check(load().stdecomp_get_kruskal(self._h, ptrs), "stdecomp_get_kruskal")
        return B

    def set_kruskal(self, B):
        """Set the Kruskal factors (and the core to their product)."""
        B = [np.ascontiguousarray(b, np.float32) for b in B]
        ptrs = (ctypes.c_void_p * self.N)(*[b.ctypes.data for b in B])
        self._check(load().stdecomp_set_kruskal(self._h, ptrs), "stdecomp_set_kruskal")

    def set_epoch(self, e):
        self._check(load().stdecomp_set_epoch(self._h, e), "stdecomp_set_epoch")

    def debug_schedule(self, epoch, batch, mode):
        M = self.batch
        entries = np.empty(M, np.int64)
        sigma = np.empty(M, np.int32)
        seg_off = np.empty(M + 1, np.int32)
        seg_row = np.empty(M, np.int32)
        nseg = np.zeros(1, np.int32)
        m = np.zeros(1, np.int32)
        self._check(load().stdecomp_debug_schedule(
            self._h, epoch, batch, mode, entries.ctypes.data_as(_i64p), sigma.ctypes.data_as(_i32p),
            seg_off.ctypes.data_as(_i32p), seg_row.ctypes.data_as(_i32p), nseg.ctypes.data_as(_i32p),
            m.ctypes.data_as(_i32p)), "stdecomp_debug_schedule")
        mm, d = int(m[0]), int(nseg[0])
        return dict(entries=entries[:mm], sigma=sigma[:mm], seg_off=seg_off[: d + 1], seg_row=seg_row[:d])

    def barrier_us(self, reps=2000):
        """Mean time of the chain's grid barrier alone, in microseconds."""
        us = ctypes.c_double(0.0)
        self._check(load().stdecomp_debug_barrier(self._h, reps, ctypes.byref(us)), "stdecomp_debug_barrier")
        return us.value

    def barrier_check(self, reps=2000):
        """Reads of another workgroup's word after a barrier that returned an
        older round (0: the barrier orders memory as the chain needs)."""
        n = ctypes.c_int64(-1)
        self._check(load().stdecomp_debug_barrier_check(self._h, reps, ctypes.byref(n)), "stdecomp_debug_barrier_check")
        return n.value

    def info(self):
        out = InfoOut()
        self._check(load().stdecomp_info(self._h, ctypes.byref(out)), "stdecomp_info")
        return {f: getattr(out, f) for f, _ in InfoOut._fields_}


def epoch_batched(handles, n_epochs=1):
    """n_epochs epochs of every model in `handles` (Stdecomp objects), their
    chains in one launch where they share a kernel."""
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*[h._h.value for h in handles])
    st = (EpochStats * n)()
    rc = load().stdecomp_epoch_batched(arr, n, n_epochs, st)
    if rc != 0:
        handles[0]._check(rc, "stdecomp_epoch_batched")
    return [{f: getattr(s, f) for f, _ in EpochStats._fields_} for s in st]


def step_batched(handles, max_minibatches):
    """Advance every model in ``handles`` by up to ``max_minibatches``
    minibatches of its current epoch (continuous batching)."""
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*[h._h.value for h in handles])
    st = (EpochStats * n)()
    rc = load().stdecomp_step_batched(arr, n, max_minibatches, st)
    if rc != 0:
        handles[0]._check(rc, "stdecomp_step_batched")
    return [{f: getattr(s, f) for f, _ in EpochStats._fields_} for s in st]


def sample_order(T, seed, epoch, device=False, stream=None):
    """The GPU sampler: pi_e(q) for q in [0, T), as a numpy array, or with
    ``device`` a torch int64 tensor written in place on the device (on
    ``stream``, a hipStream_t value, or the null stream)."""
    if device:
        import torch
        out = torch.empty(T, dtype=torch.int64, device="cuda")
        torch.cuda.current_stream().synchronize()
        rc = load().stdecomp_sample_order(T, seed, epoch, ctypes.c_void_p(out.data_ptr()), 1,
                                          ctypes.c_void_p(stream) if stream else None)
    else:
        out = np.empty(T, np.int64)
        rc = load().stdecomp_sample_order(T, seed, epoch, ctypes.c_void_p(out.ctypes.data), 0,
                                          ctypes.c_void_p(stream) if stream else None)
    if rc != STD_OK:
        raise StdecompError(rc, "stdecomp_sample_order")
    return out
