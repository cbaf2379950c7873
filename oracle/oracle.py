"""ctypes front end of the FP64 CPU oracle (``stdecomp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this module; the product path never does.  It shares no
code with the GPU library and imports nothing from it.

Arrays follow the oracle's conventions: factor matrices as a list of
``I_n x J_n`` float64 arrays (row-major), the core as a flat float64 array with
``j_0`` fastest, COO indices as an int32 ``[N, T]`` array, values float32.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stdecomp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)


def build(force=False):
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", _LIB, _SRC, "-lm"])
    return _LIB


_lib = None
_lib_path = None


def use_library(path):
    """Point the wrappers at another build of the oracle source (the mutation
    tests load deliberately broken copies); ``None`` restores the default."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None:
            build()
        L = ctypes.CDLL(_lib_path or _LIB)
        L.orc_sm64.restype = ctypes.c_uint64
        L.orc_sm64.argtypes = [ctypes.c_uint64]
        L.orc_round_key.restype = ctypes.c_uint64
        L.orc_round_key.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int]
        L.orc_feistel_half_bits.restype = ctypes.c_int
        L.orc_feistel_half_bits.argtypes = [ctypes.c_int64]
        L.orc_perm.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, _i64p]
        L.orc_segments.argtypes = [ctypes.c_int64, _i32p, _i32p, _i32p, _i32p, _i32p]
        L.orc_unfold_col.restype = ctypes.c_int64
        L.orc_unfold_col.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int]
        L.orc_predict.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, _f64p, ctypes.c_int64, _i32p, _f64p]
        L.orc_loss.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, _f64p, ctypes.c_int64, _i32p, _f32p,
                               ctypes.c_double, ctypes.c_double, _f64p]
        L.orc_core_step.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, _f64p, ctypes.c_int64, _i32p, _f32p,
                                    ctypes.c_double, ctypes.c_double]
        L.orc_mode_step.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, _f64p, ctypes.c_int64, _i32p, _f32p,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_step.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, _f64p, ctypes.c_int64, _i32p, _f32p,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_run.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, _f64p, ctypes.c_int64, _i32p, _f32p,
                              ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, _i64p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                              ctypes.c_int64, _i64p]
        L.orc_kruskal_core.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, _f64p, _f64p]
        L.orc_kruskal_W.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, ctypes.c_int64, _i32p,
                                    ctypes.c_int, ctypes.c_int, _f64p]
        L.orc_kruskal_column_step.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, ctypes.c_int, _f64p,
                                              ctypes.c_int64, _i32p, _f32p, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double]
        L.orc_kruskal_core_step.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _f64p,
                                            ctypes.c_int64, _i32p, _f32p, ctypes.c_double, ctypes.c_double]
        L.orc_step_kruskal.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _f64p,
                                       ctypes.c_int64, _i32p, _f32p, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double]
        L.orc_run_kruskal.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _f64p,
                                      ctypes.c_int64, _i32p, _f32p, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, _i64p, ctypes.c_uint64,
                                      ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i64p]
        L.orc_step_momentum.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, _f64p, _f64p, _f64p, ctypes.c_int64,
                                        _i32p, _f32p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double]
        L.orc_run_momentum.argtypes = [ctypes.c_int, _i64p, _i32p, _f64p, _f64p, _f64p, _f64p, ctypes.c_int64,
                                       _i32p, _f32p, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, _i64p, ctypes.c_uint64,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i64p]
        for f in ("orc_perm", "orc_segments", "orc_predict", "orc_loss", "orc_core_step",
                  "orc_mode_step", "orc_step", "orc_run", "orc_kruskal_core", "orc_kruskal_W",
                  "orc_kruskal_column_step", "orc_kruskal_core_step", "orc_step_kruskal", "orc_run_kruskal",
                  "orc_step_momentum", "orc_run_momentum"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError("%s failed with code %d" % (what, rc))


# --------------------------------------------------------------------- sampler
def sm64(x):
    """SplitMix64 output for state ``x`` (one generator step)."""
    return int(lib().orc_sm64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def round_key(seed, epoch, r):
    return int(lib().orc_round_key(ctypes.c_uint64(seed), epoch, r))


def feistel_half_bits(T):
    return int(lib().orc_feistel_half_bits(T))


def perm(T, seed, epoch):
    """The epoch-``epoch`` sample order pi_e of [0, T) as int64."""
    out = np.empty(T, np.int64)
    _check(lib().orc_perm(T, ctypes.c_uint64(seed), epoch, _ptr(out, _i64p)), "orc_perm")
    return out


def segments(rows):
    """sigma, seg_off, seg_row for one minibatch/mode; ``rows[p]`` = i_n of sample p."""
    rows = np.ascontiguousarray(rows, np.int32)
    m = rows.shape[0]
    sigma = np.empty(max(m, 1), np.int32)
    seg_off = np.empty(m + 1, np.int32)
    seg_row = np.empty(max(m, 1), np.int32)
    nseg = np.zeros(1, np.int32)
    _check(lib().orc_segments(m, _ptr(rows, _i32p), _ptr(sigma, _i32p), _ptr(seg_off, _i32p),
                              _ptr(seg_row, _i32p), _ptr(nseg, _i32p)), "orc_segments")
    d = int(nseg[0])
    return sigma[:m].copy(), seg_off[: d + 1].copy(), seg_row[:d].copy()


def unfold_col(dims, index, n):
    dims = np.ascontiguousarray(dims, np.int64)
    index = np.ascontiguousarray(index, np.int64)
    return int(lib().orc_unfold_col(len(dims), _ptr(dims, _i64p), _ptr(index, _i64p), n))


# ------------------------------------------------------------------ the model
class Model:
    """FP64 parameters of a sparse Tucker model (the oracle's state)."""

    def __init__(self, dims, ranks, A, G):
        self.dims = np.ascontiguousarray(dims, np.int64)
        self.ranks = np.ascontiguousarray(ranks, np.int32)
        self.N = len(self.dims)
        assert len(A) == self.N
        self.flatA = np.concatenate([np.ascontiguousarray(a, np.float64).reshape(-1) for a in A])
        self.G = np.ascontiguousarray(G, np.float64).reshape(-1).copy()
        assert self.G.size == int(np.prod(self.ranks))

    @property
    def A(self):
        out, o = [], 0
        for I, J in zip(self.dims, self.ranks):
            out.append(self.flatA[o: o + I * J].reshape(I, J))
            o += I * J
        return out

    def copy(self):
        return Model(self.dims, self.ranks, [a.copy() for a in self.A], self.G.copy())

    def _args(self):
        return (self.N, _ptr(self.dims, _i64p), _ptr(self.ranks, _i32p), _ptr(self.flatA, _f64p),
                _ptr(self.G, _f64p))

    def predict(self, idx):
        idx = np.ascontiguousarray(idx, np.int32)
        q = idx.shape[1]
        out = np.empty(max(q, 1), np.float64)
        _check(lib().orc_predict(*self._args(), q, _ptr(idx, _i32p), _ptr(out, _f64p)), "orc_predict")
        return out[:q]

    def loss(self, idx, vals, lam_A=0.0, lam_G=0.0):
        """{rmse, mae, sse, objective} over the given entries."""
        idx = np.ascontiguousarray(idx, np.int32)
        vals = np.ascontiguousarray(vals, np.float32)
        out = np.empty(4, np.float64)
        _check(lib().orc_loss(*self._args(), idx.shape[1], _ptr(idx, _i32p), _ptr(vals, _f32p),
                              lam_A, lam_G, _ptr(out, _f64p)), "orc_loss")
        return dict(rmse=out[0], mae=out[1], sse=out[2], objective=out[3])

    def core_step(self, idx, x, gam_G, lam_G):
        idx = np.ascontiguousarray(idx, np.int32)
        x = np.ascontiguousarray(x, np.float32)
        _check(lib().orc_core_step(*self._args(), idx.shape[1], _ptr(idx, _i32p), _ptr(x, _f32p),
                                   gam_G, lam_G), "orc_core_step")

    def mode_step(self, idx, x, n, gam_A, lam_A):
        idx = np.ascontiguousarray(idx, np.int32)
        x = np.ascontiguousarray(x, np.float32)
        _check(lib().orc_mode_step(*self._args(), idx.shape[1], _ptr(idx, _i32p), _ptr(x, _f32p),
                                   n, gam_A, lam_A), "orc_mode_step")

    def step(self, idx, x, gam_A, lam_A, gam_G, lam_G):
        idx = np.ascontiguousarray(idx, np.int32)
        x = np.ascontiguousarray(x, np.float32)
        _check(lib().orc_step(*self._args(), idx.shape[1], _ptr(idx, _i32p), _ptr(x, _f32p),
                              gam_A, lam_A, gam_G, lam_G), "orc_step")

    def run(self, idx, vals, M, gam_A, lam_A, gam_G, lam_G, perm=None, seed=0, epoch0=0,
            n_epochs=1, max_batches=-1):
        """Minibatch SGD epochs; ``perm`` (``[n_epochs, T]`` int64) overrides the sampler.
        Returns the number of minibatches run."""
        idx = np.ascontiguousarray(idx, np.int32)
        vals = np.ascontiguousarray(vals, np.float32)
        T = idx.shape[1]
        pp = None
        if perm is not None:
            perm = np.ascontiguousarray(perm, np.int64).reshape(-1)
            assert perm.size == n_epochs * T
            pp = _ptr(perm, _i64p)
        done = np.zeros(1, np.int64)
        _check(lib().orc_run(*self._args(), T, _ptr(idx, _i32p), _ptr(vals, _f32p), M, gam_A, lam_A,
                             gam_G, lam_G, pp, ctypes.c_uint64(seed), epoch0, n_epochs, max_batches,
                             _ptr(done, _i64p)), "orc_run")
        return int(done[0])


# --------------------------------------------------------- heavy-ball momentum
class MomentumModel(Model):
    """The model plus heavy-ball velocities: VA laid out as A (one velocity per
    factor row, zero at start), VG for the core (orc_step_momentum)."""

    def __init__(self, dims, ranks, A, G, VA=None, VG=None):
        super().__init__(dims, ranks, A, G)
        self.flatVA = (np.zeros_like(self.flatA) if VA is None else
                       np.concatenate([np.ascontiguousarray(v, np.float64).reshape(-1) for v in VA]))
        self.VG = np.zeros_like(self.G) if VG is None else np.ascontiguousarray(VG, np.float64).reshape(-1).copy()

    @property
    def VA(self):
        out, o = [], 0
        for I, J in zip(self.dims, self.ranks):
            out.append(self.flatVA[o: o + I * J].reshape(I, J))
            o += I * J
        return out

    def _margs(self):
        return (self.N, _ptr(self.dims, _i64p), _ptr(self.ranks, _i32p), _ptr(self.flatA, _f64p),
                _ptr(self.G, _f64p), _ptr(self.flatVA, _f64p), _ptr(self.VG, _f64p))

    def step(self, idx, x, gam_A, lam_A, gam_G, lam_G, mu=0.0):
        idx = np.ascontiguousarray(idx, np.int32)
        x = np.ascontiguousarray(x, np.float32)
        _check(lib().orc_step_momentum(*self._margs(), idx.shape[1], _ptr(idx, _i32p), _ptr(x, _f32p),
                                       gam_A, lam_A, gam_G, lam_G, mu), "orc_step_momentum")

    def run(self, idx, vals, M, gam_A, lam_A, gam_G, lam_G, perm=None, seed=0, epoch0=0,
            n_epochs=1, max_batches=-1, mu=0.0):
        idx = np.ascontiguousarray(idx, np.int32)
        vals = np.ascontiguousarray(vals, np.float32)
        T = idx.shape[1]
        pp = None
        if perm is not None:
            perm = np.ascontiguousarray(perm, np.int64).reshape(-1)
            assert perm.size == n_epochs * T
            pp = _ptr(perm, _i64p)
        done = np.zeros(1, np.int64)
        _check(lib().orc_run_momentum(*self._margs(), T, _ptr(idx, _i32p), _ptr(vals, _f32p), M, gam_A, lam_A,
                                      gam_G, lam_G, mu, pp, ctypes.c_uint64(seed), epoch0, n_epochs, max_batches,
                                      _ptr(done, _i64p)), "orc_run_momentum")
        return int(done[0])


# ----------------------------------------------------------- the Kruskal core
def kruskal_core(ranks, B):
    """Flat core (j_0 fastest) of the Kruskal product of the J_n x R matrices B."""
    ranks = np.ascontiguousarray(ranks, np.int32)
    R = int(np.asarray(B[0]).shape[1])
    flatB = np.concatenate([np.ascontiguousarray(b, np.float64).reshape(-1) for b in B])
    G = np.empty(int(np.prod(ranks)), np.float64)
    _check(lib().orc_kruskal_core(len(ranks), _ptr(ranks, _i32p), R, _ptr(flatB, _f64p), _ptr(G, _f64p)),
           "orc_kruskal_core")
    return G


class KruskalModel(Model):
    """FP64 parameters of a sparse Tucker model whose core is the R_core
    Kruskal product of the matrices B(n) (J_n x R); ``G`` always holds that
    product."""

    def __init__(self, dims, ranks, A, B):
        self.R = int(np.asarray(B[0]).shape[1])
        assert len(B) == len(dims) and all(np.asarray(b).shape == (J, self.R) for b, J in zip(B, ranks))
        self.flatB = np.concatenate([np.ascontiguousarray(b, np.float64).reshape(-1) for b in B])
        super().__init__(dims, ranks, A, kruskal_core(ranks, B))

    @property
    def B(self):
        out, o = [], 0
        for J in self.ranks:
            out.append(self.flatB[o: o + J * self.R].reshape(J, self.R))
            o += J * self.R
        return out

    def copy(self):
        return KruskalModel(self.dims, self.ranks, [a.copy() for a in self.A], [b.copy() for b in self.B])

    def _kargs(self):
        return (self.N, _ptr(self.dims, _i64p), _ptr(self.ranks, _i32p), _ptr(self.flatA, _f64p), self.R,
                _ptr(self.flatB, _f64p))

    def W(self, idx, n, r):
        """W_r of mode n (m x J_n) for the entries ``idx``."""
        idx = np.ascontiguousarray(idx, np.int32)
        out = np.empty((idx.shape[1], int(self.ranks[n])), np.float64)
        _check(lib().orc_kruskal_W(*self._kargs(), idx.shape[1], _ptr(idx, _i32p), n, r, _ptr(out, _f64p)),
               "orc_kruskal_W")
        return out

    def column_step(self, idx, x, n, r, gam_B, lam_B):
        idx = np.ascontiguousarray(idx, np.int32)
        x = np.ascontiguousarray(x, np.float32)
        _check(lib().orc_kruskal_column_step(*self._kargs(), idx.shape[1], _ptr(idx, _i32p), _ptr(x, _f32p),
                                             n, r, gam_B, lam_B), "orc_kruskal_column_step")
        self.G[:] = kruskal_core(self.ranks, self.B)

    def kruskal_core_step(self, idx, x, gam_B, lam_B):
        idx = np.ascontiguousarray(idx, np.int32)
        x = np.ascontiguousarray(x, np.float32)
        _check(lib().orc_kruskal_core_step(*self._kargs(), _ptr(self.G, _f64p), idx.shape[1], _ptr(idx, _i32p),
                                           _ptr(x, _f32p), gam_B, lam_B), "orc_kruskal_core_step")

    def step(self, idx, x, gam_A, lam_A, gam_B, lam_B):
        idx = np.ascontiguousarray(idx, np.int32)
        x = np.ascontiguousarray(x, np.float32)
        _check(lib().orc_step_kruskal(*self._kargs(), _ptr(self.G, _f64p), idx.shape[1], _ptr(idx, _i32p),
                                      _ptr(x, _f32p), gam_A, lam_A, gam_B, lam_B), "orc_step_kruskal")

    def run(self, idx, vals, M, gam_A, lam_A, gam_G, lam_G, perm=None, seed=0, epoch0=0,
            n_epochs=1, max_batches=-1):
        """Minibatch SGD epochs with the Kruskal core sub-step (gam_G and
        lam_G are the paper's gamma_B and lambda_B)."""
        idx = np.ascontiguousarray(idx, np.int32)
        vals = np.ascontiguousarray(vals, np.float32)
        T = idx.shape[1]
        pp = None
        if perm is not None:
            perm = np.ascontiguousarray(perm, np.int64).reshape(-1)
            assert perm.size == n_epochs * T
            pp = _ptr(perm, _i64p)
        done = np.zeros(1, np.int64)
        _check(lib().orc_run_kruskal(*self._kargs(), _ptr(self.G, _f64p), T, _ptr(idx, _i32p), _ptr(vals, _f32p),
                                     M, gam_A, lam_A, gam_G, lam_G, pp, ctypes.c_uint64(seed), epoch0, n_epochs,
                                     max_batches, _ptr(done, _i64p)), "orc_run_kruskal")
        return int(done[0])
