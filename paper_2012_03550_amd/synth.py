"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws inputs: COO indices, values, a held-out split and
initial parameters.  It contains none of the SGD_Tucker update arithmetic and
is the one module that both the GPU path's tests and the CPU oracle's tests
read their inputs from.

The paper evaluates on rating tensors (MovieLens, Netflix, Yahoo-music; its
dataset table) that are not available here.  The generators below stand in for
them with the shapes, sizes and index skew of those tensors:

* ``planted_uniform``: a 3-order tensor with uniform indices whose values come
  from a planted Tucker model plus Gaussian noise (small parity workload).
* ``ratings_zipf``: a Netflix-like 3-order rating tensor, Zipf-distributed
  indices per mode (ranks mapped through a seeded permutation so that
  popularity is not index-adjacent) and integer ratings 1..5.
* ``planted_powerlaw``: a 4-order tensor with power-law indices on the first
  two modes, uniform indices on the others, values from a planted model.

Planted values are the Tucker model evaluated at the sampled coordinates with
``numpy.einsum`` (the generative model of the data, not the solver).
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def zipf_indices(rng, I, s, count, chunk=1 << 23):
    """``count`` draws from a finite Zipf law over ranks 1..I (p_k ~ k^-s),
    mapped through a seeded permutation of [0, I)."""
    ranks = np.arange(1, I + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** (-float(s)))
    cdf /= cdf[-1]
    relabel = rng.permutation(I).astype(np.int32)
    out = np.empty(count, np.int32)
    for lo in range(0, count, chunk):
        hi = min(count, lo + chunk)
        u = rng.random(hi - lo)
        r = np.searchsorted(cdf, u, side="right")
        np.minimum(r, I - 1, out=r)
        out[lo:hi] = relabel[r]
    return out


def uniform_indices(rng, I, count):
    return rng.integers(0, I, size=count, dtype=np.int64).astype(np.int32)


def planted_model(rng, dims, ranks, scale=None):
    """Planted factors and core, entries N(0,1)/sqrt(J) (per-mode J for the
    factors, J_1 for the core) unless ``scale`` fixes the std."""
    A = []
    for I, J in zip(dims, ranks):
        sd = scale if scale is not None else 1.0 / np.sqrt(J)
        A.append(rng.standard_normal((I, J)) * sd)
    sd = scale if scale is not None else 1.0 / np.sqrt(ranks[0])
    G = rng.standard_normal(int(np.prod(ranks))) * sd
    return A, G


def evaluate_planted(A, G, ranks, idx, chunk=1 << 18):
    """Planted-model values at the coordinates ``idx`` ([N, T]) in float64."""
    N = len(A)
    T = idx.shape[1]
    core = np.asarray(G, np.float64).reshape(tuple(reversed(ranks)))  # C order: j_{N-1} slowest
    letters = "abcdefgh"[:N]
    # core axes are (j_{N-1}, ..., j_0); row operands are (t, j_k)
    spec = "".join(reversed(letters)) + "," + ",".join("z" + letters[k] for k in range(N)) + "->z"
    out = np.empty(T, np.float64)
    for lo in range(0, T, chunk):
        hi = min(T, lo + chunk)
        rows = [A[k][idx[k, lo:hi]] for k in range(N)]
        out[lo:hi] = np.einsum(spec, core, *rows, optimize=True)
    return out


def evaluate_planted_device(A, G, ranks, idx, device, chunk=1 << 20):
    """The same values as ``evaluate_planted`` (float64) computed with torch on
    ``device`` (for workloads of hundreds of millions of entries): the core is
    contracted with mode 0's rows by a matrix product, then with the other
    modes' rows one at a time."""
    import torch
    N = len(A)
    T = idx.shape[1]
    At = [torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(device) for a in A]
    # flat core index j_0 + J_0 (j_1 + J_1 (...)): rows of this view are (j_{N-1}, ..., j_1) in C order
    core = torch.from_numpy(np.asarray(G, np.float64)).to(device).view(-1, ranks[0]).t().contiguous()
    out = np.empty(T, np.float64)
    for lo in range(0, T, chunk):
        hi = min(T, lo + chunk)
        ii = torch.from_numpy(np.ascontiguousarray(idx[:, lo:hi], np.int64)).to(device)
        x = At[0][ii[0]] @ core  # (z, prod_{k>=1} J_k), j_1 fastest
        for k in range(1, N):
            rk = At[k][ii[k]]  # (z, J_k)
            x = torch.bmm(x.view(hi - lo, -1, ranks[k]), rk.unsqueeze(2).contiguous()).view(hi - lo, -1)
        out[lo:hi] = x.view(-1).cpu().numpy()
    return out


def split_holdout(rng, T, frac):
    """Boolean mask of held-out entries (each entry independently with prob. frac)."""
    return rng.random(T) < frac


class Workload:
    """COO training/held-out sets plus the planted model if there is one."""

    def __init__(self, dims, ranks, idx, vals, test_mask, planted=None, noise=None, name=""):
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(r) for r in ranks)
        self.name = name
        keep = ~test_mask
        self.train_idx = np.ascontiguousarray(idx[:, keep])
        self.train_vals = np.ascontiguousarray(vals[keep])
        self.test_idx = np.ascontiguousarray(idx[:, test_mask])
        self.test_vals = np.ascontiguousarray(vals[test_mask])
        self.planted = planted
        self.noise = noise

    @property
    def N(self):
        return len(self.dims)

    @property
    def nnz(self):
        return self.train_idx.shape[1]


def planted_uniform(dims=(1000, 1000, 1000), ranks=(5, 5, 5), nnz=100_000, sigma=0.01,
                    holdout=0.1, seed=1001):
    """Uniform indices, planted model with N(0,1)/sqrt(J) entries plus N(0, sigma^2) noise."""
    rng = _rng(seed)
    idx = np.stack([uniform_indices(rng, I, nnz) for I in dims])
    A, G = planted_model(rng, dims, ranks)
    noise = rng.standard_normal(nnz) * sigma
    vals = (evaluate_planted(A, G, ranks, idx) + noise).astype(np.float32)
    mask = split_holdout(rng, nnz, holdout)
    return Workload(dims, ranks, idx, vals, mask, planted=(A, G), noise=noise[~mask],
                    name="planted_uniform")


def planted_batch(n=64, ranks_choice=(4, 8, 16), log_dims=(3.0, 6.0), log_nnz=(4.0, 7.0), sigma=0.01,
                  seed=1004, device=None, holdout=0.0):
    """Many independent three-mode tensors: mode sizes floor(10^U(log_dims)),
    entry counts floor(10^U(log_nnz)), uniform indices, equal ranks J drawn
    from ``ranks_choice``, values from each tensor's planted model plus
    N(0, sigma^2) noise."""
    rng = _rng(seed)
    out = []
    for t in range(n):
        dims = tuple(int(10 ** rng.uniform(*log_dims)) for _ in range(3))
        nnz = int(10 ** rng.uniform(*log_nnz))
        J = int(rng.choice(ranks_choice))
        ranks = (J, J, J)
        idx = np.stack([uniform_indices(rng, I, nnz) for I in dims])
        A, G = planted_model(rng, dims, ranks)
        noise = rng.standard_normal(nnz) * sigma
        clean = evaluate_planted(A, G, ranks, idx) if device is None else evaluate_planted_device(A, G, ranks, idx, device)
        vals = (clean + noise).astype(np.float32)
        mask = split_holdout(rng, nnz, holdout) if holdout > 0 else np.zeros(nnz, bool)
        out.append(Workload(dims, ranks, idx, vals, mask, planted=(A, G), noise=noise[~mask], name="planted_batch_%d" % t))
    return out


RATING_PROBS = (0.05, 0.10, 0.25, 0.35, 0.25)


def ratings_zipf(dims=(480_000, 18_000, 2_000), ranks=(10, 10, 10), nnz=100_000_000, s=1.1,
                 probs=RATING_PROBS, holdout=0.1, seed=1002):
    """Netflix-like rating tensor: Zipf(s) indices per mode, ratings 1..5 drawn
    with the given probabilities independently of the indices."""
    rng = _rng(seed)
    idx = np.stack([zipf_indices(rng, I, s, nnz) for I in dims])
    cdf = np.cumsum(np.asarray(probs, np.float64))
    cdf /= cdf[-1]
    vals = np.empty(nnz, np.float32)
    chunk = 1 << 23
    for lo in range(0, nnz, chunk):
        hi = min(nnz, lo + chunk)
        vals[lo:hi] = (np.searchsorted(cdf, rng.random(hi - lo), side="right") + 1).astype(np.float32)
    np.minimum(vals, len(probs), out=vals)
    mask = split_holdout(rng, nnz, holdout)
    return Workload(dims, ranks, idx, vals, mask, name="ratings_zipf")


def planted_powerlaw(dims=(100_000, 100_000, 1_000, 100), ranks=(8, 8, 8, 8), nnz=200_000_000,
                     s=1.2, powerlaw_modes=2, sigma=0.05, holdout=0.1, seed=1003, device=None):
    """Power-law (Zipf s) indices on the first ``powerlaw_modes`` modes, uniform
    on the rest; planted model with N(0,1)/sqrt(J) entries plus N(0, sigma^2).
    With ``device`` the planted values are computed there (torch, float64)."""
    rng = _rng(seed)
    rows = []
    for k, I in enumerate(dims):
        rows.append(zipf_indices(rng, I, s, nnz) if k < powerlaw_modes else uniform_indices(rng, I, nnz))
    idx = np.stack(rows)
    A, G = planted_model(rng, dims, ranks)
    noise = rng.standard_normal(nnz) * sigma
    clean = evaluate_planted(A, G, ranks, idx) if device is None else evaluate_planted_device(A, G, ranks, idx, device)
    vals = (clean + noise).astype(np.float32)
    mask = split_holdout(rng, nnz, holdout)
    return Workload(dims, ranks, idx, vals, mask, planted=(A, G), noise=noise[~mask],
                    name="planted_powerlaw")


def random_tiny(N, dims, ranks, nnz, seed, skew=None):
    """Small random tensors for parity tests: uniform indices (or Zipf with
    exponent ``skew``), values N(0,1)."""
    rng = _rng(seed)
    rows = []
    for I in dims:
        rows.append(zipf_indices(rng, I, skew, nnz) if skew else uniform_indices(rng, I, nnz))
    idx = np.stack(rows) if nnz > 0 else np.zeros((N, 0), np.int32)
    vals = rng.standard_normal(nnz).astype(np.float32)
    return idx.astype(np.int32), vals


def init_params(dims, ranks, seed, kind="scaled"):
    """Initial factors and core.  ``scaled``: entries N(0, 1/J_n) (core: 1/J_1);
    ``paper``: N(0.5, 0.1^2), the initialisation of the paper's experiments."""
    rng = _rng(seed)
    A = []
    for I, J in zip(dims, ranks):
        if kind == "paper":
            A.append(0.5 + 0.1 * rng.standard_normal((I, J)))
        else:
            A.append(rng.standard_normal((I, J)) / np.sqrt(J))
    P = int(np.prod(ranks))
    if kind == "paper":
        G = 0.5 + 0.1 * rng.standard_normal(P)
    else:
        G = rng.standard_normal(P) / np.sqrt(ranks[0])
    return [a.astype(np.float32) for a in A], G.astype(np.float32)
