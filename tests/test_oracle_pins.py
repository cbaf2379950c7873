"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test states what it pins.  None of them re-types the oracle's own code:
they use the paper's worked examples, published test vectors, definitions
that reduce to library routines (numpy einsum / kron / linalg.solve), exact
rational arithmetic, finite differences and closed-form optima.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2012_03550_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ----------------------------------------------------------------------------
# independent numpy model: Definition "n-Mode Tensor-Matrix product" and
# Definition "Sparse Tucker Decomposition" via tensordot / einsum
# ----------------------------------------------------------------------------
def core_tensor(G, ranks):
    """Flat core (j_0 fastest) as an ndarray indexed [j_0, ..., j_{N-1}]."""
    return np.asarray(G, np.float64).reshape(tuple(ranks), order="F")


def dense_tucker(A, G, ranks):
    """X_hat = G x_1 A(1) x_2 ... x_N A(N), by successive n-mode products."""
    X = core_tensor(G, ranks)
    for n, a in enumerate(A):
        # (X x_n U)_{..., i_n, ...} = sum_{j_n} X_{..., j_n, ...} U_{i_n, j_n}
        X = np.moveaxis(np.tensordot(a, X, axes=([1], [n])), 0, n)
    return X


def einsum_predict(A, G, ranks, idx):
    N = len(A)
    letters = "abcdefgh"[:N]
    spec = letters + "," + ",".join("z" + l for l in letters) + "->z"
    return np.einsum(spec, core_tensor(G, ranks), *[A[k][idx[k]] for k in range(N)])


def unfold(X, n):
    """Mode-n unfolding of Definition "Tensor Unfolding": column index with the
    lowest remaining mode fastest (Fortran order over the other axes)."""
    Xn = np.moveaxis(X, n, 0)
    return Xn.reshape(Xn.shape[0], -1, order="F")


def random_model(rng, dims, ranks, scale=0.7):
    A = [rng.standard_normal((I, J)) * scale for I, J in zip(dims, ranks)]
    G = rng.standard_normal(int(np.prod(ranks))) * scale
    return A, G


# ----------------------------------------------------------------------------
# sampler
# ----------------------------------------------------------------------------
def test_splitmix64_published_vectors(oracle_mod):
    """SplitMix64 seeded with 0 yields the published first outputs
    0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f (Steele et al.
    2014, reference generator); the oracle's round function is that output."""
    g = 0x9E3779B97F4A7C15
    assert oracle_mod.sm64(0) == 0xE220A8397B1DCDAF
    assert oracle_mod.sm64(g) == 0x6E789E6AA1B965F4
    assert oracle_mod.sm64((2 * g) % 2**64) == 0x06C45D188009454F


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 17, 255, 256, 257, 1000, 65537, 300_001])
def test_perm_is_bijection(oracle_mod, T):
    """Each epoch visits every entry exactly once (an epoch is a pass over
    Omega without replacement)."""
    for e in (0, 1, 7):
        p = oracle_mod.perm(T, 12345, e)
        assert p.shape == (T,)
        assert np.array_equal(np.sort(p), np.arange(T))


def test_perm_depends_on_epoch_and_seed(oracle_mod):
    T = 10_000
    a, b, c = oracle_mod.perm(T, 1, 0), oracle_mod.perm(T, 1, 1), oracle_mod.perm(T, 2, 0)
    assert (a != b).mean() > 0.99 and (a != c).mean() > 0.99
    assert np.array_equal(a, oracle_mod.perm(T, 1, 0))


def test_perm_looks_uniform(oracle_mod):
    """Positions of the first decile are spread over the whole range (a
    Feistel network with a mixing round function is not order-preserving)."""
    T = 100_000
    p = oracle_mod.perm(T, 99, 3)
    hist = np.bincount(p[: T // 10] * 10 // T, minlength=10)
    assert hist.min() > 800 and hist.max() < 1200


def test_perm_frozen_vectors(oracle_mod):
    """Bit-exact regression vectors (written by tests/golden/make_golden.py,
    which calls only the oracle); the GPU sampler is compared to them."""
    with open(os.path.join(GOLDEN, "sampler_vectors.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        p = oracle_mod.perm(case["T"], case["seed"], case["epoch"])
        assert p[: len(case["head"])].tolist() == case["head"]
        assert int(p.sum()) == case["T"] * (case["T"] - 1) // 2


# ----------------------------------------------------------------------------
# unfolding order and row segments: the paper's worked examples
# ----------------------------------------------------------------------------
def test_unfolding_columns_paper_example(oracle_mod):
    """The improved-strategy example: row 1 of X^(1) is updated by entries
    (1,1,1), (1,2,2), (1,3,2), (1,2,3) with S^(1) columns 1, 5, 6, 8."""
    with open(os.path.join(GOLDEN, "paper_toy_coo.json")) as f:
        g = json.load(f)
    ex = g["improved_strategy_coo"]
    cols = [oracle_mod.unfold_col(g["dims"], np.array(e) - 1, 0) + 1 for e in ex["mode1_row1_entries"]]
    assert cols == ex["mode1_row1_columns"]


def test_segments_paper_example(oracle_mod):
    """Same example: the four row-1 entries form one segment of mode 1, and
    each thread's pair of entries lies in one row of X^(3)."""
    with open(os.path.join(GOLDEN, "paper_toy_coo.json")) as f:
        g = json.load(f)
    ex = g["improved_strategy_coo"]
    coo = np.array(ex["entries"])
    rows1 = (coo[:, 0] - 1).astype(np.int32)
    sigma, off, segrow = oracle_mod.segments(rows1)
    sizes = dict(zip(segrow.tolist(), np.diff(off).tolist()))
    assert sizes[0] == 4 and sizes[2] == 2
    assert sigma.tolist() == [0, 2, 3, 4, 1, 5]
    rows3 = (coo[:, 2] - 1).astype(np.int32)
    sigma, off, segrow = oracle_mod.segments(rows3)
    assert np.diff(off).tolist() == [2, 2, 2]
    for t in ex["threads"]:
        assert rows3[t[0]] == rows3[t[1]]


def test_segments_naive_example(oracle_mod):
    """Naive-strategy example: rows 1, 2, 3 of X^(3) hold 4, 2 and 1 entries."""
    with open(os.path.join(GOLDEN, "paper_toy_coo.json")) as f:
        g = json.load(f)
    ex = g["naive_strategy_mode3"]
    rows = []
    for r, cols in ex["row_columns"].items():
        rows += [int(r) - 1] * len(cols)
    rows = np.array(rows, np.int32)[np.random.default_rng(0).permutation(len(rows))]
    sigma, off, segrow = oracle_mod.segments(rows)
    assert np.diff(off).tolist() == ex["segment_sizes"]
    assert segrow.tolist() == [0, 1, 2]


@pytest.mark.parametrize("m", [0, 1, 2, 64, 1000])
def test_segments_sorted_and_stable(oracle_mod, m):
    rng = np.random.default_rng(m)
    rows = rng.integers(0, max(1, m // 3), size=m).astype(np.int32)
    sigma, off, segrow = oracle_mod.segments(rows)
    key = rows.astype(np.int64) * (m + 1) + np.arange(m)
    assert np.array_equal(sigma, np.argsort(key, kind="stable"))
    assert off[0] == 0 and off[-1] == m
    assert np.array_equal(segrow, np.unique(rows))


# ----------------------------------------------------------------------------
# forward model
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dims,ranks", [
    ((4, 3), (2, 3)),
    ((4, 3, 5), (2, 3, 2)),
    ((3, 4, 2, 3), (2, 1, 2, 3)),
    ((2, 3, 2, 2, 3), (2, 2, 1, 2, 2)),
])
def test_predict_matches_dense_tucker(oracle_mod, dims, ranks):
    """x_hat equals the dense n-mode-product reconstruction at every cell."""
    rng = np.random.default_rng(len(dims))
    A, G = random_model(rng, dims, ranks)
    X = dense_tucker(A, G, ranks)
    cells = np.array(np.unravel_index(np.arange(X.size), X.shape), np.int32)
    m = oracle_mod.Model(dims, ranks, A, G)
    np.testing.assert_allclose(m.predict(cells), X.reshape(-1), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_unfolding_kronecker_identity(oracle_mod, n):
    """X_hat^(n) = A(n) G_(n) S(n)^T with S(n) = A(N) x ... x A(n+1) x A(n-1)
    x ... x A(1) (Kronecker, Eq. optimization_for_factor): fixes the relative
    order of the unfolding, the Kronecker product and the core storage."""
    dims, ranks = (3, 4, 2, 3), (2, 3, 2, 2)
    rng = np.random.default_rng(10 + n)
    A, G = random_model(rng, dims, ranks)
    m = oracle_mod.Model(dims, ranks, A, G)
    cells = np.array(np.unravel_index(np.arange(int(np.prod(dims))), dims, order="C"), np.int32)
    X = np.empty(dims)
    X[tuple(cells)] = m.predict(cells)
    S = None
    for k in reversed(range(len(dims))):
        if k == n:
            continue
        S = A[k] if S is None else np.kron(S, A[k])
    Gn = unfold(core_tensor(G, ranks), n)
    np.testing.assert_allclose(unfold(X, n), A[n] @ Gn @ S.T, rtol=1e-12, atol=1e-12)


def test_gauge_invariance(oracle_mod):
    """A(n) Q with G x_n Q^-1 leaves every prediction unchanged."""
    dims, ranks = (5, 4, 6), (3, 2, 3)
    rng = np.random.default_rng(3)
    A, G = random_model(rng, dims, ranks)
    idx = np.stack([rng.integers(0, I, 50) for I in dims]).astype(np.int32)
    before = oracle_mod.Model(dims, ranks, A, G).predict(idx)
    Q = rng.standard_normal((3, 3)) + 3 * np.eye(3)
    A2 = [a.copy() for a in A]
    A2[2] = A[2] @ Q
    Gt = np.moveaxis(np.tensordot(np.linalg.inv(Q), core_tensor(G, ranks), axes=([1], [2])), 0, 2)
    G2 = Gt.reshape(-1, order="F")
    after = oracle_mod.Model(dims, ranks, A2, G2).predict(idx)
    np.testing.assert_allclose(after, before, rtol=1e-10, atol=1e-12)


def test_predict_rejects_bad_index(oracle_mod):
    m = oracle_mod.Model((3, 3), (2, 2), [np.ones((3, 2)), np.ones((3, 2))], np.ones(4))
    with pytest.raises(oracle_mod.OracleError):
        m.predict(np.array([[0], [3]], np.int32))


# ----------------------------------------------------------------------------
# loss formula (Section "Experimental Settings": RMSE and MAE over Gamma)
# ----------------------------------------------------------------------------
def test_loss_formula(oracle_mod):
    dims, ranks = (6, 5, 4), (2, 3, 2)
    rng = np.random.default_rng(4)
    A, G = random_model(rng, dims, ranks)
    idx = np.stack([rng.integers(0, I, 40) for I in dims]).astype(np.int32)
    vals = rng.standard_normal(40).astype(np.float32)
    r = vals.astype(np.float64) - einsum_predict(A, G, ranks, idx)
    out = oracle_mod.Model(dims, ranks, A, G).loss(idx, vals, lam_A=0.3, lam_G=0.2)
    assert out["rmse"] == pytest.approx(np.sqrt(np.mean(r ** 2)), rel=1e-12)
    assert out["mae"] == pytest.approx(np.mean(np.abs(r)), rel=1e-12)
    assert out["sse"] == pytest.approx(np.sum(r ** 2), rel=1e-12)
    reg = 0.5 * 0.3 * sum((a ** 2).sum() for a in A) + 0.5 * 0.2 * (G ** 2).sum()
    assert out["objective"] == pytest.approx(0.5 * np.mean(r ** 2) + reg, rel=1e-12)


# ----------------------------------------------------------------------------
# gradients: finite differences of the sub-objectives
# ----------------------------------------------------------------------------
def _tiny_batch(rng, dims, m, repeat_row=True):
    idx = np.stack([rng.integers(0, I, m) for I in dims]).astype(np.int32)
    if repeat_row:  # make segments with several samples in every mode
        for k in range(len(dims)):
            idx[k, : m // 2] = idx[k, 0]
    x = rng.standard_normal(m).astype(np.float32)
    return idx, x


def _fd(f, w, eps=1e-6):
    g = np.empty_like(w)
    for t in range(w.size):
        wp, wm = w.copy(), w.copy()
        wp.flat[t] += eps
        wm.flat[t] -= eps
        g.flat[t] = (f(wp) - f(wm)) / (2 * eps)
    return g


@pytest.mark.parametrize("dims,ranks", [((4, 3, 5), (2, 3, 2)), ((3, 4, 2, 3), (2, 2, 2, 3))])
def test_core_step_is_gradient_of_fC(oracle_mod, dims, ranks):
    """Core sub-step = gamma_G * grad of f_C(G) = (1/2m) sum r^2 + (lambda_G/2)||G||^2
    (Eq. approximated_core_tensor_optimization with the averaged rule of Eq. SGD):
    pins 1/m, lambda, the sign and the 1/2 convention."""
    rng = np.random.default_rng(5)
    A, G = random_model(rng, dims, ranks)
    idx, x = _tiny_batch(rng, dims, 9)
    lam, gam = 0.37, 0.05
    m = len(x)

    def fC(g):
        r = x.astype(np.float64) - einsum_predict(A, g, ranks, idx)
        return 0.5 * np.mean(r ** 2) + 0.5 * lam * np.sum(g ** 2)

    grad = _fd(fC, G.copy())
    mod = oracle_mod.Model(dims, ranks, A, G)
    mod.core_step(idx, x, gam, lam)
    np.testing.assert_allclose((G - mod.G) / gam, grad, rtol=1e-7, atol=1e-8)
    # factors untouched by the core step
    np.testing.assert_array_equal(mod.flatA, np.concatenate([a.reshape(-1) for a in A]))
    assert m == 9


@pytest.mark.parametrize("n", [0, 1, 2])
def test_mode_step_is_gradient_of_row_objective(oracle_mod, n):
    """Mode-n sub-step moves each sampled row i by gamma_A * grad of
    f_{n,i}(a) = (1/2c_i) sum_{p in seg(i)} (x_p - x_hat_p(a))^2 + (lambda_A/2)||a||^2
    (Eq. SGD_factor_matrix / Gradient_factor_matrix with the row-count
    normaliser of Algorithm 1); rows outside the minibatch do not move."""
    dims, ranks = (5, 4, 6), (2, 3, 2)
    rng = np.random.default_rng(6 + n)
    A, G = random_model(rng, dims, ranks)
    idx, x = _tiny_batch(rng, dims, 11)
    lam, gam = 0.21, 0.03
    mod = oracle_mod.Model(dims, ranks, A, G)
    mod.mode_step(idx, x, n, gam, lam)
    newA = mod.A
    for i in range(dims[n]):
        sel = np.nonzero(idx[n] == i)[0]
        if sel.size == 0:
            np.testing.assert_array_equal(newA[n][i], A[n][i])
            continue

        def f(a):
            A2 = [t.copy() for t in A]
            A2[n][i] = a
            r = x[sel].astype(np.float64) - einsum_predict(A2, G, ranks, idx[:, sel])
            return 0.5 * np.mean(r ** 2) + 0.5 * lam * np.sum(a ** 2)

        grad = _fd(f, A[n][i].copy())
        np.testing.assert_allclose((A[n][i] - newA[n][i]) / gam, grad, rtol=1e-7, atol=1e-8)
    for k in range(len(dims)):
        if k != n:
            np.testing.assert_array_equal(newA[k], A[k])
    np.testing.assert_array_equal(mod.G, G)


def test_step_order_core_then_modes(oracle_mod):
    """One minibatch = core sub-step, then modes 1..N in order, each using the
    parameters left by the previous sub-steps (Algorithm 1)."""
    dims, ranks = (5, 4, 6), (2, 3, 2)
    rng = np.random.default_rng(8)
    A, G = random_model(rng, dims, ranks)
    idx, x = _tiny_batch(rng, dims, 10)
    a = oracle_mod.Model(dims, ranks, A, G)
    a.step(idx, x, 0.05, 0.01, 0.04, 0.02)
    b = oracle_mod.Model(dims, ranks, A, G)
    b.core_step(idx, x, 0.04, 0.02)
    for n in range(3):
        b.mode_step(idx, x, n, 0.05, 0.01)
    np.testing.assert_array_equal(a.G, b.G)
    np.testing.assert_array_equal(a.flatA, b.flatA)
    c = oracle_mod.Model(dims, ranks, A, G)  # a different order gives a different result
    for n in (2, 1, 0):
        c.mode_step(idx, x, n, 0.05, 0.01)
    c.core_step(idx, x, 0.04, 0.02)
    assert not np.allclose(c.flatA, a.flatA)


# ----------------------------------------------------------------------------
# special cases with closed forms
# ----------------------------------------------------------------------------
def test_matrix_factorisation_exact(oracle_mod):
    """N = 2, G = identity, gamma_G = 0, M = 1: the method is matrix-factorisation
    SGD (x_hat = u_i . v_j; u <- u + g (r v - l u); then v <- v + g (r' u - l v)
    with the residual r' recomputed from the new u, the Gauss-Seidel order of
    Algorithm 1).  Checked against exact rational arithmetic on three entries."""
    F = Fraction
    U = [[F(1, 2), F(1, 4)], [F(-1, 3), F(1, 5)]]
    V = [[F(1, 3), F(-1, 2)], [F(2, 5), F(1, 7)]]
    entries = [(0, 1, F(3, 4)), (1, 0, F(-1, 2)), (0, 0, F(5, 4))]
    g, l = F(1, 10), F(1, 20)
    for i, j, xv in entries:
        r = xv - sum(U[i][k] * V[j][k] for k in range(2))
        U[i] = [U[i][k] + g * (r * V[j][k] - l * U[i][k]) for k in range(2)]
        r = xv - sum(U[i][k] * V[j][k] for k in range(2))
        V[j] = [V[j][k] + g * (r * U[i][k] - l * V[j][k]) for k in range(2)]
    A0 = [np.array([[0.5, 0.25], [-1 / 3, 0.2]]), np.array([[1 / 3, -0.5], [0.4, 1 / 7]])]
    mod = oracle_mod.Model((2, 2), (2, 2), A0, np.array([1.0, 0.0, 0.0, 1.0]))
    idx = np.array([[e[0] for e in entries], [e[1] for e in entries]], np.int32)
    vals = np.array([float(e[2]) for e in entries], np.float32)  # exact in binary32
    perm = np.arange(3, dtype=np.int64)
    mod.run(idx, vals, M=1, gam_A=0.1, lam_A=0.05, gam_G=0.0, lam_G=0.0, perm=perm, n_epochs=1)
    np.testing.assert_allclose(mod.A[0], np.array(U, dtype=float), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mod.A[1], np.array(V, dtype=float), rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(mod.G, [1.0, 0.0, 0.0, 1.0])


def test_core_full_batch_converges_to_ridge(oracle_mod):
    """gamma_A = 0, M = T: repeated core steps converge to the ridge solution
    g* = (H^T H / T + lambda I)^-1 H^T x / T, with H_p = a(N) x ... x a(1)."""
    dims, ranks = (6, 5, 4), (2, 3, 2)
    rng = np.random.default_rng(9)
    A, G = random_model(rng, dims, ranks)
    T = 60
    idx = np.stack([rng.integers(0, I, T) for I in dims]).astype(np.int32)
    x = rng.standard_normal(T).astype(np.float32)
    H = np.stack([np.kron(np.kron(A[2][idx[2, p]], A[1][idx[1, p]]), A[0][idx[0, p]]) for p in range(T)])
    lam = 0.1
    g_star = np.linalg.solve(H.T @ H / T + lam * np.eye(H.shape[1]), H.T @ x.astype(np.float64) / T)
    L = np.linalg.eigvalsh(H.T @ H / T).max() + lam
    mod = oracle_mod.Model(dims, ranks, A, G)
    mod.run(idx, x, M=T, gam_A=0.0, lam_A=0.0, gam_G=1.0 / L, lam_G=lam,
            perm=np.tile(np.arange(T, dtype=np.int64), 3000), n_epochs=3000)
    np.testing.assert_allclose(mod.G, g_star, rtol=1e-8, atol=1e-10)
    np.testing.assert_array_equal(mod.flatA, np.concatenate([a.reshape(-1) for a in A]))


def test_full_batch_descent(oracle_mod):
    """lambda = 0, M = T, small steps: every sub-step is a gradient step on a
    convex quadratic block, so the training SSE never increases."""
    dims, ranks = (8, 7, 6), (2, 2, 2)
    rng = np.random.default_rng(11)
    A, G = random_model(rng, dims, ranks, scale=0.5)
    T = 80
    idx = np.stack([rng.integers(0, I, T) for I in dims]).astype(np.int32)
    x = rng.standard_normal(T).astype(np.float32)
    mod = oracle_mod.Model(dims, ranks, A, G)
    prev = mod.loss(idx, x)["sse"]
    start = prev
    for _ in range(60):
        mod.core_step(idx, x, 0.05, 0.0)
        cur = mod.loss(idx, x)["sse"]
        assert cur <= prev + 1e-12
        prev = cur
        for n in range(3):
            mod.mode_step(idx, x, n, 0.05, 0.0)
            cur = mod.loss(idx, x)["sse"]
            assert cur <= prev + 1e-12
            prev = cur
    assert prev < 0.97 * start


def test_planted_model_residuals_are_the_noise(oracle_mod):
    """With the parameters set to the planted model, every residual is the
    injected noise (up to the float32 rounding of the stored values), and a
    step with lambda = 0 on noise-free planted data leaves the model in place."""
    wl = synth.planted_uniform(dims=(60, 50, 40), ranks=(3, 4, 2), nnz=4000, sigma=0.01, seed=77)
    A, G = wl.planted
    mod = oracle_mod.Model(wl.dims, wl.ranks, A, G)
    r = wl.train_vals.astype(np.float64) - mod.predict(wl.train_idx)
    # the stored float32 values carry at most half an ulp of rounding
    half_ulp = np.spacing(np.abs(wl.train_vals)).astype(np.float64) / 2
    assert np.all(np.abs(r - wl.noise.astype(np.float64)) <= half_ulp + 1e-12)
    assert mod.loss(wl.train_idx, wl.train_vals)["rmse"] == pytest.approx(
        np.sqrt(np.mean(wl.noise.astype(np.float64) ** 2)), rel=1e-4)
    clean = synth.planted_uniform(dims=(60, 50, 40), ranks=(3, 4, 2), nnz=4000, sigma=0.0, seed=77)
    mod = oracle_mod.Model(clean.dims, clean.ranks, *clean.planted)
    mod.run(clean.train_idx, clean.train_vals, M=64, gam_A=0.05, lam_A=0.0, gam_G=0.05, lam_G=0.0,
            seed=5, n_epochs=1)
    np.testing.assert_allclose(mod.G, clean.planted[1], atol=1e-6)
    for a, b in zip(mod.A, clean.planted[0]):
        np.testing.assert_allclose(a, b, atol=1e-6)


def test_run_uses_sampler_and_ragged_last_batch(oracle_mod):
    """orc_run with its own sampler equals orc_run given pi_e explicitly, and an
    epoch of T entries has ceil(T/M) minibatches, the last one shorter."""
    dims, ranks = (9, 8, 7), (2, 2, 3)
    rng = np.random.default_rng(12)
    A, G = random_model(rng, dims, ranks)
    T, M = 103, 16
    idx = np.stack([rng.integers(0, I, T) for I in dims]).astype(np.int32)
    x = rng.standard_normal(T).astype(np.float32)
    a = oracle_mod.Model(dims, ranks, A, G)
    nb = a.run(idx, x, M, 0.05, 0.01, 0.05, 0.01, seed=42, epoch0=3, n_epochs=2)
    assert nb == 2 * 7
    b = oracle_mod.Model(dims, ranks, A, G)
    perm = np.concatenate([oracle_mod.perm(T, 42, 3), oracle_mod.perm(T, 42, 4)])
    b.run(idx, x, M, 0.05, 0.01, 0.05, 0.01, perm=perm, n_epochs=2)
    np.testing.assert_array_equal(a.flatA, b.flatA)
    np.testing.assert_array_equal(a.G, b.G)
    # the last minibatch of an epoch holds the remaining 103 - 6*16 = 7 entries
    c = oracle_mod.Model(dims, ranks, A, G)
    c.run(idx, x, M, 0.05, 0.01, 0.05, 0.01, perm=perm[:T], n_epochs=1, max_batches=6)
    order = perm[:T]
    tail = order[96:]
    c.step(idx[:, tail], x[tail], 0.05, 0.01, 0.05, 0.01)
    b1 = oracle_mod.Model(dims, ranks, A, G)
    b1.run(idx, x, M, 0.05, 0.01, 0.05, 0.01, perm=perm[:T], n_epochs=1)
    np.testing.assert_array_equal(c.flatA, b1.flatA)


def test_planted_convergence_to_noise_floor(oracle_mod):
    """Planted rank-(3,3,3) tensor with noise sigma = 0.01: from a random
    initialisation the held-out RMSE falls to the noise floor (the planted
    model is recoverable, so the minimum of the expected loss is sigma).  The
    epoch count and the 1.5*sigma bound are calibrated on the oracle: no
    number in the paper fixes the curve."""
    wl = synth.planted_uniform(dims=(100, 100, 100), ranks=(3, 3, 3), nnz=60_000, sigma=0.01, seed=21)
    A0, G0 = synth.init_params(wl.dims, wl.ranks, seed=2001)
    mod = oracle_mod.Model(wl.dims, wl.ranks, A0, G0)
    r0 = mod.loss(wl.test_idx, wl.test_vals)["rmse"]
    mod.run(wl.train_idx, wl.train_vals, M=32, gam_A=0.05, lam_A=0.001, gam_G=0.05, lam_G=0.001,
            seed=3001, n_epochs=20)
    r1 = mod.loss(wl.test_idx, wl.test_vals)["rmse"]
    assert r0 > 0.5
    assert r1 < 1.5 * 0.01
