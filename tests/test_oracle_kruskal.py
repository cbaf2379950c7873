"""Pins of the oracle's Kruskal-core sub-step against what the paper and the
mathematics fix (Section "Optimization Process for the Core Tensor": Eqs.
CP-Decomposition, eventual0, Q_r, eventual1, eventual_approximated,
SGD_core_tensor and Gradient_core_tensor; Algorithm 1, core loop).

None of them re-types the oracle's construction (explicit H_Psi, Khatri-Rao
column, block matrix O_r, W_r = H_Psi O_r): they use the definition of the
Kruskal product through numpy outer products, the closed form of W_r, central
finite differences of the B-parametrised objective, exact rational arithmetic
on a case that reduces to matrix-factorisation SGD, a planted fixed point and
full-batch descent.
"""
from fractions import Fraction

import numpy as np
import pytest

from tests.test_oracle_pins import _fd, einsum_predict


def random_kruskal(rng, dims, ranks, R, scale=0.7):
    A = [rng.standard_normal((I, J)) * scale for I, J in zip(dims, ranks)]
    B = [rng.standard_normal((J, R)) * scale for J in ranks]
    return A, B


def outer_core(B):
    """sum_r b(1)_r o ... o b(N)_r (the definition), flattened with j_0 fastest."""
    N = len(B)
    letters = "abcdefgh"[:N]
    spec = ",".join(l + "z" for l in letters) + "->" + letters
    return np.einsum(spec, *B).reshape(-1, order="F")


def tiny_batch(rng, dims, m):
    idx = np.stack([rng.integers(0, I, m) for I in dims]).astype(np.int32)
    x = rng.standard_normal(m).astype(np.float32)
    return idx, x


@pytest.mark.parametrize("ranks,R", [((2, 3, 4), 2), ((3, 2, 2, 3), 3), ((4, 5), 1)])
def test_kruskal_core_is_sum_of_outer_products(oracle_mod, ranks, R):
    """Eq. CP-Decomposition: G = sum_r b(1)_r o ... o b(N)_r (flat, j_0 fastest)."""
    rng = np.random.default_rng(21)
    B = [rng.standard_normal((J, R)) for J in ranks]
    np.testing.assert_allclose(oracle_mod.kruskal_core(ranks, B), outer_core(B), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("dims,ranks,R", [((5, 4, 6), (2, 3, 2), 3), ((4, 3, 5, 3), (2, 2, 3, 2), 2)])
def test_W_closed_form_and_prediction(oracle_mod, dims, ranks, R):
    """W_r = H_Psi O_r (Algorithm 1, core loop; Eq. Q_r) has the closed form
    W_r[s, j] = a(n)_s[j] * prod_{k != n} (a(k)_s . b(k)_r), and
    sum_r W_r b(n)_r is the STD prediction with the Kruskal core, for every n."""
    rng = np.random.default_rng(22)
    A, B = random_kruskal(rng, dims, ranks, R)
    mod = oracle_mod.KruskalModel(dims, ranks, A, B)
    idx, x = tiny_batch(rng, dims, 7)
    want_pred = einsum_predict(A, outer_core(B), ranks, idx)
    for n in range(len(dims)):
        pred = np.zeros(idx.shape[1])
        for r in range(R):
            W = mod.W(idx, n, r)
            z = np.ones(idx.shape[1])
            for k in range(len(dims)):
                if k != n:
                    z *= A[k][idx[k]] @ B[k][:, r]
            np.testing.assert_allclose(W, A[n][idx[n]] * z[:, None], rtol=1e-13, atol=1e-14)
            pred += W @ B[n][:, r]
        np.testing.assert_allclose(pred, want_pred, rtol=1e-12, atol=1e-13)


def kruskal_objective(A, B, ranks, idx, x, n, r, lam):
    def f(b):
        B2 = [t.copy() for t in B]
        B2[n][:, r] = b
        res = x.astype(np.float64) - einsum_predict(A, outer_core(B2), ranks, idx)
        return 0.5 * np.mean(res ** 2) + 0.5 * lam * np.sum(b ** 2)
    return f


@pytest.mark.parametrize("dims,ranks,R,n,r", [((5, 4, 6), (2, 3, 2), 3, 0, 1), ((5, 4, 6), (2, 3, 2), 3, 2, 2),
                                              ((4, 3, 5, 3), (2, 2, 3, 2), 2, 1, 0),
                                              ((4, 3, 5, 3), (2, 2, 3, 2), 2, 3, 1)])
def test_column_step_is_gradient(oracle_mod, dims, ranks, R, n, r):
    """One block step on column r of B(n) moves it by gamma_B times the
    gradient of (1/2m) sum_s (x_s - x_hat_s(B))^2 + (lambda_B/2)||b||^2
    (Eq. eventual_approximated with the averaged SGD of Eq. SGD_core_tensor
    and the gradient of Eq. Gradient_core_tensor): pins 1/m, lambda, the sign,
    the 1/2 convention and that the residual uses every current column."""
    rng = np.random.default_rng(23 + n + r)
    A, B = random_kruskal(rng, dims, ranks, R)
    idx, x = tiny_batch(rng, dims, 9)
    lam, gam = 0.29, 0.04
    grad = _fd(kruskal_objective(A, B, ranks, idx, x, n, r, lam), B[n][:, r].copy())
    mod = oracle_mod.KruskalModel(dims, ranks, A, B)
    mod.column_step(idx, x, n, r, gam, lam)
    np.testing.assert_allclose((B[n][:, r] - mod.B[n][:, r]) / gam, grad, rtol=1e-7, atol=1e-8)
    for k in range(len(dims)):  # nothing else moves
        for c in range(R):
            if (k, c) != (n, r):
                np.testing.assert_array_equal(mod.B[k][:, c], B[k][:, c])
    np.testing.assert_allclose(mod.G, outer_core(mod.B), rtol=1e-14, atol=1e-14)


def test_core_step_is_cyclic_over_modes_then_columns(oracle_mod):
    """The Kruskal core sub-step is the block steps for n = 1..N and, within
    each mode, the columns r = 1..R in order, each from the parameters the
    previous ones left (Algorithm 1, core loop); then G is formed (Eq.
    CP-Decomposition).  Another order gives another result."""
    dims, ranks, R = (5, 4, 6), (2, 3, 2), 3
    rng = np.random.default_rng(24)
    A, B = random_kruskal(rng, dims, ranks, R)
    idx, x = tiny_batch(rng, dims, 10)
    a = oracle_mod.KruskalModel(dims, ranks, A, B)
    a.kruskal_core_step(idx, x, 0.05, 0.02)
    b = oracle_mod.KruskalModel(dims, ranks, A, B)
    for n in range(3):
        for r in range(R):
            b.column_step(idx, x, n, r, 0.05, 0.02)
    np.testing.assert_array_equal(a.flatB, b.flatB)
    np.testing.assert_allclose(a.G, outer_core(a.B), rtol=1e-14, atol=1e-14)
    c = oracle_mod.KruskalModel(dims, ranks, A, B)
    for n in (2, 1, 0):
        for r in range(R):
            c.column_step(idx, x, n, r, 0.05, 0.02)
    assert not np.allclose(c.flatB, a.flatB)
    np.testing.assert_array_equal(a.flatA, np.concatenate([t.reshape(-1) for t in A]))


def test_matrix_factorisation_exact_kruskal(oracle_mod):
    """N = 2, A(1) = A(2) = identity, gamma_A = 0: the prediction of entry
    (i, j) is sum_r B(1)[i, r] B(2)[j, r], and the Kruskal core sub-step is
    cyclic matrix-factorisation SGD on B(1) then B(2), one column at a time,
    with the minibatch-averaged gradient and the residual of the current
    columns.  Checked against exact rational arithmetic on a 3-entry batch."""
    F = Fraction
    B1 = [[F(1, 2), F(-1, 3)], [F(1, 4), F(2, 5)]]
    B2 = [[F(1, 3), F(1, 7)], [F(-1, 2), F(1, 5)]]
    entries = [(0, 1, F(3, 4)), (1, 0, F(-1, 2)), (1, 1, F(5, 4))]
    g, l, m = F(1, 10), F(1, 20), 3

    def pred(i, j):
        return sum(B1[i][r] * B2[j][r] for r in range(2))

    for r in range(2):  # mode 1
        res = [xv - pred(i, j) for i, j, xv in entries]
        grad = [-sum(res[s] * B2[entries[s][1]][r] for s in range(m) if entries[s][0] == a) / m + l * B1[a][r]
                for a in range(2)]
        for a in range(2):
            B1[a][r] -= g * grad[a]
    for r in range(2):  # mode 2
        res = [xv - pred(i, j) for i, j, xv in entries]
        grad = [-sum(res[s] * B1[entries[s][0]][r] for s in range(m) if entries[s][1] == a) / m + l * B2[a][r]
                for a in range(2)]
        for a in range(2):
            B2[a][r] -= g * grad[a]
    B0 = [np.array([[0.5, -1 / 3], [0.25, 0.4]]), np.array([[1 / 3, 1 / 7], [-0.5, 0.2]])]
    mod = oracle_mod.KruskalModel((2, 2), (2, 2), [np.eye(2), np.eye(2)], B0)
    idx = np.array([[e[0] for e in entries], [e[1] for e in entries]], np.int32)
    vals = np.array([float(e[2]) for e in entries], np.float32)  # exact in binary32
    mod.run(idx, vals, M=3, gam_A=0.0, lam_A=0.0, gam_G=0.1, lam_G=0.05, perm=np.arange(3, dtype=np.int64),
            n_epochs=1)
    np.testing.assert_allclose(mod.B[0], np.array(B1, dtype=float), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mod.B[1], np.array(B2, dtype=float), rtol=1e-14, atol=1e-15)
    G = [[sum(B1[i][r] * B2[j][r] for r in range(2)) for i in range(2)] for j in range(2)]  # G[j][i]: j_0 = i fastest
    np.testing.assert_allclose(mod.G, np.array(G, dtype=float).reshape(-1), rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(mod.A[0], np.eye(2))


def test_planted_kruskal_model_is_fixed_point(oracle_mod):
    """Noise-free entries of a Kruskal-core model and lambda = 0: every
    residual is zero, so the core sub-step leaves B where it is."""
    dims, ranks, R = (6, 5, 4), (2, 3, 2), 2
    rng = np.random.default_rng(25)
    A, B = random_kruskal(rng, dims, ranks, R)
    idx, _ = tiny_batch(rng, dims, 40)
    x = einsum_predict(A, outer_core(B), ranks, idx)
    mod = oracle_mod.KruskalModel(dims, ranks, A, B)
    # values exactly representable: use the float32 rounding and compare the move to its size
    x32 = x.astype(np.float32)
    mod.kruskal_core_step(idx, x32, 0.1, 0.0)
    err = float(np.max(np.abs(x32.astype(np.float64) - x)))
    np.testing.assert_allclose(mod.flatB, np.concatenate([b.reshape(-1) for b in B]), rtol=0, atol=10 * err + 1e-15)


def test_full_batch_descent_kruskal(oracle_mod):
    """lambda = 0, the whole set as one minibatch, small steps: each column
    step is a gradient step on a convex quadratic of that column, so the
    training SSE never increases."""
    dims, ranks, R = (7, 6, 5), (2, 3, 2), 3
    rng = np.random.default_rng(26)
    A, B = random_kruskal(rng, dims, ranks, R, scale=0.6)
    idx, x = tiny_batch(rng, dims, 60)
    mod = oracle_mod.KruskalModel(dims, ranks, A, B)
    prev = start = mod.loss(idx, x)["sse"]
    for _ in range(30):
        for n in range(3):
            for r in range(R):
                mod.column_step(idx, x, n, r, 0.05, 0.0)
                cur = mod.loss(idx, x)["sse"]
                assert cur <= prev + 1e-12
                prev = cur
    assert prev < 0.97 * start


def test_kruskal_step_then_factor_steps(oracle_mod):
    """A minibatch with the Kruskal core is its core sub-step, then the factor
    sub-steps of modes 1..N with the core that sub-step formed (Algorithm 1)."""
    dims, ranks, R = (5, 4, 6), (2, 3, 2), 2
    rng = np.random.default_rng(27)
    A, B = random_kruskal(rng, dims, ranks, R)
    idx, x = tiny_batch(rng, dims, 10)
    a = oracle_mod.KruskalModel(dims, ranks, A, B)
    a.step(idx, x, 0.05, 0.01, 0.04, 0.02)
    b = oracle_mod.KruskalModel(dims, ranks, A, B)
    b.kruskal_core_step(idx, x, 0.04, 0.02)
    for n in range(3):
        b.mode_step(idx, x, n, 0.05, 0.01)
    np.testing.assert_array_equal(a.flatA, b.flatA)
    np.testing.assert_array_equal(a.flatB, b.flatB)
    np.testing.assert_array_equal(a.G, b.G)
