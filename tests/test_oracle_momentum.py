"""Pins of the oracle's heavy-ball momentum extension (orc_step_momentum).

The paper names momentum as a way to extend SGD_Tucker (Section "Conclusion
and Future Works") without fixing its form; the oracle's reading is Polyak's
heavy ball applied to each sub-step's stochastic gradient, v <- mu v + g,
theta <- theta - gamma v, with one velocity per factor row that changes only
when its row is sampled and one velocity for the core that changes once per
minibatch.  These tests pin that reading with exact rational arithmetic, the
reduction to the plain method at mu = 0, the fixed point of full-batch heavy
ball on the core objective, and the laziness of unsampled rows.
"""
from fractions import Fraction

import numpy as np


def random_model(rng, dims, ranks, scale=0.7):
    A = [rng.standard_normal((I, J)) * scale for I, J in zip(dims, ranks)]
    G = rng.standard_normal(int(np.prod(ranks))) * scale
    return A, G


def random_entries(rng, dims, T):
    idx = np.stack([rng.integers(0, I, T) for I in dims]).astype(np.int32)
    x = rng.standard_normal(T).astype(np.float32)
    return idx, x


def test_mu_zero_is_the_plain_method(oracle_mod):
    """mu = 0: every velocity equals the current gradient, so the iterates are
    those of the plain method bit for bit, over several epochs."""
    dims, ranks = (9, 7, 8), (3, 2, 4)
    rng = np.random.default_rng(21)
    A, G = random_model(rng, dims, ranks)
    idx, x = random_entries(rng, dims, 150)
    plain = oracle_mod.Model(dims, ranks, A, G)
    mom = oracle_mod.MomentumModel(dims, ranks, A, G)
    kw = dict(M=16, gam_A=0.05, lam_A=0.01, gam_G=0.03, lam_G=0.02, seed=5, n_epochs=3)
    plain.run(idx, x, **kw)
    mom.run(idx, x, mu=0.0, **kw)
    np.testing.assert_array_equal(mom.flatA, plain.flatA)
    np.testing.assert_array_equal(mom.G, plain.G)


def test_heavy_ball_matrix_factorisation_exact(oracle_mod):
    """N = 2, G = identity, gamma_G = 0, M = 1: heavy-ball matrix factorisation
    SGD.  For entry (i, j, x): r = x - u_i . v_j; w_i <- mu w_i + (-r v_j + l u_i);
    u_i <- u_i - g w_i; then r' from the new u_i, z_j <- mu z_j + (-r' u_i + l v_j);
    v_j <- v_j - g z_j.  Rows 0 of both modes are sampled twice, so their
    velocities carry over.  Checked against exact rational arithmetic."""
    F = Fraction
    U = [[F(1, 2), F(1, 4)], [F(-1, 3), F(1, 5)]]
    V = [[F(1, 3), F(-1, 2)], [F(2, 5), F(1, 7)]]
    WU = [[F(0)] * 2 for _ in range(2)]
    WV = [[F(0)] * 2 for _ in range(2)]
    entries = [(0, 1, F(3, 4)), (1, 0, F(-1, 2)), (0, 0, F(5, 4)), (1, 1, F(1, 4))]
    g, l, mu = F(1, 10), F(1, 20), F(3, 4)
    for i, j, xv in entries:
        r = xv - sum(U[i][k] * V[j][k] for k in range(2))
        WU[i] = [mu * WU[i][k] + (-r * V[j][k] + l * U[i][k]) for k in range(2)]
        U[i] = [U[i][k] - g * WU[i][k] for k in range(2)]
        r = xv - sum(U[i][k] * V[j][k] for k in range(2))
        WV[j] = [mu * WV[j][k] + (-r * U[i][k] + l * V[j][k]) for k in range(2)]
        V[j] = [V[j][k] - g * WV[j][k] for k in range(2)]
    A0 = [np.array([[0.5, 0.25], [-1 / 3, 0.2]]), np.array([[1 / 3, -0.5], [0.4, 1 / 7]])]
    mod = oracle_mod.MomentumModel((2, 2), (2, 2), A0, np.array([1.0, 0.0, 0.0, 1.0]))
    idx = np.array([[e[0] for e in entries], [e[1] for e in entries]], np.int32)
    vals = np.array([float(e[2]) for e in entries], np.float32)  # exact in binary32
    perm = np.arange(len(entries), dtype=np.int64)
    mod.run(idx, vals, M=1, gam_A=0.1, lam_A=0.05, gam_G=0.0, lam_G=0.0, perm=perm, mu=0.75)
    np.testing.assert_allclose(mod.A[0], np.array(U, dtype=float), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mod.A[1], np.array(V, dtype=float), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mod.VA[0], np.array(WU, dtype=float), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(mod.VA[1], np.array(WV, dtype=float), rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(mod.G, [1.0, 0.0, 0.0, 1.0])


def test_heavy_ball_core_exact(oracle_mod):
    """gamma_A = 0, N = 2, ranks (2, 2), minibatches of two entries: the core
    takes heavy-ball steps on f(G) = (1/2m) sum_p (x_p - u_{i_p}^T G v_{j_p})^2
    + (lambda/2)||G||^2, whose gradient is -(1/m) sum_p r_p u_{i_p} v_{j_p}^T
    + lambda G (Definition "Sparse Tucker Decomposition" with N = 2: the core is
    a matrix and the model is a bilinear form).  The core is flat with j_0
    fastest, so G[a, b] sits at a + 2 b.  Exact rational arithmetic."""
    F = Fraction
    U = [[F(1, 2), F(-1, 4)], [F(1, 3), F(2, 5)], [F(-3, 4), F(1, 8)]]
    V = [[F(1, 5), F(1, 2)], [F(-2, 3), F(1, 4)]]
    Gm = [[F(1, 4), F(-1, 2)], [F(1, 8), F(3, 4)]]          # Gm[a][b]
    W = [[F(0)] * 2 for _ in range(2)]
    entries = [(0, 1, F(1, 2)), (2, 0, F(-3, 4)), (1, 1, F(5, 8)), (0, 0, F(1, 4)),
               (2, 1, F(3, 2)), (1, 0, F(-1, 8))]
    g, lam, mu, m = F(1, 5), F(1, 10), F(1, 2), 2
    for b0 in range(0, len(entries), m):
        grad = [[lam * Gm[a][b] for b in range(2)] for a in range(2)]
        for i, j, xv in entries[b0:b0 + m]:
            xh = sum(U[i][a] * Gm[a][b] * V[j][b] for a in range(2) for b in range(2))
            r = xv - xh
            for a in range(2):
                for b in range(2):
                    grad[a][b] -= r * U[i][a] * V[j][b] / m
        W = [[mu * W[a][b] + grad[a][b] for b in range(2)] for a in range(2)]
        Gm = [[Gm[a][b] - g * W[a][b] for b in range(2)] for a in range(2)]
    A0 = [np.array(U, dtype=float), np.array(V, dtype=float)]
    G0 = np.array([0.25, 0.125, -0.5, 0.75])
    mod = oracle_mod.MomentumModel((3, 2), (2, 2), A0, G0)
    idx = np.array([[e[0] for e in entries], [e[1] for e in entries]], np.int32)
    vals = np.array([float(e[2]) for e in entries], np.float32)
    perm = np.arange(len(entries), dtype=np.int64)
    mod.run(idx, vals, M=m, gam_A=0.0, lam_A=0.0, gam_G=0.2, lam_G=0.1, perm=perm, mu=0.5)
    want_G = [float(Gm[a][b]) for b in range(2) for a in range(2)]
    want_W = [float(W[a][b]) for b in range(2) for a in range(2)]
    np.testing.assert_allclose(mod.G, want_G, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mod.VG, want_W, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(mod.A[0], A0[0], rtol=0, atol=0)


def test_core_heavy_ball_converges_to_ridge(oracle_mod):
    """gamma_A = 0, M = T, mu = 0.6: full-batch heavy ball on the strongly
    convex core objective converges (gamma = 1/L < 2(1 + mu)/L) to the same
    ridge solution g* = (H^T H / T + lambda I)^-1 H^T x / T as plain descent,
    and its velocity goes to zero."""
    dims, ranks = (6, 5, 4), (2, 3, 2)
    rng = np.random.default_rng(9)
    A, G = random_model(rng, dims, ranks)
    T = 60
    idx, x = random_entries(rng, dims, T)
    H = np.stack([np.kron(np.kron(A[2][idx[2, p]], A[1][idx[1, p]]), A[0][idx[0, p]]) for p in range(T)])
    lam = 0.1
    g_star = np.linalg.solve(H.T @ H / T + lam * np.eye(H.shape[1]), H.T @ x.astype(np.float64) / T)
    L = np.linalg.eigvalsh(H.T @ H / T).max() + lam
    mod = oracle_mod.MomentumModel(dims, ranks, A, G)
    mod.run(idx, x, M=T, gam_A=0.0, lam_A=0.0, gam_G=1.0 / L, lam_G=lam,
            perm=np.tile(np.arange(T, dtype=np.int64), 2000), n_epochs=2000, mu=0.6)
    np.testing.assert_allclose(mod.G, g_star, rtol=1e-8, atol=1e-10)
    assert np.abs(mod.VG).max() < 1e-9
    np.testing.assert_array_equal(mod.flatA, np.concatenate([a.reshape(-1) for a in A]))


def test_unsampled_rows_keep_row_and_velocity(oracle_mod):
    """Lazy rows: a factor row that no entry of the minibatches touches keeps
    both its parameters and its (nonzero) velocity, while every sampled row
    and the core move."""
    dims, ranks = (12, 10, 9), (2, 3, 2)
    rng = np.random.default_rng(33)
    A, G = random_model(rng, dims, ranks)
    VA = [rng.standard_normal(a.shape) for a in A]
    VG = rng.standard_normal(G.shape)
    T = 20
    idx = np.stack([rng.integers(0, I // 2, T) for I in dims]).astype(np.int32)  # upper halves never sampled
    x = rng.standard_normal(T).astype(np.float32)
    mod = oracle_mod.MomentumModel(dims, ranks, A, G, VA, VG)
    mod.run(idx, x, M=7, gam_A=0.05, lam_A=0.01, gam_G=0.05, lam_G=0.01, seed=2, mu=0.9)
    for n, I in enumerate(dims):
        sampled = np.zeros(I, bool)
        sampled[idx[n]] = True
        np.testing.assert_array_equal(mod.A[n][~sampled], A[n][~sampled])
        np.testing.assert_array_equal(mod.VA[n][~sampled], VA[n][~sampled])
        assert np.all(np.any(mod.A[n][sampled] != A[n][sampled], axis=1))
        assert np.all(np.any(mod.VA[n][sampled] != VA[n][sampled], axis=1))
    assert np.all(mod.VG != VG) and np.all(mod.G != G)


def test_momentum_rejects_bad_mu(oracle_mod):
    """mu outside [0, 1) is refused."""
    dims, ranks = (4, 4), (2, 2)
    rng = np.random.default_rng(1)
    A, G = random_model(rng, dims, ranks)
    idx, x = random_entries(rng, dims, 5)
    mod = oracle_mod.MomentumModel(dims, ranks, A, G)
    for mu in (-0.1, 1.0, float("nan")):
        try:
            mod.run(idx, x, M=2, gam_A=0.1, lam_A=0.0, gam_G=0.1, lam_G=0.0, mu=mu)
        except Exception:
            continue
        raise AssertionError(f"mu={mu} accepted")
