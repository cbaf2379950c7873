"""The Kruskal core on the GPU (options.r_core = R > 0) against the FP64
oracle's Kruskal sub-step (oracle.KruskalModel; Section "Optimization Process
for the Core Tensor", Eqs. CP-Decomposition, eventual_approximated and
Gradient_core_tensor; Algorithm 1, core loop), through the C ABI.

The GPU forms, per mode, the Gram matrix of [W_0 .. W_{R-1} | x] and takes
the column steps on it; the oracle forms W_r = H_Psi O_r explicitly and takes
each column step on the samples.  The two agree in exact arithmetic; FP32
results must match to the FP32 bar: per epoch from a common state, relative
Frobenius error <= 1e-5 for every A(n), every B(n) and the core, and every
row after one and two minibatches to 1e-6 absolute.
"""
import numpy as np
import pytest

from paper_2012_03550_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
BF16_TOL = 2.5e-3


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_03550_amd import binding
    binding.load()
    return binding


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    n = np.linalg.norm(b.ravel())
    d = np.linalg.norm((a - b).ravel())
    return d / n if n > 0 else d


def init_kruskal(dims, ranks, R, seed):
    rng = np.random.default_rng(seed)
    A = [(rng.standard_normal((I, J)) / np.sqrt(J)).astype(np.float32) for I, J in zip(dims, ranks)]
    sd = (1.0 / (R * ranks[0])) ** (0.5 / len(dims))
    B = [(rng.standard_normal((J, R)) * sd).astype(np.float32) for J in ranks]
    return A, B


def make(lib, dims, ranks, R, idx, vals, A0, B0, M, chunk, lr, lam, seed=55, dtype="f32"):
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=M, lr_factor=lr, lr_core=lr, lam_factor=lam, lam_core=lam,
                     seed_sample=seed, init="caller", chunk=chunk, r_core=R, dtype=dtype)
    G0 = np.zeros(int(np.prod(ranks)), np.float32)
    h.set_params(A0, G0)
    h.set_kruskal(B0)
    return h


def test_kruskal_params_and_predict(lib, oracle_mod):
    """set_kruskal / get_kruskal round-trip B bit for bit; the core becomes
    their Kruskal product (predictions match the oracle's)."""
    dims, ranks, R = (40, 30, 20), (4, 3, 5), 3
    idx, vals = synth.random_tiny(3, dims, ranks, 2000, seed=1)
    A, B = init_kruskal(dims, ranks, R, 2)
    h = make(lib, dims, ranks, R, idx, vals, A, B, 64, 16, 0.01, 0.01)
    for b, b2 in zip(B, h.get_kruskal()):
        np.testing.assert_array_equal(b, b2)
    ref = oracle_mod.KruskalModel(dims, ranks, [a.astype(np.float64) for a in A], [b.astype(np.float64) for b in B])
    _, G = h.get_params()
    assert rel(G, ref.G) <= 1e-6
    q = idx[:, :500]
    want = ref.predict(q)
    assert np.max(np.abs(h.predict(q) - want)) <= 1e-5 * np.sqrt(np.mean(want ** 2))
    h.close()
    dense = lib.Stdecomp(dims, ranks, idx, vals, batch=64)
    with pytest.raises(lib.StdecompError) as ei:
        dense.get_kruskal()
    assert ei.value.code == lib.STD_E_STATE
    dense.close()


KR_CASES = [
    # name, dims, ranks, R, nnz, M, chunk, skew
    ("n3_r1_w1", (60, 50, 40), (3, 3, 3), 1, 3000, 64, 64, None),
    ("n3_r3_mixed_w4", (60, 50, 40), (2, 3, 4), 3, 3000, 128, 32, 1.2),
    ("n3_j5_r5_w8_ragged", (200, 150, 100), (5, 5, 5), 5, 9001, 512, 64, 1.1),
    ("n2_r2_w2", (80, 70), (4, 4), 2, 4000, 128, 64, None),
    ("n4_r2_w4", (30, 25, 20, 15), (3, 3, 3, 3), 2, 5000, 256, 64, None),
    ("n4_j8_r8_w16", (60, 50, 30, 20), (8, 8, 8, 8), 8, 12000, 1024, 64, 1.2),
    ("n3_j5_r10_w4", (100, 90, 80), (5, 5, 5), 10, 6000, 256, 64, None),
]


@pytest.mark.parametrize("case", KR_CASES, ids=[c[0] for c in KR_CASES])
def test_kruskal_epochs_match_oracle(lib, oracle_mod, case):
    name, dims, ranks, R, nnz, M, chunk, skew = case
    idx, vals = synth.random_tiny(len(dims), dims, ranks, nnz, seed=len(name) + 7, skew=skew)
    vals = (vals * 0.5).astype(np.float32)
    A0, B0 = init_kruskal(dims, ranks, R, len(name))
    lr, lam, seed = 0.02, 0.01, 55
    h = make(lib, dims, ranks, R, idx, vals, A0, B0, M, chunk, lr, lam, seed)
    say(name, "chain", h.info())
    As, Bs = A0, B0
    for e in range(2):
        h.epoch(1)
        Ag, Gg = h.get_params()
        Bg = h.get_kruskal()
        ref = oracle_mod.KruskalModel(dims, ranks, [a.astype(np.float64) for a in As],
                                      [b.astype(np.float64) for b in Bs])
        ref.run(idx, vals, M, lr, lam, lr, lam, seed=seed, epoch0=e, n_epochs=1)
        errs = [rel(Ag[n], ref.A[n]) for n in range(len(dims))] + [rel(Bg[n], ref.B[n]) for n in range(len(dims))]
        errs.append(rel(Gg, ref.G))
        say(name, "epoch", e, "rel errors A..., B..., G:", ["%.2e" % x for x in errs])
        assert max(errs) <= TOL, (name, e, errs)
        As, Bs = Ag, Bg
    h.close()


@pytest.mark.parametrize("dims,ranks,R,chunk", [((200, 150, 100), (4, 4, 4), 4, 32),
                                                ((60, 50, 30, 20), (8, 8, 8, 8), 8, 64)])
def test_kruskal_rows_after_minibatches(lib, oracle_mod, dims, ranks, R, chunk):
    """Every parameter after one and two minibatches, to 1e-6 absolute."""
    idx, vals = synth.random_tiny(len(dims), dims, ranks, 20000, seed=9, skew=1.2)
    A0, B0 = init_kruskal(dims, ranks, R, 9)
    for nb in (1, 2):
        ref = oracle_mod.KruskalModel(dims, ranks, [a.astype(np.float64) for a in A0],
                                      [b.astype(np.float64) for b in B0])
        ref.run(idx, vals, 512, 0.01, 0.01, 0.01, 0.01, seed=77, epoch0=0, n_epochs=1, max_batches=nb)
        h = make(lib, dims, ranks, R, idx, vals, A0, B0, 512, chunk, 0.01, 0.01, seed=77)
        h.run_minibatches(0, 0, nb)
        A, G = h.get_params()
        B = h.get_kruskal()
        h.close()
        errs = ([float(np.max(np.abs(a - r))) for a, r in zip(A, ref.A)] +
                [float(np.max(np.abs(b - r))) for b, r in zip(B, ref.B)] + [float(np.max(np.abs(G - ref.G)))])
        say("kruskal rows", dims, "R", R, "minibatches", nb, "max abs errors", ["%.1e" % x for x in errs])
        assert max(errs) <= 1e-6, errs


def test_kruskal_bf16_close_to_oracle(lib, oracle_mod):
    dims, ranks, R = (200, 150, 100), (5, 5, 5), 5
    idx, vals = synth.random_tiny(3, dims, ranks, 9001, seed=31, skew=1.1)
    vals = (vals * 0.5).astype(np.float32)
    A0, B0 = init_kruskal(dims, ranks, R, 32)
    h = make(lib, dims, ranks, R, idx, vals, A0, B0, 512, 64, 0.02, 0.01, dtype="bf16")
    h.epoch(1)
    Ag, Gg = h.get_params()
    Bg = h.get_kruskal()
    ref = oracle_mod.KruskalModel(dims, ranks, [a.astype(np.float64) for a in A0], [b.astype(np.float64) for b in B0])
    ref.run(idx, vals, 512, 0.02, 0.01, 0.02, 0.01, seed=55, epoch0=0, n_epochs=1)
    errs = [rel(Ag[n], ref.A[n]) for n in range(3)] + [rel(Bg[n], ref.B[n]) for n in range(3)] + [rel(Gg, ref.G)]
    say("kruskal bf16 rel errors", ["%.2e" % x for x in errs])
    assert max(errs) <= BF16_TOL, errs
    h.close()


def test_kruskal_planted_converges(lib, oracle_mod):
    """A planted model whose core is a Kruskal product of rank 3 (100^3,
    J = 3, core entries of variance 1/J, 60k entries, noise 0.01, 10% held
    out), fitted with R = 3, M = 32, lr = 0.05, lambda = 1e-4 for 20 epochs
    (the scaled initialisation sits near the zero model, which both runs
    leave after about eight epochs).  Both the GPU and the free-running
    oracle must bring the held-out RMSE below 60% of the data RMS, and end
    within 1% of each other: a free run through that escape amplifies
    rounding differences, so the parity gate is the per-epoch comparison
    above, and this test checks that the GPU trajectory reaches the oracle's
    fit (parity of the converged value is unpinned by the paper)."""
    rng = np.random.default_rng(41)
    dims, ranks, R = (100, 100, 100), (3, 3, 3), 3
    Ap = [rng.standard_normal((I, J)) / np.sqrt(J) for I, J in zip(dims, ranks)]
    Bp = [rng.standard_normal((J, R)) * (1.0 / (R * 3)) ** (1.0 / 6) for J in ranks]
    Gp = oracle_mod.kruskal_core(ranks, Bp)
    T = 60000
    idx = np.stack([rng.integers(0, I, T) for I in dims]).astype(np.int32)
    vals = (synth.evaluate_planted(Ap, Gp, ranks, idx) + 0.01 * rng.standard_normal(T)).astype(np.float32)
    tr, te = slice(0, 54000), slice(54000, T)
    A0, B0 = init_kruskal(dims, ranks, R, 42)
    lr, lam, M, E = 0.05, 1e-4, 32, 20
    h = make(lib, dims, ranks, R, idx[:, tr], vals[tr], A0, B0, M, 0, lr, lam, seed=43)
    h.epoch(E)
    rg = h.loss(idx[:, te], vals[te])["rmse"]
    h.close()
    ref = oracle_mod.KruskalModel(dims, ranks, [a.astype(np.float64) for a in A0], [b.astype(np.float64) for b in B0])
    ref.run(idx[:, tr], vals[tr], M, lr, lam, lr, lam, seed=43, epoch0=0, n_epochs=E)
    ro = ref.loss(idx[:, te], vals[te])["rmse"]
    rms = float(np.sqrt(np.mean(vals[te].astype(np.float64) ** 2)))
    say("kruskal planted: held-out RMSE GPU %.6f oracle %.6f (data RMS %.4f, relative gap %.2e)" %
        (rg, ro, rms, (rg - ro) / ro))
    assert ro < 0.6 * rms and rg < 0.6 * rms
    assert abs(rg - ro) <= 1e-2 * ro
