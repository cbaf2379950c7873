"""GPU path (libstdecomp through its C ABI) against the FP64 CPU oracle.

Integer work (sampler, sorted row sets, segments) must match bit for bit.
Floating-point results must match to the FP32 tolerance: per epoch, from a
common starting state, the relative Frobenius error of every factor matrix
and of the core, and the relative RMSE error, are at most 1e-5.
"""
import os
import sys

import numpy as np
import pytest

from paper_2012_03550_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


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
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def row_rel_max(A, ref):
    """max over rows i of ||A[i] - ref[i]|| / ||ref[i]|| (rows whose reference
    norm is below 1e-3 of the matrix's RMS row norm are measured against that
    floor instead).  A handful of wrong rows barely moves a Frobenius norm
    over thousands of rows; this catches them."""
    A = np.asarray(A, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.linalg.norm(A - ref, axis=1)
    n = np.linalg.norm(ref, axis=1)
    floor = 1e-3 * np.sqrt(np.mean(n ** 2)) if n.size else 0.0
    return float(np.max(d / np.maximum(n, max(floor, 1e-30)))) if n.size else 0.0


# Per-row bound for FP32 (each factor row against the FP64 oracle after one
# epoch from a common state): the FP32 bar itself, per row.  The rows seen
# stay below 1e-6; a row that missed or doubled an update is off by
# gamma * |gradient| / |row| ~ 1e-3 .. 1e-1.
ROW_REL_TOL = 1e-5


def oracle_epoch_errors(oracle_mod, dims, ranks, idx, vals, M, lr, lam, seed, epoch, A_start, G_start, Ag, Gg):
    """The oracle runs epoch `epoch` from (A_start, G_start); returns the
    relative Frobenius errors of (Ag, Gg) per factor and core, and the
    largest per-row relative error of the factors."""
    ref = oracle_mod.Model(dims, ranks, [a.astype(np.float64) for a in A_start], G_start.astype(np.float64))
    ref.run(idx, vals, M, lr, lam, lr, lam, seed=seed, epoch0=epoch, n_epochs=1)
    errs = [rel(Ag[n], ref.A[n]) for n in range(len(dims))] + [rel(Gg, ref.G)]
    rows = max(row_rel_max(Ag[n], ref.A[n]) for n in range(len(dims)))
    return errs, rows


def make_handle(lib, dims, ranks, idx, vals, A0, G0, M, lr=0.01, lam=0.01, lr_core=None, lam_core=None,
                seed=3001, chunk=0, dtype="f32"):
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=M, lr_factor=lr, lr_core=lr if lr_core is None else lr_core,
                     lam_factor=lam, lam_core=lam if lam_core is None else lam_core, seed_sample=seed,
                     init="caller", chunk=chunk, dtype=dtype)
    h.set_params(A0, G0)
    return h


def compare_epochs(lib, oracle_mod, name, dims, ranks, idx, vals, M, epochs, lr=0.01, lam=0.01, seed=3001,
                   chunk=0, init_seed=2001, test=None, tol=TOL, dtype="f32", rmse_tol=None):
    """Run `epochs` epochs on the GPU; after each, run the oracle for the same
    epoch from the GPU's starting state of that epoch and compare."""
    A0, G0 = synth.init_params(dims, ranks, seed=init_seed)
    say(name, "dims", dims, "ranks", ranks, "T", idx.shape[1], "M", M, "chunk", chunk)
    h = make_handle(lib, dims, ranks, idx, vals, A0, G0, M, lr, lam, seed=seed, chunk=chunk, dtype=dtype)
    info = h.info()
    say(name, "chain", info)
    free_run = oracle_mod.Model(dims, ranks, [a.astype(np.float64) for a in A0], G0.astype(np.float64))
    A_start, G_start = A0, G0
    worst = worst_row = 0.0
    for e in range(epochs):
        say(name, "epoch", e)
        h.epoch(1)
        Ag, Gg = h.get_params()
        errs, rows = oracle_epoch_errors(oracle_mod, dims, ranks, idx, vals, M, lr, lam, seed, e, A_start, G_start,
                                         Ag, Gg)
        worst = max(worst, max(errs))
        worst_row = max(worst_row, rows)
        say(name, "epoch", e, "rel errors", ["%.2e" % x for x in errs], "max row rel error %.2e" % rows)
        assert max(errs) <= tol, (name, e, errs)
        assert rows <= (ROW_REL_TOL if dtype == "f32" else BF16_ROW_TOL), (name, e, rows)
        if test is not None:
            rg = h.loss(test[0], test[1])["rmse"]
            ro = oracle_mod.Model(dims, ranks, [a.astype(np.float64) for a in Ag],
                                  Gg.astype(np.float64)).loss(test[0], test[1])["rmse"]
            assert abs(rg - ro) <= TOL * ro, (name, e, rg, ro)
        free_run.run(idx, vals, M, lr, lam, lr, lam, seed=seed, epoch0=e, n_epochs=1)
        A_start, G_start = Ag, Gg
    drift = max([rel(Ag[n], free_run.A[n]) for n in range(len(dims))] + [rel(Gg, free_run.G)])
    say(name, dtype, "worst per-epoch rel err %.3g (row %.3g), free-running drift after %d epochs %.3g" %
        (worst, worst_row, epochs, drift))
    gap = None
    if test is not None:
        rg = h.loss(test[0], test[1])["rmse"]
        ro = free_run.loss(test[0], test[1])["rmse"]
        gap = (rg - ro) / ro
        say(name, dtype, "held-out RMSE %.6f vs free-running FP64 oracle %.6f (relative gap %.3g)" % (rg, ro, gap))
        if rmse_tol is not None:
            assert abs(gap) <= rmse_tol, (name, rg, ro)
    h.close()
    return worst, drift, info


# ----------------------------------------------------------------- sampler
@pytest.mark.parametrize("T", [1, 2, 3, 17, 1000, 65537, 1 << 20, (1 << 20) + 1])
def test_sampler_bit_exact(lib, oracle_mod, T):
    for seed, epoch in ((0, 0), (3001, 5), (0xDEADBEEFCAFE, 123)):
        say("sampler T", T, "seed", seed, "epoch", epoch)
        np.testing.assert_array_equal(lib.sample_order(T, seed, epoch), oracle_mod.perm(T, seed, epoch))


def test_sampler_golden_vectors(lib):
    import json
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sampler_vectors.json")))
    for c in g["cases"]:
        say("sampler golden", c["T"], c["seed"], c["epoch"])
        p = lib.sample_order(c["T"], c["seed"], c["epoch"])
        assert p[: len(c["head"])].tolist() == c["head"]


# ------------------------------------------------------- schedule (integers)
@pytest.mark.parametrize("skew", [None, 1.2])
def test_schedule_bit_exact(lib, oracle_mod, skew):
    dims, ranks = (300, 50, 7), (3, 2, 2)
    idx, vals = synth.random_tiny(3, dims, ranks, 10_007, seed=5, skew=skew)
    M = 1000
    A0, G0 = synth.init_params(dims, ranks, seed=1)
    h = make_handle(lib, dims, ranks, idx, vals, A0, G0, M, seed=77, chunk=64)
    T = idx.shape[1]
    for epoch in (0, 3):
        order = oracle_mod.perm(T, 77, epoch)
        for b in (0, 4, T // M):  # includes the ragged last minibatch
            for mode in range(3):
                say("schedule skew", skew, "epoch", epoch, "batch", b, "mode", mode)
                got = h.debug_schedule(epoch, b, mode)
                ent = order[b * M: min((b + 1) * M, T)]
                np.testing.assert_array_equal(got["entries"], ent)
                sigma, off, segrow = oracle_mod.segments(idx[mode][ent])
                np.testing.assert_array_equal(got["sigma"], sigma)
                np.testing.assert_array_equal(got["seg_off"], off)
                np.testing.assert_array_equal(got["seg_row"], segrow)
    h.close()


# ---------------------------------------------------------- predict / loss
@pytest.mark.parametrize("dims,ranks", [((40, 30, 20), (4, 4, 4)), ((10, 12, 9, 8), (2, 3, 2, 3)),
                                        ((7, 6), (5, 7)), ((9, 8, 7, 6, 5), (2, 2, 2, 2, 2)),
                                        ((50, 40, 30), (10, 10, 10)), ((20, 20, 20), (16, 16, 16))])
def test_predict_and_loss(lib, oracle_mod, dims, ranks):
    say("predict", dims, ranks)
    rng = np.random.default_rng(3)
    A = [rng.standard_normal((I, J)).astype(np.float32) / np.sqrt(J) for I, J in zip(dims, ranks)]
    G = (rng.standard_normal(int(np.prod(ranks))) / np.sqrt(ranks[0])).astype(np.float32)
    idx, vals = synth.random_tiny(len(dims), dims, ranks, 5000, seed=4)
    h = make_handle(lib, dims, ranks, idx, vals, A, G, 64)
    ref = oracle_mod.Model(dims, ranks, [a.astype(np.float64) for a in A], G.astype(np.float64))
    q = np.stack([rng.integers(0, I, 3001) for I in dims]).astype(np.int32)
    got = h.predict(q)
    want = ref.predict(q)
    scale = np.sqrt(np.mean(want ** 2))
    assert np.max(np.abs(got - want)) <= 1e-5 * max(scale, 1e-3)
    lg, lo = h.loss(q, vals[:3001]), ref.loss(q, vals[:3001], lam_A=0.01, lam_G=0.01)
    for k in ("rmse", "mae", "sse", "objective"):
        assert abs(lg[k] - lo[k]) <= 1e-5 * abs(lo[k]), k
    tr = h.loss()
    assert tr["count"] == idx.shape[1]
    assert abs(tr["rmse"] - ref.loss(idx, vals)["rmse"]) <= 1e-5 * ref.loss(idx, vals)["rmse"]
    h.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("dims,ranks", [((7, 6), (5, 7)), ((10, 12, 9, 8), (2, 3, 2, 3)), ((40, 30, 20), (4, 4, 4)),
                                        ((3000, 50, 20), (6, 6, 6))])
def test_params_round_trip(lib, oracle_mod, dims, ranks, dtype):
    """set_params / get_params return the FP32 masters bit for bit (rows of
    J_n values stored at a padded stride), and a second set_params replaces
    the first everywhere (predictions follow the second set)."""
    say("params round trip", dims, ranks, dtype)
    rng = np.random.default_rng(11)
    idx, vals = synth.random_tiny(len(dims), dims, ranks, 2000, seed=6)
    sets = []
    for _ in range(2):
        A = [rng.standard_normal((I, J)).astype(np.float32) for I, J in zip(dims, ranks)]
        G = rng.standard_normal(int(np.prod(ranks))).astype(np.float32)
        sets.append((A, G))
    h = make_handle(lib, dims, ranks, idx, vals, sets[0][0], sets[0][1], 64, dtype=dtype)
    for A, G in sets:
        h.set_params(A, G)
        A1, G1 = h.get_params()
        assert all(np.array_equal(a, b) for a, b in zip(A, A1)) and np.array_equal(G, G1)
    A, G = sets[1]
    ref = oracle_mod.Model(dims, ranks, [a.astype(np.float64) for a in A], G.astype(np.float64))
    q = np.stack([rng.integers(0, I, 1001) for I in dims]).astype(np.int32)
    want = ref.predict(q)
    assert np.max(np.abs(h.predict(q) - want)) <= 1e-5 * max(np.sqrt(np.mean(want ** 2)), 1e-3)
    h.close()


def test_predict_rejects_bad_index(lib):
    say("predict bad index")
    dims, ranks = (10, 10, 10), (2, 2, 2)
    idx, vals = synth.random_tiny(3, dims, ranks, 100, seed=1)
    A0, G0 = synth.init_params(dims, ranks, seed=1)
    h = make_handle(lib, dims, ranks, idx, vals, A0, G0, 16)
    bad = np.array([[0, 1], [0, 10], [0, 1]], np.int32)
    with pytest.raises(lib.StdecompError) as ei:
        h.predict(bad)
    assert ei.value.code == lib.STD_E_INVAL
    h.close()


def test_init_rejects_bad_problem(lib):
    say("init bad problem")
    dims, ranks = (10, 10, 10), (2, 2, 2)
    idx, vals = synth.random_tiny(3, dims, ranks, 100, seed=1)
    idx[1, 5] = 10
    with pytest.raises(lib.StdecompError):
        lib.Stdecomp(dims, ranks, idx, vals, batch=16)
    idx[1, 5] = 0
    with pytest.raises(lib.StdecompError):
        lib.Stdecomp(dims, (2, 2, 33), idx, vals, batch=16)
    # a core that does not fit one workgroup's LDS: refused, with the reason
    with pytest.raises(lib.StdecompError) as ei:
        lib.Stdecomp((30, 30, 30), (24, 24, 24), idx, vals, batch=4096)
    assert "LDS" in str(ei.value), str(ei.value)
    with pytest.raises(lib.StdecompError):
        lib.Stdecomp(dims, ranks, idx, vals, batch=0)


# ------------------------------------------------------- the SGD epochs
CASES = [
    # name, dims, ranks, nnz, M, chunk, skew
    ("n3_mixed_generic_w4", (60, 50, 40), (2, 3, 4), 3000, 32, 8, None),
    ("n2_uniform_w1", (80, 70), (4, 4), 4000, 64, 0, None),
    ("n4_uniform_w8", (30, 25, 20, 15), (3, 3, 3, 3), 5000, 128, 16, None),
    ("n4_j8_tables_per_phase_w8", (60, 50, 30, 20), (8, 8, 8, 8), 12000, 1024, 128, 1.2),
    ("n4_j8_two_level_core_w16", (60, 50, 30, 20), (8, 8, 8, 8), 12000, 1024, 64, 1.2),
    ("n5_uniform", (12, 11, 10, 9, 8), (2, 2, 2, 2, 2), 3000, 64, 16, None),
    ("n3_zipf_long_runs_w8", (500, 400, 30), (4, 4, 4), 30000, 512, 64, 1.3),
    ("n3_j10_w4_ragged", (300, 200, 100), (10, 10, 10), 9001, 1024, 256, 1.1),
    ("n3_j16", (100, 90, 80), (16, 16, 16), 6000, 256, 64, None),
    ("n3_j5_chunk1", (50, 40, 30), (5, 5, 5), 700, 8, 1, 1.5),
    # the largest order (eight modes, the generic-order kernel with every mode loop at its bound)
    ("n8_j2_w4", (9, 8, 7, 6, 6, 5, 5, 4), (2, 2, 2, 2, 2, 2, 2, 2), 2000, 64, 16, 1.2),
    # an epoch shorter than one minibatch: a single ragged minibatch of 37 entries
    ("n3_one_ragged_minibatch", (30, 20, 10), (3, 4, 2), 37, 64, 16, None),
    # unequal ranks on four modes with the largest rank 16 (generic kernel, two-stage contraction)
    ("n4_unequal_j16_w8", (40, 30, 20, 10), (16, 4, 2, 3), 6000, 256, 32, 1.1),
    # rank 20: the generic-rank kernel; at M = 4096 the automatic chunk (64, 64
    # workgroups) leaves 88 floats of the workgroup's LDS unused
    ("n3_j20_w4", (100, 90, 80), (20, 20, 20), 6000, 256, 64, None),
    ("n3_j20_auto_m4096", (400, 300, 200), (20, 20, 20), 2 * 4096 + 100, 4096, 0, 1.2),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_epochs_match_oracle(lib, oracle_mod, case):
    name, dims, ranks, nnz, M, chunk, skew = case
    idx, vals = synth.random_tiny(len(dims), dims, ranks, nnz, seed=len(name), skew=skew)
    vals = (vals * 0.5).astype(np.float32)
    compare_epochs(lib, oracle_mod, name, dims, ranks, idx, vals, M, epochs=3, lr=0.02, lam=0.01, chunk=chunk)


# Chains of more than 64 workgroups: rows straddling chunk boundaries are
# finished by the grouped quad-DPP path (four and more modes) or by one thread
# per run in chunk order (three modes), not by the one-wave scan of W <= 64.
# The automatic chunk reaches these geometries on its own (four modes, J = 8,
# M = 16384: 128 workgroups of 128; three modes, J = 16, M = 8192: 128 of 64).
WIDE_CASES = [
    # name, dims, ranks, nnz, M, chunk, skew
    ("n4_j8_auto_m16384", (200, 150, 60, 40), (8, 8, 8, 8), 2 * 16384 + 777, 16384, 0, 1.2),
    ("n3_j16_auto_m8192", (400, 300, 200), (16, 16, 16), 2 * 8192 + 501, 8192, 0, 1.2),
    ("n3_j4_chunk64_m8192", (2000, 500, 50), (4, 4, 4), 3 * 8192 + 1000, 8192, 64, 1.3),
    ("n3_j5_chunk32_m8192", (3000, 100, 40), (5, 5, 5), 2 * 8192 + 33, 8192, 32, 1.4),
]


@pytest.mark.parametrize("case", WIDE_CASES, ids=[c[0] for c in WIDE_CASES])
def test_wide_chains_match_oracle(lib, oracle_mod, case):
    name, dims, ranks, nnz, M, chunk, skew = case
    idx, vals = synth.random_tiny(len(dims), dims, ranks, nnz, seed=len(name) + 100, skew=skew)
    vals = (vals * 0.5).astype(np.float32)
    _, _, info = compare_epochs(lib, oracle_mod, name, dims, ranks, idx, vals, M, epochs=2, lr=0.02, lam=0.01,
                                chunk=chunk)
    assert info["workgroups"] > 64, info


def test_planted_config_c1(lib, oracle_mod):
    """The small planted workload: 1000^3, 100k entries (10% held out), J = 5,
    M = 256, lr = lambda = 0.01, 10 epochs; per-epoch parameters and held-out
    RMSE against the oracle."""
    wl = synth.planted_uniform(seed=1001)
    compare_epochs(lib, oracle_mod, "c1", wl.dims, wl.ranks, wl.train_idx, wl.train_vals, 256, epochs=10,
                   lr=0.01, lam=0.01, test=(wl.test_idx, wl.test_vals))


def test_deterministic_and_resumable(lib):
    dims, ranks = (200, 150, 100), (4, 4, 4)
    idx, vals = synth.random_tiny(3, dims, ranks, 20000, seed=9, skew=1.2)
    A0, G0 = synth.init_params(dims, ranks, seed=9)
    say("determinism")
    runs = []
    for _ in range(2):
        h = make_handle(lib, dims, ranks, idx, vals, A0, G0, 512, chunk=64)
        h.epoch(2)
        runs.append(h.get_params())
        h.close()
    for a, b in zip(runs[0][0], runs[1][0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    say("resume at epoch 1")
    h = make_handle(lib, dims, ranks, idx, vals, A0, G0, 512, chunk=64)
    h.epoch(1)
    A1, G1 = h.get_params()
    h.close()
    h = make_handle(lib, dims, ranks, idx, vals, A1, G1, 512, chunk=64)
    h.set_epoch(1)
    h.epoch(1)
    A2, G2 = h.get_params()
    h.close()
    for a, b in zip(A2, runs[0][0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(G2, runs[0][1])
    say("resume mid-epoch")
    h = make_handle(lib, dims, ranks, idx, vals, A0, G0, 512, chunk=64)
    nb = h.info()["minibatches"]
    h.run_minibatches(0, 0, 7)
    h.run_minibatches(0, 7, nb)
    h.run_minibatches(1, 0, nb)
    A3, G3 = h.get_params()
    h.close()
    for a, b in zip(A3, runs[0][0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(G3, runs[0][1])


def test_diverged_is_reported(lib):
    say("divergence")
    dims, ranks = (20, 20, 20), (3, 3, 3)
    idx, vals = synth.random_tiny(3, dims, ranks, 2000, seed=2)
    A0, G0 = synth.init_params(dims, ranks, seed=2)
    A0 = [a * 5 for a in A0]
    h = make_handle(lib, dims, ranks, idx, vals * 100, A0, G0 * 5, 16, lr=5.0, lam=0.0)
    with pytest.raises(lib.StdecompError) as ei:
        for _ in range(5):
            h.epoch(1)
    assert ei.value.code == lib.STD_E_DIVERGED
    # the report names where the first non-finite value was written
    say("divergence report:", str(ei.value))
    assert "first at epoch" in str(ei.value) and "minibatch" in str(ei.value), str(ei.value)
    h.close()


# ------------------------------------------------------------ BF16 mode
# BF16 operands carry a relative rounding error of at most u = 2^-9 (round to
# nearest even, 8 significant bits); the masters, accumulations and updates
# stay FP32.  One SGD step changes a parameter by gamma * (gradient), whose
# error from the rounded operands is O(u) of the step, and the steps of an
# epoch are a fraction of the parameter, so the epoch's error relative to the
# parameters stays below u.  The bound, 2.5e-3 (1.3 u) relative Frobenius per
# epoch from a common state, sits above the largest error seen (7.4e-4, on a
# mode of rank 20) and below what a path that rounded the masters themselves
# to BF16 would accumulate (about u per step a row takes, several per epoch).
# Per row the bound is 1e-2 (rows of small norm see relatively larger
# rounding).
BF16_TOL = 2.5e-3
BF16_ROW_TOL = 1e-2
BF_CASES = [
    ("bf16_n3_j10_w4", (300, 200, 100), (10, 10, 10), 9001, 1024, 256, 1.1),
    ("bf16_n4_j8_w8", (40, 30, 20, 15), (8, 8, 8, 8), 8000, 512, 64, None),
    ("bf16_n4_j8_w16", (40, 30, 20, 15), (8, 8, 8, 8), 8000, 1024, 64, 1.2),
    ("bf16_n3_mixed_generic", (60, 50, 40), (2, 3, 20), 3000, 64, 16, 1.3),
    ("bf16_n3_j16", (100, 90, 80), (16, 16, 16), 6000, 256, 64, None),
]


@pytest.mark.parametrize("case", BF_CASES, ids=[c[0] for c in BF_CASES])
def test_bf16_epochs_close_to_oracle(lib, oracle_mod, case):
    name, dims, ranks, nnz, M, chunk, skew = case
    idx, vals = synth.random_tiny(len(dims), dims, ranks, nnz, seed=len(name), skew=skew)
    vals = (vals * 0.5).astype(np.float32)
    compare_epochs(lib, oracle_mod, name, dims, ranks, idx, vals, M, epochs=2, lr=0.02, lam=0.01, chunk=chunk,
                   dtype="bf16", tol=BF16_TOL)


def test_bf16_planted_rmse_gap(lib, oracle_mod):
    """BF16 on the small planted workload (1000^3, 100k entries, J = 5,
    M = 256, 10 epochs): the held-out RMSE gap to the free-running FP64
    oracle is reported and must stay under 1e-4 relative."""
    wl = synth.planted_uniform(seed=1001)
    compare_epochs(lib, oracle_mod, "c1_bf16", wl.dims, wl.ranks, wl.train_idx, wl.train_vals, 256, epochs=10,
                   lr=0.01, lam=0.01, test=(wl.test_idx, wl.test_vals), dtype="bf16", tol=BF16_TOL, rmse_tol=1e-4)


# ------------------------------------------- every row after a few minibatches
# Row-level check after one and two minibatches, in one launch and in one
# launch per minibatch: the largest absolute error of any parameter against
# the oracle.  Rows that straddle chunk boundaries are finished by the next
# sub-step (or at the end of a launch) and patched into other workgroups'
# samples; an error there touches a handful of rows, which the per-epoch
# relative norms above can miss.  FP32 rounding of O(1) parameters after a
# few steps stays far below the bound.
ROW_TOL = 1e-6
ROW_CASES = [((200, 150, 100), (4, 4, 4), 32, 512), ((200, 150, 100), (4, 4, 4), 64, 512),
             ((200, 150, 100), (4, 4, 4), 128, 512), ((60, 50, 30, 20), (8, 8, 8, 8), 64, 512),
             ((60, 50, 30, 20), (8, 8, 8, 8), 128, 512),
             # more than 64 workgroups (grouped and per-thread finishing of straddling rows)
             ((200, 150, 60, 40), (8, 8, 8, 8), 128, 16384), ((2000, 500, 50), (4, 4, 4), 64, 8192),
             ((400, 300, 200), (16, 16, 16), 64, 8192)]


@pytest.mark.parametrize("dims,ranks,chunk,M", ROW_CASES,
                         ids=["n%d_j%d_chunk%d_m%d" % (len(c[0]), c[1][0], c[2], c[3]) for c in ROW_CASES])
def test_rows_after_minibatches(lib, oracle_mod, dims, ranks, chunk, M):
    idx, vals = synth.random_tiny(len(dims), dims, ranks, max(20000, 3 * M), seed=9, skew=1.2)
    A0, G0 = synth.init_params(dims, ranks, seed=9)
    say("rows", dims, ranks, "chunk", chunk, "M", M)
    for nb in (1, 2):
        ref = oracle_mod.Model(dims, ranks, [a.astype(np.float64) for a in A0], G0.astype(np.float64))
        ref.run(idx, vals, M, 0.01, 0.01, 0.01, 0.01, seed=77, epoch0=0, n_epochs=1, max_batches=nb)
        for split in (False, True):
            h = make_handle(lib, dims, ranks, idx, vals, A0, G0, M, seed=77, chunk=chunk)
            if not split:
                say("  chain", h.info())
            if split:
                for k in range(nb):
                    h.run_minibatches(0, k, k + 1)
            else:
                h.run_minibatches(0, 0, nb)
            A, G = h.get_params()
            h.close()
            errs = [float(np.max(np.abs(a - r))) for a, r in zip(A, ref.A)] + [float(np.max(np.abs(G - ref.G)))]
            say("  minibatches", nb, "split launches" if split else "one launch", "max abs errors", errs)
            assert max(errs) <= ROW_TOL, errs


# ------------------------------------------------ several models, one launch
# stdecomp_epoch_batched runs the chains of independent models in one
# launch, slots of W workgroups each running a balanced list of chains; every
# model must end exactly where it ends alone (the same chain body, arguments
# and workgroup count), and a batch the single launch cannot take (different
# workgroup counts) falls back to running the models one after another.
BATCH_SETS = {
    # (dims, ranks, nnz, M, chunk): one launch needs the same workgroup count W = ceil(M / chunk)
    "n3_j4_w8": [((200, 150, 100), (4, 4, 4), 20000, 512, 64), ((120, 90, 60), (4, 4, 4), 9000, 256, 32),
                 ((300, 40, 70), (4, 4, 4), 15000, 1024, 128), ((50, 50, 50), (4, 4, 4), 3000, 128, 16)],
    "n3_mixed_ranks_w8": [((200, 150, 100), (4, 4, 4), 20000, 512, 64), ((80, 70, 60), (5, 5, 5), 6000, 256, 32),
                          ((100, 90, 80), (8, 8, 8), 8000, 512, 64), ((60, 50, 40), (16, 16, 16), 5000, 512, 64),
                          ((70, 60, 50), (3, 4, 6), 4000, 128, 16)],
    # W = 64: four slots of the device's compute units, seven chains, so slots run chains one after another
    "n3_more_chains_than_slots_w64": [((200, 150, 100), (4, 4, 4), 20000, 512, 8), ((120, 90, 60), (8, 8, 8), 9000, 512, 8),
                                      ((300, 40, 70), (4, 4, 4), 15000, 512, 8), ((50, 50, 50), (3, 3, 3), 3000, 512, 8),
                                      ((90, 80, 70), (5, 5, 5), 7000, 512, 8), ((40, 30, 20), (4, 4, 4), 2000, 512, 8),
                                      ((110, 100, 90), (6, 6, 6), 11000, 512, 8)],
    "n4_j8_w16": [((60, 50, 30, 20), (8, 8, 8, 8), 12000, 1024, 64), ((40, 30, 20, 15), (8, 8, 8, 8), 8000, 512, 32)],
    "different_w_fallback": [((200, 150, 100), (4, 4, 4), 20000, 512, 64), ((80, 70, 60), (5, 5, 5), 6000, 256, 64)],
}


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("name", list(BATCH_SETS))
def test_batched_models_match_alone(lib, oracle_mod, name, dtype):
    models = BATCH_SETS[name]
    say("batched", name, dtype)
    inputs = []
    for k, (dims, ranks, nnz, M, chunk) in enumerate(models):
        idx, vals = synth.random_tiny(len(dims), dims, ranks, nnz, seed=40 + k, skew=1.2)
        A0, G0 = synth.init_params(dims, ranks, seed=50 + k)
        inputs.append((dims, ranks, idx, (vals * 0.5).astype(np.float32), A0, G0, M, chunk))
    alone = []
    for (dims, ranks, idx, vals, A0, G0, M, chunk) in inputs:
        h = make_handle(lib, dims, ranks, idx, vals, A0, G0, M, lr=0.02, seed=77, chunk=chunk, dtype=dtype)
        h.epoch(2)
        alone.append(h.get_params())
        h.close()
    hs = [make_handle(lib, dims, ranks, idx, vals, A0, G0, M, lr=0.02, seed=77, chunk=chunk, dtype=dtype)
          for (dims, ranks, idx, vals, A0, G0, M, chunk) in inputs]
    # two batched epochs, one call each: after each, every model against the
    # FP64 oracle run for that epoch from the model's state before it
    starts = [(A0, G0) for (_, _, _, _, A0, G0, _, _) in inputs]
    tol = TOL if dtype == "f32" else BF16_TOL
    for e in range(2):
        stats = lib.epoch_batched(hs, 1)
        if not name.endswith("fallback"):  # one launch: every model reports the same launch time
            assert len({s["chain_seconds"] for s in stats}) == 1, stats
        mixed = [h.get_params() for h in hs]
        for k, ((dims, ranks, idx, vals, _, _, M, _), (As, Gs_), (Ag, Gg), s) in enumerate(
                zip(inputs, starts, mixed, stats)):
            assert s["epochs_run"] == 1
            errs, rows = oracle_epoch_errors(oracle_mod, dims, ranks, idx, vals, M, 0.02, 0.01, 77, e, As, Gs_,
                                             Ag, Gg)
            say("  model", k, "epoch", e, "vs oracle: rel errors", ["%.2e" % x for x in errs],
                "max row rel error %.2e" % rows)
            assert max(errs) <= tol, (k, e, errs)
            assert rows <= (ROW_REL_TOL if dtype == "f32" else BF16_ROW_TOL), (k, e, rows)
        starts = mixed
    for h in hs:
        h.close()
    for k, ((A1, G1), (A2, G2)) in enumerate(zip(alone, mixed)):
        diff = max([float(np.max(np.abs(a - b))) for a, b in zip(A1, A2)] + [float(np.max(np.abs(G1 - G2)))])
        say("  model", k, "max |alone - batched|", diff)
        assert diff == 0.0, (k, diff)


@pytest.mark.parametrize("name", ["n3_mixed_ranks_w8", "different_w_fallback"])
def test_step_batched_windows_match_whole_epochs(lib, name):
    """Continuous batching: advancing the models by windows of 7 minibatches
    (models joining the batch at different times, finishing their epochs at
    different windows) ends every model bit for bit where two whole epochs
    alone end; a model inside an epoch refuses stdecomp_epoch."""
    models = BATCH_SETS[name]
    say("windows", name)
    inputs = []
    for k, (dims, ranks, nnz, M, chunk) in enumerate(models):
        idx, vals = synth.random_tiny(len(dims), dims, ranks, nnz, seed=40 + k, skew=1.2)
        A0, G0 = synth.init_params(dims, ranks, seed=50 + k)
        inputs.append((dims, ranks, idx, (vals * 0.5).astype(np.float32), A0, G0, M, chunk))
    alone = []
    for (dims, ranks, idx, vals, A0, G0, M, chunk) in inputs:
        h = make_handle(lib, dims, ranks, idx, vals, A0, G0, M, lr=0.02, seed=77, chunk=chunk)
        h.epoch(2)
        alone.append(h.get_params())
        h.close()
    hs = [make_handle(lib, dims, ranks, idx, vals, A0, G0, M, lr=0.02, seed=77, chunk=chunk)
          for (dims, ranks, idx, vals, A0, G0, M, chunk) in inputs]
    joined, calls = 1, 0
    while True:
        active = [h for h in hs[:joined] if h.info()["epoch"] < 2]
        if not active and joined >= len(hs):
            break
        if active:
            lib.step_batched(active, 7)
        calls += 1
        if calls == 1:  # the first model is 7 minibatches into its first epoch
            with pytest.raises(lib.StdecompError) as ei:
                hs[0].epoch(1)
            assert ei.value.code == lib.STD_E_STATE
        if calls % 2 == 0 and joined < len(hs):  # one more model joins every second window
            joined += 1
    say("  windows:", calls)
    for k, (h, (A1, G1)) in enumerate(zip(hs, alone)):
        assert h.info()["epoch"] == 2 and h.info()["cursor"] == 0
        A2, G2 = h.get_params()
        diff = max([float(np.max(np.abs(a - b))) for a, b in zip(A1, A2)] + [float(np.max(np.abs(G1 - G2)))])
        say("  model", k, "max |alone - windows|", diff)
        assert diff == 0.0, (k, diff)
        h.close()


def test_serving_loop_results_match_alone(lib, oracle_mod):
    """Jobs that train through the serving loop (admission, rounds of
    batched epochs, retirement) end exactly where they end alone, and each
    served epoch matches the FP64 oracle run for that epoch from the job's
    state before it."""
    from paper_2012_03550_amd import serve
    say("serving loop")
    specs = [((200, 150, 100), (4, 4, 4), 20000), ((120, 90, 60), (4, 4, 4), 9000), ((60, 50, 30, 20), (8, 8, 8, 8), 8000),
             ((80, 70, 60), (5, 5, 5), 6000)]
    jobs = []
    for k, (dims, ranks, nnz) in enumerate(specs):
        idx, vals = synth.random_tiny(len(dims), dims, ranks, nnz, seed=60 + k, skew=1.2)
        jobs.append(serve.Job(k, 0.0, dims, ranks, idx, (vals * 0.5).astype(np.float32), epochs=2 + (k % 2),
                              batch=512, seed=500 + 7 * k))
    final = {}
    states = {}  # job id -> parameters after each served epoch
    srv = serve.Server(hbm_budget=1 << 34, chunk=64, on_finish=lambda j: final.__setitem__(j.jid, j.handle.get_params()),
                       on_epoch=lambda j: states.setdefault(j.jid, []).append(j.handle.get_params()))
    for j in jobs:
        srv.submit(j)
    srv.admit(0.0)
    while srv.active:
        srv.round(lambda: 0.0)
    assert len(srv.done) == len(jobs)
    for j in jobs:
        h = lib.Stdecomp(j.dims, j.ranks, j.idx, j.vals, batch=512, lr_factor=0.01, lr_core=0.01, lam_factor=0.01,
                         lam_core=0.01, seed_sample=j.seed, seed_init=j.seed + 1, chunk=64)
        start = h.get_params()  # the library's own initial parameters (same seed as the served job)
        h.epoch(j.epochs)
        A, G = h.get_params()
        h.close()
        assert len(states[j.jid]) == j.epochs
        for e, (Ag, Gg) in enumerate(states[j.jid]):
            errs, rows = oracle_epoch_errors(oracle_mod, j.dims, j.ranks, j.idx, j.vals, 512, 0.01, 0.01, j.seed, e,
                                             start[0], start[1], Ag, Gg)
            say("  job", j.jid, "epoch", e, "vs oracle: rel errors", ["%.2e" % x for x in errs],
                "max row rel error %.2e" % rows)
            assert max(errs) <= TOL and rows <= ROW_REL_TOL, (j.jid, e, errs, rows)
            start = (Ag, Gg)
        A2, G2 = final[j.jid]
        diff = max([float(np.max(np.abs(a - b))) for a, b in zip(A, A2)] + [float(np.max(np.abs(G - G2)))])
        say("  job", j.jid, "epochs", j.epochs, "max |alone - served|", diff)
        assert diff == 0.0


def test_chunk_tuner(lib):
    """The tuner times each candidate chunk that fits and returns the fastest;
    a handle built with it trains."""
    from paper_2012_03550_amd import tune
    dims, ranks = (300, 200, 100), (8, 8, 8)
    idx, vals = synth.random_tiny(3, dims, ranks, 30000, seed=70, skew=1.1)
    best, times = tune.tune_chunk(dims, ranks, idx, vals, 1024, candidates=(32, 64, 128, 256), minibatches=16)
    say("tuner", times, "->", best)
    assert best in times and times[best] == min(times.values()) and len(times) >= 2
    assert tune.tune_chunk(dims, ranks, idx, vals, 1024)[0] == best  # cached
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=1024, chunk=best)
    assert h.info()["chunk"] == best
    h.epoch(1)
    h.close()


def test_batch_tuner(lib):
    """The batch tuner times one batched epoch of every model with each
    candidate chunk (one chunk for all: the chains must share the workgroup
    count) and returns the highest rate; the batch trains with it in one
    launch; the decision is cached per set of shapes."""
    from paper_2012_03550_amd import tune
    models = []
    for k, (dims, ranks, nnz) in enumerate([((200, 150, 100), (4, 4, 4), 20000), ((120, 90, 60), (8, 8, 8), 9000),
                                            ((300, 40, 70), (5, 5, 5), 15000)]):
        idx, vals = synth.random_tiny(3, dims, ranks, nnz, seed=80 + k, skew=1.2)
        models.append((dims, ranks, idx, (vals * 0.5).astype(np.float32)))
    best, rates = tune.tune_batch(models, 512, candidates=(32, 64, 128))
    say("batch tuner", rates, "->", best)
    assert set(rates) == {32, 64, 128} and best == max(rates, key=rates.get) and min(rates.values()) > 0
    assert tune.tune_batch(models, 512, candidates=(32, 64, 128))[0] == best  # cached
    hs = [lib.Stdecomp(d, r, i, v, batch=512, chunk=best) for d, r, i, v in models]
    st = lib.epoch_batched(hs, 1)
    assert len({s["chain_seconds"] for s in st}) == 1 and all(s["epochs_run"] == 1 for s in st)
    for h in hs:
        h.close()


def test_barrier_probe(lib):
    """The grid-barrier timing aid returns a positive time and rejects bad
    arguments."""
    dims, ranks = (200, 150, 100), (4, 4, 4)
    idx, vals = synth.random_tiny(3, dims, ranks, 20000, seed=9)
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=512, chunk=64)
    t = h.barrier_us(500)
    say("barrier", h.info()["workgroups"], "workgroups:", t, "us")
    assert 0.0 < t < 1000.0
    with pytest.raises(lib.StdecompError):
        h.barrier_us(0)
    h.epoch(1)  # the chain still runs after the probe
    h.close()
