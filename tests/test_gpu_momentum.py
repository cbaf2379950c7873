"""Heavy-ball momentum on the GPU (options.momentum = mu > 0) against the FP64
oracle's orc_run_momentum, through the C ABI.

The reading (the paper names momentum as an extension without fixing it,
Section "Conclusion and Future Works"): on every sub-step v <- mu v + g,
theta <- theta - gamma v, one core velocity updated once per minibatch and
one velocity per factor row, updated only when the row is sampled.  FP32
results must match to the FP32 bar: per epoch from a common state (parameters
and velocities), relative Frobenius error <= 1e-5 for every A(n), G and their
velocities, every factor row to 1e-5 and every row velocity to 5e-5 relative
(a velocity is proportional to the residuals x - x_hat, whose relative
rounding grows as |x| / |x - x_hat| where the model fits well; the
parameters take that error times gamma only), and after one
and two minibatches every parameter to 1e-6 absolute and every velocity to
1e-6 of its array's largest magnitude (velocities are running sums of
gradients, not O(1) values: their FP32 rounding scales with them).  In BF16
the velocities carry the BF16 rounding of the contraction operands directly
(the parameters only through gamma times it): 1e-2 relative, about 2.6 BF16
unit roundoffs, against 2.5e-3 for the parameters.  The cases cover the
one- and two-level core updates and all three ways rows that straddle chunk
boundaries are finished (one-wave scan for W <= 64, one thread per run and
the grouped quad butterfly for W > 64), whose carry slots hold the old
velocity.
"""
import numpy as np
import pytest

from paper_2012_03550_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
ROW_REL_TOL = 1e-5
VEL_ROW_REL_TOL = 5e-5
BF16_TOL = 2.5e-3
BF16_VEL_TOL = 1e-2
BF16_ROW_TOL = 1e-2
MU = 0.5


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
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def row_rel_max(A, ref):
    """max over rows of ||A[i] - ref[i]|| / ||ref[i]||, with a floor of 1e-3
    of the RMS row norm (rows of zero velocity are measured against it)."""
    A = np.asarray(A, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.linalg.norm(A - ref, axis=1)
    n = np.linalg.norm(ref, axis=1)
    floor = 1e-3 * np.sqrt(np.mean(n ** 2)) if n.size else 0.0
    return float(np.max(d / np.maximum(n, max(floor, 1e-30)))) if n.size else 0.0


def make(lib, dims, ranks, idx, vals, A0, G0, M, chunk, lr, lam, seed=77, dtype="f32", mu=MU):
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=M, lr_factor=lr, lr_core=lr, lam_factor=lam, lam_core=lam,
                     seed_sample=seed, init="caller", chunk=chunk, dtype=dtype, momentum=mu)
    h.set_params(A0, G0)
    return h


def oracle_from(oracle_mod, dims, ranks, A, G, VA, VG):
    return oracle_mod.MomentumModel(dims, ranks, [a.astype(np.float64) for a in A], G.astype(np.float64),
                                    [v.astype(np.float64) for v in VA], VG.astype(np.float64))


def errors(dims, got, ref):
    (A, G, VA, VG) = got
    N = len(dims)
    errs = ([rel(A[n], ref.A[n]) for n in range(N)] + [rel(G, ref.G)] +
            [rel(VA[n], ref.VA[n]) for n in range(N)] + [rel(VG, ref.VG)])
    rows = max(row_rel_max(A[n], ref.A[n]) for n in range(N))
    vrows = max(row_rel_max(VA[n], ref.VA[n]) for n in range(N))
    return errs, (rows, vrows)


def test_momentum_options_and_velocity_calls(lib):
    dims, ranks = (40, 30, 20), (4, 3, 5)
    idx, vals = synth.random_tiny(3, dims, ranks, 2000, seed=1)
    for bad in (1.0, -0.5, float("nan")):
        with pytest.raises(lib.StdecompError) as ei:
            lib.Stdecomp(dims, ranks, idx, vals, batch=64, momentum=bad)
        assert ei.value.code == lib.STD_E_INVAL
    with pytest.raises(lib.StdecompError) as ei:  # the Kruskal core takes no momentum
        lib.Stdecomp(dims, ranks, idx, vals, batch=64, momentum=0.5, r_core=2)
    assert ei.value.code == lib.STD_E_INVAL
    plain = lib.Stdecomp(dims, ranks, idx, vals, batch=64)
    with pytest.raises(lib.StdecompError) as ei:
        plain.get_velocity()
    assert ei.value.code == lib.STD_E_STATE
    plain.close()
    h = lib.Stdecomp(dims, ranks, idx, vals, batch=64, momentum=0.9)
    VA, VG = h.get_velocity()
    assert all(np.all(v == 0) for v in VA) and np.all(VG == 0)  # zero at init
    rng = np.random.default_rng(3)
    VA1 = [rng.standard_normal(v.shape).astype(np.float32) for v in VA]
    VG1 = rng.standard_normal(VG.shape).astype(np.float32)
    h.set_velocity(VA1, VG1)
    VA2, VG2 = h.get_velocity()
    for a, b in zip(VA1, VA2):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(VG1, VG2)
    h.close()


CASES = [
    # name, dims, ranks, nnz, M, chunk, skew
    ("n3_mixed_generic_w4", (60, 50, 40), (2, 3, 4), 3000, 32, 8, None),
    ("n2_uniform_w2", (80, 70), (4, 4), 4000, 64, 32, None),
    ("n3_zipf_long_runs_w8", (500, 400, 30), (4, 4, 4), 30000, 512, 64, 1.3),
    ("n3_j10_w4_ragged", (300, 200, 100), (10, 10, 10), 9001, 1024, 256, 1.1),
    ("n4_j8_two_level_core_w16", (60, 50, 30, 20), (8, 8, 8, 8), 12000, 1024, 64, 1.2),
    ("n4_j8_tables_per_phase_w8", (60, 50, 30, 20), (8, 8, 8, 8), 12000, 1024, 128, 1.2),
    ("n5_uniform", (12, 11, 10, 9, 8), (2, 2, 2, 2, 2), 3000, 64, 16, None),
    # more than 64 workgroups: grouped (four modes) and per-thread (three modes) finishing
    ("n4_j8_auto_m16384", (200, 150, 60, 40), (8, 8, 8, 8), 2 * 16384 + 777, 16384, 0, 1.2),
    ("n3_j4_chunk64_m8192", (2000, 500, 50), (4, 4, 4), 3 * 8192 + 1000, 8192, 64, 1.3),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_momentum_epochs_match_oracle(lib, oracle_mod, case):
    name, dims, ranks, nnz, M, chunk, skew = case
    idx, vals = synth.random_tiny(len(dims), dims, ranks, nnz, seed=len(name) + 300, skew=skew)
    vals = (vals * 0.5).astype(np.float32)
    A0, G0 = synth.init_params(dims, ranks, seed=len(name) + 400)
    lr, lam, seed = 0.02, 0.01, 77
    h = make(lib, dims, ranks, idx, vals, A0, G0, M, chunk, lr, lam, seed)
    say(name, "chain", h.info())
    start = (A0, G0) + h.get_velocity()
    free = oracle_from(oracle_mod, dims, ranks, *start)
    worst = worst_row = 0.0
    for e in range(2):
        h.epoch(1)
        got = h.get_params() + h.get_velocity()
        ref = oracle_from(oracle_mod, dims, ranks, *start)
        ref.run(idx, vals, M, lr, lam, lr, lam, seed=seed, epoch0=e, n_epochs=1, mu=MU)
        errs, (rows, vrows) = errors(dims, got, ref)
        worst, worst_row = max(worst, max(errs)), max(worst_row, rows)
        say(name, "epoch", e, "rel errors A.., G, VA.., VG:", ["%.2e" % x for x in errs],
            "row %.2e, row velocity %.2e" % (rows, vrows))
        assert max(errs) <= TOL, (name, e, errs)
        assert rows <= ROW_REL_TOL and vrows <= VEL_ROW_REL_TOL, (name, e, rows, vrows)
        free.run(idx, vals, M, lr, lam, lr, lam, seed=seed, epoch0=e, n_epochs=1, mu=MU)
        start = got
    drift = max(errors(dims, got, free)[0])
    say(name, "momentum: worst per-epoch rel err %.3g (row %.3g), free-running drift after 2 epochs %.3g" %
        (worst, worst_row, drift))
    h.close()


ROW_CASES = [((200, 150, 100), (4, 4, 4), 32, 512), ((60, 50, 30, 20), (8, 8, 8, 8), 64, 512),
             ((200, 150, 60, 40), (8, 8, 8, 8), 128, 16384), ((2000, 500, 50), (4, 4, 4), 64, 8192),
             ((400, 300, 200), (16, 16, 16), 64, 8192)]


@pytest.mark.parametrize("dims,ranks,chunk,M", ROW_CASES,
                         ids=["n%d_j%d_chunk%d_m%d" % (len(c[0]), c[1][0], c[2], c[3]) for c in ROW_CASES])
def test_momentum_values_after_minibatches(lib, oracle_mod, dims, ranks, chunk, M):
    """Every parameter and velocity after one and two minibatches (one launch,
    and one launch per minibatch), to 1e-6 absolute."""
    idx, vals = synth.random_tiny(len(dims), dims, ranks, max(20000, 3 * M), seed=19, skew=1.2)
    A0, G0 = synth.init_params(dims, ranks, seed=19)
    VA0 = [np.zeros_like(a) for a in A0]
    VG0 = np.zeros_like(G0)
    for nb in (1, 2):
        ref = oracle_from(oracle_mod, dims, ranks, A0, G0, VA0, VG0)
        ref.run(idx, vals, M, 0.01, 0.01, 0.01, 0.01, seed=78, epoch0=0, n_epochs=1, max_batches=nb, mu=0.9)
        for split in (False, True):
            h = make(lib, dims, ranks, idx, vals, A0, G0, M, chunk, 0.01, 0.01, seed=78, mu=0.9)
            if split:
                for k in range(nb):
                    h.run_minibatches(0, k, k + 1)
            else:
                h.run_minibatches(0, 0, nb)
            A, G = h.get_params()
            VA, VG = h.get_velocity()
            h.close()
            errs = [float(np.max(np.abs(a - r))) for a, r in zip(A, ref.A)] + [float(np.max(np.abs(G - ref.G)))]
            verrs = ([float(np.max(np.abs(a - r)) / max(1.0, np.max(np.abs(r)))) for a, r in zip(VA, ref.VA)] +
                     [float(np.max(np.abs(VG - ref.VG)) / max(1.0, np.max(np.abs(ref.VG))))])
            say("momentum values", dims, "chunk", chunk, "M", M, "minibatches", nb,
                "split" if split else "one launch", "max abs errors", ["%.1e" % x for x in errs],
                "velocities (scaled)", ["%.1e" % x for x in verrs])
            assert max(errs) <= 1e-6, errs
            assert max(verrs) <= 1e-6, verrs


def test_momentum_bf16_close_to_oracle(lib, oracle_mod):
    dims, ranks = (60, 50, 30, 20), (8, 8, 8, 8)
    idx, vals = synth.random_tiny(4, dims, ranks, 12000, seed=31, skew=1.2)
    vals = (vals * 0.5).astype(np.float32)
    A0, G0 = synth.init_params(dims, ranks, seed=32)
    h = make(lib, dims, ranks, idx, vals, A0, G0, 1024, 64, 0.02, 0.01, dtype="bf16")
    start = (A0, G0) + h.get_velocity()
    h.epoch(1)
    got = h.get_params() + h.get_velocity()
    h.close()
    ref = oracle_from(oracle_mod, dims, ranks, *start)
    ref.run(idx, vals, 1024, 0.02, 0.01, 0.02, 0.01, seed=77, epoch0=0, n_epochs=1, mu=MU)
    errs, (rows, vrows) = errors(dims, got, ref)
    say("momentum bf16 rel errors A.., G, VA.., VG:", ["%.2e" % x for x in errs],
        "row %.2e, row velocity %.2e" % (rows, vrows))
    n = len(dims) + 1
    assert max(errs[:n]) <= BF16_TOL, errs
    assert max(errs[n:]) <= BF16_VEL_TOL, errs
    assert rows <= BF16_ROW_TOL, rows


def test_momentum_resume_is_bit_identical(lib):
    """Parameters and velocities saved after one epoch, loaded into a new
    handle at epoch 1: the second epoch ends bit for bit where the
    uninterrupted run ends (also resuming mid-epoch from run_minibatches)."""
    dims, ranks = (200, 150, 100), (4, 4, 4)
    idx, vals = synth.random_tiny(3, dims, ranks, 20000, seed=5, skew=1.2)
    A0, G0 = synth.init_params(dims, ranks, seed=6)
    h = make(lib, dims, ranks, idx, vals, A0, G0, 512, 64, 0.02, 0.01)
    h.epoch(1)
    A1, G1 = h.get_params()
    VA1, VG1 = h.get_velocity()
    h.epoch(1)
    A2, G2 = h.get_params()
    VA2, VG2 = h.get_velocity()
    h.close()
    r = make(lib, dims, ranks, idx, vals, A1, G1, 512, 64, 0.02, 0.01)
    r.set_velocity(VA1, VG1)
    r.set_epoch(1)
    r.epoch(1)
    A3, G3 = r.get_params()
    VA3, VG3 = r.get_velocity()
    r.close()
    for x, y in zip(A2 + [G2] + VA2 + [VG2], A3 + [G3] + VA3 + [VG3]):
        np.testing.assert_array_equal(x, y)
    # mid-epoch: minibatches [0, 10) then [10, nb) of epoch 1 in two launches
    r = make(lib, dims, ranks, idx, vals, A1, G1, 512, 64, 0.02, 0.01)
    r.set_velocity(VA1, VG1)
    nb = -(-idx.shape[1] // 512)
    r.run_minibatches(1, 0, 10)
    r.run_minibatches(1, 10, nb)
    A4, G4 = r.get_params()
    VA4, VG4 = r.get_velocity()
    r.close()
    for x, y in zip(A2 + [G2] + VA2 + [VG2], A4 + [G4] + VA4 + [VG4]):
        np.testing.assert_array_equal(x, y)


MOM_BATCHES = {
    # every model with momentum (different mu, ranks and sizes): one launch
    "all_momentum": [((200, 150, 100), (4, 4, 4), 20000, 512, 64, 0.5), ((80, 70, 60), (5, 5, 5), 6000, 256, 32, 0.2),
                     ((100, 90, 80), (8, 8, 8), 8000, 512, 64, 0.9), ((60, 50, 40), (16, 16, 16), 5000, 512, 64, 0.3)],
    # with and without momentum: the models run one after another
    "mixed_fallback": [((200, 150, 100), (4, 4, 4), 20000, 512, 64, 0.5), ((80, 70, 60), (5, 5, 5), 6000, 256, 32, 0.0)],
}


@pytest.mark.parametrize("name", list(MOM_BATCHES))
def test_momentum_in_batched_launch(lib, oracle_mod, name):
    """Models with momentum in one batched launch end bit for bit where they
    end alone, and each matches its oracle; a batch that mixes models with
    and without momentum runs them one after another, with the same results."""
    models = MOM_BATCHES[name]
    inputs = []
    for k, (dims, ranks, nnz, M, chunk, mu) in enumerate(models):
        idx, vals = synth.random_tiny(3, dims, ranks, nnz, seed=60 + k, skew=1.2)
        A0, G0 = synth.init_params(dims, ranks, seed=70 + k)
        inputs.append((dims, ranks, idx, (vals * 0.5).astype(np.float32), A0, G0, M, chunk, mu))
    alone = []
    for (dims, ranks, idx, vals, A0, G0, M, chunk, mu) in inputs:
        h = make(lib, dims, ranks, idx, vals, A0, G0, M, chunk, 0.02, 0.01, mu=mu)
        h.epoch(1)
        alone.append(h.get_params() + (h.get_velocity() if mu > 0 else ()))
        h.close()
    hs = [make(lib, dims, ranks, idx, vals, A0, G0, M, chunk, 0.02, 0.01, mu=mu)
          for (dims, ranks, idx, vals, A0, G0, M, chunk, mu) in inputs]
    stats = lib.epoch_batched(hs, 1)
    if name == "all_momentum":
        assert len({s["chain_seconds"] for s in stats}) == 1, stats  # one launch
    for k, (h, (dims, ranks, idx, vals, A0, G0, M, chunk, mu), a) in enumerate(zip(hs, inputs, alone)):
        got = h.get_params() + (h.get_velocity() if mu > 0 else ())
        for x, y in zip(got[0] + [got[1]], a[0] + [a[1]]):
            np.testing.assert_array_equal(x, y)
        if mu > 0:
            for x, y in zip(got[2] + [got[3]], a[2] + [a[3]]):
                np.testing.assert_array_equal(x, y)
            ref = oracle_from(oracle_mod, dims, ranks, A0, G0, [np.zeros_like(x) for x in A0], np.zeros_like(G0))
            ref.run(idx, vals, M, 0.02, 0.01, 0.02, 0.01, seed=77, epoch0=0, n_epochs=1, mu=mu)
            errs, (rows, vrows) = errors(dims, got, ref)
        else:
            ref = oracle_mod.Model(dims, ranks, [x.astype(np.float64) for x in A0], G0.astype(np.float64))
            ref.run(idx, vals, M, 0.02, 0.01, 0.02, 0.01, seed=77, epoch0=0, n_epochs=1)
            errs = [rel(got[0][n], ref.A[n]) for n in range(3)] + [rel(got[1], ref.G)]
            rows, vrows = max(row_rel_max(got[0][n], ref.A[n]) for n in range(3)), 0.0
        say("batched", name, "model", k, "mu", mu, "rel errors", ["%.2e" % x for x in errs],
            "row %.2e, row velocity %.2e" % (rows, vrows))
        assert max(errs) <= TOL and rows <= ROW_REL_TOL and vrows <= VEL_ROW_REL_TOL, (k, errs, rows, vrows)
    for h in hs:
        h.close()
