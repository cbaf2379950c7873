"""Chain placement (options.placement) on the GPU, through the C ABI.

A chain of W <= (CUs per XCC) workgroups can run on one XCC, where its grid
barrier orders memory in that XCC's L2 instead of at device scope.  The
placement changes no arithmetic and no order of it: every result must be
bit-identical to the spread placement.  The barrier's memory ordering is also
checked directly (stdecomp_debug_barrier_check): after each barrier every
workgroup must read every other workgroup's write of that round.
"""
import numpy as np
import pytest

from paper_2012_03550_amd import synth

pytestmark = pytest.mark.gpu

ONE_XCC, SPREAD = 2, 1


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


def test_auto_places_a_narrow_chain_on_one_xcc(lib):
    dims, ranks = (300, 200, 100), (5, 5, 5)
    idx, vals = synth.random_tiny(3, dims, ranks, 20000, seed=3)
    with lib.Stdecomp(dims, ranks, idx, vals, batch=1024, chunk=32) as h:  # W = 32
        inf = h.info()
        say("auto W=32", inf)
        assert inf["workgroups"] == 32 and inf["placement"] == ONE_XCC
    with lib.Stdecomp(dims, ranks, idx, vals, batch=2048, chunk=32) as h:  # W = 64: too wide
        inf = h.info()
        say("auto W=64", inf)
        assert inf["workgroups"] == 64 and inf["placement"] == SPREAD
    with pytest.raises(lib.StdecompError) as ei:
        lib.Stdecomp(dims, ranks, idx, vals, batch=2048, chunk=32, placement="one_xcc")
    assert ei.value.code == lib.STD_E_INVAL
    with lib.Stdecomp(dims, ranks, idx, vals, batch=1024, chunk=32, placement="spread") as h:
        assert h.info()["placement"] == SPREAD


def test_one_xcc_only_for_the_dense_core(lib):
    """The one-XCC kernels are those of the dense core (with or without
    momentum): the Kruskal core runs spread (auto) or is refused (one XCC)."""
    dims, ranks = (200, 150, 90), (5, 5, 5)
    idx, vals = synth.random_tiny(3, dims, ranks, 15000, seed=6)
    with lib.Stdecomp(dims, ranks, idx, vals, batch=512, chunk=32, r_core=3) as h:
        assert h.info()["placement"] == SPREAD
    with pytest.raises(lib.StdecompError) as ei:
        lib.Stdecomp(dims, ranks, idx, vals, batch=512, chunk=32, placement="one_xcc", r_core=3)
    assert ei.value.code == lib.STD_E_INVAL
    with lib.Stdecomp(dims, ranks, idx, vals, batch=512, chunk=32, momentum=0.5) as h:
        assert h.info()["placement"] == ONE_XCC


@pytest.mark.parametrize("W", [2, 16, 32])
def test_barrier_orders_memory_in_both_placements(lib, W):
    dims, ranks = (300, 200, 100), (4, 4, 4)
    idx, vals = synth.random_tiny(3, dims, ranks, 20000, seed=4)
    for place in ("one_xcc", "spread"):
        with lib.Stdecomp(dims, ranks, idx, vals, batch=32 * W, chunk=32, placement=place) as h:
            assert h.info()["workgroups"] == W
            stale = h.barrier_check(4000)
            us = h.barrier_us(2000)
            say(f"W={W} {place}: stale reads {stale}, {us:.2f} us per barrier")
            assert stale == 0


CASES = [
    # name, dims, ranks, nnz, M, chunk, dtype, extra options
    ("n3_j5_f32_w32", (400, 300, 60), (5, 5, 5), 30000, 1024, 32, "f32", {}),
    ("n3_j10_bf16_w8", (300, 200, 100), (10, 10, 10), 9001, 1024, 128, "bf16", {}),
    ("n4_j8_two_level_w16", (60, 50, 30, 20), (8, 8, 8, 8), 12000, 1024, 64, "f32", {}),
    ("n4_j4_bf16_w32", (80, 60, 40, 30), (4, 4, 4, 4), 20000, 2048, 64, "bf16", {}),
    ("n3_mixed_generic_w4", (60, 50, 40), (2, 3, 4), 3000, 32, 8, "f32", {}),
    ("n3_mixed_generic_bf16_w16", (300, 200, 100), (6, 4, 5), 12000, 1024, 64, "bf16", {}),
    ("n3_j6_momentum_w16", (200, 150, 90), (6, 6, 6), 15000, 512, 32, "f32", {"momentum": 0.5}),
    ("n4_j4_momentum_bf16_w8", (80, 60, 40, 30), (4, 4, 4, 4), 20000, 512, 64, "bf16", {"momentum": 0.3}),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_placements_give_identical_bits(lib, case):
    name, dims, ranks, nnz, M, chunk, dtype, extra = case
    N = len(dims)
    idx, vals = synth.random_tiny(N, dims, ranks, nnz, seed=11, skew=1.2)
    out = {}
    for place in ("one_xcc", "spread"):
        say(name, place)
        with lib.Stdecomp(dims, ranks, idx, vals, batch=M, chunk=chunk, dtype=dtype, seed_init=5,
                          lr_factor=0.02, lr_core=0.02, lam_factor=0.01, lam_core=0.01, placement=place,
                          **extra) as h:
            assert h.info()["placement"] == (ONE_XCC if place == "one_xcc" else SPREAD)
            h.epoch(2)
            A, G = h.get_params()
            res = [a.copy() for a in A] + [G.copy()]
            if extra.get("momentum"):
                VA, VG = h.get_velocity()
                res += [v.copy() for v in VA] + [VG.copy()]
            out[place] = res
    for a, b in zip(out["one_xcc"], out["spread"]):
        assert np.all(np.isfinite(a))
        np.testing.assert_array_equal(a, b)
