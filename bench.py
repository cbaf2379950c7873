"""Throughput of the SGD_Tucker minibatch update on one MI355X.

Default workload (the precision comparison the metric is quoted on): a
4-order tensor 100000 x 100000 x 1000 x 100 with 200M nonzeros, power-law
(Zipf 1.2) indices on modes 1-2 and uniform indices on modes 3-4, values from
a planted rank-(8,8,8,8) Tucker model plus N(0, 0.05^2) noise, 10% held out;
core ranks J = (8,8,8,8), minibatches of M = 8192 (synthetic data, random
initial parameters).  One step = one epoch over the 180M training entries
(sampler, row-set sort, minibatch chain) followed by the held-out RMSE.  The
FP32 path is the headline value; the BF16 path (BF16 operands, FP32 masters
and accumulation) runs the same steps from the same initial parameters and is
reported beside it, each with its held-out RMSE gap to the FP64 oracle on the
first minibatches of epoch 0.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config c3|c2|c4|c5|ranks]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "nonzero-updates/sec/GPU at fixed held-out RMSE (FP32 vs BF16); serve p50/p99"

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp32_TFs": 157.3,
    "bf16_TFs": 2500.0,
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--nnz", type=int, default=0, help="entries before the held-out split (0: the config's)")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--chunk", type=int, default=0, help="chain chunk (c2, c3, c4; 0: automatic, c4: tuned)")
    ap.add_argument("--placement", default="auto", choices=["auto", "spread", "one_xcc"],
                    help="(c2, c3) where the chain's workgroups run (auto: one XCC when W fits one)")
    ap.add_argument("--cpu-batches", type=int, default=-1,
                    help="minibatches of the CPU oracle baseline (0: skip; -1: the config's default, c3: 48, c2: 60)")
    ap.add_argument("--prefix", type=int, default=200,
                    help="(c3) minibatches of epoch 0 on which each dtype is compared with the FP64 oracle "
                         "(0: skip; the oracle runs them in a thread beside the GPU steps)")
    ap.add_argument("--traffic-json", default=None,
                    help="(c2) counter record of the chain (default: profiles/chain_traffic_ratings_zipf[_bf16].json)")
    ap.add_argument("--duration", type=float, default=3.0, help="(c5) seconds of job arrivals")
    ap.add_argument("--config", default="c3", choices=["c2", "c3", "c4", "c5", "ranks"],
                    help="c3 (default): 4-order planted power-law tensor, FP32 vs BF16; c2: Netflix-shaped ratings; "
                         "c4: 64 independent planted tensors, batched launches vs one model at a time; "
                         "c5: serving loop (Poisson jobs and queries), p50/p99 latency; "
                         "ranks: core-rank sweep J = 4..24 on a ratings tensor")
    ap.add_argument("--dtypes", default="f32,bf16", help="(c3) precisions to run, the first is the headline")
    ap.add_argument("--rcore", type=int, default=0,
                    help="(c3) 0: dense core; R > 0: the paper's Kruskal core of rank R (the oracle prefix then "
                         "defaults to 2 minibatches, 1 of them timed)")
    ap.add_argument("--momentum", type=float, default=0.0,
                    help="(c3) heavy-ball momentum mu in [0, 1) on every sub-step (0: the plain method)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes 5 times (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(5):
            dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        sec = ev[0].elapsed_time(ev[1]) * 1e-3 / 5
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "repeats": 6,
                          "copy_GBs_read_plus_write": round(2 * n * 4 / sec / 1e9, 1)}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.config == "c3":
        run_c3(args)
        return
    if args.config == "c2":
        run_c2(args)
        return
    if args.config == "c4":
        run_c4(args)
        return
    if args.config == "c5":
        run_c5(args)
        return
    if args.config == "ranks":
        run_ranks(args)
        return


def run_c2(args):
    """Netflix-shaped ratings: 480000 x 18000 x 2000, 100M entries (Zipf 1.1
    per mode, ratings 1..5, 10% held out), J = (10,10,10), M = 4096,
    lr = lambda = 0.01; step = one epoch + held-out RMSE."""
    import numpy as np
    import torch

    from paper_2012_03550_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t = time.time()
    wl = synth.ratings_zipf(nnz=args.nnz or 100_000_000)
    log("generated %d training / %d held-out entries in %.1fs" % (wl.nnz, wl.test_vals.size, time.time() - t))
    M = args.batch
    lr = lam = 0.01
    h = binding.Stdecomp(wl.dims, wl.ranks, wl.train_idx, wl.train_vals, batch=M, lr_factor=lr, lr_core=lr,
                         lam_factor=lam, lam_core=lam, seed_sample=3002, seed_init=2002, dtype=args.dtype,
                         chunk=args.chunk, placement=args.placement)
    info = h.info()
    log("chain", info)
    A0, G0 = h.get_params()
    test_idx = torch.from_numpy(wl.test_idx).cuda()
    test_vals = torch.from_numpy(wl.test_vals).cuda()

    for w in range(args.warmup):
        st = h.epoch(1)
        h.loss(test_idx, test_vals)
        log("warmup epoch %d: %.3fs device" % (w, st["device_seconds"]))
    torch.cuda.synchronize()
    acc = None
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = h.epoch(1)
        ls = h.loss(test_idx, test_vals)
        if acc is None:
            acc = dict(st)
        else:
            for key in st:
                acc[key] += st[key]
        log("step %d: chain %.3fs schedule %.4fs held-out RMSE %.5f" % (k, st["chain_seconds"],
                                                                       st["schedule_seconds"], ls["rmse"]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    updates = acc["updates"]
    value = updates / elapsed

    # roofline of the dominant kernel (the minibatch chain), from the
    # library's HIP events on its own stream
    tpath = args.traffic_json or traffic_path("ratings_zipf", args.dtype)
    roofline = chain_roofline(acc, args.dtype, stored_traffic(tpath, args.dtype, wl.nnz, M, info),
                              latency_bound(h, M, len(wl.dims), updates / acc["chain_seconds"]))

    cpu = None
    cpu_batches = 60 if args.cpu_batches < 0 else args.cpu_batches
    if cpu_batches > 0:
        cpu = cpu_baseline(h, wl, A0, G0, M, lr, lam, cpu_batches)
    h.close()

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "nonzero-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "ratings_zipf 480000x18000x2000 100M nnz (Zipf 1.1, ratings 1-5, 10% held out), "
                               "J=(10,10,10), M=4096, lr=lambda=0.01; step = 1 epoch + held-out RMSE",
                   "train_entries": int(wl.nnz), "batch": M, "chain_workgroups": info["workgroups"],
                   "chain_chunk": info["chunk"], "chain_placement": PLACEMENT_NAMES[info["placement"]]},
        "heldout_rmse": round(ls["rmse"], 6),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_c3(args):
    """The precision comparison (default): 4-order planted power-law tensor
    100000x100000x1000x100, 200M entries (Zipf 1.2 on modes 1-2, uniform on
    3-4), planted rank (8,8,8,8) plus N(0, 0.05^2) noise, 10% held out;
    J = (8,8,8,8), M = 8192, lr = 0.05, lambda = 1e-4 (at lr = lambda = 0.01,
    or lambda = 1e-3, the model decays to the zero saddle and stays there; at
    lr = 0.1 it diverges in the first epoch).  Each dtype runs W warm-up and
    K timed steps (one epoch + held-out RMSE each) from the same initial
    parameters.  Before that, each runs the first ``--prefix`` minibatches of
    epoch 0, and the FP64 oracle runs the same minibatches from the same
    parameters in a thread beside the GPU work: the parameter and held-out
    RMSE gaps of each dtype to the oracle are reported, and the oracle's
    first ``--cpu-batches`` minibatches are its timed baseline."""
    import threading

    import numpy as np
    import torch
    from paper_2012_03550_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    nnz = args.nnz or 200_000_000
    t = time.time()
    wl = synth.planted_powerlaw(nnz=nnz, device="cuda")
    log("generated %d training / %d held-out entries in %.1fs" % (wl.nnz, wl.test_vals.size, time.time() - t))
    M, lr, lam, sample = 8192, 0.05, 1e-4, 200_000
    seed_s, seed_i = 3003, 2003
    R = max(0, args.rcore)
    mu = args.momentum
    prefix = max(0, args.prefix) if (R == 0 or args.prefix != 200) else 2
    cpu_batches = (48 if R == 0 else 1) if args.cpu_batches < 0 else args.cpu_batches
    cpu_batches = min(cpu_batches, prefix) if prefix else cpu_batches
    dtypes = [d for d in args.dtypes.split(",") if d]
    test_idx = torch.from_numpy(wl.test_idx).cuda()
    test_vals = torch.from_numpy(wl.test_vals).cuda()
    s_idx = np.ascontiguousarray(wl.test_idx[:, :sample])
    s_vals = np.ascontiguousarray(wl.test_vals[:sample])
    res, orc = {}, {}
    A0 = G0 = B0 = None
    worker = None
    for dtype in dtypes:
        h = binding.Stdecomp(wl.dims, wl.ranks, wl.train_idx, wl.train_vals, batch=M, lr_factor=lr, lr_core=lr,
                             lam_factor=lam, lam_core=lam, seed_sample=seed_s, seed_init=seed_i, dtype=dtype,
                             r_core=R, momentum=mu, chunk=args.chunk, placement=args.placement)
        if A0 is None:
            A0, G0 = h.get_params()
            B0 = h.get_kruskal() if R else None
            if prefix > 0 or cpu_batches > 0:
                worker = threading.Thread(target=oracle_prefix, daemon=True,
                                          args=(wl, A0, G0, M, lr, lam, seed_s, max(prefix, cpu_batches),
                                                cpu_batches, s_idx, s_vals, orc, B0, mu))
                worker.start()
        info = h.info()
        log("c3 %s chain" % dtype, info)
        r = {"chain_workgroups": info["workgroups"], "chain_chunk": info["chunk"],
             "chain_placement": PLACEMENT_NAMES[info["placement"]]}
        if prefix > 0:
            h.run_minibatches(0, 0, prefix)
            r["prefix_params"] = h.get_params() + ((h.get_kruskal(),) if R else ())
            r["prefix_heldout_rmse_sample"] = h.loss(s_idx, s_vals)["rmse"]
        h.set_params(A0, G0)
        if R:
            h.set_kruskal(B0)
        if mu > 0:  # the velocities start at zero again
            VA, VG = h.get_velocity()
            h.set_velocity([np.zeros_like(v) for v in VA], np.zeros_like(VG))
        A1, G1 = h.get_params()
        if not (all(np.array_equal(a, b) for a, b in zip(A0, A1)) and np.array_equal(G0, G1)):
            raise RuntimeError("c3 %s: parameters read back after set_params differ from those set" % dtype)
        h.set_epoch(0)
        for w in range(args.warmup):
            st = h.epoch(1)
            ls = h.loss(test_idx, test_vals)
            log("c3 %s warmup epoch %d: %.3fs device, held-out RMSE %.5f" % (dtype, w, st["device_seconds"],
                                                                           ls["rmse"]))
        acc, rmse = None, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            st = h.epoch(1)
            rmse.append(h.loss(test_idx, test_vals)["rmse"])
            acc = dict(st) if acc is None else {key: acc[key] + st[key] for key in st}
            log("c3 %s step %d: chain %.3fs schedule %.4fs held-out RMSE %.5f" % (
                dtype, k, st["chain_seconds"], st["schedule_seconds"], rmse[-1]))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        updates = acc["updates"]
        lat = latency_bound(h, M, len(wl.dims), updates / acc["chain_seconds"])
        h.close()
        r.update({"value": round(updates / elapsed, 1), "ms_per_step": round(elapsed / args.steps * 1e3, 3),
                  "device_updates_per_s": round(updates / acc["device_seconds"], 1),
                  "heldout_rmse_per_step": [round(x, 6) for x in rmse],
                  "roofline": chain_roofline(acc, dtype, stored_traffic(traffic_path("planted_powerlaw", dtype),
                                                                         dtype, wl.nnz, M, info), lat)})
        res[dtype] = r
    if worker is not None:
        log("waiting for the oracle")
        worker.join()
    head = res[dtypes[0]]
    precision = None
    if prefix > 0 and "A" in orc:
        precision = {"prefix_minibatches": prefix, "heldout_sample": sample,
                     "rmse_oracle_f64": round(orc["rmse"], 9)}
        for dtype in dtypes:
            pp = res[dtype].pop("prefix_params")
            Ag, Gg = pp[0], pp[1]
            rg = res[dtype].pop("prefix_heldout_rmse_sample")
            errs = [rel_err(Ag[n], orc["A"][n]) for n in range(len(wl.dims))] + [rel_err(Gg, orc["G"])]
            if R:
                errs += [rel_err(pp[2][n], orc["B"][n]) for n in range(len(wl.dims))]
            precision[dtype] = {"rmse": round(rg, 9), "rmse_rel_gap": (rg - orc["rmse"]) / orc["rmse"],
                                "params_max_rel_err": max(errs)}
    else:
        for dtype in dtypes:
            res[dtype].pop("prefix_params", None)
            res[dtype].pop("prefix_heldout_rmse_sample", None)
    cpu = None
    if cpu_batches > 0 and "seconds" in orc:
        cpu = dict({"value": round(cpu_batches * M / orc["seconds"], 1), "unit": "nonzero-updates/s", "cores": 1,
                    "kind": "oracle",
                    "sample": "first %d minibatches (%d updates) of epoch 0 from the same initial parameters, FP64 C, "
                              "one thread" % (cpu_batches, cpu_batches * M)}, **host_cpu())
    if len(dtypes) > 1 and head["value"]:
        for dtype in dtypes[1:]:
            res[dtype]["speedup_vs_%s" % dtypes[0]] = round(res[dtype]["value"] / head["value"], 4)
    out = {"metric": METRIC, "value": head["value"],
           "unit": "nonzero-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtypes[0], "data": "synthetic",
           "config": {"workload": "planted_powerlaw 100000x100000x1000x100, %d entries (Zipf 1.2 on modes 1-2, "
                                  "uniform on 3-4), planted rank 8^4 + N(0,0.05^2), 10%% held out; J=(8,8,8,8), "
                                  "M=8192, lr=0.05, lambda=1e-4%s%s; step = 1 epoch + held-out RMSE" % (
                                      nnz, "; Kruskal core R=%d" % R if R else "",
                                      "; heavy-ball momentum mu=%g" % mu if mu > 0 else ""),
                      "train_entries": int(wl.nnz), "batch": M, "r_core": R, "momentum": mu, "chain_workgroups": head["chain_workgroups"],
                      "chain_chunk": head["chain_chunk"], "chain_placement": head["chain_placement"]},
           "heldout_rmse": head["heldout_rmse_per_step"][-1] if head["heldout_rmse_per_step"] else None,
           "roofline": head["roofline"], "precision": precision, "cpu_baseline": cpu}
    for dtype in dtypes[1:]:
        out[dtype] = res[dtype]
    print(json.dumps(out), flush=True)


def oracle_prefix(wl, A0, G0, M, lr, lam, seed, nb, nb_timed, s_idx, s_vals, out, B0=None, mu=0.0):
    """The FP64 oracle on minibatches [0, nb) of epoch 0 from (A0, G0): the
    entries of those minibatches are taken in the oracle's own epoch order
    and run as a tensor of nb * M entries in identity order (the same
    minibatches); the first nb_timed are timed apart.  Fills out['A'],
    out['G'], out['rmse'] (held-out sample) and out['seconds'].  mu > 0:
    with heavy-ball momentum from zero velocities."""
    import numpy as np
    from oracle import oracle
    oracle.build()
    T = wl.nnz
    order = oracle.perm(T, seed, 0)[: min(T, nb * M)]
    idx = np.ascontiguousarray(wl.train_idx[:, order])
    vals = np.ascontiguousarray(wl.train_vals[order])
    del order
    kw = {}
    if mu > 0:
        ref = oracle.MomentumModel(wl.dims, wl.ranks, [a.astype(np.float64) for a in A0], G0.astype(np.float64))
        kw = {"mu": mu}
    elif B0 is None:
        ref = oracle.Model(wl.dims, wl.ranks, [a.astype(np.float64) for a in A0], G0.astype(np.float64))
    else:  # the Kruskal core: the model's core is the product of B0
        ref = oracle.KruskalModel(wl.dims, wl.ranks, [a.astype(np.float64) for a in A0],
                                  [b.astype(np.float64) for b in B0])
    cut = min(idx.shape[1], nb_timed * M)
    log("oracle: running %d minibatches of epoch 0 (%d timed)" % (nb, nb_timed))
    t = time.perf_counter()
    if cut > 0:
        ref.run(idx[:, :cut], vals[:cut], M, lr, lam, lr, lam, perm=np.arange(cut, dtype=np.int64), **kw)
    out["seconds"] = time.perf_counter() - t
    if idx.shape[1] > cut:
        rest = idx.shape[1] - cut
        ref.run(idx[:, cut:], vals[cut:], M, lr, lam, lr, lam, perm=np.arange(rest, dtype=np.int64), **kw)
    out["rmse"] = ref.loss(s_idx, s_vals)["rmse"]
    out["A"] = [a.copy() for a in ref.A]
    out["G"] = ref.G.copy()
    if B0 is not None:
        out["B"] = [b.copy() for b in ref.B]
    log("oracle: %d minibatches in %.1fs (first %d in %.1fs), sample held-out RMSE %.6f" % (
        nb, time.perf_counter() - t, nb_timed, out["seconds"], out["rmse"]))


def rel_err(a, ref):
    import numpy as np
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    n = np.linalg.norm(ref.ravel())
    d = np.linalg.norm((a - ref).ravel())
    return float(d / n) if n > 0 else float(d)


def chain_roofline(acc, dtype, traffic, lat):
    """Roofline object of the minibatch chain from the library's HIP-event
    times on its own stream: MFMA (the contractions) against the dtype's dense
    peak, and HBM, algorithmic bytes and counter traffic per launch against
    the 8 TB/s peak."""
    launches = acc["chain_launches"]
    avg = acc["chain_seconds"] / launches
    flops = acc["flops_alg"] / launches
    alg = acc["bytes_alg"] / launches
    peak = PEAK["bf16_TFs"] if dtype == "bf16" else PEAK["fp32_TFs"]
    ach = flops / avg / 1e12
    hbm = {"alg_bytes_per_launch": int(alg), "alg_GBs": round(alg / avg / 1e9, 3),
           "alg_frac": round(alg / avg / 1e9 / PEAK["hbm_GBs"], 6), "peak_GBs": PEAK["hbm_GBs"]}
    if traffic:
        hbm.update({"traffic_bytes_per_launch": int(traffic), "traffic_GBs": round(traffic / avg / 1e9, 3),
                    "traffic_frac": round(traffic / avg / 1e9 / PEAK["hbm_GBs"], 6),
                    "traffic_over_alg": round(traffic / alg, 3)})
    return {"bound": "mfma", "achieved": round(ach, 4), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 6),
            "traffic": int(traffic) if traffic else None, "kernel": "k_chain", "launches": launches,
            "avg_launch_ms": round(avg * 1e3, 3), "hbm": hbm, "latency_bound": lat}


def run_c4(args):
    """64 independent three-mode tensors (mode sizes 10^U(3,6), 10^U(4,7)
    entries, uniform indices, equal ranks from {4, 8, 16}, planted models plus
    N(0, 0.01^2) noise); M = 1024, lr = lambda = 0.01.  The chunk (and so the
    workgroups per chain) is one for the whole batch: --chunk, or by default
    the tuner's pick from timing one batched epoch with each candidate.  One
    batched call per epoch runs all 64 chains in one cooperative launch:
    slots of W workgroups, as many as the device holds, each running a list
    of chains balanced on the host (longest first).  The comparison runs
    every model alone, one after another.  value = all models'
    nonzero-updates per second of batched epochs."""
    import numpy as np
    import torch
    from oracle import oracle
    from paper_2012_03550_amd import binding, synth, tune

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t = time.time()
    wls = synth.planted_batch(n=64, device="cuda")
    total = sum(w.nnz for w in wls)
    log("generated %d tensors, %d entries in %.1fs" % (len(wls), total, time.time() - t))
    M, lr, lam = 1024, 0.01, 0.01
    res = {}
    for dtype in ("f32", "bf16"):
        if args.chunk > 0:
            chunk, rates = args.chunk, None
        else:  # one chunk for the whole batch, by timing a batched epoch with each candidate
            t = time.time()
            chunk, rates = tune.tune_batch([(w.dims, w.ranks, w.train_idx, w.train_vals) for w in wls], M, dtype=dtype,
                                           lr=lr, lam=lam)
            log("c4 %s tuner (%.1fs): %s -> chunk %d" % (dtype, time.time() - t,
                                                       {c: "%.3e" % r for c, r in rates.items()}, chunk))
        hs = [binding.Stdecomp(w.dims, w.ranks, w.train_idx, w.train_vals, batch=M, lr_factor=lr, lr_core=lr,
                               lam_factor=lam, lam_core=lam, seed_sample=3004 + k, seed_init=2004 + k, chunk=chunk,
                               dtype=dtype) for k, w in enumerate(wls)]
        for _ in range(max(1, args.warmup)):
            binding.epoch_batched(hs, 1)
        torch.cuda.synchronize()
        acc = {"chain_seconds": 0.0, "chain_launches": 0, "flops_alg": 0.0, "bytes_alg": 0.0}
        t0 = time.perf_counter()
        for _ in range(args.steps):
            st = binding.epoch_batched(hs, 1)
            acc["chain_seconds"] += st[0]["chain_seconds"]
            acc["chain_launches"] += st[0]["chain_launches"]
            acc["flops_alg"] += sum(x["flops_alg"] for x in st)
            acc["bytes_alg"] += sum(x["bytes_alg"] for x in st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        batched = total * args.steps / wall
        t0 = time.perf_counter()
        for h in hs:
            h.epoch(1)
        torch.cuda.synchronize()
        alone = total / (time.perf_counter() - t0)
        rmse = [h.loss()["rmse"] for h in hs]
        for h in hs:
            h.close()
        log("c4 %s: batched %.3e updates/s, one model at a time %.3e" % (dtype, batched, alone))
        Js = sorted({w.ranks[0] for w in wls})
        res[dtype] = {"chunk": chunk, "workgroups_per_chain": -(-M // chunk),
                      "tuner_updates_per_s": {str(c): round(r, 1) for c, r in rates.items()} if rates else None,
                      "updates_per_s": round(batched, 1), "alone_updates_per_s": round(alone, 1),
                      "speedup": round(batched / alone, 3), "ms_per_step": round(wall / args.steps * 1e3, 3),
                      "ranks": {str(j): sum(1 for w in wls if w.ranks[0] == j) for j in Js},
                      "roofline": chain_roofline(acc, dtype, None, None),
                      "train_rmse_max": round(max(rmse), 6), "train_rmse_median": round(float(np.median(rmse)), 6)}
    # CPU baseline: the oracle over the four smallest tensors, one epoch each
    oracle.build()
    small = sorted(range(len(wls)), key=lambda k: wls[k].nnz)[:4]
    upd = 0
    t = time.perf_counter()
    for k in small:
        w = wls[k]
        A0, G0 = synth.init_params(w.dims, w.ranks, seed=2004 + k)
        ref = oracle.Model(w.dims, w.ranks, [a.astype(np.float64) for a in A0], G0.astype(np.float64))
        ref.run(w.train_idx, w.train_vals, M, lr, lam, lr, lam, seed=3004 + k, epoch0=0, n_epochs=1)
        upd += w.nnz
    dt = time.perf_counter() - t
    out = {"metric": METRIC, "value": res["f32"]["updates_per_s"],
           "unit": "nonzero-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": max(1, args.warmup),
           "ms_per_step": res["f32"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "64 planted three-mode tensors, mode sizes 10^U(3,6), 10^U(4,7) entries, J from "
                                  "{4,8,16}, M=1024, lr=lambda=0.01; step = 1 epoch of every tensor, one batched launch",
                      "tensors": len(wls), "entries": int(total), "batch": M, "chunk": res["f32"]["chunk"]},
           "roofline": res["f32"]["roofline"], "f32": res["f32"], "bf16": res["bf16"],
           "cpu_baseline": dict({"value": round(upd / dt, 1), "unit": "nonzero-updates/s", "cores": 1, "kind": "oracle",
                                 "sample": "one epoch of each of the 4 smallest tensors (%d updates), FP64 C, one "
                                           "thread, from the host initialiser's own draw (a timing sample)" % upd},
                                **host_cpu())}
    print(json.dumps(out), flush=True)


def run_c5(args):
    """Serving: decomposition jobs arrive by a Poisson process (20/s for
    --duration seconds), each a planted tensor of order 3, 4 or 5 with
    10^U(4,8) entries, mode sizes 10^U(3,6), equal ranks J uniform in 4..16,
    N(0, 0.01^2) noise, 5 epochs, M = 1024; completion queries (random index
    tuples of a resident model) arrive at 10^5/s.  A background thread admits
    jobs by device footprint (a job whose core and tables exceed one
    workgroup's LDS is rejected with the library's reason) and runs rounds of
    one epoch of every resident job, batched launches over the device's
    slots; the main thread submits arrivals and answers the queries that have
    arrived, every 2 ms, on the handles' query streams beside the training
    launches.  value = nonzero-updates/s over the whole run; offered load =
    the arriving jobs' updates (entries x epochs) per second of arrivals."""
    import threading

    import numpy as np
    import torch
    from paper_2012_03550_amd import serve, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    rng = np.random.default_rng(1005)
    D = args.duration
    jobs, t = [], 0.0
    t_gen = time.time()
    while True:
        t += rng.exponential(1 / 20.0)
        if t > D:
            break
        N = int(rng.choice([3, 4, 5]))
        J = int(rng.integers(4, 17))
        dims = tuple(int(10 ** rng.uniform(3, 6)) for _ in range(N))
        nnz = int(10 ** rng.uniform(4, 8))
        idx = np.stack([synth.uniform_indices(rng, I, nnz) for I in dims])
        A, G = synth.planted_model(rng, dims, (J,) * N)
        P = J ** N
        if P <= 1 << 14:  # (chunks of entries sized so the contraction's product stays near 1 GB)
            clean = synth.evaluate_planted_device(A, G, (J,) * N, idx, "cuda", chunk=max(1024, (1 << 27) // P))
        else:  # a core this large does not fit one workgroup's LDS: the library rejects the job at admission
            clean = np.zeros(nnz)
        vals = (clean + rng.standard_normal(nnz) * 0.01).astype(np.float32)
        jobs.append(serve.Job(len(jobs), t, dims, (J,) * N, idx, vals, epochs=5, seed=3005 + len(jobs)))
    qarr = np.sort(rng.uniform(0.0, D, rng.poisson(1e5 * D)))
    offered = sum(j.idx.shape[1] * j.epochs for j in jobs) / D
    log("trace: %d jobs (%d entries), %d queries; generated in %.1fs; offered %.3e updates/s" %
        (len(jobs), sum(j.idx.shape[1] for j in jobs), qarr.size, time.time() - t_gen, offered))
    srv = serve.Server(hbm_budget=200 << 30, chunk=0, dtype=args.dtype)
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0  # noqa: E731
    stop = threading.Event()
    trainer = threading.Thread(target=srv.run, args=(clock, stop), daemon=True)
    trainer.start()
    qlat, qpos, ji, dropped = [], 0, 0, 0
    last_log = 0.0
    while True:
        now = clock()
        while ji < len(jobs) and jobs[ji].arrival <= now:
            srv.submit(jobs[ji])
            ji += 1
        if ji == len(jobs):
            stop.set()
        hi = int(np.searchsorted(qarr, now, side="right"))
        if hi > qpos:
            got = srv.answer(hi - qpos, rng)
            if got:
                done = clock()
                qlat.extend((done - qarr[qpos:hi]).tolist())
                dropped += (hi - qpos) - got
                qpos = hi
        if now - last_log > 10.0:
            last_log = now
            log("t=%.1fs: %d done, %d active, %d waiting, %d rejected, %d queries answered" % (
                now, len(srv.done), len(srv.active), len(srv.pending), len(srv.rejected), len(qlat)))
        if stop.is_set() and not trainer.is_alive():
            break
        if now > D + 900:
            log("stopping: the run exceeded its time limit")
            stop.set()
            break
        time.sleep(0.002)
    trainer.join(timeout=60)
    wall = clock()
    jl = [j.finished - j.arrival for j in srv.done]
    reasons = {}
    for j in srv.rejected:
        reasons[j.rejected.split(":")[-1].strip()[:80]] = reasons.get(j.rejected.split(":")[-1].strip()[:80], 0) + 1
    out = {"metric": METRIC, "value": round(srv.updates / wall, 1),
           "unit": "nonzero-updates/s", "n_gpus": 1, "steps": srv.rounds, "warmup": 0, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": "serving: Poisson jobs 20/s for %gs (order 3-5, 10^U(4,8) entries, mode sizes "
                                  "10^U(3,6), J uniform 4..16, 5 epochs, M=1024) + completion queries 1e5/s" % D,
                      "jobs": len(jobs), "queries": int(qarr.size)},
           "serve": {"jobs_done": len(srv.done), "jobs_rejected": len(srv.rejected), "rejected_reasons": reasons,
                     "job_latency_s_p50": percentile_or_none(jl, 50), "job_latency_s_p99": percentile_or_none(jl, 99),
                     "queries_answered": len(qlat), "queries_dropped": dropped,
                     "query_latency_ms_p50": ms_or_none(percentile_or_none(qlat, 50)),
                     "query_latency_ms_p99": ms_or_none(percentile_or_none(qlat, 99)),
                     "offered_updates_per_s": round(offered, 1),
                     "achieved_updates_per_s": round(srv.updates / wall, 1),
                     "job_train_rmse_median": percentile_or_none([j.rmse for j in srv.done], 50),
                     "wall_s": round(wall, 3), "rounds": srv.rounds}}
    print(json.dumps(out), flush=True)


def percentile_or_none(xs, p):
    import numpy as np
    return round(float(np.percentile(np.asarray(xs, np.float64), p)), 6) if len(xs) else None


def ms_or_none(x):
    return None if x is None else round(1e3 * x, 3)


def run_ranks(args):
    """Core-rank sweep: the ratings workload of config 2 at 20M entries, equal
    ranks J in {4, 6, 8, 10, 12, 16, 20, 24}, M = 4096, two epochs each from
    the scaled initialisation; updates/s of the second epoch and the
    held-out RMSE after it (a rank whose chain does not fit one workgroup's
    LDS is reported as such)."""
    import numpy as np
    import torch
    from paper_2012_03550_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    nnz = 20_000_000
    rows = []
    wl = synth.ratings_zipf(nnz=nnz)
    for J in (4, 6, 8, 10, 12, 16, 20, 24):
        try:
            h = binding.Stdecomp(wl.dims, (J, J, J), wl.train_idx, wl.train_vals, batch=4096, seed_sample=3002,
                                 seed_init=2002, dtype=args.dtype)
        except binding.StdecompError as e:
            rows.append({"J": J, "fits": False, "error": str(e)})
            log("J=%d: %s" % (J, e))
            continue
        h.epoch(1)
        st = h.epoch(1)
        rmse = h.loss(wl.test_idx, wl.test_vals)["rmse"]
        info = h.info()
        h.close()
        per_mb = st["chain_seconds"] / st["minibatches"]
        rows.append({"J": J, "fits": True, "updates_per_s": round(st["updates"] / st["device_seconds"], 1),
                     "us_per_minibatch": round(per_mb * 1e6, 2), "heldout_rmse": round(rmse, 6),
                     "kernel_variant": info["variant"], "workgroups": info["workgroups"],
                     "mfma_TFs": round(st["flops_alg"] / st["chain_seconds"] / 1e12, 4)})
        log("J=%d: %.3e updates/s, %.1f us per minibatch, held-out RMSE %.5f" % (J, rows[-1]["updates_per_s"],
                                                                             per_mb * 1e6, rmse))
    best = max((r["updates_per_s"] for r in rows if r.get("fits")), default=None)
    out = {"metric": METRIC, "value": rows[3].get("updates_per_s") if len(rows) > 3 else best,
           "unit": "nonzero-updates/s", "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": "ratings_zipf 480000x18000x2000 at 20M entries, equal ranks J = 4..24, M=4096; "
                                  "value = J=10", "entries": nnz},
           "sweep": rows}
    print(json.dumps(out), flush=True)


def latency_bound(h, M, N, chain_rate):
    """The chain's grid barrier timed alone: a minibatch is N + 1 dependent
    sub-steps, so no chain exceeds M / ((N + 1) t_sync) updates/s."""
    t = h.barrier_us(2000)
    bound = M / ((N + 1) * t * 1e-6)
    return {"t_sync_us": round(t, 3), "sub_steps": N + 1, "updates_per_s": round(bound, 1),
            "chain_frac": round(chain_rate / bound, 4)}


def host_cpu():
    """The host's CPU model and hardware thread count (where the oracle baseline ran)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"host_cpu": model, "host_threads": os.cpu_count()}


PLACEMENT_NAMES = {1: "spread", 2: "one_xcc"}


def traffic_path(workload, dtype):
    return os.path.join(ROOT, "profiles", "chain_traffic_%s%s.json" % (workload, "" if dtype == "f32" else "_" + dtype))


def stored_traffic(path, dtype, train_entries, batch, info):
    """HBM bytes per chain launch (FETCH_SIZE and WRITE_SIZE scaled by the
    copy-kernel factors) from a stored counter record, if it was taken on this
    kernel source, dtype, training-set size, minibatch size and chain geometry
    (workgroups, chunk, placement); else None."""
    if not os.path.exists(path):
        return None
    tj = json.load(open(path))
    want = {"kernel_source_hash": kernel_source_hash(), "dtype": dtype, "train_entries": int(train_entries),
            "batch": int(batch), "workgroups": int(info["workgroups"]), "chunk": int(info["chunk"]),
            "placement": PLACEMENT_NAMES[info["placement"]]}
    if any(tj.get(k) != v for k, v in want.items()):
        return None
    return tj.get("bytes_per_launch")


def kernel_source_hash():
    import hashlib
    hsh = hashlib.sha256()
    for f in ("stdecomp_chain_body.h", "stdecomp_chain.hip", "stdecomp_chain_xcc.hip", "stdecomp_device.h", "stdecomp_internal.h"):
        hsh.update(open(os.path.join(ROOT, "paper_2012_03550_amd", "csrc", f), "rb").read())
    return hsh.hexdigest()[:16]


def cpu_baseline(h, wl, A0, G0, M, lr, lam, nbatches):
    """The FP64 oracle (single thread) on the first `nbatches` minibatches of
    epoch 0 from the same initial parameters, plus the GPU's result on the
    same prefix for a parity check."""
    import numpy as np
    from oracle import oracle
    from paper_2012_03550_amd import binding
    oracle.build()
    ref = oracle.Model(wl.dims, wl.ranks, [a.astype(np.float64) for a in A0], G0.astype(np.float64))
    log("oracle: running %d minibatches of epoch 0" % nbatches)
    t = time.perf_counter()
    ref.run(wl.train_idx, wl.train_vals, M, lr, lam, lr, lam, seed=3002, epoch0=0, n_epochs=1,
            max_batches=nbatches)
    dt = time.perf_counter() - t
    g = binding.Stdecomp(wl.dims, wl.ranks, wl.train_idx, wl.train_vals, batch=M, lr_factor=lr, lr_core=lr,
                         lam_factor=lam, lam_core=lam, seed_sample=3002, init="caller")
    g.set_params(A0, G0)
    g.run_minibatches(0, 0, nbatches)
    Ag, Gg = g.get_params()
    g.close()
    err = max([float(np.linalg.norm(Ag[n] - ref.A[n]) / np.linalg.norm(ref.A[n])) for n in range(3)] +
              [float(np.linalg.norm(Gg - ref.G) / np.linalg.norm(ref.G))])
    log("cpu oracle: %d minibatches in %.2fs; GPU vs oracle on that prefix: max rel err %.3g" % (nbatches, dt, err))
    return dict({"value": round(nbatches * M / dt, 1), "unit": "nonzero-updates/s", "cores": 1, "kind": "oracle",
                 "sample": "first %d minibatches (%d updates) of epoch 0 from the same initial parameters, FP64 C, "
                           "one thread" % (nbatches, nbatches * M),
                 "gpu_prefix_max_rel_err": err}, **host_cpu())


if __name__ == "__main__":
    main()
