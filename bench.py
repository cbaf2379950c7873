"""Throughput of the SGD_Tucker minibatch update on one MI355X.

Workload: the Netflix-shaped rating tensor -- 480000 x 18000 x 2000, 100M
nonzeros with Zipf(1.1) indices per mode and ratings 1..5, 10% held out --
with core ranks J = (10, 10, 10) and minibatches of M = 4096 (synthetic data,
random initial parameters).  One step = one epoch over the ~90M training
entries (sampler, row-set sort, minibatch chain) followed by the held-out
RMSE.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--dtype f32|bf16]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

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
    ap.add_argument("--nnz", type=int, default=100_000_000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--cpu-batches", type=int, default=60,
                    help="minibatches of the CPU oracle baseline (0: skip)")
    ap.add_argument("--traffic-json", default=None,
                    help="counter record of the chain (default: profiles/chain_traffic.json for FP32, "
                         "profiles/chain_traffic_bf16.json for BF16)")
    ap.add_argument("--duration", type=float, default=10.0, help="(c5) seconds of job arrivals")
    ap.add_argument("--config", default="c2", choices=["c2", "c3", "c4", "c5", "ranks"],
                    help="c2: Netflix-shaped ratings (default); c3: 4-order planted power-law tensor, FP32 vs BF16; "
                         "c4: 64 independent planted tensors, batched launches vs one model at a time; "
                         "c5: serving loop (Poisson jobs and queries), p50/p99 latency; "
                         "ranks: core-rank sweep J = 4..24 on a ratings tensor")
    ap.add_argument("--epochs", type=int, default=5, help="(c3) epochs per precision")
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
        print("bench.py runs on one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.config == "c3":
        run_c3(args)
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

    import numpy as np
    import torch

    from paper_2012_03550_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t = time.time()
    wl = synth.ratings_zipf(nnz=args.nnz)
    log("generated %d training / %d held-out entries in %.1fs" % (wl.nnz, wl.test_vals.size, time.time() - t))
    M = args.batch
    lr = lam = 0.01
    h = binding.Stdecomp(wl.dims, wl.ranks, wl.train_idx, wl.train_vals, batch=M, lr_factor=lr, lr_core=lr,
                         lam_factor=lam, lam_core=lam, seed_sample=3002, seed_init=2002, dtype=args.dtype,
                         chunk=args.chunk)
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
    launches = acc["chain_launches"]
    avg_launch = acc["chain_seconds"] / launches
    flops_per_launch = acc["flops_alg"] / launches
    achieved = flops_per_launch / avg_launch / 1e12
    peak = PEAK["bf16_TFs"] if args.dtype == "bf16" else PEAK["fp32_TFs"]
    traffic = None
    tpath = args.traffic_json or os.path.join(
        ROOT, "profiles", "chain_traffic.json" if args.dtype == "f32" else "chain_traffic_%s.json" % args.dtype)
    if os.path.exists(tpath):
        tj = json.load(open(tpath))
        if tj.get("kernel_source_hash") == kernel_source_hash() and tj.get("dtype") == args.dtype:
            traffic = tj.get("bytes_per_launch")
    roofline = {"bound": "mfma", "achieved": round(achieved, 4), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 6), "traffic": traffic,
                "kernel": "k_chain", "avg_launch_ms": round(avg_launch * 1e3, 3),
                "hbm_alg_GBs": round(acc["bytes_alg"] / acc["chain_seconds"] / 1e9, 2),
                "latency_bound": latency_bound(h, M, len(wl.dims), updates / acc["chain_seconds"])}

    cpu = None
    if args.cpu_batches > 0:
        cpu = cpu_baseline(h, wl, A0, G0, M, lr, lam, args.cpu_batches)
    h.close()

    out = {
        "metric": "nonzero-updates/sec/GPU at fixed held-out RMSE",
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
                   "chain_chunk": info["chunk"]},
        "heldout_rmse": round(ls["rmse"], 6),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_c3(args):
    """4-order planted power-law tensor 100000x100000x1000x100, 200M entries
    (Zipf 1.2 on modes 1-2, uniform on 3-4), planted rank (8,8,8,8) plus
    N(0, 0.05^2) noise, 10% held out; J = (8,8,8,8), M = 8192, lr = 0.05,
    lambda = 1e-4 (at lr = lambda = 0.01, or lambda = 1e-3, the model decays
    to the zero saddle and stays there; at lr = 0.1 it diverges in the first
    epoch), ``--epochs`` epochs in FP32 and in BF16 from the same initial
    parameters.  Precision: the FP64 oracle, the FP32 chain and the BF16 chain
    run the same first 200 minibatches of epoch 0 and their held-out RMSE is
    compared on a 200,000-entry sample of the held-out set."""
    import numpy as np
    import torch
    from oracle import oracle
    from paper_2012_03550_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    nnz = args.nnz if args.nnz != 100_000_000 else 200_000_000
    t = time.time()
    wl = synth.planted_powerlaw(nnz=nnz, device="cuda")
    log("generated %d training / %d held-out entries in %.1fs" % (wl.nnz, wl.test_vals.size, time.time() - t))
    M, lr, lam, prefix, sample = 8192, 0.05, 1e-4, 200, 200_000
    test_idx = torch.from_numpy(wl.test_idx).cuda()
    test_vals = torch.from_numpy(wl.test_vals).cuda()
    s_idx = np.ascontiguousarray(wl.test_idx[:, :sample])
    s_vals = np.ascontiguousarray(wl.test_vals[:sample])
    res = {}
    A0 = G0 = None
    for dtype in ("f32", "bf16"):
        h = binding.Stdecomp(wl.dims, wl.ranks, wl.train_idx, wl.train_vals, batch=M, lr_factor=lr, lr_core=lr,
                             lam_factor=lam, lam_core=lam, seed_sample=3003, seed_init=2003, dtype=dtype)
        if A0 is None:
            A0, G0 = h.get_params()
        h.run_minibatches(0, 0, prefix)
        prefix_rmse = h.loss(s_idx, s_vals)["rmse"]
        h.set_params(A0, G0)
        A1, G1 = h.get_params()
        if not (all(np.array_equal(a, b) for a, b in zip(A0, A1)) and np.array_equal(G0, G1)):
            raise RuntimeError("c3 %s: parameters read back after set_params differ from those set" % dtype)
        h.set_epoch(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dev = 0.0
        chain_s = 0.0
        launches = 0
        bytes_alg = 0.0
        rmse = []
        done = 0
        for e in range(args.epochs):
            try:
                st = h.epoch(1)
            except binding.StdecompError as ex:
                log("c3 %s epoch %d: %s" % (dtype, e, ex))
                rmse.append("diverged")
                break
            done += 1
            dev += st["device_seconds"]
            chain_s += st["chain_seconds"]
            launches += st["chain_launches"]
            bytes_alg += st["bytes_alg"]
            rmse.append(round(h.loss(test_idx, test_vals)["rmse"], 6))
            log("c3 %s epoch %d: chain %.3fs held-out RMSE %.5f" % (dtype, e, st["chain_seconds"], rmse[-1]))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        info = h.info()
        lat = latency_bound(h, M, len(wl.dims), wl.nnz * done / chain_s) if done else None
        h.close()
        flops = (2 * len(wl.dims) + 4) * int(np.prod(wl.ranks))  # per nonzero-update
        peak = 157.3 if dtype == "f32" else 2500.0
        ach = wl.nnz * done * flops / chain_s / 1e12 if done else None
        res[dtype] = {"updates_per_s": round(wl.nnz * done / wall, 1) if done else None, "device_updates_per_s":
                      round(wl.nnz * done / dev, 1) if done else None,
                      "roofline": {"bound": "mfma", "achieved": round(ach, 4) if done else None, "peak": peak,
                                   "unit": "TFLOP/s", "frac": round(ach / peak, 6) if done else None,
                                   "traffic": c3_traffic(dtype, wl.nnz), "kernel": "k_chain",
                                   "chain_seconds": round(chain_s, 4), "chain_launches": launches,
                                   "avg_launch_ms": round(chain_s / launches * 1e3, 3) if launches else None,
                                   "alg_bytes_per_launch": int(bytes_alg / launches) if launches else None,
                                   "latency_bound": lat},
                      "heldout_rmse_per_epoch": rmse,
                      "prefix_heldout_rmse_sample": prefix_rmse, "chain_workgroups": info["workgroups"],
                      "chain_chunk": info["chunk"]}
    precision = cpu = None
    if args.cpu_batches > 0:  # (--cpu-batches 0: no oracle, for profiling runs)
        oracle.build()
        ref = oracle.Model(wl.dims, wl.ranks, [a.astype(np.float64) for a in A0], G0.astype(np.float64))
        log("oracle: running %d minibatches of epoch 0" % prefix)
        t = time.perf_counter()
        ref.run(wl.train_idx, wl.train_vals, M, lr, lam, lr, lam, seed=3003, epoch0=0, n_epochs=1, max_batches=prefix)
        dt = time.perf_counter() - t
        orc = ref.loss(s_idx, s_vals)["rmse"]
        log("oracle: %d minibatches in %.1fs, sample held-out RMSE %.6f" % (prefix, dt, orc))
        precision = {"prefix_minibatches": prefix, "heldout_sample": sample, "rmse_oracle_f64": orc,
                     "rmse_f32": res["f32"]["prefix_heldout_rmse_sample"],
                     "rmse_bf16": res["bf16"]["prefix_heldout_rmse_sample"],
                     "f32_rel_gap": (res["f32"]["prefix_heldout_rmse_sample"] - orc) / orc,
                     "bf16_rel_gap": (res["bf16"]["prefix_heldout_rmse_sample"] - orc) / orc}
        cpu = dict({"value": round(prefix * M / dt, 1), "unit": "nonzero-updates/s", "cores": 1, "kind": "oracle",
                    "sample": "first %d minibatches of epoch 0, FP64 C, one thread" % prefix}, **host_cpu())
    out = {"metric": "nonzero-updates/sec/GPU at fixed held-out RMSE", "value": res["f32"]["updates_per_s"],
           "unit": "nonzero-updates/s", "n_gpus": 1, "steps": args.epochs, "warmup": 0, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "planted_powerlaw 100000x100000x1000x100, %d entries (Zipf 1.2 on modes 1-2, "
                                  "uniform on 3-4), planted rank 8^4 + N(0,0.05^2), 10%% held out; J=(8,8,8,8), "
                                  "M=8192, lr=0.05, lambda=1e-4; step = 1 epoch + held-out RMSE" % nnz,
                      "train_entries": int(wl.nnz), "batch": M},
           "roofline": res["f32"]["roofline"], "f32": res["f32"], "bf16": res["bf16"], "precision": precision,
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def run_c4(args):
    """64 independent three-mode tensors (mode sizes 10^U(3,6), 10^U(4,7)
    entries, uniform indices, equal ranks from {4, 8, 16}, planted models plus
    N(0, 0.01^2) noise); M = 1024, lr = lambda = 0.01, 128-entry chunks.
    Models of one rank share a kernel and run as one batched launch per
    epoch; the comparison runs every model alone.  value = all models'
    nonzero-updates per second of batched epochs."""
    import numpy as np
    import torch
    from oracle import oracle
    from paper_2012_03550_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t = time.time()
    wls = synth.planted_batch(n=64, device="cuda")
    total = sum(w.nnz for w in wls)
    log("generated %d tensors, %d entries in %.1fs" % (len(wls), total, time.time() - t))
    M, lr, lam, chunk = 1024, 0.01, 0.01, 128
    res = {}
    for dtype in ("f32", "bf16"):
        hs = [binding.Stdecomp(w.dims, w.ranks, w.train_idx, w.train_vals, batch=M, lr_factor=lr, lr_core=lr,
                               lam_factor=lam, lam_core=lam, seed_sample=3004 + k, seed_init=2004 + k, chunk=chunk,
                               dtype=dtype) for k, w in enumerate(wls)]
        groups = {}
        for h, w in zip(hs, wls):
            groups.setdefault(w.ranks[0], []).append(h)
        for g in groups.values():  # warm-up epoch
            binding.epoch_batched(g, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for g in groups.values():
                binding.epoch_batched(g, 1)
        torch.cuda.synchronize()
        batched = total * args.steps / (time.perf_counter() - t0)
        t0 = time.perf_counter()
        for h in hs:
            h.epoch(1)
        torch.cuda.synchronize()
        alone = total / (time.perf_counter() - t0)
        rmse = [h.loss()["rmse"] for h in hs]
        for h in hs:
            h.close()
        log("c4 %s: batched %.3e updates/s, one model at a time %.3e" % (dtype, batched, alone))
        res[dtype] = {"updates_per_s": round(batched, 1), "alone_updates_per_s": round(alone, 1),
                      "speedup": round(batched / alone, 3), "groups": {str(j): len(g) for j, g in groups.items()},
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
    out = {"metric": "nonzero-updates/sec/GPU at fixed held-out RMSE", "value": res["f32"]["updates_per_s"],
           "unit": "nonzero-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "64 planted three-mode tensors, mode sizes 10^U(3,6), 10^U(4,7) entries, J from "
                                  "{4,8,16}, M=1024, lr=lambda=0.01; step = 1 epoch of every tensor, batched per rank",
                      "tensors": len(wls), "entries": int(total), "batch": M, "chunk": chunk},
           "f32": res["f32"], "bf16": res["bf16"],
           "cpu_baseline": dict({"value": round(upd / dt, 1), "unit": "nonzero-updates/s", "cores": 1, "kind": "oracle",
                                 "sample": "one epoch of each of the 4 smallest tensors (%d updates), FP64 C, one "
                                           "thread, from the host initialiser's own draw (a timing sample)" % upd},
                                **host_cpu())}
    print(json.dumps(out), flush=True)


def run_c5(args):
    """Serving: decomposition jobs arrive by a Poisson process (20/s for
    --duration seconds), each a planted tensor of order 3 or 4 with
    10^U(4,6) entries, mode sizes 10^U(3,5), equal ranks from {4, 8, 16}
    (order 4: {4, 8}), N(0, 0.01^2) noise, 5 epochs, M = 1024; completion
    queries (random index tuples of a resident model) arrive at 10^5/s.
    Jobs are admitted by device footprint and advance one epoch per round,
    jobs with the same kernel in one batched launch; queries are answered
    between rounds.  value = nonzero-updates/s over the whole run."""
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
        N = int(rng.choice([3, 4]))
        J = int(rng.choice([4, 8, 16] if N == 3 else [4, 8]))
        dims = tuple(int(10 ** rng.uniform(3, 5)) for _ in range(N))
        nnz = int(10 ** rng.uniform(4, 6))
        idx = np.stack([synth.uniform_indices(rng, I, nnz) for I in dims])
        A, G = synth.planted_model(rng, dims, (J,) * N)
        clean = synth.evaluate_planted_device(A, G, (J,) * N, idx, "cuda")
        vals = (clean + rng.standard_normal(nnz) * 0.01).astype(np.float32)
        jobs.append(serve.Job(len(jobs), t, dims, (J,) * N, idx, vals, epochs=5, seed=3005 + len(jobs)))
    qarr = np.sort(rng.uniform(0.0, D, rng.poisson(1e5 * D)))
    log("trace: %d jobs (%d entries), %d queries; generated in %.1fs" %
        (len(jobs), sum(j.idx.shape[1] for j in jobs), qarr.size, time.time() - t_gen))
    srv = serve.Server(hbm_budget=100 << 30, dtype=args.dtype)
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0  # noqa: E731
    qlat = []
    qpos = [0]

    def answer_queries():  # every query that has arrived, if a model is resident
        hi = int(np.searchsorted(qarr, clock(), side="right"))
        if hi > qpos[0] and srv.answer(hi - qpos[0], rng):
            done = clock()
            qlat.extend((done - qarr[qpos[0]:hi]).tolist())
            qpos[0] = hi

    ji = 0
    rounds = 0
    while ji < len(jobs) or srv.pending or srv.active:
        now = clock()
        while ji < len(jobs) and jobs[ji].arrival <= now:
            srv.submit(jobs[ji])
            ji += 1
        srv.admit(now)
        if srv.active:
            srv.round(clock, answer_queries)
            rounds += 1
        elif ji < len(jobs):
            time.sleep(max(0.0, jobs[ji].arrival - clock()))
        answer_queries()
        if rounds and rounds % 50 == 0:
            log("round %d: t=%.1fs, %d done, %d active, %d waiting" % (rounds, clock(), len(srv.done),
                                                                    len(srv.active), len(srv.pending)))
        if clock() > D + 600:
            log("stopping: the run exceeded its time limit")
            break
    wall = clock()
    jl = [j.finished - j.arrival for j in srv.done]
    out = {"metric": "nonzero-updates/sec/GPU at fixed held-out RMSE", "value": round(srv.updates / wall, 1),
           "unit": "nonzero-updates/s", "n_gpus": 1, "steps": rounds, "warmup": 0, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": "serving: Poisson jobs 20/s for %gs (order 3-4, 10^U(4,6) entries, J in {4,8,16}, "
                                  "5 epochs, M=1024) + completion queries 1e5/s" % D,
                      "jobs": len(jobs), "queries": int(qarr.size)},
           "serve": {"jobs_done": len(srv.done), "job_latency_s_p50": percentile_or_none(jl, 50),
                     "job_latency_s_p99": percentile_or_none(jl, 99),
                     "queries_answered": len(qlat), "query_latency_ms_p50": ms_or_none(percentile_or_none(qlat, 50)),
                     "query_latency_ms_p99": ms_or_none(percentile_or_none(qlat, 99)),
                     "job_train_rmse_median": percentile_or_none([j.rmse for j in srv.done], 50),
                     "wall_s": round(wall, 3), "rounds": rounds}}
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
    out = {"metric": "nonzero-updates/sec/GPU at fixed held-out RMSE", "value": rows[3].get("updates_per_s") if len(rows) > 3 else best,
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


def c3_traffic(dtype, train_entries):
    """HBM bytes per chain launch of the config-3 epoch (FETCH_SIZE and
    WRITE_SIZE scaled by the copy-kernel factors), if the stored counter record
    was taken on this kernel source, dtype and training-set size; else None."""
    path = os.path.join(ROOT, "profiles", "chain_traffic_planted_powerlaw%s.json" % ("" if dtype == "f32" else "_bf16"))
    if not os.path.exists(path):
        return None
    tj = json.load(open(path))
    if (tj.get("kernel_source_hash") != kernel_source_hash() or tj.get("dtype") != dtype
            or tj.get("train_entries") != train_entries):
        return None
    return tj.get("bytes_per_launch")


def kernel_source_hash():
    import hashlib
    hsh = hashlib.sha256()
    for f in ("stdecomp_chain.hip", "stdecomp_device.h", "stdecomp_internal.h"):
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
