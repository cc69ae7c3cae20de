#!/usr/bin/env python3
"""End-to-end DPar2 benchmark on one MI355X.

Workload: a US-Stock-shaped irregular tensor (K = 4000 slices, J = 88
features, lognormal history lengths I_k in [200, 8000] with median 1500,
rank-10 PARAFAC2 entries with feature scales over 1e-2..1e3 and 5% noise;
N ~ 7.66M rows, 2.70 GB float32), R = 10, oversampling 10 (L = 20), 32
iterations.  One step = one whole decomposition from the same initial
factors: two-stage compression (one read of the slab), 32 compressed ALS
iterations and the fitness against the original slices, all on the device
with the slab already resident in HBM.

Prints one JSON line: slices/s, ms per decomposition, the roofline of the
slab-pass kernel (timed with HIP events recorded around it on its launch
stream), and the FP64 oracle timed on a bounded sample of the same workload
on the host cores (with the fitness of both on that sample)."""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
INT8_MFMA_PEAK_TOPS = 5000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=2000,
                    help="slices of the workload the CPU oracle runs on (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the precision form (bf16 and fp8-e4m3 slabs) and the power step timed on "
                         "the same workload")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batching form (256 independent tensors of mixed J, R, K, I_k)")
    ap.add_argument("--batch-tensors", type=int, default=256)
    ap.add_argument("--item-rows", type=int, default=0,
                    help="fixed work-item size of the slab pass (0: choose it with the autotuner)")
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the precision form at J = 2049 (K = 8000, spectrogram-like, R = 10 and 20)")
    ap.add_argument("--wide-k", type=int, default=8000)
    ap.add_argument("--scalability", action="store_true",
                    help="run only the tenrand scalability workloads (five sizes at R = 10, R = 10..50 at "
                         "2000 x 2000 x 4000); one JSON line")
    ap.add_argument("--scale-ranks", default="10,20,30,40,50",
                    help="with --scalability: ranks of the rank sweep at 2000 x 2000 x 4000")
    ap.add_argument("--scale-no-sizes", action="store_true",
                    help="with --scalability: leave out the size sweep at R = 10")
    ap.add_argument("--scalability-plain", action="store_true",
                    help="with --scalability: also time PARAFAC2-ALS (Alg. 2) at every point")
    ap.add_argument("--wide-only", action="store_true",
                    help="run only the J = 2049 form (one JSON line with its figures; for profiling)")
    ap.add_argument("--wide-ranks", default="10,20", help="ranks of the J = 2049 form")
    ap.add_argument("--wide-q", default="0,1", help="power steps of the J = 2049 form")
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the learned warm-start form (train the set encoder, compare on held-out tensors)")
    ap.add_argument("--warm-train", type=int, default=400, help="training tensors of the warm-start form")
    ap.add_argument("--warm-test", type=int, default=32, help="held-out tensors of the warm-start form")
    ap.add_argument("--warm-steps", type=int, default=3000, help="Adam steps (minibatch 32) of the warm-start training")
    ap.add_argument("--warm-no-match", action="store_true",
                    help="warm-start training compares components in the targets' own order (no matching)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip PARAFAC2-ALS on the uncompressed slices (Alg. 2) on the same workload")
    ap.add_argument("--no-down", action="store_true",
                    help="skip the post-processing leg (Sec. IV-E: PCC, Eq. 9 similarity, top-k, RWR)")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the streaming leg (the last 10%% of the slices appended to a decomposition of the rest)")
    ap.add_argument("--cpu-runs", type=int, default=3, help="timed runs of the CPU oracle (mean and median)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter_collection.csv "
                         "files (FETCH_SIZE, WRITE_SIZE) of a --calib-copy run, then exit")
    return ap.parse_args()


SLAB_KERNEL = "k_sketch_q"
CALIB_BYTES = 1 << 30          # the --calib-copy copy reads and writes 1 GiB


def write_traffic(fetch_csv, write_csv):
    """HBM bytes per slab-pass launch from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled so that the 1 GiB calibration copy reads as 1 GiB."""
    import csv

    def per_dispatch(path, counter):
        # the slab pass of the decomposition is the last one launched (the
        # autotuner's launches come first); the copy is the largest copy
        slab, copy = {}, []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            if SLAB_KERNEL in r["Kernel_Name"]:
                d = int(r["Dispatch_Id"])
                slab[d] = slab.get(d, 0.0) + v
            elif "copyBuffer" in r["Kernel_Name"]:
                copy.append(v)
        return slab[max(slab)], max(copy)

    f_slab, f_copy = per_dispatch(fetch_csv, "FETCH_SIZE")
    w_slab, w_copy = per_dispatch(write_csv, "WRITE_SIZE")
    f_scale, w_scale = CALIB_BYTES / f_copy, CALIB_BYTES / w_copy
    rec = {"kernel": SLAB_KERNEL, "source_sha256": slab_source_sha(),
           "fetch_counter_bytes": f_slab, "write_counter_bytes": w_slab,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "bytes_per_launch": int(round(f_slab * f_scale + w_slab * w_scale)),
           "calibration": "1 GiB device copy: FETCH_SIZE and WRITE_SIZE scaled to read as 1 GiB each"}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


SLAB_SOURCES = ("sketch_impl.h", "k_slab_f32.hip", "common.h", "internal.h")


def slab_source_sha():
    """SHA-256 over the sources the FP32 slab-pass kernel is built from."""
    h = hashlib.sha256()
    for name in SLAB_SOURCES:
        with open(os.path.join(ROOT, "paper_2203_12798_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record():
    """HBM bytes per slab-pass launch from the committed counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != slab_source_sha():
        return None
    return rec


def gen_batch(n, d, torch, np):
    """The batching workload: n independent tensors; tensor t draws K ~ U{16..256},
    J from {32, 64, 128}, R from {5, 10, 20} and I_k ~ U{32..2048} from
    numpy's SeedSequence(4).spawn(n)[t]; its entries are a rank-R PARAFAC2
    model (Q_k column-orthonormal from the QR of a Gaussian I_k x R matrix,
    H, V ~ N(0, 1), W ~ U(0.5, 1.5)) plus N(0, 0.05^2) noise, drawn on the
    GPU with torch's generator seeded by t, float32."""
    specs, tensors = [], []
    for t, ss in enumerate(np.random.SeedSequence(4).spawn(n)):
        rng = np.random.default_rng(ss)
        K = int(rng.integers(16, 257))
        J = int(rng.choice([32, 64, 128]))
        R = int(rng.choice([5, 10, 20]))
        rows = rng.integers(32, 2049, size=K)
        g = torch.Generator(device="cuda").manual_seed(t)
        imax = int(rows.max())
        mask = torch.arange(imax, device="cuda")[None, :] < torch.from_numpy(rows).cuda()[:, None]
        G = torch.randn(K, imax, R, device="cuda", generator=g) * mask[:, :, None]
        Q = torch.linalg.qr(G).Q                                     # zero rows stay zero
        H = torch.randn(R, R, device="cuda", generator=g)
        V = torch.randn(J, R, device="cuda", generator=g)
        W = 0.5 + torch.rand(K, R, device="cuda", generator=g)
        Mk = (H[None, :, :] * W[:, None, :]) @ V.t()                 # K x R x J
        Xp = torch.bmm(Q.contiguous(), Mk.contiguous())
        slab = Xp[mask] + 0.05 * torch.randn(int(rows.sum()), J, device="cuda", generator=g)
        offs = np.concatenate([[0], np.cumsum(rows)]).astype(np.int64)
        tensors.append(d.Tensor(slab.contiguous(), torch.from_numpy(offs).cuda(), offs))
        specs.append((K, J, R))
        del G, Q, Xp, Mk
    return specs, tensors


def bench_batch(args, d, torch, np):
    n = args.batch_tensors
    iters = 32
    t = time.perf_counter()
    specs, Ts = gen_batch(n, d, torch, np)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    rows = sum(T.offsets_host[-1] for T in Ts)
    slices = sum(K for K, _, _ in specs)
    print(f"[bench] batch: {n} tensors, {slices} slices, {rows} rows (gen {gen_s:.1f}s)", file=sys.stderr,
          flush=True)
    res = {"tensors": n, "slices": int(slices), "rows": int(rows),
           "slab_gb": round(sum(T.slab.numel() * 4 for T in Ts) / 1e9, 3), "iterations": iters,
           "groups": len({(J, R) for _, J, R in specs})}
    g = torch.Generator(device="cuda").manual_seed(12345)
    om1 = [torch.randn(J, min(R + 10, J), device="cuda", generator=g) for K, J, R in specs]
    om2 = [torch.randn(K * R, min(R + 10, J), device="cuda", generator=g) for K, J, R in specs]
    # all factors in one buffer (views per tensor), re-initialised by one copy
    sizes = [R * R + J * R + K * R for K, J, R in specs]
    init = torch.empty(sum(sizes), dtype=torch.float64, device="cuda")
    flat = torch.empty_like(init)
    fs, at = [], 0
    for (K, J, R), n_el in zip(specs, sizes):
        Hi, Vi, Wi = (init[at:at + R * R].view(R, R), init[at + R * R:at + R * R + J * R].view(J, R),
                      init[at + R * R + J * R:at + n_el].view(K, R))
        Hi.copy_(torch.eye(R, dtype=torch.float64, device="cuda"))
        Vi.copy_(torch.randn(J, R, dtype=torch.float64, device="cuda", generator=g))
        Wi.fill_(1.0)
        fs.append(d.Factors(flat[at:at + R * R].view(R, R), flat[at + R * R:at + R * R + J * R].view(J, R),
                            flat[at + R * R + J * R:at + n_el].view(K, R)))
        at += n_el
    # slab tiling per (J, R) group: dpar2_autotune_slab on the group's largest
    # tensor (rows per work item x whole-row or 128-column-chunk pass), applied
    # to every tensor of the group
    from paper_2203_12798_amd import binding
    cands = [(2048, False), (4096, False), (8192, False), (16384, False), (4096, True), (16384, True)]
    tuned = {}
    for key in sorted({(J, R) for _, J, R in specs}):
        idx = max((i for i, (_, J, R) in enumerate(specs) if (J, R) == key), key=lambda i: Ts[i].offsets_host[-1])
        K, J, R = specs[idx]
        L = min(R + 10, J)
        o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters)
        wst = d.alloc_workspace(Ts[idx], d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters, item_rows=2048,
                                                   wide_slab=True))
        (ir, wide), times = binding.autotune_slab(Ts[idx], o, om1[idx], wst, cands)
        tuned[key] = (ir, wide)
        del wst
    res["autotune"] = {f"J{J}_R{R}": {"item_rows": ir, "pass": "128-column chunks" if wide else "whole rows"}
                       for (J, R), (ir, wide) in tuned.items()}
    for graph, tune in ((False, False), (True, False), (True, True)):
        os_ = [d.Options(rank=R, sketch=min(R + 10, J), sketch2=min(R + 10, J), max_iter=iters, graph=graph,
                         item_rows=tuned[(J, R)][0] if tune else 0, wide_slab=tuned[(J, R)][1] if tune else False)
               for K, J, R in specs]
        ws = d.alloc_batch_workspace(Ts, os_)

        def step():
            flat.copy_(init)
            d.decompose_batch(Ts, os_, om1, om2, fs, ws)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
        reps = d.batch_report_read(Ts, os_, ws)
        key = ("graph" if graph else "eager") + ("_autotuned" if tune else "")
        res[key] = {"ms_per_batch": round(ms, 3), "tensors_per_s": round(n / (ms / 1e3), 1),
                    "slices_per_s": round(slices / (ms / 1e3), 1),
                    "rows_per_s": round(rows / (ms / 1e3), 1)}
        fits = np.array([r["fit_true"] for r in reps])
        res[key]["fitness_min"] = float(fits.min())
        res[key]["fitness_mean"] = float(fits.mean())
        print(f"[bench] batch {key}: {ms:.3f} ms", file=sys.stderr, flush=True)
        del ws
    return res


def gen_warm_tensor(t, seed, d, torch, np):
    """One tensor of the warm-start workload: K ~ U{32..512}, J = 64,
    I_k ~ U{64..1024}, rank-10 PARAFAC2 plus Gaussian noise of 0.01 x the RMS
    of the clean entries; numpy SeedSequence(seed).spawn for the shape,
    torch's generator seeded by (seed, t) for the entries.  Q_k has
    orthonormal columns: the Gaussian I_k x R block made orthonormal by two
    rounds of Cholesky QR in FP64 (batched over the slices; a tall Gaussian
    block is well conditioned, so two rounds reach rounding-level
    orthogonality)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, t]))
    K, J, R = int(rng.integers(32, 513)), 64, 10
    rows = rng.integers(64, 1025, size=K)
    g = torch.Generator(device="cuda").manual_seed(seed * 100003 + t)
    imax = int(rows.max())
    mask = torch.arange(imax, device="cuda")[None, :] < torch.from_numpy(rows).cuda()[:, None]
    Q = (torch.randn(K, imax, R, device="cuda", generator=g) * mask[:, :, None]).double()
    for _ in range(2):
        C = torch.linalg.cholesky(torch.bmm(Q.transpose(1, 2).contiguous(), Q))
        Q = torch.linalg.solve_triangular(C.transpose(1, 2).contiguous(), Q, upper=True, left=False)
    Q = Q.float()
    H = torch.randn(R, R, device="cuda", generator=g)
    V = torch.randn(J, R, device="cuda", generator=g)
    W = 0.5 + torch.rand(K, R, device="cuda", generator=g)
    clean = torch.bmm(Q.contiguous(), ((H[None] * W[:, None, :]) @ V.t()).contiguous())[mask]
    slab = clean + 0.01 * clean.pow(2).mean().sqrt() * torch.randn(clean.shape, device="cuda", generator=g)
    offs = np.concatenate([[0], np.cumsum(rows)]).astype(np.int64)
    return d.Tensor(slab.contiguous(), torch.from_numpy(offs).cuda(), offs), K, J, R


def bench_warm(args, d, torch, np):
    """Learned warm start: trains the set encoder on tensors labelled by their
    own 150-iteration decompositions (batched), then on held-out tensors measures the
    iterations and device time each start needs to reach the random start's
    300-iteration fitness minus 1e-3 (|delta fitness| <= 1e-3)."""
    from paper_2203_12798_amd import warm
    R, L, max_it = 10, 20, 300
    t0 = time.perf_counter()

    def setup(T, K, J, seed):
        o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=max_it)
        g = torch.Generator(device="cuda").manual_seed(seed)
        om1 = torch.randn(J, L, device="cuda", generator=g)
        om2 = torch.randn(K * R, L, device="cuda", generator=g)
        init = (torch.eye(R, dtype=torch.float64, device="cuda"),
                torch.randn(J, R, dtype=torch.float64, device="cuda", generator=g),
                torch.ones(K, R, dtype=torch.float64, device="cuda"))
        return o, om1, om2, init

    # labels: the training tensors are decomposed 64 at a time in one batch
    # call (bit for bit the single-tensor decompositions), then each is
    # compressed on its own workspace for its tokens and targets
    train = []
    nb = 64
    for t0b in range(0, args.warm_train, nb):
        batch = []
        for t in range(t0b, min(t0b + nb, args.warm_train)):
            T, K, J, _ = gen_warm_tensor(t, 5, d, torch, np)
            o, om1, om2, init = setup(T, K, J, t)
            o.max_iter = 150
            batch.append((T, o, om1, om2, d.Factors(*(a.clone() for a in init))))
        Ts, os_ = [b[0] for b in batch], [b[1] for b in batch]
        wsb = d.alloc_batch_workspace(Ts, os_)
        d.decompose_batch(Ts, os_, [b[2] for b in batch], [b[3] for b in batch], [b[4] for b in batch], wsb)
        d.release(wsb)
        del wsb
        for T, o, om1, om2, f in batch:
            ws = d.alloc_workspace(T, o)
            d.compress(T, o, om1, om2, ws)
            s = warm.label(T, o, ws, f)
            if float(s.tW.abs().max()) < 10.0:       # degenerate ALS solutions are not labels
                train.append(s)
            d.release(ws)
            del ws
        del batch, Ts
        if (t0b // nb) % 16 == 15:
            print(f"[bench] warm: {t0b + nb} tensors labelled", file=sys.stderr, flush=True)
    label_s = time.perf_counter() - t0
    net = warm.WarmNet(R, seed=1)
    t1 = time.perf_counter()
    net.train(train, steps=args.warm_steps, batch=32, lr=1e-3, match=not args.warm_no_match)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    print(f"[bench] warm: {len(train)} labels ({label_s:.1f}s), trained in {train_s:.1f}s", file=sys.stderr,
          flush=True)
    its_r, its_w, ms_r, ms_w, dfit = [], [], [], [], []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for t in range(args.warm_test):
        T, K, J, _ = gen_warm_tensor(t, 6, d, torch, np)
        o, om1, om2, init = setup(T, K, J, 10 ** 6 + t)
        ws = d.alloc_workspace(T, o)
        d.compress(T, o, om1, om2, ws)
        f = d.Factors(*(a.clone() for a in init))
        ev[0].record()
        _, fit_r = warm.iterations_to(T, o, ws, f, 2.0, max_it)
        ev[1].record()
        torch.cuda.synchronize()
        per_it = ev[0].elapsed_time(ev[1]) / max_it
        target = fit_r[-1] - 1e-3
        tr = int(np.nonzero(fit_r >= target)[0][0]) + 1
        d.compress(T, o, om1, om2, ws)
        fw = d.Factors(*(a.clone() for a in init))
        ev[2].record()
        net.init_factors(T, o, ws, fw)
        ev[3].record()
        tw, fit_w = warm.iterations_to(T, o, ws, fw, target, max_it)
        torch.cuda.synchronize()
        its_r.append(tr)
        its_w.append(max_it if tw is None else tw)
        ms_r.append(tr * per_it)
        ms_w.append(ev[2].elapsed_time(ev[3]) + its_w[-1] * per_it)
        dfit.append(fit_w[-1] - fit_r[-1])
        del T, ws
        if t % 200 == 199:
            print(f"[bench] warm: {t + 1} held-out tensors", file=sys.stderr, flush=True)
    return {"workload": "K~U{32..512}, J=64, I_k~U{64..1024}, rank-10 PARAFAC2 + 1% noise; R=10 L=20",
            "train_tensors": len(train), "train_steps": args.warm_steps, "matched_loss": not args.warm_no_match, "label_s": round(label_s, 1),
            "train_s": round(train_s, 2), "test_tensors": args.warm_test,
            "target": "random start's 300-iteration compressed fitness - 1e-3",
            "iters_random_mean": float(np.mean(its_r)), "iters_warm_mean": float(np.mean(its_w)),
            "iters_random_median": float(np.median(its_r)), "iters_warm_median": float(np.median(its_w)),
            "reached_warm": int(sum(1 for i in its_w if i < max_it)),
            "ms_to_target_random_mean": round(float(np.mean(ms_r)), 3),
            "ms_to_target_warm_mean": round(float(np.mean(ms_w)), 3),
            "speedup_vs_random": round(float(np.sum(ms_r) / np.sum(ms_w)), 3),
            "fit_after_300_warm_minus_random_mean": float(np.mean(dfit))}


def gen_wide(K, d, torch, np, seed=3, chunk=256):
    """Spectrogram-shaped workload: K slices, J = 2049 bins, I_k ~ U{100..704}
    (numpy default_rng(3)); each slice a rank-20 PARAFAC2 whose first
    component is a DC term (Q_k(:, 0) = 1 / sqrt(I_k), the other columns
    orthonormal to it, from the QR of [1, Gaussian]), V(:, 0) a decaying
    positive envelope exp(-j / 400) and W(k, 0) in [3, 4] so that the model is
    mostly positive, H = I + 0.3 N(0, 1), the other V and W entries N(0, 1)
    and U(0.5, 1.5); clipped at 0, plus exponential noise of mean 0.1 x the
    clipped model's mean.  Drawn on the GPU with torch's generator, float32."""
    J, Rt = 2049, 20
    rng = np.random.default_rng(seed)
    rows = rng.integers(100, 705, size=K)
    g = torch.Generator(device="cuda").manual_seed(seed)
    H = torch.eye(Rt, device="cuda") + 0.3 * torch.randn(Rt, Rt, device="cuda", generator=g)
    V = torch.randn(J, Rt, device="cuda", generator=g)
    V[:, 0] = torch.exp(-torch.arange(J, device="cuda", dtype=torch.float32) / 400.0)
    offs = np.concatenate([[0], np.cumsum(rows)]).astype(np.int64)
    slab = torch.empty((int(offs[-1]), J), dtype=torch.float32, device="cuda")
    for k0 in range(0, K, chunk):
        r = rows[k0:k0 + chunk]
        kc, imax = len(r), int(r.max())
        mask = torch.arange(imax, device="cuda")[None, :] < torch.from_numpy(r).cuda()[:, None]
        G = torch.randn(kc, imax, Rt, device="cuda", generator=g)
        G[:, :, 0] = 1.0
        Q = torch.linalg.qr(G * mask[:, :, None]).Q
        Q = Q * torch.sign(Q[:, :1, :1] + 1e-30)                     # DC column positive
        W = 0.5 + torch.rand(kc, Rt, device="cuda", generator=g)
        W[:, 0] = 3.0 + torch.rand(kc, device="cuda", generator=g)
        X = torch.bmm(Q.contiguous(), ((H[None] * W[:, None, :]) @ V.t()).contiguous())[mask].clamp_min(0.0)
        noise = torch.empty_like(X).exponential_(1.0, generator=g)
        slab[int(offs[k0]):int(offs[k0 + kc])] = X + 0.1 * X.mean() * noise
        del G, Q, X, noise
    return d.Tensor(slab, torch.from_numpy(offs).cuda(), offs), rows


SCALE_SIZES = [(1000, 1000, 1000), (1000, 1000, 2000), (2000, 1000, 2000), (2000, 2000, 2000), (2000, 2000, 4000)]


def bench_scalability(args, d, torch, np, binding):
    """The paper's synthetic scalability workloads (Sec. IV-C): tenrand-style
    tensors of K slices of I x J entries uniform in [0, 1) (torch's generator
    on the GPU, seed 5), float32; the five sizes I x J x K at R = 10, and
    R = 10, 20, 30, 40, 50 at 2000 x 2000 x 4000 (64 GB).  As in those experiments the
    randomized SVD runs at the target rank (L = L2 = R) and 32 iterations.
    Per point: ms per decomposition (mean of the timed runs), the slab-pass
    time, the fitness, and PARAFAC2-ALS on the GPU (Alg. 2, same factors and
    iterations) where --scalability-plain asks for it."""
    out = {"workload": "tenrand I x J x K uniform [0, 1) float32; L = R; 32 iterations", "points": []}
    g = torch.Generator(device="cuda").manual_seed(5)
    runs = max(1, args.steps // 2)
    ranks = [int(r) for r in args.scale_ranks.split(",")]
    cases = [] if args.scale_no_sizes else [(I, J, K, 10) for I, J, K in SCALE_SIZES]
    cases += [(2000, 2000, 4000, R) for R in ranks if R != 10 or args.scale_no_sizes]
    cur = None
    for I, J, K, R in cases:
        if cur is None or cur[0] != (I, J, K):
            cur = None
            torch.cuda.empty_cache()
            slab = torch.rand((I * K, J), device="cuda", generator=g)
            offs = np.arange(K + 1, dtype=np.int64) * I
            cur = ((I, J, K), d.Tensor(slab, torch.from_numpy(offs).cuda(), offs))
        T = cur[1]
        L = R
        o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=32)
        om1 = torch.randn(J, L, device="cuda", generator=g)
        om2 = torch.randn(K * R, L, device="cuda", generator=g)
        init = (torch.eye(R, dtype=torch.float64, device="cuda"),
                torch.randn(J, R, dtype=torch.float64, device="cuda", generator=g),
                torch.ones(K, R, dtype=torch.float64, device="cuda"))
        ws = d.alloc_workspace(T, o)
        f = d.Factors(*(a.clone() for a in init))

        def step():
            f.H.copy_(init[0])
            f.V.copy_(init[1])
            f.W.copy_(init[2])
            d.decompose(T, o, om1, om2, f, ws)

        step()
        torch.cuda.synchronize()
        binding.profile_enable(True)
        binding.profile_read()
        t0 = time.perf_counter()
        for _ in range(runs):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / runs
        nl, sk = binding.profile_read()
        binding.profile_enable(False)
        rep = d.report_read(T, o, ws)
        pt = {"I": I, "J": J, "K": K, "R": R, "L": L, "gb_f32": round(I * J * K * 4 / 1e9, 2),
              "ms_per_decomposition": round(ms, 2), "slab_pass_ms": round(sk / max(nl, 1), 3),
              "fitness": rep["fit_true"], "iters": rep["iters"]}
        d.release(ws)
        del ws
        if args.scalability_plain:
            op = d.Options(rank=R, sketch=R, sketch2=R, max_iter=32)
            wsp = d.alloc_plain_workspace(T, op)
            fp = d.Factors(*(a.clone() for a in init))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rp = d.als_plain(T, op, fp, wsp, report=True)
            torch.cuda.synchronize()
            pt["plain_als_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
            pt["plain_als_fitness"] = rp["fit_true"]
            pt["dpar2_speedup"] = round(pt["plain_als_ms"] / ms, 2)
            del wsp
        print(f"[bench] scalability {I}x{J}x{K} R={R}: {ms:.2f} ms", file=sys.stderr, flush=True)
        out["points"].append(pt)
    return out


def bench_downstream(args, d, torch, np):
    """Post-processing of Sec. IV-E on a decomposition computed here: a
    stock-shaped tensor of K = 2000 slices of equal length (I = 250 rows,
    J = 88 features, rank-10 PARAFAC2 with feature scales 10^U(-2, 3) and 5%
    noise, drawn on the GPU with torch's generator, seed 9), DPar2 at R = 10
    (L = 20, 32 iterations) with U_k; then the feature PCC over the rows of V
    (J x J), the Eq. 9 similarity of all K slices (K x K, gamma = 1 / mean
    ||U_k||^2), the top 10 of slice 0 and the random walk with restart from
    slice 0 (c = 0.15, 100 iterations), each timed with HIP events (mean of
    the timed runs).  The similarity kernel's rate is given against the FP64
    vector peak: K^2 I R (subtract + fused multiply-add) = 3 K^2 I R flops."""
    K, I, J, R, L = 2000, 250, 88, 10, 20
    g = torch.Generator(device="cuda").manual_seed(9)
    G = torch.randn(K, I, R, device="cuda", generator=g)
    Q = torch.linalg.qr(G).Q
    H = torch.randn(R, R, device="cuda", generator=g)
    V = torch.randn(J, R, device="cuda", generator=g)
    W = 0.5 + torch.rand(K, R, device="cuda", generator=g)
    X = torch.bmm(Q.contiguous(), ((H[None] * W[:, None, :]) @ V.t()).contiguous())
    X = X * (10.0 ** (-2.0 + 5.0 * torch.rand(J, device="cuda", generator=g)))[None, None, :]
    rms = X.pow(2).mean(dim=(0, 1)).sqrt()
    X = X + 0.05 * rms[None, None, :] * torch.randn(X.shape, device="cuda", generator=g)
    slab = X.reshape(K * I, J).contiguous().float()
    del G, Q, X
    offs = np.arange(K + 1, dtype=np.int64) * I
    T = d.Tensor(slab, torch.from_numpy(offs).cuda(), offs)
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=32)
    om1 = torch.randn(J, L, device="cuda", generator=g)
    om2 = torch.randn(K * R, L, device="cuda", generator=g)
    f = d.Factors(torch.eye(R, dtype=torch.float64, device="cuda"),
                  torch.randn(J, R, dtype=torch.float64, device="cuda", generator=g),
                  torch.ones(K, R, dtype=torch.float64, device="cuda"))
    ws = d.alloc_workspace(T, o)
    U = torch.zeros((K * I, R), dtype=torch.float64, device="cuda")
    rep = d.decompose(T, o, om1, om2, f, ws, U=U, report=True)
    gamma = 1.0 / float(U.pow(2).sum() / K)
    C = torch.empty((J, J), dtype=torch.float64, device="cuda")
    S = torch.empty((K, K), dtype=torch.float64, device="cuda")
    top = torch.empty(10, dtype=torch.int32, device="cuda")
    r = torch.empty(K, dtype=torch.float64, device="cuda")
    work = torch.empty(3 * K, dtype=torch.float64, device="cuda")   # 3 n doubles of scratch
    runs = max(3, args.steps)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(runs):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / runs

    ms_pcc = timed(lambda: d.feature_pcc(f.V, C))
    ms_sim = timed(lambda: d.slice_similarity(T, U, range(K), gamma, S))
    ms_top = timed(lambda: d.top_k(S[0], 0, 10, top))
    ms_rwr = timed(lambda: d.rwr(S, 0, r, work, c=0.15, iters=100))
    sim_flops = 3.0 * K * K * I * R
    out = {"workload": f"K={K} slices of I={I} rows, J={J}, rank-10 PARAFAC2 (feature scales 10^U(-2,3), 5% noise); "
                       f"DPar2 R={R} L={L}, 32 iterations, U_k",
           "fitness": rep["fit_true"],
           "pcc_ms": round(ms_pcc, 4), "similarity_ms": round(ms_sim, 3), "top10_ms": round(ms_top, 4),
           "rwr_100_iterations_ms": round(ms_rwr, 3),
           "similarity_fp64_tflops": round(sim_flops / (ms_sim / 1e3) / 1e12, 2),
           "similarity_frac_of_fp64_vector_peak": round(sim_flops / (ms_sim / 1e3) / 1e12 / 78.6, 4),
           "rwr_hbm_gbs": round(100 * K * K * 8 / (ms_rwr / 1e3) / 1e9, 1),
           "top10_of_slice_0": [int(x) for x in top.cpu().numpy()]}
    print(f"[bench] post-processing: pcc {ms_pcc:.3f} ms, similarity {ms_sim:.2f} ms, top-10 {ms_top:.3f} ms, "
          f"rwr {ms_rwr:.2f} ms", file=sys.stderr, flush=True)
    d.release(ws)
    return out


def bench_wide(args, d, torch, np, binding):
    """Precision form at the spectrogram shape (J = 2049): float32, bf16 and
    fp8-e4m3 (per-slice power-of-two scales) slabs, R = 10 (L = 20) and
    R = 20 (L = 30), 32 iterations, each without and with one power step
    (q = 1, the form's accuracy recovery); ms per decomposition, the
    slab-pass time (both kernels of the wide pass) with its rate against HBM
    peak (one read of the slab's bytes), and the fitness each form reports
    (against the slab it was given).  Also decomposes the first 128 slices in
    every form and returns their factors, so that the oracle leg can state
    each form's error against the FP64 oracle on the float32 data."""
    t0 = time.perf_counter()
    T, rows = gen_wide(args.wide_k, d, torch, np)
    torch.cuda.synchronize()
    K, J = T.K, T.J
    res = {"workload": f"spectrogram-shaped K={K} J={J} I_k~U{{100..704}}, rank-20 PARAFAC2 (DC component), "
                       "clipped, exponential noise; 32 iterations",
           "K": K, "J": J, "N": int(T.offsets_host[-1]), "slab_gb_f32": round(T.slab.numel() * 4 / 1e9, 2),
           "gen_s": round(time.perf_counter() - t0, 1)}
    amax = torch.zeros(K, device="cuda")
    rid = torch.repeat_interleave(torch.arange(K, device="cuda"), torch.from_numpy(rows).cuda())
    amax.scatter_reduce_(0, rid, T.slab.abs().amax(dim=1), reduce="amax")
    scale = torch.exp2(torch.ceil(torch.log2(torch.clamp(amax, min=1e-30) / 448.0)))
    forms = {"f32": T,
             "bf16": d.Tensor(T.slab.to(torch.bfloat16).view(torch.int16), T.offsets_dev, T.offsets_host,
                              binding.DPAR2_BF16),
             "fp8": d.Tensor((T.slab / scale[rid][:, None]).to(torch.float8_e4m3fn).view(torch.uint8).contiguous(),
                             T.offsets_dev, T.offsets_host, binding.DPAR2_FP8_E4M3, scale.contiguous())}
    g = torch.Generator(device="cuda").manual_seed(99)
    N = int(T.offsets_host[-1])
    qs = [int(q) for q in args.wide_q.split(",")]
    for R in [int(r) for r in args.wide_ranks.split(",")]:
        L = R + 10
        om1 = torch.randn(J, L, device="cuda", generator=g)
        om1b = om1.to(torch.bfloat16).to(torch.float32)
        om2 = torch.randn(K * R, L, device="cuda", generator=g)
        init = (torch.eye(R, dtype=torch.float64, device="cuda"),
                torch.randn(J, R, dtype=torch.float64, device="cuda", generator=g),
                torch.ones(K, R, dtype=torch.float64, device="cuda"))
        out = {}
        for name, Tk, q in [(n, t, q) for n, t in forms.items() for q in qs]:
            o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=32, power_iters=q)
            name = name if q == 0 else name + "_q1"
            ws = d.alloc_workspace(Tk, o)
            f = d.Factors(*(a.clone() for a in init))
            om = om1 if name == "f32" else om1b

            def step():
                f.H.copy_(init[0])
                f.V.copy_(init[1])
                f.W.copy_(init[2])
                d.decompose(Tk, o, om, om2, f, ws)

            step()
            torch.cuda.synchronize()
            binding.profile_enable(True)
            binding.profile_read()
            ta = time.perf_counter()
            for _ in range(2):
                step()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - ta) * 1e3 / 2
            nl, sk = binding.profile_read()
            binding.profile_enable(False)
            rep = d.report_read(Tk, o, ws)
            esz = {"f32": 4, "bf16": 2, "fp8": 1}[name.split("_")[0]]
            sk_ms = sk / max(nl, 1)
            gbs = N * J * esz / (sk_ms / 1e3) / 1e9
            out[name] = {"ms_per_step": round(ms, 2), "slices_per_s": round(K / (ms / 1e3), 1),
                         "slab_pass_ms": round(sk_ms, 3),
                         "slab_pass_gbs": round(gbs, 1), "slab_pass_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                         "fitness": rep["fit_true"], "warn_bits": rep["warn_bits"]}
            print(f"[bench] wide R={R} {name}: {ms:.2f} ms", file=sys.stderr, flush=True)
            del ws
        for name in [n for n in ("bf16", "fp8", "f32_q1", "bf16_q1", "fp8_q1") if n in out and "f32" in out]:
            out[name]["speedup_vs_f32"] = round(out["f32"]["ms_per_step"] / out[name]["ms_per_step"], 3)
            out[name]["fitness_delta_vs_f32"] = out[name]["fitness"] - out["f32"]["fitness"]
        res[f"R{R}"] = out
    res["note"] = ("slab_pass_ms is the first slab pass of a decomposition (the sketch and projection kernels); "
                   "slab_pass_gbs = N J bytes-per-entry / slab_pass_ms (one read of the slab's bytes; the wide pass "
                   "reads it twice); the fitness of a bf16 / fp8 form is against the slab it was given, so it "
                   "includes the encoding noise (see sample for the error against the float32 data)")
    # the first 128 slices in every form (R = 10, L = 20, 32 iterations):
    # factors and U for the oracle leg
    if args.wide_only:
        return res, None
    Ks = min(128, K)
    off_s = T.offsets_host[:Ks + 1].copy()
    ns = int(off_s[-1])
    od = torch.from_numpy(off_s).cuda()
    samp = {"K": Ks, "offsets": off_s, "slab": T.slab[:ns].cpu().numpy(), "runs": {}}
    R, L = 10, 20
    gs = torch.Generator(device="cuda").manual_seed(7)
    om1 = torch.randn(J, L, device="cuda", generator=gs)
    om1b = om1.to(torch.bfloat16).to(torch.float32)
    om2 = torch.randn(Ks * R, L, device="cuda", generator=gs)
    V0 = torch.randn(J, R, dtype=torch.float64, device="cuda", generator=gs)
    samp.update({"om1": om1.cpu().numpy(), "om2": om2.cpu().numpy(), "V0": V0.cpu().numpy()})
    sub = {"f32": d.Tensor(T.slab[:ns], od, off_s),
           "bf16": d.Tensor(forms["bf16"].slab[:ns], od, off_s, binding.DPAR2_BF16),
           "fp8": d.Tensor(forms["fp8"].slab[:ns], od, off_s, binding.DPAR2_FP8_E4M3, forms["fp8"].scale[:Ks])}
    for name, Tk in sub.items():
        for q in (0, 1):
            o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=32, power_iters=q)
            ws = d.alloc_workspace(Tk, o)
            f = d.Factors(torch.eye(R, dtype=torch.float64, device="cuda"), V0.clone(),
                          torch.ones(Ks, R, dtype=torch.float64, device="cuda"))
            U = torch.zeros((ns, R), dtype=torch.float64, device="cuda")
            d.decompose(Tk, o, om1 if name == "f32" else om1b, om2, f, ws, U=U)
            H, V, W = f.numpy()
            samp["runs"][name + ("_q1" if q else "")] = (U.cpu().numpy(), H, V, W)
            del ws
    return res, samp


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(slices would shard across GPUs by longest-first partitioning of I_k)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2203_12798_amd as d
    from paper_2203_12798_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.scalability:
        print(json.dumps({"scalability": bench_scalability(args, d, torch, np, binding)}), flush=True)
        return
    if args.wide_only:
        res, _ = bench_wide(args, d, torch, np, binding)
        print(json.dumps({"precision_wide": res}), flush=True)
        return
    print("[bench] generating workload", file=sys.stderr, flush=True)
    t = time.perf_counter()
    X = synth.stock_like()
    gen_s = time.perf_counter() - t
    K, J = X.K, X.J
    R, L, L2, iters = 10, 20, 20, 32
    om1, om2 = synth.omegas(J, L, K * R)
    H0, V0, W0 = synth.init_factors(J, K, R)
    print(f"[bench] K={K} J={J} N={X.N} slab={X.slab.nbytes / 1e9:.2f} GB (gen {gen_s:.1f}s)",
          file=sys.stderr, flush=True)

    T = d.Tensor.from_numpy(X.slab, X.offsets)
    # tiling of the slab pass from the autotuner (median of 3 timed launches
    # each): work-item size, whole-row or 128-column-chunk pass
    cands = [(2048, False), (4096, False), (8192, False), (16384, False), (4096, True), (16384, True)]
    ws = d.alloc_workspace(T, d.Options(rank=R, sketch=L, sketch2=L2, max_iter=iters, item_rows=2048,
                                        wide_slab=True))
    o1 = torch.from_numpy(om1).cuda()
    if args.item_rows:
        item_rows, wide, tune_ms, tune_wide_ms = args.item_rows, False, None, None
    else:
        (item_rows, wide), times = binding.autotune_slab(
            T, d.Options(rank=R, sketch=L, sketch2=L2, max_iter=iters), o1, ws, cands)
        tune_ms = {str(r): t for (r, w), t in zip(cands, times) if not w}
        tune_wide_ms = {str(r): t for (r, w), t in zip(cands, times) if w}
    print(f"[bench] autotune: whole-row {tune_ms}, 128-column chunks {tune_wide_ms} -> "
          f"{item_rows} rows per item{', chunked' if wide else ''}", file=sys.stderr, flush=True)
    o = d.Options(rank=R, sketch=L, sketch2=L2, max_iter=iters, item_rows=item_rows, wide_slab=wide)
    o2 = torch.from_numpy(om2).cuda()
    init = [torch.from_numpy(a).cuda() for a in (H0, V0, W0)]
    f = d.Factors.from_numpy(H0, V0, W0)

    def step():
        f.H.copy_(init[0])
        f.V.copy_(init[1])
        f.W.copy_(init[2])
        d.decompose(T, o, o1, o2, f, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    binding.profile_enable(True)
    binding.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, sketch_ms_total = binding.profile_read()
    binding.profile_enable(False)
    rep = d.report_read(T, o, ws)
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)
    ms_f32 = (t1 - t0) * 1e3 / max(args.steps, 1)

    # where the step's time goes: the compression alone, the iterations
    # alone, and a first call on a fresh workspace (schedule built, iteration
    # graph captured) against the later ones
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    f.H.copy_(init[0])
    f.V.copy_(init[1])
    f.W.copy_(init[2])
    ev[0].record()
    d.compress(T, o, o1, o2, ws)
    ev[1].record()
    d.als_step(T, o, f, iters, ws)
    ev[2].record()
    torch.cuda.synchronize()
    compress_ms, als_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    ws_cold = d.alloc_workspace(T, o)
    f.H.copy_(init[0])
    f.V.copy_(init[1])
    f.W.copy_(init[2])
    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    d.decompose(T, o, o1, o2, f, ws_cold)
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - tc0) * 1e3
    d.release(ws_cold)
    del ws_cold
    timing = {"compress_ms": round(compress_ms, 3), "iterations_ms": round(als_ms, 3),
              "us_per_iteration": round(als_ms * 1e3 / iters, 2), "cold_call_ms": round(cold_ms, 3),
              "note": "compress and the 32 iterations timed apart with HIP events; the cold call is the first "
                      "decomposition on a fresh workspace (schedule built and uploaded, iteration graph captured)"}

    plain = None
    if not args.no_plain:
        # Alg. 2 (PARAFAC2-ALS on the uncompressed slices) on the same tensor,
        # initial factors and iteration count: the method DPar2 accelerates
        try:
            op = d.Options(rank=R, sketch=R, sketch2=R, max_iter=iters, item_rows=item_rows)
            wsp = d.alloc_plain_workspace(T, op)
            fp = d.Factors.from_numpy(H0, V0, W0)

            def stepp():
                fp.H.copy_(init[0])
                fp.V.copy_(init[1])
                fp.W.copy_(init[2])
                return d.als_plain(T, op, fp, wsp)

            stepp()
            torch.cuda.synchronize()
            tp0 = time.perf_counter()
            for _ in range(max(1, args.steps // 2)):
                stepp()
            torch.cuda.synchronize()
            ms_plain = (time.perf_counter() - tp0) * 1e3 / max(1, args.steps // 2)
            fp.H.copy_(init[0])
            fp.V.copy_(init[1])
            fp.W.copy_(init[2])
            rp = d.als_plain(T, op, fp, wsp, report=True)
            plain = {"ms_per_decomposition": round(ms_plain, 3), "ms_per_iteration": round(ms_plain / iters, 4),
                     "fitness": rp["fit_true"], "iters": rp["iters"],
                     "dpar2_speedup": round(ms_plain / ms_f32, 2),
                     "dpar2_fitness_minus_plain": rep["fit_true"] - rp["fit_true"],
                     "note": "Alg. 2 on the GPU: every iteration reads the slab once (X_k V on the first-stage "
                             "slab kernel), polar factors, Y_k = Q_k^T X_k and a CP-ALS sweep in FP64"}
            print(f"[bench] plain ALS: {ms_plain:.2f} ms", file=sys.stderr, flush=True)
            del wsp
        except Exception as exc:   # reported, not fatal
            plain = {"error": str(exc)[:300]}

    stream = None
    if not args.no_stream:
        # streaming: the first 90% of the slices decomposed, the last 10%
        # appended (first stage of the new slices only, second stage over the
        # whole M, the same 32 iterations from the earlier H and V and the
        # mean of the earlier W rows), against the one-call decomposition
        try:
            kp = K - K // 10
            Tp = d.Tensor(T.slab, T.offsets_dev, X.offsets[:kp + 1].copy())
            wsp = d.alloc_workspace(Tp, o)
            fpv = d.Factors.from_numpy(H0, V0, W0[:kp])
            d.decompose(Tp, o, o1, o2[:kp * R].contiguous(), fpv, wsp)
            Hp, Vp, Wp = fpv.numpy()
            Ww = np.concatenate([Wp, np.repeat(Wp.mean(axis=0, keepdims=True), K - kp, axis=0)])
            wsa = d.alloc_append_workspace(T, kp, o)
            warm = [torch.from_numpy(a).cuda() for a in (Hp, Vp, Ww)]
            fa = d.Factors(*(a.clone() for a in warm))

            def stepa():
                fa.H.copy_(warm[0])
                fa.V.copy_(warm[1])
                fa.W.copy_(warm[2])
                d.append(T, kp, o, o1, o2, wsp, fa, wsa)

            stepa()
            torch.cuda.synchronize()
            ta0 = time.perf_counter()
            for _ in range(args.steps):
                stepa()
            torch.cuda.synchronize()
            ms_app = (time.perf_counter() - ta0) * 1e3 / args.steps
            ra = d.report_read(T, o, wsa)
            new_bytes = int(X.offsets[-1] - X.offsets[kp]) * J * 4
            stream = {"k_prev": kp, "k_appended": K - kp, "ms_per_append": round(ms_app, 3),
                      "ms_full_decomposition": round(ms_f32, 3), "speedup_vs_full": round(ms_f32 / ms_app, 2),
                      "slab_bytes_read": new_bytes, "fitness": ra["fit_true"],
                      "fitness_minus_full": ra["fit_true"] - rep["fit_true"],
                      "note": "first stage of the appended slices, second stage over all of M, 32 iterations "
                              "warm-started from the earlier factors; slab rows of the earlier slices not read"}
            print(f"[bench] append {K - kp} slices to {kp}: {ms_app:.2f} ms", file=sys.stderr, flush=True)
            d.release(wsp)
            d.release(wsa)
            del wsp, wsa
        except Exception as exc:   # reported, not fatal
            stream = {"error": str(exc)[:300]}

    forms = None
    if not args.no_forms:
        # the same workload as bf16 bit patterns and as per-slice-scaled fp8
        # e4m3 codes (scale 2^ceil(log2(amax_k / 448))), encoded on the device
        # with torch's round-to-nearest casts; and float32 with one power step
        forms = {}
        amax = np.maximum.reduceat(np.abs(X.slab).max(axis=1), X.offsets[:-1])
        scale = np.exp2(np.ceil(np.log2(np.maximum(amax, 1e-30) / 448.0))).astype(np.float32)
        rows = torch.repeat_interleave(torch.arange(K, device="cuda"),
                                       torch.from_numpy(np.diff(X.offsets)).cuda())
        o1b = torch.from_numpy(synth.round_bf16(om1)).cuda()
        def run_form(kind):
            if kind == "bf16":
                Tk = d.Tensor(T.slab.to(torch.bfloat16).view(torch.int16), T.offsets_dev, X.offsets,
                              binding.DPAR2_BF16)
                ok, om = o, o1b
            elif kind == "fp8":
                sc = torch.from_numpy(scale).cuda()
                codes = (T.slab / sc[rows][:, None]).to(torch.float8_e4m3fn).view(torch.uint8)
                Tk = d.Tensor(codes.contiguous(), T.offsets_dev, X.offsets, binding.DPAR2_FP8_E4M3, sc)
                ok, om = o, o1b
            else:
                Tk, om = T, o1
                ok = d.Options(rank=R, sketch=L, sketch2=L2, max_iter=iters, power_iters=1)
            wsk = d.alloc_workspace(Tk, ok)

            def stepk():
                f.H.copy_(init[0])
                f.V.copy_(init[1])
                f.W.copy_(init[2])
                d.decompose(Tk, ok, om, o2, f, wsk)

            for _ in range(args.warmup):
                stepk()
            torch.cuda.synchronize()
            tk0 = time.perf_counter()
            for _ in range(args.steps):
                stepk()
            torch.cuda.synchronize()
            msk = (time.perf_counter() - tk0) * 1e3 / max(args.steps, 1)
            rk = d.report_read(Tk, ok, wsk)
            print(f"[bench] form {kind}: {msk:.3f} ms", file=sys.stderr, flush=True)
            return {"ms_per_step": round(msk, 3), "slices_per_s": round(K / (msk / 1e3), 1),
                    "speedup_vs_f32": round(ms_f32 / msk, 3), "fitness": rk["fit_true"],
                    "fitness_delta_vs_f32": rk["fit_true"] - rep["fit_true"]}

        for kind in ("bf16", "fp8", "f32_q1"):
            try:
                forms[kind] = run_form(kind)
            except Exception as exc:   # a form that cannot run is reported, not fatal
                forms[kind] = {"error": str(exc)[:200]}

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    ms_per_step = (t1 - t0) * 1e3 / max(args.steps, 1)
    sec = ms_per_step / 1e3
    # slab-pass roofline: the algorithmic bytes are one read of the slab
    # (the per-item partial sums the pass also writes are the implementation's)
    alg_bytes = X.N * J * 4
    alg_flops = 2.0 * X.N * J * L * 2 + 2.0 * X.N * L * L
    sk_ms = sketch_ms_total / max(launches, 1)
    achieved = alg_bytes / (sk_ms / 1e3) / 1e9
    tr = traffic_record()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if (tr is None or wide) else tr["bytes_per_launch"],
                "kernel": ("k_wide_y + k_wide_p (slab pass in 128-column chunks: FP32 MFMA sketch, Gram and "
                           "projection of the 22-bit per-tile fixed point as exact int8 MFMA digit products; the slab "
                           "is read twice)") if wide else
                          ("k_sketch_q (slab pass: sketch from three-piece bf16 MFMA products, Gram and projection of "
                           "the 22-bit per-tile fixed point as exact int8 MFMA digit products)"),
                "kernel_ms": round(sk_ms, 4), "algorithmic_bytes": int(alg_bytes),
                "timed_launches": launches}
    sketch_tf = alg_flops / (sk_ms / 1e3) / 1e12
    # matrix-core work the whole-row pass issues per 64-row tile (J <= 128):
    # the sketch as six bf16 16x16x32 products per 32-column chunk and
    # 16-column tile of L in each of the 4 waves (float32 slab: three-piece
    # splits), the Gram and projection as nine int8 16x16x64 products per
    # 16x16 output tile (L/16 x J/16 projection tiles, 1 or 3 Gram tiles)
    lt_, jt_ = (L + 15) // 16, (J + 15) // 16
    jt_ = jt_ if jt_ <= 4 else (6 if jt_ <= 6 else 8)
    tiles = int(sum(-(-int(r) // 64) for r in X.rows))
    bf16_flops = tiles * 4 * ((jt_ + 1) // 2) * lt_ * 6 * (16 * 16 * 32 * 2)
    int8_ops = tiles * (lt_ * jt_ + (1 if lt_ == 1 else 3)) * 9 * (16 * 16 * 64 * 2)
    out = {
        "metric": "end-to-end DPar2 s & slices/s at R=10; sketch-GEMM % peak; fitness vs FP64",
        "value": round(K / sec, 1), "unit": "slices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "seconds": round(sec, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "us-stock-shaped irregular tensor K=4000 J=88 I_k lognormal[200,8000] "
                               "median 1500, rank-10 PARAFAC2 + 5% noise; R=10 L=20 L2=20 32 iterations",
                   "K": K, "J": J, "N": int(X.N), "rank": R, "sketch": L, "iterations": iters},
        "roofline": roofline,
        "autotune": {"item_rows": item_rows, "pass": "128-column chunks" if wide else "whole rows",
                     "slab_pass_ms_by_item_rows": tune_ms, "chunked_slab_pass_ms_by_item_rows": tune_wide_ms},
        "sketch_gemm": {"useful_tflops": round(sketch_tf, 2),
                        "useful_frac_of_fp32_mfma_peak": round(sketch_tf / FP32_MFMA_PEAK_TFLOPS, 4),
                        "bf16_mfma_issued_tflops": round(bf16_flops / (sk_ms / 1e3) / 1e12, 1),
                        "bf16_mfma_frac_of_peak": round(bf16_flops / (sk_ms / 1e3) / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4),
                        "int8_mfma_issued_tops": round(int8_ops / (sk_ms / 1e3) / 1e12, 1),
                        "int8_mfma_frac_of_peak": round(int8_ops / (sk_ms / 1e3) / 1e12 / INT8_MFMA_PEAK_TOPS, 4),
                        "note": "useful flops 4NJL+2NL^2 of the float32 method against the FP32 matrix-core peak; the "
                                "pass issues them as bf16 products (sketch: three-piece splits of X and Omega) and "
                                "int8 digit products (Gram and projection, exact for the 22-bit per-tile fixed point), each against the dense peak of "
                                "its own type"},
        "fitness": {"gpu": rep["fit_true"], "iters": rep["iters"], "warn_bits": rep["warn_bits"]},
    }
    out["timing"] = timing
    if plain is not None:
        out["plain_als"] = plain
    if stream is not None:
        out["stream"] = stream
    if not args.no_down:
        try:
            out["post_processing"] = bench_downstream(args, d, torch, np)
        except Exception as exc:   # reported, not fatal
            out["post_processing"] = {"error": str(exc)[:300]}
    if forms is not None:
        out["forms"] = forms
    if not args.no_batch:
        try:
            out["batch"] = bench_batch(args, d, torch, np)
        except Exception as exc:   # reported, not fatal
            out["batch"] = {"error": str(exc)[:300]}
    wide_sample = None
    if not args.no_wide:
        try:
            out["precision_wide"], wide_sample = bench_wide(args, d, torch, np, binding)
        except Exception as exc:   # reported, not fatal
            out["precision_wide"] = {"error": str(exc)[:300]}
    if not args.no_warm:
        try:
            out["warm_start"] = bench_warm(args, d, torch, np)
        except Exception as exc:   # reported, not fatal
            out["warm_start"] = {"error": str(exc)[:300]}

    if not args.no_cpu_baseline and args.cpu_sample > 0:
        from threadpoolctl import threadpool_info, threadpool_limits

        from oracle import dpar2_oracle as O
        Ks = min(args.cpu_sample, K)
        off = X.offsets[:Ks + 1]
        slab = X.slab[:off[-1]]
        oms1, oms2 = synth.omegas(J, L, Ks * R)
        Hs, Vs, Ws = synth.init_factors(J, Ks, R)
        cores = len(os.sched_getaffinity(0))
        blas = sorted({f"{i.get('internal_api')} {i.get('version')}" for i in threadpool_info()
                       if i.get("user_api") == "blas"})
        print(f"[bench] oracle on {Ks} slices, {cores} threads, BLAS {blas}", file=sys.stderr, flush=True)
        runs = []
        with threadpool_limits(limits=1, user_api="blas"):
            for _ in range(max(1, args.cpu_runs)):
                tc = time.perf_counter()
                comp = O.compress(slab, off, R, oms1, oms2, threads=cores)
                tm = time.perf_counter()
                st = O.als_compressed(comp, Hs, Vs, Ws, iters)
                ta = time.perf_counter()
                fit_ref = O.fitness(slab, off, O.output_U(comp, st), st.W, st.V)
                te = time.perf_counter()
                runs.append((te - tc, tm - tc, ta - tm))
        tot = np.array([r[0] for r in runs])
        Ts = d.Tensor.from_numpy(slab, off)
        wss = d.alloc_workspace(Ts, o)
        fs = d.Factors.from_numpy(Hs, Vs, Ws)
        d.decompose(Ts, o, torch.from_numpy(oms1).cuda(), torch.from_numpy(oms2).cuda(), fs, wss)
        reps = d.report_read(Ts, o, wss)
        out["cpu_baseline"] = {"value": round(Ks / float(np.mean(tot)), 2), "unit": "slices/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"first {Ks} of the {K} slices (same generator, own Omega and "
                                         f"init of that size), full DPar2: compression + {iters} "
                                         f"iterations + fitness; mean of {len(runs)} runs",
                               "seconds_mean": round(float(np.mean(tot)), 3),
                               "seconds_median": round(float(np.median(tot)), 3),
                               "compress_s_mean": round(float(np.mean([r[1] for r in runs])), 3),
                               "ms_per_iteration_mean": round(float(np.mean([r[2] for r in runs])) * 1e3 / iters, 3),
                               "threads": f"{cores} slice workers (Alg. 4 partition), 1 BLAS thread each",
                               "blas": blas}
        out["fitness"].update({"sample_gpu": reps["fit_true"], "sample_oracle": fit_ref,
                               "sample_abs_diff": abs(reps["fit_true"] - fit_ref)})
        if wide_sample is not None:
            # each precision form's model against the float32 data of the
            # first 128 slices of the spectrogram workload, next to the FP64
            # oracle's own decomposition of those slices (same Omega, start)
            sw = wide_sample
            Ksw, offw, slw = sw["K"], sw["offsets"], sw["slab"]
            Rw = 10
            with threadpool_limits(limits=1, user_api="blas"):
                refs = {q: O.dpar2(slw, offw, Rw, sw["om1"], sw["om2"], np.eye(Rw), sw["V0"], np.ones((Ksw, Rw)), 32,
                                   q=q, threads=cores) for q in (0, 1)}
                errs = {}
                for name, (U, H, V, W) in sw["runs"].items():
                    Ul = [U[offw[k]:offw[k + 1]] for k in range(Ksw)]
                    fw = O.fitness(slw, offw, Ul, W, V)
                    ref = refs[1 if name.endswith("_q1") else 0]
                    errs[name] = {"fitness_vs_float32_data": fw, "delta_vs_fp64_oracle": fw - ref.fit}
            out["precision_wide"]["sample"] = {
                "slices": Ksw, "rank": Rw, "oracle_fitness": refs[0].fit, "oracle_fitness_q1": refs[1].fit,
                "forms": errs,
                "note": "every form's factors scored against the float32 slices with the oracle's fitness; "
                        "the oracle decomposes the float32 slices in FP64 with the same power steps as the "
                        "form (q = 0, or q = 1 for the _q1 forms)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
