"""Benchmark of the H-matrix product C = A B on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere256k|...] [--mode learned|plain|mixed|learned-mixed] [--eps E]

One step is one whole product hmat_multiply(A, B, eps): every farfield block
compressed, every nearfield block evaluated, on inputs already resident in HBM.
Tree construction and assembly happen before the timed region. In learned mode
the rank predictor is trained first (also untimed) on the farfield ranks of
plain products of other workloads (the 65536-point sphere and the
262144-point ellipsoid), then every timed product starts each compression
with the predicted width; the plain adaptive form is timed after it for
comparison. Prints one JSON
line with the throughput (effective GFLOP/s = minimum algorithmic flops of the
method / wall time), the roofline position of the dominant kernel family
(measured with HIP events inside the timed steps) and the CPU oracle's rate on
a stratified sample of the same workload.
"""

import argparse
import ctypes
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H×H product time (s) & effective GFLOP/s at ε=1e-6, n=2^18; learned vs plain"
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 (vector and matrix)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def leaf_arrays(H, tree):
    cl = H.hmat_tree_clusters(tree)
    bl = H.hmat_tree_blocks(tree)
    ids = np.nonzero(bl["kind"] != 0)[0]
    t, s = bl["tau"][ids], bl["sigma"][ids]
    r0 = cl["begin"][t].astype(np.int64)
    c0 = cl["begin"][s].astype(np.int64)
    return dict(r0=r0, r1=r0 + cl["size"][t], c0=c0, c1=c0 + cl["size"][s], kind=bl["kind"][ids],
                level=bl["level"][ids])


def host_cpus():
    """Logical CPUs of the host as lscpu reports them (None if lscpu is missing)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:
        return None
    for line in out.splitlines():
        if line.startswith("CPU(s):"):
            return int(line.split(":")[1])
    return None


def cpu_baseline(H, tree, A, B, C, eps, seconds=20.0, max_rows=256, seed=0):
    """The CPU oracle (exact block from densified strips of the library's A_H and
    B_H, singular values for farfield blocks) timed on a stratified sample: per
    (level, kind) a few leaves of at most max_rows rows, about `seconds` of oracle
    time in all. Reported as measured: seconds per block for each sampled
    (level, kind), and the effective rate on the sample, i.e. the algorithmic
    flops the product charged to the sampled blocks (hmat_product_block_flops) /
    the oracle's time on them. Nothing is extrapolated to the whole product.
    Each sampled exact block is also compared with C's block after the timing:
    relative error / eps and rank - eps-rank for farfield blocks, relative
    error for nearfield blocks."""
    from oracle.product import LeafStrips, oracle_block
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    la = leaf_arrays(H, tree)
    n = H.hmat_tree_info(tree)["n"]
    bflops = H.hmat_product_block_flops(C)

    def src(M):
        def get(i):
            d, U, V = H.hmat_block_get(M, i)
            return (U @ V.T) if d["kind"] == 1 else V
        return LeafStrips(n, la["r0"], la["r1"], la["c0"], la["c1"], get)

    sa, sb = src(A), src(B)
    parity = {"far_err": [], "slack": [], "near_err": []}
    rng = np.random.default_rng(seed)
    levels = np.unique(la["level"])
    per = {}
    f_sample, t_sample, sampled = 0.0, 0.0, 0
    budget_per = seconds / max(1, 2 * len(levels))
    for L in levels[::-1]:
        for kind in (1, 2):
            cand = np.nonzero((la["level"] == L) & (la["kind"] == kind) & (la["r1"] - la["r0"] <= max_rows)
                              & (la["c1"] - la["c0"] <= max_rows))[0]
            total = int(np.sum((la["level"] == L) & (la["kind"] == kind)))
            if cand.size == 0:
                if total:
                    per[f"{int(L)}/{'far' if kind == 1 else 'near'}"] = {"blocks_in_product": total,
                                                                          "sampled": 0}
                continue
            cnt, tt, ff = 0, 0.0, 0.0
            for i in rng.permutation(cand)[:64]:
                r0, r1, c0, c1 = la["r0"][i], la["r1"][i], la["c0"][i], la["c1"][i]
                for j in sa.rows_needed(r0, r1):  # fetch the inputs first: only the oracle is timed
                    sa.leaf(j)
                for j in sb.cols_needed(c0, c1):
                    sb.leaf(j)
                ts = time.perf_counter()
                D, sv, kstar = oracle_block(sa, sb, r0, r1, c0, c1, kind, eps)
                dt = time.perf_counter() - ts
                d, U, V = H.hmat_block_get(C, int(i))
                nd = float(np.linalg.norm(D))
                if kind == 1:
                    e = float(np.linalg.norm(D - U @ V.T)) / max(nd, 1e-300)
                    parity["far_err"].append(e / eps)
                    parity["slack"].append(int(d["rank"]) - int(kstar))
                else:
                    parity["near_err"].append(float(np.linalg.norm(D - V)) / max(nd, 1e-300))
                cnt += 1
                tt += dt
                ff += float(bflops[i])
                sa.cache.clear()
                sb.cache.clear()
                if tt > budget_per:
                    break
            per[f"{int(L)}/{'far' if kind == 1 else 'near'}"] = {
                "blocks_in_product": total, "sampled": cnt, "seconds_per_block": tt / cnt,
                "max_rows": int(np.max((la["r1"] - la["r0"])[cand]))}
            f_sample += ff
            t_sample += tt
            sampled += cnt
    out = {
        "value": f_sample / t_sample / 1e9,
        "unit": "GFLOP/s (effective: algorithmic flops of the sampled blocks / oracle seconds on them)",
        "cores": int(threads),
        "host_cpus_lscpu": host_cpus(),
        "kind": "oracle",
        "sample": f"{sampled} leaves of this workload (<= {max_rows} rows, up to 64 per level and kind, "
                  f"{t_sample:.1f} s of oracle time): exact block from densified strips of the library's "
                  f"A_H and B_H, plus the singular values of farfield blocks; one process, BLAS threads = cores",
        "seconds_measured": t_sample,
        "flops_of_sampled_blocks": f_sample,
        "seconds_per_block": per,
    }
    if parity["far_err"]:
        fe = np.array(parity["far_err"])
        sl = np.array(parity["slack"])
        ne = np.array(parity["near_err"]) if parity["near_err"] else np.zeros(1)
        out["sampled_parity"] = {
            "blocks_far": int(fe.size), "blocks_near": len(parity["near_err"]),
            "far_err_over_eps_max": float(fe.max()), "far_err_over_eps_p99": float(np.percentile(fe, 99)),
            "far_err_over_eps_median": float(np.median(fe)), "rank_minus_kstar_max": int(sl.max()),
            "near_rel_err_max": float(ne.max()),
            "far_outside_bound": int(np.sum((fe > 1.01) | (sl > 2))),
        }
    return out


def train_predictor(H, configs, names, epochs, cache=None, eps=None, target="widths"):
    """Rank predictor trained on plain products of other workloads (untimed), at their
    own accuracy or at `eps` when given. Its label per farfield block is the sketch
    width at which the residual check passed (target "widths": the width a first
    sketch needs to avoid growth rounds) or the block's final rank ("ranks"). Returns
    the model handle and a summary. With `cache`, the training features are read
    from that .npz file when it exists (written by an earlier run with the same
    options), else computed and saved there."""
    feats, ranks = [], []
    t0 = time.perf_counter()
    if cache and os.path.exists(cache):
        with np.load(cache) as z:
            feats, ranks = [z["feats"]], [z["ranks"]]
            names = [str(x) for x in z["names"]] if "names" in z.files else names
        log(f"[bench] predictor data from {cache}: {len(ranks[0])} farfield blocks")
    for name in (names if not feats else []):
        wl = configs[name]
        tr = H.hmat_build_tree(wl.points(), wl.leaf, wl.eta, wl.split)
        A, _ = H.hmat_assemble(tr, wl.kernel_a.kind, wl.kernel_a.diag, wl.kernel_a.shift, wl.eps_in)
        B = A if wl.same_ab else H.hmat_assemble(tr, wl.kernel_b.kind, wl.kernel_b.diag, wl.kernel_b.shift,
                                                  wl.eps_in)[0]
        st = H.hmat_stats()
        o = H.hmat_opts_default()
        o.stats = ctypes.pointer(st)
        C, _ = H.hmat_multiply(A, B, wl.eps if eps is None else eps, o, allow_not_converged=True)
        f, r = H.hmat_product_features(C)
        if target == "widths":
            r = H.hmat_product_widths(C)
        feats.append(f)
        ranks.append(r)
        for h in ([A, C] if wl.same_ab else [A, B, C]):
            H.hmat_destroy(h)
        H.hmat_tree_destroy(tr)
        log(f"[bench] predictor data: {name}: {len(r)} farfield blocks")
    f = np.concatenate(feats)
    r = np.concatenate(ranks)
    if cache and not os.path.exists(cache):
        np.savez(cache, feats=f, ranks=r, names=np.array(names))
    model = H.hmat_rank_model_create(1)
    t1 = time.perf_counter()
    losses = H.hmat_rank_model_train(model, f, r, H.hmat_train_opts_default(epochs=epochs, batch=512, lr=2e-3))
    t2 = time.perf_counter()
    pred = H.hmat_rank_model_predict(model, f)
    rmse = float(np.sqrt(np.mean((pred - r) ** 2)))
    log(f"[bench] predictor trained on {len(r)} blocks in {t2 - t1:.1f}s (data {t1 - t0:.1f}s), "
        f"loss {losses[0]:.4f} -> {losses[-1]:.4f}, rank rmse {rmse:.2f}")
    return model, {"train_on": names, "train_eps": eps, "target": target, "samples": int(len(r)), "epochs": epochs,
                   "train_seconds": t2 - t1, "rank_rmse_train": rmse, "loss_first": float(losses[0]), "loss_last": float(losses[-1])}


def copy_probe():
    """A plain device copy of known size (1 GiB read, 1 GiB written per launch,
    five launches), the calibration run for the HBM traffic counters. Also reports the
    rates the device reaches on plain streaming work (the copy, and a sum that only
    reads), timed with events on the stream the copies run on: the practical ceiling
    against which the apply kernels' measured HBM traffic rates are read."""
    import torch
    nbytes = 1 << 30
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    y.copy_(x)  # the first launch of each is not timed
    ev[0].record()
    for _ in range(4):
        y.copy_(x)
    ev[1].record()
    x.sum()
    ev[2].record()
    for _ in range(4):
        x.sum()
    ev[3].record()
    torch.cuda.synchronize()
    copy_s = ev[0].elapsed_time(ev[1]) / 1e3 / 4
    read_s = ev[2].elapsed_time(ev[3]) / 1e3 / 4
    # no device-to-host read of the sum: it would add a small copy kernel to the counters'
    # calibration, which averages the copy kernel's dispatches
    print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "launches": 5,
                      "copy_GB_s": 2 * nbytes / copy_s / 1e9, "read_GB_s": nbytes / read_s / 1e9}))


def product_source_hash():
    """Hash of the apply-kernel sources and of the driver that sizes their launches:
    traffic figures measured on other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    for f in ("product.hip", "product_kernels.h", "multiply.cpp"):
        with open(os.path.join(ROOT, "paper_1805_08998_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3
    counter summary (a line 'traffic <kernel> <workload> <bytes> <source hash>'),
    or None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    want = product_source_hash()
    with open(path) as fh:
        for line in fh:
            f = line.strip().strip("`").split()
            if len(f) == 5 and f[0] == "traffic" and f[1] == kernel and f[2] == workload and f[4] == want:
                return float(f[3])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere256k")
    ap.add_argument("--mode", default="learned", choices=["learned", "plain", "mixed", "learned-mixed"],
                    help="learned: predicted first widths; mixed: float32 sketch panels; learned-mixed: both")
    ap.add_argument("--train-on", default="sphere64k,ellipsoid256k",
                    help="workloads whose plain products provide the predictor's training data")
    ap.add_argument("--train-epochs", type=int, default=30)
    ap.add_argument("--train-target", default="widths", choices=["widths", "ranks"],
                    help="predictor label: sketch width at which the check passed, or final rank")
    ap.add_argument("--features-cache", default=None,
                    help=".npz file of predictor training features (read if present, else written)")
    ap.add_argument("--compare-steps", type=int, default=None,
                    help="timed plain float64 products after the learned or mixed ones (default: min(--steps, 5))")
    ap.add_argument("--eps", type=float, default=None,
                    help="product accuracy (default: the workload's); the predictor is then trained at it too")
    ap.add_argument("--scheme", default="randomized", choices=["randomized", "aca", "lanczos"],
                    help="low-rank scheme of the farfield blocks (Section 4); aca and lanczos run plain")
    ap.add_argument("--k-fixed", type=int, default=0,
                    help="fixed-rank mode: ACA/Lanczos stop after k steps, randomized runs Algorithm 9")
    ap.add_argument("--exact-lowrank", action="store_true",
                    help="targets without H-pairs are truncated exactly by Algorithm 5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the copy kernel that calibrates the traffic counters")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the product runs on a "
              "single MI355X (sharding the product over GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs as a single process on one GPU", file=sys.stderr)
        sys.exit(2)

    from workloads import CONFIGS
    from paper_1805_08998_amd import hmat as H

    if args.workload == "batched64":
        print("bench.py: the batched64 workload is switched off. hmat_multiply_batched calls on this "
              "64-product batch stopped making progress when the library's device footprint neared the "
              "whole device; the allocator now keeps to three quarters of it, which has not been run on "
              "this batch yet. Small batches are covered by tests/test_gpu_batched.py.", file=sys.stderr)
        sys.exit(2)
    w = CONFIGS[args.workload]
    scheme_code = {"randomized": H.HMAT_SCHEME_RANDOMIZED, "aca": H.HMAT_SCHEME_ACA,
                   "lanczos": H.HMAT_SCHEME_LANCZOS}[args.scheme]
    if (args.scheme != "randomized" or args.k_fixed) and args.mode != "plain":
        log(f"[bench] scheme {args.scheme}, k_fixed {args.k_fixed}: runs in plain mode (the predictor sizes "
            "the first sketch of the adaptive randomized scheme only)")
        args.mode = "plain"
    if args.eps is not None:
        w = dataclasses.replace(w, eps=args.eps)
    model = None
    train_info = None
    if args.mode in ("learned", "learned-mixed"):
        model, train_info = train_predictor(H, CONFIGS, args.train_on.split(","), args.train_epochs,
                                            args.features_cache, eps=args.eps, target=args.train_target)
    pts = w.points()
    t0 = time.perf_counter()
    tree = H.hmat_build_tree(pts, w.leaf, w.eta, w.split)
    info = H.hmat_tree_info(tree)
    t1 = time.perf_counter()
    log(f"[bench] tree n={info['n']} depth={info['depth']} far={info['n_far']} near={info['n_near']} "
        f"csp={info['csp']} ({t1 - t0:.2f}s)")
    A, _ = H.hmat_assemble(tree, w.kernel_a.kind, w.kernel_a.diag, w.kernel_a.shift, w.eps_in)
    B, _ = H.hmat_assemble(tree, w.kernel_b.kind, w.kernel_b.diag, w.kernel_b.shift, w.eps_in)
    t2 = time.perf_counter()
    log(f"[bench] assembly of A and B {t2 - t1:.2f}s")

    def run(time_kernels, mode=args.mode):
        st = H.hmat_stats()
        o = H.hmat_opts_default()
        if mode in ("mixed", "learned-mixed"):
            o.precision = H.HMAT_FP32_APPLY
        if mode in ("learned", "learned-mixed"):
            o.rank_mode = H.HMAT_RANK_PREDICT
            o.rank_model = model
        o.time_kernels = 1 if time_kernels else 0
        o.scheme = scheme_code
        o.k_fixed = args.k_fixed
        o.exact_lowrank = 1 if args.exact_lowrank else 0
        o.stats = ctypes.pointer(st)
        ts = time.perf_counter()
        C, code = H.hmat_multiply(A, B, w.eps, o, allow_not_converged=True)
        te = time.perf_counter()
        return C, st.as_dict(), te - ts

    for i in range(args.warmup):
        C, st, dt = run(False)
        H.hmat_destroy(C)
        log(f"[bench] warmup {i}: {dt:.3f}s plan {st['t_plan']:.3f} restrict {st['t_restrict']:.3f} "
            f"near {st['t_near']:.3f} sketch {st['t_sketch']:.3f} project {st['t_project']:.3f} "
            f"core {st['t_core']:.3f} growth rounds {st['n_growth_rounds']} not converged {st['n_not_converged']} "
            f"batches {st['n_batches']} grown {st['n_grown_blocks']} columns {st['sketch_columns']}")

    times, stats = [], []
    C = None
    for i in range(args.steps):
        if C is not None:
            H.hmat_destroy(C)
        C, st, dt = run(False)
        times.append(dt)
        stats.append(st)
        log(f"[bench] step {i}: {dt:.3f}s batches {st['n_batches']} restrict {st['t_restrict']:.3f} "
            f"near {st['t_near']:.3f} sketch {st['t_sketch']:.3f} project {st['t_project']:.3f} "
            f"grown {st['n_grown_blocks']} fallback {st['n_fallback']} columns {st['sketch_columns']} "
            f"growth {st['t_growth']:.3f}s "
            f"alloc {st['t_alloc']:.3f}s releases {st['n_cache_release']}")
    t = sum(times) / len(times)
    st = stats[-1]
    flops = st["flops_alg"]
    spread = {"mean_s": t, "median_s": float(np.median(times)), "min_s": min(times), "max_s": max(times),
              "steps": len(times), "cache_releases": int(sum(x["n_cache_release"] for x in stats)),
              "alloc_s_max": max(x["t_alloc"] for x in stats)}
    # one more product with every kernel launch bracketed by HIP events on the
    # library's stream: per-family launch durations for the roofline (event
    # records slow the product down, so this step is not part of `value`)
    H.hmat_destroy(C)
    C, kst, kdt = run(True)
    log(f"[bench] instrumented step: {kdt:.3f}s")
    plain = None
    compare_steps = min(args.steps, 5) if args.compare_steps is None else args.compare_steps
    if args.mode != "plain" and compare_steps > 0:
        pt = []
        for i in range(compare_steps):
            Cp, pst, dt = run(False, "plain")
            H.hmat_destroy(Cp)
            pt.append(dt)
            log(f"[bench] plain step {i}: {dt:.3f}s batches {pst['n_batches']} grown {pst['n_grown_blocks']} "
                f"growth {pst['t_growth']:.3f}s "
                f"columns {pst['sketch_columns']} sketch {pst['t_sketch']:.3f} project {pst['t_project']:.3f}")
        tp = sum(pt) / len(pt)
        plain = {"seconds_per_product": tp, "median_s": float(np.median(pt)), "min_s": min(pt), "max_s": max(pt),
                 "gflops_effective": pst["flops_alg"] / tp / 1e9,
                 "steps": len(pt), "n_growth_rounds": pst["n_growth_rounds"],
                 "n_grown_blocks": pst["n_grown_blocks"], "sketch_columns": pst["sketch_columns"],
                 "target_passes": pst["target_passes"],
                 "speedup_over_plain_mean": tp / t,
                 "speedup_over_plain_median": float(np.median(pt)) / float(np.median(times))}

    # roofline of the dominant kernel family (largest summed launch time)
    ktime = np.array(kst["kern_time"])
    kb = np.array(kst["kern_bytes"])
    kf = np.array(kst["kern_flops"])
    kl = np.array(kst["kern_launches"])
    cand = [0, 1, 2, 3, 5, 6, 7]
    dom = cand[int(np.argmax(ktime[cand]))]
    avg = ktime[dom] / max(1, kl[dom])
    bytes_per_launch = kb[dom] / max(1, kl[dom])
    achieved = bytes_per_launch / avg / 1e9 if avg > 0 else None
    roofline = {
        "bound": "hbm",
        "kernel": H.KERN_SYMBOLS[dom],
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
        "traffic": measured_traffic(H.KERN_SYMBOLS[dom], w.name),
        "avg_launch_us": 1e6 * avg,
        "instrumented_step_s": kdt,
        "launches": int(kl[dom]),
        "alg_bytes_per_launch": bytes_per_launch,
        "alg_flops_per_launch": kf[dom] / max(1, kl[dom]),
        "fp64_tflops_achieved": kf[dom] / max(ktime[dom], 1e-30) / 1e12,
        "fp64_peak_tflops": FP64_PEAK_TFLOPS,
        "families": {H.KERN_NAMES[k]: {"time_s": ktime[k], "launches": int(kl[k]),
                                       "GB_s": (kb[k] / ktime[k] / 1e9) if ktime[k] > 0 else None,
                                       "TFLOP_s": (kf[k] / ktime[k] / 1e12) if ktime[k] > 0 else None}
                     for k in range(8)},
    }
    # whole product against the roofline: the floor is the larger of the algorithmic
    # flops at the fp64 peak and the algorithmic bytes at the HBM peak; the compulsory
    # bytes read every input panel once per operator pass (range and projection) and
    # write the output once
    pool_bytes = {name: 8.0 * H.hmat_pool_len(M) for name, M in (("A", A), ("B", B), ("C", C))}
    compulsory = 2.0 * (pool_bytes["A"] + pool_bytes["B"]) + pool_bytes["C"]
    floor = max(flops / (FP64_PEAK_TFLOPS * 1e12), st["bytes_alg"] / (HBM_PEAK_GBS * 1e9))
    roofline["whole_product"] = {
        "flops_alg": flops, "bytes_alg": st["bytes_alg"], "floor_s": floor, "frac": floor / t,
        "compulsory_bytes": compulsory, "compulsory_floor_s": compulsory / (HBM_PEAK_GBS * 1e9),
        "bytes_alg_over_compulsory": st["bytes_alg"] / compulsory, "pool_bytes": pool_bytes}
    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(H, tree, A, B, C, w.eps, seconds=args.cpu_seconds)
        except Exception as e:  # the baseline is reported, never the target
            log(f"[bench] cpu baseline failed: {e!r}")
    out = {
        "metric": METRIC,
        "value": (flops / t / 1e9) if flops > 0 else None,
        "unit": "GFLOP/s (effective: minimum algorithmic flops of the method / wall time)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.mode in ("mixed", "learned-mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "geometry": w.geometry, "jitter": w.jitter, "leaf": w.leaf,
                   "eta": w.eta, "split": "midpoint" if w.split == 0 else "median",
                   "kernels": [f"{w.kernel_a.kind}+{w.kernel_a.shift}I", f"{w.kernel_b.kind}+{w.kernel_b.shift}I"],
                   "eps": w.eps, "eps_in": w.eps_in, "mode": args.mode, "scheme": args.scheme,
                   "k_fixed": args.k_fixed, "exact_lowrank": bool(args.exact_lowrank), "seconds_per_product": t,
                   "alg_flops": flops, "alg_bytes": st["bytes_alg"], "predictor": train_info,
                   "timing": spread, "plain": plain},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stats": {k: v for k, v in st.items() if k not in ("rank_hist",)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
