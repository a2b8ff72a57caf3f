"""Benchmark of the H-matrix product C = A B on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere256k] [--mode plain|learned|mixed]

One step is one whole product hmat_multiply(A, B, eps) (all farfield blocks
compressed, all nearfield blocks evaluated) on inputs already resident in HBM;
tree construction and assembly happen before the timed region. Prints one JSON
line (see the keys below).
"""

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H×H product time (s) & effective GFLOP/s at ε=1e-6, n=2^18; learned vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere256k")
    ap.add_argument("--mode", default="plain", choices=["plain", "learned", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the product runs on a single MI355X; see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    from workloads import CONFIGS
    from paper_1805_08998_amd import hmat as H

    w = CONFIGS[args.workload]
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

    def opts():
        o = H.hmat_opts_default()
        if args.mode == "mixed":
            o.precision = H.HMAT_FP32_APPLY
        return o

    for i in range(args.warmup):
        st = H.hmat_stats()
        o = opts()
        o.stats = ctypes.pointer(st)
        C, code = H.hmat_multiply(A, B, w.eps, o, allow_not_converged=True)
        H.hmat_destroy(C)
        log(f"[bench] warmup {i}: {st.t_total:.3f}s plan {st.t_plan:.3f} restrict {st.t_restrict:.3f} "
            f"near {st.t_near:.3f} sketch {st.t_sketch:.3f} project {st.t_project:.3f} core {st.t_core:.3f} "
            f"growth rounds {st.n_growth_rounds} not converged {st.n_not_converged}")

    times, stats = [], []
    for i in range(args.steps):
        st = H.hmat_stats()
        o = opts()
        o.stats = ctypes.pointer(st)
        ts = time.perf_counter()
        C, code = H.hmat_multiply(A, B, w.eps, o, allow_not_converged=True)
        te = time.perf_counter()
        times.append(te - ts)
        stats.append(st.as_dict())
        if i + 1 < args.steps:
            H.hmat_destroy(C)
        log(f"[bench] step {i}: {te - ts:.3f}s")
    t = sum(times) / len(times)
    st = stats[-1]
    flops = st["flops_alg"]
    out = {
        "metric": METRIC,
        "value": (flops / t / 1e9) if flops > 0 else None,
        "unit": "GFLOP/s (effective: algorithmic flops / wall time)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.mode != "mixed" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "geometry": w.geometry, "leaf": w.leaf, "eta": w.eta,
                   "kernels": [w.kernel_a.kind, w.kernel_b.kind + "+I"], "eps": w.eps, "eps_in": w.eps_in,
                   "mode": args.mode, "seconds_per_product": t},
        "stats": {k: v for k, v in st.items() if k != "rank_hist"},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
