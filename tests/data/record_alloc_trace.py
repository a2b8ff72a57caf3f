"""Records the device allocations of the 64-product batch (n log-uniform in
[4096, 65536], workloads.batched_geometries(64, seed=0), eps 1e-6), its products run one
at a time, and writes them in the compact form tests/alloc_sim.cpp replays:

    p <product> <n>                 a product starts
    a <id> <bytes> <gap_us>         allocation number id of the product (block bytes)
    f <id> <gap_us>                 free of allocation id

gap_us: microseconds since the product's previous allocation or free. Blocks allocated
before a product starts (its inputs) are left out; blocks still live at its end are its
output.

    python tests/data/record_alloc_trace.py record <raw> <marks>   (on a GPU)
    python tests/data/record_alloc_trace.py convert <raw> <marks> <out.gz>
"""
import ctypes
import gzip
import os
import sys
import time


def record(raw, marks):
    os.environ["HMAT_ALLOC_TRACE"] = raw  # read when the library's allocator starts
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
    from paper_1805_08998_amd import hmat as H
    from workloads import batched_geometries
    H.lib()
    with open(marks, "w") as mk:
        for i, sp in enumerate(batched_geometries(64, seed=0)):
            t = H.hmat_build_tree(sp["points"], 64, 0.8, 0)
            A, _ = H.hmat_assemble(t, sp["kernel_a"], 1.0, 0.0, eps_in=1e-8)
            B, _ = H.hmat_assemble(t, sp["kernel_b"], 1.0, 0.0, eps_in=1e-8)
            st = H.hmat_stats()
            o = H.hmat_opts_default()
            o.stats = ctypes.pointer(st)
            ta = time.monotonic()
            C, _ = H.hmat_multiply(A, B, 1e-6, o)
            tb = time.monotonic()
            mk.write(f"{i} {len(sp['points'])} {ta:.6f} {tb:.6f}\n")
            mk.flush()
            print(f"product {i}: n {len(sp['points'])}, {tb - ta:.3f} s", flush=True)
            for h in (A, B, C):
                H.hmat_destroy(h)
            H.hmat_tree_destroy(t)


def convert(raw, marks, out):
    mk = [tuple(map(float, line.split())) for line in open(marks)]
    lines, k, live, nid, last = [], 0, {}, 0, None
    started = -1
    for line in open(raw):
        f = line.split()
        if f[0] not in ("a", "f"):
            continue
        t = float(f[-1])
        while k < len(mk) and t > mk[k][3]:
            k += 1
        if k >= len(mk) or t < mk[k][2]:
            continue
        if started != k:
            lines.append(f"p {k} {int(mk[k][1])}")
            started, live, nid, last = k, {}, 0, t
        gap = int(round((t - last) * 1e6))
        last = t
        if f[0] == "a":
            live[f[3]] = nid
            lines.append(f"a {nid} {f[5]} {gap}")
            nid += 1
        elif f[3] in live:
            lines.append(f"f {live.pop(f[3])} {gap}")
    with gzip.open(out, "wt") as g:
        g.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "record":
        record(sys.argv[2], sys.argv[3])
    else:
        convert(sys.argv[2], sys.argv[3], sys.argv[4])
