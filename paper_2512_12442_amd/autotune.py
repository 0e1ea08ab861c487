"""Autotuner of the batched posterior's tiles (tile width and waves per work-group).

For each precision and size class c (m_pad = 128 (c + 1)), the models of the batched
local-models workload (256 SE models, m ~ U{64..1024}, grids 16^3..64^3) that fall in the
class are evaluated with lcp_dense_batch for every candidate (16 or 32 columns, 4, 8 or 16
waves) whose B tile fits the LDS.  The posterior launch is timed with the library's HIP-event
stage timer (median of --reps runs after a warm-up) and the fastest candidate becomes the
class's default.  Writes csrc/tune_table.inc (the measured times in its comments; rebuild
to take it in) and a JSON record of every measurement.  Needs a GPU.

    python -m paper_2512_12442_amd.autotune [--out DIR] [--reps R]
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PRECS = ["fp64", "fp32", "bf16x3", "f16x3"]          # the order of lcp_precision
CANDIDATES = [(16, 4), (16, 8), (16, 16), (32, 4), (32, 8), (32, 16)]


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=os.path.join(HERE, "csrc"), help="directory of tune_table.inc")
    ap.add_argument("--json", default=None, help="write the measurements here as JSON")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import numpy as np
    import torch
    import paper_2512_12442_amd as lcp
    import workloads

    dev = torch.device("cuda:0")
    Ws = workloads.local_blocks(args.seed)
    zb = torch.as_tensor(Ws[0].zbank, device=dev)
    classes = {}
    for W in Ws:
        classes.setdefault((W.m + 127) // 128 - 1, []).append(W)
    record = {"workload": "local_blocks seed %d" % args.seed, "reps": args.reps, "classes": {}}
    table = {p: [None] * 8 for p in PRECS}
    for c in range(8):
        sub = classes.get(c, [])
        if not sub:
            for p in PRECS:
                table[p][c] = (lcp.batch_tiles(p, c), None, {})
            continue
        B = lcp.GPModelBatch.from_workloads(sub, dev)
        grids, th = [lcp.grid_of(W) for W in sub], [W.theta for W in sub]
        flop = sum(W.n_vertices * W.m * (W.m + 1) for W in sub)
        for p in PRECS:
            times = {}
            out, ws = B.lcp_dense(grids, th, zb, p)
            for nt, nw in CANDIDATES:
                try:
                    lcp.batch_tiles(p, c, nt, nw)
                except lcp.LcpError:
                    continue                    # tile exceeds the LDS at this size
                B.lcp_dense(grids, th, zb, p, out=out, ws=ws)
                ms = []
                for _ in range(args.reps):
                    with lcp.StageTimer(["posterior"]) as st:
                        B.lcp_dense(grids, th, zb, p, out=out, ws=ws)
                    ms.append(st.ms["posterior"])
                times[f"{nt}x{nw}"] = float(np.median(ms))
            lcp.batch_tiles(p, c, 0)
            best = min(times, key=times.get)
            nt, nw = (int(v) for v in best.split("x"))
            table[p][c] = ((nt, nw), times[best], times)
            record["classes"].setdefault(str(c), {})[p] = {"models": len(sub), "flop": flop, "ms": times,
                                                          "best": best}
            print(f"class {c} ({len(sub)} models) {p}: " + ", ".join(f"{k} {v:.3f}" for k, v in times.items()) +
                  f" -> {best}", flush=True)
        del B
        torch.cuda.empty_cache()
    lines = ["// Batched posterior tiles {tile width, waves} per precision (LCP_FP64, LCP_FP32,",
             "// LCP_MIXED_BF16X3, LCP_MIXED_F16X3) and size class c (m_pad = 128 (c + 1)), chosen by",
             "// paper_2512_12442_amd/autotune.py on the batched local-models workload: the fastest",
             "// posterior launch (ms, median of %d) over the candidates that fit the LDS." % args.reps]
    for p in PRECS:
        for c in range(8):
            cfg, best, times = table[p][c]
            if times:
                lines.append("//   %-6s class %d: " % (p, c) + ", ".join(f"{k} {v:.3f}" for k, v in times.items()))
    lines.append("static const TileCfg kTunedTiles[4][kSizeClasses] = {")
    for p in PRECS:
        lines.append("    {" + ", ".join("{%d, %d}" % table[p][c][0] for c in range(8)) + "},")
    lines.append("};")
    path = os.path.join(args.out, "tune_table.inc")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(record, f, indent=1)


if __name__ == "__main__":
    main()
