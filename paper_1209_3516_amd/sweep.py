"""The paper's p-theta balance experiment (Table 4) and its 3-digit force
point at N = 10^6 (section 3.5), run on one GPU with synthetic inputs.

  python -m paper_1209_3516_amd.sweep [--n 100000] [--ncrit 30] [--json out.json]

Table 4 analogue: bodies uniform in the unit cube (the paper does not state
its distribution), charges U[-1, 1], ncrit = 30; for p = 3..6 and force
errors 1e-2..1e-5, the largest theta meeting the error, and the time of list
construction (GPU traversal and work plan) plus the M2L and P2P kernels.  The paper's theta
is a different quantity (it uses B_max and R_max and exceeds 1), so the theta
values are not comparable; the trend is.

3-digit point: N = 10^6, force error <= 1e-3 on 1000 sampled targets, for
p = 3..6; time of tree build + traversal + the first evaluation, once with
the host tree and traversal (upload of tree, lists and plan included) and
once with tree, lists and plan built on the GPU from positions already on
the device; and the time of a warm evaluation.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import fmm
from . import tuning
from . import workloads as W


def table4(n, ncrit, ps=(3, 4, 5, 6), targets=(1e-2, 1e-3, 1e-4, 1e-5)):
    x = W.uniform_cube(n)
    q = W.charges(n)
    prob = tuning.Problem(x, q)
    rows = []
    for p in ps:
        for err in targets:
            th, _ = tuning.largest_theta(prob, p, err, ncrit, device=True)
            if th is None:
                rows.append(dict(p=p, target=err, theta=None))
                continue
            r = prob.run(p, th, ncrit, device=True)  # timed, serial phases
            ms = r["phase_ms"]
            rows.append(dict(p=p, target=err, theta=th, e_force=r["e_force"], e_phi=r["e_phi"],
                             traverse_ms=1e3 * r["traverse_s"], m2l_ms=ms["m2l"],
                             p2p_ms=ms["p2p"], dtt_ms=1e3 * r["traverse_s"] + ms["m2l"]
                             + ms["p2p"], eval_ms=ms["total"],
                             m2l_entries=r["stats"]["m2l_entries"],
                             p2p_pairs=r["stats"]["p2p_pairs"]))
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return rows


def three_digit_point(n, ncrit=64, ps=(3, 4, 5, 6), target=1e-3):
    import torch

    x = W.uniform_cube(n)
    q = W.charges(n)
    prob = tuning.Problem(x, q, targets=W.sample_targets(n, 1000))
    rows = []
    for p in ps:
        th, _ = tuning.largest_theta(prob, p, target, ncrit, step=0.05, refine=5,
                                     device=True)
        if th is None:
            continue
        qt = torch.tensor(q, dtype=torch.float32, device="cuda:0")
        xt = torch.tensor(x, device="cuda:0")
        cold = {}
        for where in ("host", "gpu", "gpu"):  # the second GPU run is the one kept
            tree = lists = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if where == "host":
                tree = fmm.Tree(x, ncrit)
                lists = fmm.Lists(tree, th)
            else:
                tree = fmm.Tree.from_device(xt, ncrit)
                lists = fmm.Lists(tree, th, device=True)
            phi, g = fmm.evaluate(tree, lists, qt, p)
            torch.cuda.synchronize()
            cold[where] = time.perf_counter() - t0
        t0 = time.perf_counter()
        phi, g = fmm.evaluate(tree, lists, qt, p)
        torch.cuda.synchronize()
        warm = time.perf_counter() - t0
        e = tuning.errors(phi.double().cpu().numpy()[prob.targets],
                          g.double().cpu().numpy()[prob.targets], prob.ref_phi, prob.ref_grad,
                          q[prob.targets])
        rows.append(dict(p=p, theta=th, ncrit=ncrit, end_to_end_s=cold["host"],
                         end_to_end_gpu_s=cold["gpu"], warm_eval_s=warm, **e))
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return rows


def markdown(t4, pt):
    out = ["| target e_F | " + " | ".join("p = %d" % p for p in (3, 4, 5, 6)) + " |",
           "|---|---|---|---|---|"]
    for err in (1e-2, 1e-3, 1e-4, 1e-5):
        cells = []
        for p in (3, 4, 5, 6):
            r = [x for x in t4 if x["p"] == p and x["target"] == err]
            if not r or r[0]["theta"] is None:
                cells.append("n/a")
            else:
                r = r[0]
                cells.append("θ=%.3f, %.2f ms (lists %.2f + M2L %.2f + P2P %.2f)" % (
                    r["theta"], r["dtt_ms"], r["traverse_ms"], r["m2l_ms"], r["p2p_ms"]))
        out.append("| %.0e | " % err + " | ".join(cells) + " |")
    out.append("")
    out.append("| p | θ | e_F | e_φ | tree+lists+first eval, host-built [s] | "
               "same, GPU-built [s] | warm eval [ms] |")
    out.append("|---|---|---|---|---|---|---|")
    for r in pt:
        out.append("| %d | %.3f | %.2e | %.2e | %.3f | %.4f | %.2f |" % (
            r["p"], r["theta"], r["e_force"], r["e_phi"], r["end_to_end_s"],
            r["end_to_end_gpu_s"], 1e3 * r["warm_eval_s"]))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--ncrit", type=int, default=30)
    ap.add_argument("--n-large", type=int, default=1_000_000)
    ap.add_argument("--json", default=None)
    ap.add_argument("--skip-table4", action="store_true")
    args = ap.parse_args()
    t4 = [] if args.skip_table4 else table4(args.n, args.ncrit)
    pt = three_digit_point(args.n_large)
    print(markdown(t4, pt))
    if args.json:
        with open(args.json, "w") as f:
            json.dump(dict(table4=t4, three_digit=pt), f, indent=1)


if __name__ == "__main__":
    main()
