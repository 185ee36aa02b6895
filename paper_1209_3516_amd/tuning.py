"""Accuracy-driven choice of the opening angle theta (section 3.2, Table 4), and
auto-tuning of the bodies per leaf and of the M2L/M2P choice.

For a given order p the paper searches for the largest theta whose FMM result
meets a target relative L2 error of the force against a direct sum.  The same
search here: the FMM runs on the GPU (mixed precision by default), the
reference is the library's FP64 direct sum on the GPU, the error is taken over
a set of target bodies, and the search is a coarse scan of theta followed by
bisection inside the bracketing step.

Errors: relative L2 norms over the sampled targets against the FP64 direct
sum, of phi (e_phi), of grad phi (e_grad) and of the paper's force
F_i = -q_i grad_i (e_F).
"""
import time

import numpy as np

from . import fmm


def errors(phi, grad, ref_phi, ref_grad, q_t):
    f = -q_t[:, None] * grad
    fr = -q_t[:, None] * ref_grad
    return dict(e_phi=float(np.linalg.norm(phi - ref_phi) / np.linalg.norm(ref_phi)),
                e_grad=float(np.linalg.norm(grad - ref_grad) / np.linalg.norm(ref_grad)),
                e_force=float(np.linalg.norm(f - fr) / np.linalg.norm(fr)))


class Problem:
    """Bodies, charges and the FP64 direct-sum reference at the target bodies."""

    def __init__(self, x, q, targets=None, device="cuda:0"):
        import torch

        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.q = np.ascontiguousarray(q, dtype=np.float64)
        n = self.x.shape[0]
        self.targets = np.arange(n, dtype=np.int64) if targets is None else np.asarray(
            targets, dtype=np.int64)
        self.device = device
        ph, g = fmm.direct(torch.tensor(self.x, device=device), torch.tensor(self.q, device=device),
                           torch.tensor(self.targets, device=device))
        torch.cuda.synchronize()
        self.ref_phi = ph.cpu().numpy()
        self.ref_grad = g.cpu().numpy()

    def run(self, p, theta, ncrit, precision="mixed", tree=None, timed=True, device=False):
        """One FMM at (p, theta): errors and times (tree build, traversal on the
        host or with device=True on the GPU, GPU phases)."""
        import torch

        xd = torch.tensor(self.x, device=self.device) if device and tree is None else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if tree is None:
            tree = fmm.Tree.from_device(xd, ncrit) if device else fmm.Tree(self.x, ncrit)
        t1 = time.perf_counter()
        # timed runs report the median of three list builds (each previous
        # one freed before the next is timed), after one untimed build: after
        # the host-side work between two points the GPU clock is still low
        builds = []
        lists = None
        for k in range(4 if timed else 1):
            lists = None
            tb = time.perf_counter()
            lists = fmm.Lists(tree, theta, device=device)
            if k > 0 or not timed:
                builds.append(time.perf_counter() - tb)
        traverse_s = sorted(builds)[len(builds) // 2]
        dt = torch.float64 if precision == "fp64" else torch.float32
        qt = torch.tensor(self.q, dtype=dt, device=self.device)
        fmm.evaluate(tree, lists, qt, p, precision)  # first call uploads the lists
        torch.cuda.synchronize()
        phi, g = fmm.evaluate(tree, lists, qt, p, precision, timing=timed, serial=True)
        ms = fmm.last_timings(lists) if timed else {}
        torch.cuda.synchronize()
        out = errors(phi.double().cpu().numpy()[self.targets],
                     g.double().cpu().numpy()[self.targets], self.ref_phi, self.ref_grad,
                     self.q[self.targets])
        out.update(p=p, theta=theta, ncrit=ncrit, tree_s=t1 - t0, traverse_s=traverse_s,
                   phase_ms=ms, stats=lists.stats())
        return out


def largest_theta(problem, p, target, ncrit, metric="e_force", lo=0.02, hi=0.98, step=0.04,
                  refine=7, precision="mixed", device=False):
    """Largest theta in [lo, hi] whose error metric is <= target: scan from
    large theta downwards in `step`, then bisect inside the bracketing step.
    Returns (theta, run) or (None, None) if even `lo` misses the target."""
    tree = fmm.Tree(problem.x, ncrit)
    grid = np.arange(hi, lo - 1e-12, -step)
    good = None
    bad = None
    for th in grid:
        r = problem.run(p, float(th), ncrit, precision, tree=tree, timed=False, device=device)
        if r[metric] <= target:
            good = (float(th), r)
            break
        bad = float(th)
    if good is None:
        return None, None
    if bad is None:
        return good
    a, b = good[0], bad
    best = good
    for _ in range(refine):
        mid = 0.5 * (a + b)
        r = problem.run(p, mid, ncrit, precision, tree=tree, timed=False, device=device)
        if r[metric] <= target:
            a, best = mid, (mid, r)
        else:
            b = mid
    return best


def autotune(x, q, p, theta, ncrits=(16, 24, 32, 48, 64, 96, 128), m2p_values=(0, 2, 4, 8),
             n_targets=1000, reps=5, device="cuda:0"):
    """Time the evaluation for every (ncrit, m2p_max) and return the fastest,
    with the table of all options (the auto-tuning of the hybrid codes that the
    paper's section 2 describes: bodies per leaf trades P2P against M2L work,
    and M2P replaces M2L for small target leaves).  Times are device times of a
    warm evaluation (median of `reps`); errors are against the FP64 direct sum
    on `n_targets` sampled targets.  m2p_max = 0 uses the GPU-built lists."""
    import torch

    from . import workloads as W

    n = x.shape[0]
    tg = W.sample_targets(n, min(n_targets, n))
    xd = torch.tensor(x, device=device)
    ref = fmm.direct(xd, torch.tensor(q, device=device), torch.tensor(tg, device=device))
    torch.cuda.synchronize()
    ref_phi, ref_grad = ref[0].cpu().numpy(), ref[1].cpu().numpy()
    qt = torch.tensor(q, dtype=torch.float32, device=device)
    rows = []
    for ncrit in ncrits:
        tree = fmm.Tree.from_device(xd, ncrit)
        for m in m2p_values:
            lists = fmm.Lists(tree, theta, device=(m == 0), m2p_max=m)
            phi, g = fmm.evaluate(tree, lists, qt, p)
            ts = []
            for _ in range(reps):
                fmm.evaluate(tree, lists, qt, p, timing=True, out=(phi, g))
                ts.append(fmm.last_timings(lists)["total"])
            torch.cuda.synchronize()
            e = errors(phi.double().cpu().numpy()[tg], g.double().cpu().numpy()[tg], ref_phi,
                       ref_grad, q[tg])
            st = lists.stats()
            rows.append(dict(ncrit=ncrit, m2p_max=m, eval_ms=float(np.median(ts)),
                             p2p_pairs=st["p2p_pairs"], m2l_entries=st["m2l_entries"],
                             m2p_entries=st["m2p_entries"], **e))
            del lists
        del tree
    best = min(rows, key=lambda r: r["eval_ms"])
    return best, rows


def _main():
    import argparse
    import json
    import sys

    from . import workloads as W

    ap = argparse.ArgumentParser(description="auto-tune ncrit and the M2P threshold")
    ap.add_argument("--config", default="uniform-1e6-p4")
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    cfg = W.CONFIGS[args.config]
    x = W.positions(cfg["n"], cfg["dist"])
    q = W.charges(cfg["n"], cfg["charges"])
    best, rows = autotune(x, q, cfg["p"], cfg["theta"])
    print("| ncrit | m2p_max | eval ms | P2P pairs | M2L entries | M2P entries | e_phi | e_grad |")
    print("|---|---|---|---|---|---|---|---|")
    for r in rows:
        mark = " **(fastest)**" if r is best else ""
        print("| %d | %d | %.3f%s | %d | %d | %d | %.2e | %.2e |" % (
            r["ncrit"], r["m2p_max"], r["eval_ms"], mark, r["p2p_pairs"], r["m2l_entries"],
            r["m2p_entries"], r["e_phi"], r["e_grad"]))
    sys.stdout.flush()
    if args.json:
        with open(args.json, "w") as f:
            json.dump(dict(best=best, rows=rows), f, indent=1)


if __name__ == "__main__":
    _main()
