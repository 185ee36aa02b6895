"""Benchmark: FMM evaluations per second on one MI355X.

Workload (default): 3-D Laplace FMM, N = 10^6 bodies uniform in the unit
cube, charges uniform in [-1, 1], expansion order p = 4, theta = 0.4,
ncrit = 64, potential and gradient outputs, P2P/M2L in FP32 with
Kahan-compensated P2P sums.  One step = one full evaluation (gather, P2P,
P2M, M2M, M2L, L2L, L2P + combine) on inputs already resident in GPU memory;
the tree, the interaction lists and the P2P work plan are built once
beforehand on the GPU (and, for reference, on the host) and timed separately.

Printed: one JSON line with the throughput, the P2P roofline (FP32 vector
peak, 20 flop per pair), per-phase device times, accuracy against an FP64
direct sum on 1000 sampled targets, fwd+bwd / fwd of the differentiable
wrapper, and the FP64 CPU oracle timed on this host (cpu_baseline).
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X, 256 CUs at 2.4 GHz
FLOP_PER_PAIR = 20               # potential + gradient per body pair (section 3.4, Table 6)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_p2p_uniform_N1e6_p4.txt")


def p2p_source_digest():
    """Identity of the P2P kernel as built: its sources and the device flags."""
    import hashlib

    from paper_1209_3516_amd import build_lib

    h = hashlib.sha256()
    for name in ("p2p.hip", "device_common.h", "fmm_internal.h"):
        with open(os.path.join(build_lib.CSRC, name), "rb") as f:
            h.update(f.read())
    h.update(" ".join(build_lib.DEVICE_FLAGS[:-2]).encode())
    return h.hexdigest()


def measured_traffic(config_name):
    """HBM bytes per P2P launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or None if the
    summary is missing, is for another workload, or the P2P kernel changed."""
    if config_name != "uniform-1e6-p4" or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("p2p_source_sha256") != p2p_source_digest():
        return None
    return float(vals["p2p_traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="uniform-1e6-p4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-cpu-one-thread", action="store_true",
                    help="skip the single-thread evaluation of the CPU baseline")
    ap.add_argument("--share-gpus", type=int, default=8,
                    help="also time one GPU's share of the targets when they are split into "
                         "this many Morton ranges (0: skip)")
    ap.add_argument("--box-centres", action="store_true",
                    help="cell centres at the centres of the Morton cubes (tree and lists built "
                         "on the host; the GPU build is not timed)")
    ap.add_argument("--m2l-mfma", action="store_true",
                    help="M2L batched by translation vector on the matrix cores (needs "
                         "--box-centres)")
    ap.add_argument("--mutual-p2p", action="store_true",
                    help="mutual P2P: each unordered pair of P2P leaves evaluated once for both "
                         "(measured slower than the one-sided kernel at the default workload)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first, as a reference "
                         "for hardware memory-traffic counters")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus 1); sharding the evaluation over several "
              "GPUs is not implemented (one GPU's share is timed with --share-gpus)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1209_3516_amd import fmm
    from paper_1209_3516_amd import workloads as W

    cfg = W.CONFIGS[args.config]
    n, p, theta, ncrit = cfg["n"], cfg["p"], cfg["theta"], cfg["ncrit"]
    dev = "cuda:0"
    x = W.positions(n, cfg["dist"])
    q = W.charges(n, cfg["charges"])
    w = W.weights(n)

    t0 = time.perf_counter()
    htree = fmm.Tree(x, ncrit)
    t_tree = time.perf_counter() - t0
    t0 = time.perf_counter()
    hlists = fmm.Lists(htree, theta)
    t_trav = time.perf_counter() - t0
    print("host: tree %.3fs traverse %.3fs" % (t_tree, t_trav), file=sys.stderr, flush=True)
    del hlists, htree

    # Tree, lists and work plan built on the GPU from positions on the device;
    # the second build is the one timed (the first pays one-time set-up).
    xd = torch.tensor(x, device=dev)
    qt = torch.tensor(q, dtype=torch.float32, device=dev)
    phi = torch.empty(n, dtype=torch.float32, device=dev)
    grad = torch.empty(n, 3, dtype=torch.float32, device=dev)
    gpu_build = None
    mf = args.m2l_mfma
    mu = args.mutual_p2p
    for _ in range(0 if args.box_centres else 2):
        tree = lists = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tree = fmm.Tree.from_device(xd, ncrit)
        t1 = time.perf_counter()
        lists = fmm.Lists(tree, theta, device=True)
        t2 = time.perf_counter()
        fmm.evaluate(tree, lists, qt, p, out=(phi, grad))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        gpu_build = {"tree_ms": 1e3 * (t1 - t0), "lists_and_plan_ms": 1e3 * (t2 - t1),
                     "first_eval_ms": 1e3 * (t3 - t2), "total_ms": 1e3 * (t3 - t0)}
    if args.box_centres:
        tree = fmm.Tree(x, ncrit, box_centres=True)
        lists = fmm.Lists(tree, theta)
        t0 = time.perf_counter()
        fmm.evaluate(tree, lists, qt, p, out=(phi, grad), m2l_mfma=mf)
        torch.cuda.synchronize()
        gpu_build = {"host_built_box_centres": True,
                     "first_eval_ms": 1e3 * (time.perf_counter() - t0)}
    print("gpu: %s" % gpu_build, file=sys.stderr, flush=True)

    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib * 2 ** 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        fmm.evaluate(tree, lists, qt, p, out=(phi, grad), m2l_mfma=mf, mutual_p2p=mu)
    torch.cuda.synchronize()

    # Timed region: K evaluations back to back, each recording per-phase HIP
    # events on the streams its kernels run on; the events are read after the
    # region (the mean over the last min(K, TIMING_HISTORY) evaluations), so
    # that no step waits for the previous one.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fmm.evaluate(tree, lists, qt, p, timing=True, out=(phi, grad), m2l_mfma=mf,
                     mutual_p2p=mu)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print("timed %d steps in %.3fs" % (args.steps, elapsed), file=sys.stderr, flush=True)
    phase_ms = fmm.mean_timings(lists, min(args.steps, fmm.TIMING_HISTORY))
    sclk = gpu_sclk_mhz()  # right after the timed region
    ms_per_step = 1e3 * elapsed / args.steps
    stats = lists.stats()
    pairs = stats["p2p_pairs"]
    p2p_s = phase_ms["p2p"] * 1e-3
    achieved = FLOP_PER_PAIR * pairs / p2p_s / 1e12

    # One GPU's share: the targets split into G weighted Morton ranges, each
    # range evaluated alone (P2P, M2L, L2L, L2P for its cells; the upward
    # pass in full), device time per range.
    share = None
    if args.share_gpus > 0 and not mf and not mu:
        G = args.share_gpus
        bounds = fmm.partition(tree, lists, G, p=p)
        per = []
        for k in range(G):
            rng = (bounds[k], bounds[k + 1])
            fmm.evaluate(tree, lists, qt, p, out=(phi, grad), body_range=rng)
            tot = 0.0
            for _ in range(5):
                fmm.evaluate(tree, lists, qt, p, timing=True, out=(phi, grad), body_range=rng)
                tot += fmm.last_timings(lists)["total"]
            per.append(tot / 5)
        torch.cuda.synchronize()
        share = {"n_ranges": G, "range_ms": per, "max_ms": max(per),
                 "mean_ms": sum(per) / G, "imbalance": max(per) / (sum(per) / G),
                 "full_eval_ms": phase_ms["total"],
                 "bodies": [int(b) for b in bounds]}
        print("share: max %.3f ms mean %.3f ms (full %.3f ms)" % (
            share["max_ms"], share["mean_ms"], share["full_eval_ms"]), file=sys.stderr, flush=True)
        fmm.evaluate(tree, lists, qt, p, out=(phi, grad))  # restore the full result

    # accuracy against an FP64 direct sum on 1000 sampled targets
    tg = W.sample_targets(n, 1000)
    dphi, dg = fmm.direct(torch.tensor(x, device=dev), torch.tensor(q, device=dev),
                          torch.tensor(tg, device=dev))
    torch.cuda.synchronize()
    dphi, dg = dphi.cpu().numpy(), dg.cpu().numpy()
    ph = phi.double().cpu().numpy()[tg]
    gr = grad.double().cpu().numpy()[tg]
    e_phi = float(np.linalg.norm(ph - dphi) / np.linalg.norm(dphi))
    e_grad = float(np.linalg.norm(gr - dg) / np.linalg.norm(dg))
    f_num = -q[tg][:, None] * gr
    f_ref = -q[tg][:, None] * dg
    e_force = float(np.linalg.norm(f_num - f_ref) / np.linalg.norm(f_ref))

    # differentiable wrapper: fwd+bwd / fwd for L = sum w_i phi_i
    fb = None
    if not args.no_backward:
        xt = torch.tensor(x, dtype=torch.float32, device=dev, requires_grad=True)
        qg = torch.tensor(q, dtype=torch.float32, device=dev, requires_grad=True)
        wt = torch.tensor(w, dtype=torch.float32, device=dev)
        for _ in range(2):
            (wt * fmm.potential(xt, qg, tree, lists, p)).sum().backward()
        torch.cuda.synchronize()
        kk = max(3, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(kk):
            fmm.potential(xt, qg, tree, lists, p)
        torch.cuda.synchronize()
        t_f = (time.perf_counter() - t0) / kk
        t0 = time.perf_counter()
        for _ in range(kk):
            (wt * fmm.potential(xt, qg, tree, lists, p)).sum().backward()
        torch.cuda.synchronize()
        t_fb = (time.perf_counter() - t0) / kk
        fb = dict(fwd_ms=1e3 * t_f, fwd_bwd_ms=1e3 * t_fb, ratio=t_fb / t_f)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(x, q, ncrit, theta, p, one_thread=not args.no_cpu_one_thread)

    line = {
        "metric": "FMM evals/s at N=1e6 p=4 (P2P Gpairs/s, % FP32 peak); fwd+bwd/fwd time",
        "value": args.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "laplace3d-%s-N%d-p%d-theta%g-ncrit%d" % (
            cfg["dist"], n, p, theta, ncrit), "n": n, "distribution": cfg["dist"],
            "charges": cfg["charges"], "p": p, "theta": theta, "ncrit": ncrit,
            "outputs": "potential+gradient", "precision": "fp32 P2P/M2L, Kahan P2P sums",
            "cell_centres": "morton-cube" if args.box_centres else "bounding-box",
            "m2l": "mfma-batched" if mf else "per-entry",
            "p2p": "mutual" if mu else "one-sided"},
        "roofline": {"bound": "alu", "kernel": "p2p_mutual" if mu else "p2p",
                     "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": None if mu else measured_traffic(args.config),
                     "work": "%d pairs x %d flop" % (pairs, FLOP_PER_PAIR),
                     "p2p_ms": phase_ms["p2p"]},
        "p2p_gpairs_per_s": pairs / p2p_s / 1e9,
        "phase_ms": phase_ms,
        "host_s": {"tree_build": t_tree, "traverse": t_trav},
        "gpu_sclk_mhz_after_timing": sclk,
        "gpu_build": gpu_build,
        "one_gpu_share": share,
        "lists": stats,
        "accuracy_vs_fp64_direct_1000": {"e_phi": e_phi, "e_grad": e_grad, "e_force": e_force},
        "fwd_bwd": fb,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def gpu_sclk_mhz():
    """Current shader clock of the GPU (MHz) from the amdgpu driver's sysfs
    files (the hwmon sclk input, else the level marked current in
    pp_dpm_sclk), or None.  Read directly: no helper program is started from
    this process once it has used the GPU."""
    import glob
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        try:
            for lab in sorted(glob.glob(dev + "/hwmon/hwmon*/freq*_label")):
                with open(lab) as f:
                    if f.read().strip().lower() == "sclk":
                        with open(lab.replace("_label", "_input")) as g:
                            return int(g.read().strip()) / 1e6
            with open(dev + "/pp_dpm_sclk") as f:
                for line in f:
                    m = re.search(r"(\d+(?:\.\d+)?)\s*mhz\s*\*", line, re.I)
                    if m:
                        return float(m.group(1))
        except (OSError, ValueError):
            continue
    return None


def cpu_model():
    """The host CPU's model name and the processors it offers."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name


def cpu_baseline(x, q, ncrit, theta, p, min_seconds=10.0, max_evals=20, one_thread=True):
    """The FP64 oracle evaluating the same workload on this host's cores:
    full evaluations repeated until at least `min_seconds` have passed, with
    the oracle's own phase times (median over the evaluations) and the
    wall-clock times of its tree build and traversal; then, unless disabled,
    one full evaluation on a single thread."""
    from oracle import oracle as O

    O.set_threads(int(os.environ.get("OMP_NUM_THREADS", "0") or 0))
    cores = O.get_threads()
    o = O.OracleFMM(x, ncrit, theta)
    t_tree, t_dtt = o.build_seconds
    k = 0
    phases = []
    t0 = time.perf_counter()
    while k < max_evals:
        o.evaluate(q, p)
        phases.append(O.last_phase_seconds())
        k += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    t = time.perf_counter() - t0
    med = {ph: float(np.median([d[ph] for d in phases])) for ph in O.PHASES}
    out = {"value": k / t, "unit": "evals/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(), "host_processors": os.cpu_count(),
           "sample": "%d full FP64 evaluations of the same workload (N=%d, p=%d), %.1f s; "
                     "tree and lists built beforehand, timed separately"
                     % (k, x.shape[0], p, t),
           "seconds": t,
           "phase_s": dict(tree=t_tree, traversal=t_dtt, **med)}
    if one_thread:
        O.set_threads(1)
        t0 = time.perf_counter()
        o.evaluate(q, p)
        t1 = time.perf_counter() - t0
        O.set_threads(cores)
        out["one_thread"] = {"value": 1.0 / t1, "unit": "evals/s", "cores": 1,
                             "sample": "one full FP64 evaluation of the same workload",
                             "phase_s": O.last_phase_seconds()}
    return out


if __name__ == "__main__":
    main()
