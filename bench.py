"""Benchmark: TreeCode force evaluation on one MI355X.

Workload (default): Plummer sphere, N = 1e7, FP32 positions and masses,
theta = 0.5, eps = 0.005, G = 1 (seed 1002).  One step = the whole hot path
through the C ABI: root cube + Morton keys, radix sort, octree build, upward
moments, Barnes-Hut walk, unsort and FP64 momentum diagnostic (tc_build +
tc_moments + tc_forces).  The headline is particle-forces/s = N / step time
for the compensated-FP32 walk; the plain-FP64 walk is timed the same way and
reported beside it, each with its error against the FP64 oracle on a seeded
sample of targets.

Prints one JSON line.  Options:
  --gpus N        only 1 is supported (one GPU per run)
  --steps K       timed steps per walk (default 10)
  --warmup W      untimed steps per walk (default 3)
  --no-cpu        skip the oracle leg (CPU baseline + accuracy)
  --no-adjoint    skip the fwd+adjoint leg (Plummer N = 2^18, log-normal masses)
  --mode M        headline (default) | precision | nscan | disc100m | kdk | host-scaling (see bench_modes.py)
  --calib-copy    also run a device copy of 1 GiB (calibrates rocprofv3 byte counters)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_INTERACTION = 20          # acc + pot, rsqrt counted as one
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_f32c_plummer1e7_traffic.txt")
WALK_SRC = os.path.join(ROOT, "paper_2412_01733_amd", "csrc", "walk.hip")
BUILD_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "build_plummer1e7_traffic.md")
BUILD_SRCS = ["keys.hip", "sort.hip", "scan.hip", "build.hip", "moments.hip", "order.hip"]
PEAK_FP32_TFLOPS = 157.3             # MI355X FP32 vector (packed FMA)
PEAK_FP32_NONPACKED_TFLOPS = 78.6    # one FMA per lane per clock: 256 CU x 64 lanes x 2 x 2.4 GHz
PEAK_FP64_TFLOPS = 78.6


def code_hash(path):
    """sha256 of a C++ source with its comments removed and whitespace collapsed:
    it changes with the code, not with an edit of a comment."""
    import hashlib
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return hashlib.sha256(" ".join(src.split()).encode()).hexdigest()


def walk_traffic_bytes():
    """HBM bytes per walk launch from the committed rocprofv3 counter summary,
    or None if the walk's code changed since the counters were taken."""
    try:
        kv = read_kv(TRAFFIC_FILE)
        if kv.get("walk_hip_code_sha256") != code_hash(WALK_SRC):
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])
        return (fetch + write) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def read_kv(path):
    """`key = value` lines of a committed profile summary."""
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    return kv


def build_counter_bytes():
    """Per-stage HBM bytes of one build at Plummer N = 1e7 from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None if a build source
    changed since the counters were taken."""
    import hashlib
    try:
        kv = read_kv(BUILD_TRAFFIC_FILE)
        h = hashlib.sha256()
        for f in BUILD_SRCS:
            h.update(code_hash(os.path.join(ROOT, "paper_2412_01733_amd", "csrc", f)).encode())
        if kv.get("build_src_sha256") != h.hexdigest():
            return None
        return {k: float(kv["stage_%s_bytes" % k]) for k in ("keys", "sort", "tree", "moments")}
    except (OSError, KeyError, ValueError):
        return None


PEAK_HBM_GBPS = 8000.0               # MI355X HBM3E


def stage_bytes(n, nn, p=4):
    """Compulsory HBM bytes of each build stage: what its kernels read and
    write once (no re-reads), for n particles, nn nodes and p-byte inputs."""
    keys = n * (4 * p + (4 * p + 8 + 4 + 4 * p))            # bounds; keys + index + packed record
    sort = n * (8 * (8 + 24) + (4 + 4 * p + 32))             # 8 radix passes (count + move); gather
    tree = n * (9 + 5 + 8 + 13) + nn * (14 + 13 + 13 + 32 + 8)  # adjacent, counts, scan, emit; node passes
    # leaf particles; per node: index, pre-order fields and octant, first child, children's moments, record,
    # parent link, dense topology record; then the target order: per node its topology record (read by
    # itself and by its parent) and its {offset, Hilbert state} (written by the parent, read by itself),
    # per particle its place
    moments = n * 32 + nn * (4 + 13 + 4 + 32 + 48 + 4 + 16) + nn * (16 + 16 + 8 + 8) + n * 4
    return dict(keys=keys, sort=sort, tree=tree, moments=moments)


def copy_bandwidth(torch, dev):
    """Device-to-device copy of 1 GiB: (read + write bytes) / time, GB/s."""
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def gpu_clocks():
    """Current shader and memory clock levels of the visible cards, read from
    the driver's sysfs tables (the active level is marked '*'); None if the
    tables are not readable."""
    import glob
    out = {}
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        card = {}
        for kind in ("sclk", "mclk"):
            try:
                for line in open(os.path.join(dev, "pp_dpm_" + kind)):
                    if line.rstrip().endswith("*"):
                        card[kind] = line.split(":", 1)[1].strip(" *\n")
            except OSError:
                pass
        if card:
            out[os.path.basename(os.path.dirname(dev))] = card
    return out or None


def sem(x):
    x = np.asarray(x, np.float64)
    if len(x) < 2:
        return 0.0
    return float(np.sqrt(((x - x.mean()) ** 2).sum() / (len(x) * (len(x) - 1))))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def adjoint_leg(tc, workloads, torch, dev, args, n=1 << 18, eps=0.01, seeds=(1003, 2003), stored=True):
    """fwd+adjoint ms against forward-only ms: a Plummer sphere (N = 2^18 by
    default, the fitting workload; also run at N = 1e7, the headline size, where
    the walk fills the GPU), masses perturbed log-normally (sigma = 0.2), loss =
    mean |a - a*|^2 with a* the field of the unperturbed masses, theta = 0.5, FP32
    walk.  The backward re-walks the tree with the forward's decisions; the
    variant whose forward stores the interaction lists for the backward to
    replay is timed beside it (where the lists fit)."""
    theta = 0.5
    pos_np, _ = workloads.plummer(n, seeds[0], dtype=np.float32)
    m_np = workloads.lognormal_masses(n, seeds[1]).astype(np.float32)
    pos = torch.from_numpy(pos_np).to(dev)
    m_true = torch.full((n,), 1.0 / n, dtype=torch.float32, device=dev)
    mass = torch.from_numpy(m_np).to(dev)
    tree = tc.Tree()
    astar, _ = tree.build(pos, m_true).moments().forces(theta, eps, walk="f64")
    astar = astar.float()

    def fwd(store=False):
        tree.build(pos, mass).moments()
        a, _ = tree.forces(theta, eps, walk="f32c", store_lists=store)
        return a

    def fwd_adj(store=False):
        a = fwd(store)
        g = (2.0 / n) * (a - astar)
        return tree.backward(g, None)

    res = {}
    legs = (("fwd", fwd), ("fwd_adj", fwd_adj)) + ((("fwd_adj_stored", lambda: fwd_adj(True)),) if stored else ())
    for name, fn in legs:
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) * 1e3 / args.steps
    tree.set_timing(True)
    fwd_adj(False)
    st = tree.stats()
    st_sl = None
    if stored:
        fwd_adj(True)
        st_sl = tree.stats()
    tree.set_timing(False)
    log("bench: adjoint leg N=%d: fwd %.3f ms, fwd+adjoint %.3f ms (walks %.3f / %.3f ms)" %
        (n, res["fwd"], res["fwd_adj"], st["stage_ms"][4], st["stage_ms"][6]))
    out = dict(workload="plummer-N%d-lognormal-masses-theta0.5-eps%g" % (n, eps), n=n, walk="f32c",
               fwd_ms=res["fwd"], fwd_adj_ms=res["fwd_adj"], ratio=res["fwd_adj"] / res["fwd"],
               fwd_walk_ms=st["stage_ms"][4], bwd_walk_ms=st["stage_ms"][6], bwd_down_ms=st["stage_ms"][7],
               walk_ratio=st["stage_ms"][6] / st["stage_ms"][4])
    if stored:
        out["stored_lists"] = dict(fwd_adj_ms=res["fwd_adj_stored"], lists_stored=st_sl["lists_stored"],
                                   fwd_walk_ms=st_sl["stage_ms"][4], bwd_walk_ms=st_sl["stage_ms"][6])
    return out


def bh_gradient_error(tc, workloads, torch, dev, oracle):
    """The direct-sum reference gradient at N = 4096 (Plummer, log-normal
    masses, eps = 0.01, L = mean |a - a*|^2, a* the direct field of the
    unperturbed masses): the gradient with the Barnes-Hut field (FP64 walk and
    its adjoint) at theta = 0 and 0.5 against the one with the direct-sum field
    (the oracle's frozen-list adjoint of the theta = 0 lists).  At theta = 0.5 the
    difference is the method's own approximation error."""
    n, eps = 4096, 0.01
    x, _ = workloads.plummer(n, 4003)
    m = workloads.lognormal_masses(n, 4004)
    astar, _ = oracle.direct(x, np.full(n, 1.0 / n), eps)
    T = oracle.Tree(x, m)
    ad, _ = oracle.direct(x, m, eps)
    gx_d, gm_d = T.frozen_adjoint(T.lists(0.0), eps, (2.0 / n) * (ad - astar))
    t = tc.Tree().build(torch.from_numpy(x).to(dev), torch.from_numpy(m).to(dev)).moments()
    out = dict(n=n, eps=eps, walk="f64")
    for theta in (0.0, 0.5):
        a, _ = t.forces(theta, eps, walk="f64")
        g = (2.0 / n) * (a.cpu().numpy() - astar)
        gpos, gmass = t.backward(torch.from_numpy(g).to(dev))
        ex = np.linalg.norm(gpos.cpu().numpy() - gx_d, axis=1) / np.linalg.norm(gx_d, axis=1)
        em = np.abs(gmass.cpu().numpy() - gm_d) / np.abs(gm_d)
        out["theta%g" % theta] = dict(dLdx_median=float(np.median(ex)), dLdx_p99=float(np.quantile(ex, 0.99)),
                                      dLdm_median=float(np.median(em)), dLdm_p99=float(np.quantile(em, 0.99)))
    return out


def cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--eps", type=float, default=0.005)
    ap.add_argument("--seed", type=int, default=1002)
    ap.add_argument("--walks", default="f32c,f64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 18)
    ap.add_argument("--acc-sample", type=int, default=1 << 16)
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--mode", default="headline", choices=["headline", "precision", "nscan", "disc100m", "kdk", "host-scaling"])
    args = ap.parse_args()
    if args.mode != "headline":
        import bench_modes
        return bench_modes.run(args)

    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the TreeCode path here is a single-GPU build "
              "(targets would shard by contiguous ranges of the walk's Hilbert target order over a replicated tree); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_01733_amd as tc
    import workloads

    dev = torch.device("cuda:0")
    n = args.n
    log("bench: generating Plummer N=%d seed=%d" % (n, args.seed))
    pos_np, m_np = workloads.plummer(n, args.seed, dtype=np.float32)
    pos = torch.from_numpy(pos_np).to(dev)
    mass = torch.from_numpy(m_np).to(dev)
    torch.cuda.synchronize()

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    tree = tc.Tree()
    walks = [w for w in args.walks.split(",") if w]
    res = {}
    for walk in walks:
        dt = torch.float32 if walk == "f32c" else torch.float64
        acc = torch.empty((n, 3), dtype=dt, device=dev)
        pot = torch.empty((n,), dtype=dt, device=dev)

        def step():
            tree.build(pos, mass)
            tree.moments()
            tree.forces(args.theta, args.eps, walk=walk, out=(acc, pot))

        # counted pass: the interaction total (the algorithmic work) of this walk
        tree.set_timing(False)
        tree.build(pos, mass).moments()
        tree.forces(args.theta, args.eps, walk=walk, count=True, out=(acc, pot))
        st = tree.stats()
        inter = st["interactions"]
        n_nodes = st["n_nodes"]
        util = dict(active=inter / max(st["lane_visits"], 1), all=inter / max(64 * st["node_visits"], 1),
                    node_visits=st["node_visits"], leaves=st["n_leaves"], multi_leaves=st["n_multi_leaves"])
        log("bench: %s interactions %d (%.1f per target), nodes %d" % (walk, inter, inter / n, n_nodes))
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        tree.set_timing(True)
        stage = []
        step_ms = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s0 = time.perf_counter()
            step()
            st = tree.stats()  # synchronises the stream and reads this step's stage events
            step_ms.append((time.perf_counter() - s0) * 1e3)
            stage.append(st["stage_ms"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tree.set_timing(False)
        total_ms = (t1 - t0) * 1e3 / args.steps
        stage = np.array(stage)
        walk_ms = stage[:, 4]
        res[walk] = dict(
            ms_per_step=total_ms, ms_per_step_sem=sem(step_ms),
            value=n / (total_ms * 1e-3),
            walk_ms=float(walk_ms.mean()), walk_ms_sem=sem(walk_ms),
            stage_ms={k: round(float(stage[:, i].mean()), 4) for i, k in
                      enumerate(["keys", "sort", "tree", "moments", "walk", "diag"])},
            interactions=int(inter), n_nodes=int(n_nodes), util=util,
            momentum_ratio=float(np.linalg.norm(st["momentum"]) / st["sum_m_abs_a"]),
            acc=acc, pot=pot,
        )
        log("bench: %s step %.3f ms (walk %.3f ms) -> %.4g particle-forces/s" %
            (walk, total_ms, walk_ms.mean(), n / (total_ms * 1e-3)))

    adj = None
    if not args.no_adjoint:
        adj = adjoint_leg(tc, workloads, torch, dev, args)
        adj["full_size"] = adjoint_leg(tc, workloads, torch, dev, args, n=n, eps=args.eps, seeds=(args.seed, 2002),
                                       stored=False)

    out_acc = {}
    cpu = None
    if not args.no_cpu:
        import oracle
        nthreads = max(1, min(16, os.cpu_count() or 1))
        log("bench: oracle build at full N (1 thread) ...")
        tb0 = time.perf_counter()
        T = oracle.Tree(pos_np, m_np)
        t_build = time.perf_counter() - tb0
        tg = workloads.target_sample(n, args.cpu_sample, 2002)
        log("bench: oracle walk on %d sampled targets (%d threads) ..." % (len(tg), nthreads))
        tw0 = time.perf_counter()
        ra, rp, rn = T.forces(args.theta, args.eps, targets=tg, nthreads=nthreads)
        t_walk = time.perf_counter() - tw0
        t_full = t_build + t_walk * n / len(tg)
        cpu = dict(value=n / t_full, unit="particle-forces/s", cores=nthreads, model=cpu_model(), kind="oracle",
                   sample="full-N build (1 thread, %.2f s) + walk of %d seeded targets (%d threads, %.2f s), "
                          "extrapolated to N" % (t_build, len(tg), nthreads, t_walk))
        k = min(args.acc_sample, len(tg))
        sel = tg[:k]
        for walk in walks:
            a = res[walk]["acc"][torch.from_numpy(sel).to(dev)].double().cpu().numpy()
            p = res[walk]["pot"][torch.from_numpy(sel).to(dev)].double().cpu().numpy()
            e = np.linalg.norm(a - ra[:k], axis=1) / np.linalg.norm(ra[:k], axis=1)
            ep = np.abs(p - rp[:k]) / np.abs(rp[:k])
            out_acc[walk] = dict(median=float(np.median(e)), p99=float(np.quantile(e, 0.99)),
                                 pot_median=float(np.median(ep)), pot_p99=float(np.quantile(ep, 0.99)),
                                 targets=int(k))
        oracle_inter = int(rn.sum())
        cpu["oracle_interactions_per_target"] = oracle_inter / len(tg)
        if adj is not None:
            log("bench: Barnes-Hut gradient against the direct-sum gradient, N=4096 ...")
            adj["bh_vs_direct_gradient"] = bh_gradient_error(tc, workloads, torch, dev, oracle)

    head = walks[0]
    r = res[head]
    sb = stage_bytes(n, r["n_nodes"])
    cb = build_counter_bytes() if (n == 10_000_000 and args.seed == 1002) else None
    hbm = {}
    for k, b in sb.items():
        ms = r["stage_ms"][k]
        gbps = b / (ms * 1e-3) / 1e9 if ms > 0 else None
        hbm[k] = dict(bytes=int(b), ms=ms, GBps=gbps, frac=(gbps / PEAK_HBM_GBPS) if gbps else None)
        if cb is not None:
            cg = cb[k] / (ms * 1e-3) / 1e9 if ms > 0 else None
            hbm[k].update(counter_bytes=int(cb[k]), counter_GBps=cg, counter_frac=(cg / PEAK_HBM_GBPS) if cg else None)
    copy_gbps = copy_bandwidth(torch, dev)
    flops = FLOPS_PER_INTERACTION * r["interactions"]
    achieved = flops / (r["walk_ms"] * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if head == "f32c" else PEAK_FP64_TFLOPS
    line = {
        "metric": "particle-forces/sec at N=1e7, theta=0.5 (FP32 vs FP64 walk); fwd+adjoint ms",
        "value": r["value"],
        "unit": "particle-forces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "f32c" else "f64",
        "data": "synthetic",
        "config": {"workload": "plummer-N%d-theta%g-eps%g" % (n, args.theta, args.eps), "n": n,
                   "theta": args.theta, "eps": args.eps, "walk": head, "inputs": "fp32, seed %d" % args.seed},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": walk_traffic_bytes() if head == "f32c" else None,
                     "kernel": "k_walk<%s>" % ("F32C" if head == "f32c" else "F64"),
                     "flops_per_interaction": FLOPS_PER_INTERACTION, "interactions": r["interactions"],
                     "walk_ms": r["walk_ms"],
                     "frac_nonpacked_fp32": (achieved / PEAK_FP32_NONPACKED_TFLOPS) if head == "f32c" else None},
        "build_hbm": {"peak_GBps": PEAK_HBM_GBPS, "copy_GBps": copy_gbps, "stages": hbm,
                      "note": "bytes: compulsory bytes per stage (stage_bytes); counter_bytes: rocprofv3 FETCH_SIZE x 2 + "
                              "WRITE_SIZE of the same build (profiles/build_plummer1e7_traffic.md, null if the build "
                              "code changed); both over the stage's HIP-event time"},
        "gpu_clocks": gpu_clocks(),
        "cpu_baseline": cpu,
        "adjoint": adj,
        "walks": {},
        "accuracy_vs_oracle": out_acc,
    }
    for walk in walks:
        rr = res[walk]
        fl = FLOPS_PER_INTERACTION * rr["interactions"] / (rr["walk_ms"] * 1e-3) / 1e12
        line["walks"][walk] = dict(
            value=rr["value"], ms_per_step=rr["ms_per_step"], ms_per_step_sem=rr["ms_per_step_sem"],
            walk_ms=rr["walk_ms"], walk_ms_sem=rr["walk_ms_sem"], walk_only_rate=n / (rr["walk_ms"] * 1e-3),
            walk_tflops=fl, stage_ms=rr["stage_ms"], interactions=rr["interactions"],
            interactions_per_target=rr["interactions"] / n, n_nodes=rr["n_nodes"],
            lane_utilisation=rr["util"],
            momentum_ratio=rr["momentum_ratio"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
