"""Extra measurement modes of bench.py (each prints one JSON line).

  nscan         GPU particle-forces/s for Plummer spheres N = 2^17 ... 2^24
                (theta = 0.5, eps = 0.005, FP32), the N range of the paper's
                efficiency-versus-N figure, plus the paper's own theta = 1 on a
                1e6 disc galaxy.
  disc100m      the paper's top size: disc (2e7) + Hernquist halo (8e7), FP32,
                theta = 0.5, eps = 0.01: one build + force evaluation and one
                leapfrog step (interaction lists recomputed, never stored), with
                the oracle on a seeded sample of 2^12 targets (--no-cpu skips it).
  kdk           disc (8e5) + halo (2e5), FP32, theta = 0.5, eps = 0.02,
                tau = 1e-3: 10 kick-drift-kick steps with a rebuild every step,
                per-step time (mean +- SEM, Eq.(8)) and FP64 energy / momentum.
  precision     Plummer N = 1e7, FP32 storage, eps = 0.005, theta in {0.3, 0.5,
                0.8}: compensated-FP32 walk and plain-FP64 walk against the FP64
                oracle on 2^16 seeded targets (median / p99 relative error of
                acceleration and potential, interaction-count mismatches), the
                momentum ratio R_P = |sum m a| / sum m |a| of each walk over all N,
                and walk and step times.
  host-scaling  the oracle's own parallel efficiency on the host cores, the
                paper's measurement method: T(M) over 10 repetitions (mean +- SEM,
                Eq.(8)), S(M) = T(1)/T(M), E(M) = S/M and E^(P)(M) = T(1)/(T(M) M_P)
                (Eqs.(6)-(7)) with ratio errors by Eq.(9), on 2^14 seeded targets
                of a 1e6 Plummer sphere at theta = 0.5.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sem(x):
    x = np.asarray(x, np.float64)
    return float(np.sqrt(((x - x.mean()) ** 2).sum() / (len(x) * (len(x) - 1)))) if len(x) > 1 else 0.0


def _timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.mean(ts)), sem(ts)


def run_nscan(args):
    import torch
    import paper_2412_01733_amd as tc
    import workloads
    dev = torch.device("cuda:0")
    rows = []
    tree = tc.Tree()
    for e in range(17, 25):
        n = 1 << e
        pos, m = workloads.plummer(n, 1002, dtype=np.float32)
        p, mm = torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev)
        acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
        pot = torch.empty(n, dtype=torch.float32, device=dev)

        def step():
            tree.build(p, mm).moments()
            tree.forces(0.5, 0.005, walk="f32c", out=(acc, pot))

        ms, err = _timed(step, args.steps, args.warmup, torch)
        tree.build(p, mm).moments()
        tree.forces(0.5, 0.005, walk="f32c", count=True, out=(acc, pot))
        st = tree.stats()
        rows.append(dict(n=n, ms=ms, ms_sem=err, rate=n / (ms * 1e-3), interactions_per_target=st["interactions"] / n))
        log("nscan N=2^%d: %.3f ms, %.4g particle-forces/s" % (e, ms, n / (ms * 1e-3)))
    pos, vel, m = workloads.disc_galaxy(800_000, 200_000, 1001)
    p, mm = torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev)

    def disc_step():
        tree.build(p, mm).moments()
        tree.forces(1.0, 0.02, walk="f32c")

    ms, err = _timed(disc_step, args.steps, args.warmup, torch)
    return dict(mode="nscan", unit="particle-forces/s", theta=0.5, eps=0.005, walk="f32c", rows=rows,
                disc_theta1=dict(n=1_000_000, theta=1.0, eps=0.02, ms=ms, ms_sem=err, rate=1e6 / (ms * 1e-3)))


def run_disc100m(args):
    import torch
    import paper_2412_01733_amd as tc
    import workloads
    dev = torch.device("cuda:0")
    n_disc, n_halo = 20_000_000, 80_000_000
    log("disc100m: drawing %d + %d particles" % (n_disc, n_halo))
    pos, vel, m = workloads.disc_galaxy(n_disc, n_halo, 1004)
    n = pos.shape[0]
    theta, eps, tau = 0.5, 0.01, 1e-3
    p = torch.from_numpy(pos).to(dev)
    v = torch.from_numpy(vel).to(dev)
    mm = torch.from_numpy(m).to(dev)
    acc = torch.empty((n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty(n, dtype=torch.float32, device=dev)
    tree = tc.Tree()
    tree.build(p, mm)  # creates the handle and its buffers (not timed)
    tree.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree.build(p, mm).moments()
    tree.forces(theta, eps, walk="f32c", out=(acc, pot))
    st = tree.stats()
    t_eval = (time.perf_counter() - t0) * 1e3
    log("disc100m: build+forces %.1f ms (stages %s)" % (t_eval, st["stage_ms"][:6]))
    a0 = acc.clone()
    keys = None if args.no_cpu else tree.export(moments=False)["keys"].cpu().numpy().view(np.uint64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tc.leapfrog_step(p, v, mm, acc, tau, theta, eps, walk="f32c", pot=pot, tree=tree)
    st2 = tree.stats()
    t_step = (time.perf_counter() - t1) * 1e3
    out = dict(mode="disc100m", n=n, theta=theta, eps=eps, walk="f32c", eval_ms=t_eval,
               rate=n / (t_eval * 1e-3), stage_ms=st["stage_ms"][:6], n_nodes=st["n_nodes"],
               multi_leaves=st["n_multi_leaves"], leapfrog_step_ms=t_step,
               energy=dict(kinetic=st2["kinetic"], potential=st2["potential"]),
               torch_mem_peak_gb=torch.cuda.max_memory_allocated() / 1e9)
    if not args.no_cpu:
        import oracle
        tg = workloads.target_sample(n, 1 << 12, 2004)
        log("disc100m: oracle build at N=1e8 (1 thread) ...")
        tb = time.perf_counter()
        T = oracle.Tree(pos, m)
        tb = time.perf_counter() - tb
        ok, _ = T.sorted()
        tw = time.perf_counter()
        ra, rp, _ = T.forces(theta, eps, targets=tg, nthreads=min(16, os.cpu_count() or 1))
        tw = time.perf_counter() - tw
        a = a0[torch.from_numpy(tg).to(dev)].double().cpu().numpy()
        e = np.linalg.norm(a - ra, axis=1) / np.linalg.norm(ra, axis=1)
        out.update(keys_bitexact=bool((keys == ok).all()), nodes_match=bool(T.nnodes == st["n_nodes"]),
                   accuracy=dict(median=float(np.median(e)), p99=float(np.quantile(e, 0.99)), targets=len(tg)),
                   oracle_build_s=tb, oracle_walk_s_per_target=tw / len(tg))
    return out


def run_kdk(args):
    import torch
    import paper_2412_01733_amd as tc
    import workloads
    dev = torch.device("cuda:0")
    pos, vel, m = workloads.disc_galaxy(800_000, 200_000, 1001)
    n = pos.shape[0]
    theta, eps, tau, steps = 0.5, 0.02, 1e-3, 10
    p, v, mm = (torch.from_numpy(a).to(dev) for a in (pos, vel, m))
    tree = tc.Tree()
    acc, pot = tree.build(p, mm).moments().forces(theta, eps, walk="f32c")
    diag, ts = [], []
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tc.leapfrog_step(p, v, mm, acc, tau, theta, eps, walk="f32c", pot=pot, tree=tree)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
        st = tree.stats()
        diag.append(dict(kinetic=st["kinetic"], potential=st["potential"], lin_momentum=st["lin_momentum"],
                         ang_momentum_z=st["ang_momentum"][2]))
    e = [d["kinetic"] + d["potential"] for d in diag]
    return dict(mode="kdk", n=n, theta=theta, eps=eps, tau=tau, steps=steps, step_ms=float(np.mean(ts)),
                step_ms_sem=sem(ts), rate=n / (np.mean(ts) * 1e-3), energy_drift=(e[-1] - e[0]) / abs(e[0]),
                diagnostics=diag)


def run_precision(args):
    import torch
    import oracle
    import paper_2412_01733_amd as tc
    import workloads
    dev = torch.device("cuda:0")
    n, eps, seed = 10_000_000, 0.005, 1002
    pos, m = workloads.plummer(n, seed, dtype=np.float32)
    p, mm = torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev)
    tree = tc.Tree()
    tg = workloads.target_sample(n, 1 << 16, 2002)
    sel = torch.from_numpy(tg).to(dev)
    log("precision: oracle build at N=1e7 (1 thread) ...")
    T = oracle.Tree(pos, m)
    threads = min(16, os.cpu_count() or 1)
    rows = []
    for theta in (0.3, 0.5, 0.8):
        ra, rp, rn = T.forces(theta, eps, targets=tg, nthreads=threads)
        row = dict(theta=theta, oracle_interactions_per_target=float(rn.mean()), walks={})
        for walk in ("f32c", "f64"):
            dt = torch.float32 if walk == "f32c" else torch.float64
            acc = torch.empty((n, 3), dtype=dt, device=dev)
            pot = torch.empty(n, dtype=dt, device=dev)
            tree.build(p, mm).moments()
            tree.forces(theta, eps, walk=walk, count=True, out=(acc, pot))
            st = tree.stats()
            cnt = tree.interaction_counts()[sel].cpu().numpy()
            a = acc[sel].double().cpu().numpy()
            pp = pot[sel].double().cpu().numpy()
            e = np.linalg.norm(a - ra, axis=1) / np.linalg.norm(ra, axis=1)
            ep = np.abs(pp - rp) / np.abs(rp)

            def step():
                tree.build(p, mm).moments()
                tree.forces(theta, eps, walk=walk, out=(acc, pot))

            ms, ms_err = _timed(step, args.steps, args.warmup, torch)
            tree.set_timing(True)
            wl = []
            for _ in range(3):
                step()
                wl.append(tree.stats()["stage_ms"][4])
            tree.set_timing(False)
            row["walks"][walk] = dict(
                acc_median=float(np.median(e)), acc_p99=float(np.quantile(e, 0.99)),
                pot_median=float(np.median(ep)), pot_p99=float(np.quantile(ep, 0.99)),
                count_mismatch=float(np.mean(cnt != rn)),
                R_P=float(np.linalg.norm(st["momentum"]) / st["sum_m_abs_a"]),
                interactions_per_target=st["interactions"] / n,
                step_ms=ms, step_ms_sem=ms_err, rate=n / (ms * 1e-3), walk_ms=float(np.mean(wl)),
                walk_tflops=20 * st["interactions"] / (np.mean(wl) * 1e-3) / 1e12)
            log("precision theta=%g %s: median %.3g p99 %.3g R_P %.3e step %.2f ms" %
                (theta, walk, np.median(e), np.quantile(e, 0.99), row["walks"][walk]["R_P"], ms))
        rows.append(row)
    return dict(mode="precision", workload="plummer-N1e7-fp32-eps0.005", targets=len(tg), oracle_threads=threads,
                rows=rows)


def run_host_scaling(args):
    import oracle
    import workloads
    n, k = 1_000_000, 1 << 14
    pos, m = workloads.plummer(n, 1002, dtype=np.float32)
    T = oracle.Tree(pos, m)
    tg = workloads.target_sample(n, k, 2002)
    cores = os.cpu_count() or 1
    ms = sorted({1, 2, 4, 8, 16, cores} & set(range(1, min(cores, 64) + 1)))
    reps = 10
    rows = {}
    for M in ms:
        T.forces(0.5, 0.005, targets=tg[:256], nthreads=M)  # warm-up
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            T.forces(0.5, 0.005, targets=tg, nthreads=M)
            ts.append(time.perf_counter() - t0)
        rows[M] = (float(np.mean(ts)), sem(ts))
        log("host-scaling M=%d: T=%.4f s +- %.4f" % (M, rows[M][0], rows[M][1]))
    T1, dT1 = rows[1]
    out = []
    for M in ms:
        TM, dTM = rows[M]
        S = T1 / TM
        dS = (T1 * dTM + TM * dT1) / (TM * TM)  # Eq.(9)
        out.append(dict(M=M, T=TM, T_sem=dTM, S=S, S_err=dS, E=S / M, E_err=dS / M))
    return dict(mode="host-scaling", workload="plummer-N1e6-theta0.5-eps0.005, %d seeded targets" % k,
                cores_visible=cores, note="E^(P) = T(1)/(T(M) M_P) equals E for M <= M_P physical cores",
                rows=out, cpu=_cpu_model())


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run(args):
    fn = {"precision": run_precision, "nscan": run_nscan, "disc100m": run_disc100m, "kdk": run_kdk, "host-scaling": run_host_scaling}[args.mode]
    out = fn(args)
    print(json.dumps(out), flush=True)
