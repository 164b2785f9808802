"""Throughput of the TMOP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload q2_cube_64]

A step is one pass of the element operations over the whole mesh: energy
(with min det A) and gradient, computed together as the Newton line search
does (tmop_energy_gradient), and the Hessian action, each over all
elements.  The metric is DOF-iterations/s = (dim * n_node) / (seconds per
step), inputs resident in HBM.  Printed as one JSON line.  The FP64 path is the headline
value; the mixed FP32 path, per-operation times, the roofline of the
Hessian-action kernel, Newton wall time to the F tolerance (truncated CG
with a fixed or an inexact-Newton inner tolerance, Jacobi preconditioned or
not, and Jacobi-preconditioned MINRES), the Section 4 objectives
(displacement penalty, second metric term, replication composite: their
kernels' cost and Newton with the penalty) and the CPU oracle baseline are
reported alongside.
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
sys.path.insert(0, ROOT)

from paper_1807_09807_amd import meshgen  # noqa: E402

# Algorithmic work per element: the sum-factorized contractions plus the
# per-point arithmetic of the element kernels (an FMA counts 2 flops, a
# division or cube root 1), counted from the kernel source.
HBM_PEAK = 8.0e12          # B/s
FP64_PEAK = 78.6e12        # FLOP/s, vector FP64 (dense MFMA FP64 is the same)
FP32_PEAK = 157.3e12       # FLOP/s, published FP32 vector peak


def contraction_macs(dim, P, Q):
    """MACs of one sum-factorized forward (or transposed) contraction of a
    dim-vector field: all d x d entries of A at all Q^dim points."""
    if dim == 3:
        return 3 * (P * P * Q * P * 2) + 3 * (P * Q * Q * P * 3) + 9 * Q ** 3 * P
    return 2 * (P * Q * P * 2) + 4 * Q * Q * P


# Per quadrature point, beyond the contractions: (energy, gradient, Hessian)
# flops of the point formulas with an isotropic target W = s I (every
# workload here), counted from the kernel source: 1/s rides in the G table,
# so the contraction yields T and the transposed contraction takes Y = k P
# with the weight k = w det W folded into the metric's scalar coefficients.
#   energy    det T, det A = det W det T, mu(T), w det W, accumulation
#   gradient  cof T, I1, tau, the partials, P = k1 T + kt cof T (+ k2 dI2)
#   Hessian   cof T, dcof[E], I1, T:E, cof T:E, tau, the partials, and
#             dP = kE E + kd dcof + sT T + sC cof T (+ the I2 terms of mu_302)
POINT_FLOPS = {2: (15, 31, 72), 7: (21, 32, 74), 303: (40, 87, 232), 302: (85, 242, 717)}

# HBM traffic of one Hessian-action launch (FP64) of the workload's default
# scatter, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes (KiB per
# dispatch), valid for the element-kernel sources whose SHA-256 is recorded
# with them.  The counters are scaled by what they read for a 256 MiB device
# copy in the same profile: FETCH_SIZE 131,089 KiB (factor 2.0), WRITE_SIZE
# 262,144 KiB (1.0).
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
KERNEL_SOURCES = ("tmop_elem.h", "tmop_metrics.h", "tmop_launch.h")
MEASURED_TRAFFIC = {
    # colour launch of 32,768 elements
    ("q2_cube_64", "colours"): dict(src_sha256="aa216c61c303be4cf830bdfab16ac8fd415554b74081a6a2cf94206f3f901cee",
                                    fetch_kib=41952.1, write_kib=27968.3),
    # element-vector launch over all 262,144 elements (the gather is a kernel of its own)
    ("q2_cube_64", "elements"): dict(src_sha256="aa216c61c303be4cf830bdfab16ac8fd415554b74081a6a2cf94206f3f901cee",
                                     fetch_kib=102673.6, write_kib=227995.8),
}


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1807_09807_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, scatter):
    """Calibrated HBM bytes per Hessian-action launch of the given scatter
    ("colours" or "elements"), or None when no counters were taken for it at
    the current kernel sources."""
    m = MEASURED_TRAFFIC.get((workload, scatter))
    if m is None or m["src_sha256"] != kernel_digest():
        return None
    return 1024.0 * (FETCH_SCALE * m["fetch_kib"] + WRITE_SCALE * m["write_kib"])


def algorithmic(w):
    """(flops, bytes) per element for energy, gradient, Hessian action."""
    dim, P, Q, metric = w["dim"], w["p"] + 1, w["Q"], w["metric"]
    nq = Q ** dim
    c = contraction_macs(dim, P, Q) * 2
    pf = POINT_FLOPS[metric]
    flops = (c + nq * pf[0], 2 * c + nq * pf[1], 3 * c + nq * pf[2])
    m = w["n"] * w["p"] + 1
    node_bytes = dim * 8 * m ** dim / w["n"] ** dim      # unique L-vector bytes per element, one field
    return flops, (node_bytes, 2 * node_bytes, 3 * node_bytes)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 20 warmup steps: the first calls load the kernels' code objects and the
    # first tens of milliseconds of work run below the steady clock (20-step
    # blocks from a cold start on 64^3 Q2: 2.42, 0.688, then 0.662-0.668 ms per
    # step); 100 timed steps are well under a second of work
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="q2_cube_64", choices=sorted(meshgen.WORKLOADS))
    ap.add_argument("--no-newton", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-elems", type=int, default=65536)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy a 256 MiB buffer, so a profile holds a kernel of known HBM traffic")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-initial-guess pipeline")
    ap.add_argument("--train-meshes", type=int, default=2000)
    ap.add_argument("--eval-seeds", type=int, default=8)
    ap.add_argument("--other-workloads", default="q3_square_256,q3_cube_48,q2_square_512,q2_cube_32",
                    help="further workloads whose element operations are timed and reported (comma list)")
    ap.add_argument("--no-section4", action="store_true", help="skip the Section 4 objectives")
    ap.add_argument("--no-targets", action="store_true", help="skip the per-point target and sliding runs")
    ap.add_argument("--no-dfo", action="store_true", help="skip the derivative-free solver")
    ap.add_argument("--section4-2d", default="q3_square_256",
                    help="2D workload for the second metric term and the replication composite")
    return ap.parse_args()


def learned_guess(args, log):
    """The learned initial guess on the 512^2 Q2 mu_2 workload: training data
    from the library's Newton solutions of seeded 64^2 meshes, Adam
    training, then plain vs learned Newton to F_tol on unseen meshes."""
    from paper_1807_09807_amd import mlp as ML
    log(f"# learned guess: {args.train_meshes} training meshes of 64^2")
    data = ML.generate_training_data(n_mesh=args.train_meshes, n=64, seed0=1000)
    log(f"#   data {data.info['seconds']:.1f} s ({data.X.shape[0]} element samples, Newton status per union solve "
        f"{sorted(set(data.info['newton_status']))}, worst |g|/|g0| {data.info['max_rel_gnorm']:.1e})")
    net, tinfo = ML.train(data, epochs=6, batch_meshes=2, lr=2e-3, seed=0)
    log(f"#   training {tinfo['seconds']:.1f} s, {tinfo['steps']} Adam steps of {tinfo['batch']} samples, "
        f"last-batch loss per epoch {[round(l, 6) for l in tinfo['loss_history']]}")
    rows = ML.evaluate(net, n=512, seeds=tuple(10000 + k for k in range(args.eval_seeds)), log=log)
    # wall-time ratio over the seeds where both runs reached F_tol; losses (ratio < 1) included
    both = [r for r in rows if r["plain"]["reached_F_tol"] and r["learned"]["reached_F_tol"]]
    sp = [r["plain"]["wall_s"] / r["learned"]["wall_s"] for r in both]
    return dict(train_meshes=args.train_meshes, samples=int(data.X.shape[0]), data_s=data.info["seconds"],
                train_s=tinfo["seconds"], train_samples_per_s=tinfo["steps"] * tinfo["batch"] / tinfo["seconds"],
                loss_history=tinfo["loss_history"], eval=rows,
                speedup_wall_per_seed=[round(x, 3) for x in sp],
                speedup_wall_median=float(np.median(sp)) if sp else None,
                seeds_learned_slower=[r["seed"] for r in both if r["learned"]["wall_s"] > r["plain"]["wall_s"]],
                seeds_fallback=[r["seed"] for r in rows if not r["used_proposal"] or r["learned"]["fell_back_after_solve"]],
                reference_converged=[r["reference"]["converged"] for r in rows],
                proposal_F_over_F0=[r["F_proposal"] / r["F0"] for r in rows],
                newton_iters_plain=[r["plain"]["iters"] for r in rows],
                newton_iters_learned=[r["learned"]["iters"] for r in rows])


def copy_calibration(torch, dev):
    """One device-to-device copy of 256 MiB (read 256 MiB, write 256 MiB)."""
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


_CPU_JOB = {}


def _oracle_chunk(e0, e1):
    """Worker of the multi-process CPU baseline: energy + gradient + Hessian
    action of the FP64 oracle on elements [e0, e1), one thread; returns
    (F part, seconds).  The mesh arrays come from the parent by fork."""
    from threadpoolctl import threadpool_limits
    from oracle import tmop_oracle as O
    j = _CPU_JOB
    w = j["w"]
    with threadpool_limits(1):
        prob = O.Problem(w["dim"], w["p"], w["Q"], j["en"][e0:e1], w["metric"], j["h"] * np.eye(w["dim"]))
        t0 = time.perf_counter()
        F, _ = prob.energy(j["x"])
        prob.gradient(j["x"])
        prob.hessian_apply(j["x"], j["v"])
        return F, time.perf_counter() - t0


def cpu_baseline(w, mesh, x, v, n_elem_sample, chunk=4096, workers=None):
    """The FP64 oracle (energy + gradient + Hessian action) on the first
    n_elem_sample elements, scaled to DOF-iterations/s, (i) in one process
    and thread and (ii) over a pool of worker processes (fork, one thread
    each, at most 16: the host share of one GPU) on element chunks of the
    whole mesh, merged with math.fsum.  The sample is fed to the oracle in
    element chunks (its dense per-point tables would not fit in memory at
    once)."""
    import math
    import multiprocessing as mp
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    _CPU_JOB.update(w=w, en=mesh.elem_node, h=mesh.h, x=x, v=v)
    frac = n_elem_sample / mesh.n_elem
    bounds = [(e0, min(e0 + chunk, n_elem_sample)) for e0 in range(0, n_elem_sample, chunk)]
    dt = sum(_oracle_chunk(a, b)[1] for a, b in bounds)            # (i) one process, one thread
    single = dict(value=mesh.n_dof * frac / dt, cores=1, seconds=round(dt, 2))
    n_work = workers or min(16, os.cpu_count() or 1)
    sample2 = min(mesh.n_elem, n_elem_sample * n_work)              # (ii) the same work per core
    bounds2 = [(e0, min(e0 + chunk, sample2)) for e0 in range(0, sample2, chunk)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(n_work) as pool:
        parts = pool.starmap(_oracle_chunk, bounds2)
    wall = time.perf_counter() - t0
    math.fsum(p[0] for p in parts)
    frac2 = sample2 / mesh.n_elem
    return dict(value=mesh.n_dof * frac2 / wall, unit="DOF-iterations/s", cores=n_work, kind="oracle",
                sample=f"energy+gradient+Hessian action of the FP64 oracle on {sample2} of {mesh.n_elem} elements "
                       f"in chunks of {chunk} over {n_work} worker processes of one thread ({wall:.1f} s wall), "
                       f"scaled by the element fraction; host {cpu}, {os.cpu_count()} CPUs visible",
                single_thread=dict(single, sample=f"{n_elem_sample} elements in one thread"))


def build_mesh(T, torch, dev, name, gpu_repair=False):
    """The named workload's seeded mesh and its target W = h I.  With
    gpu_repair, inverted elements of the seeded mesh are redrawn using the
    library's own det A (the W_3 sizes kernel), as the test suite does with
    the oracle's."""
    w = meshgen.WORKLOADS[name]
    W = None
    bad = None
    if gpu_repair:
        topo = meshgen.box_mesh(w["dim"], w["n"], w["p"])
        W = topo.h * np.eye(w["dim"])
        cctx = T.Context(w["dim"], w["p"], topo.elem_node, topo.n_node, w["Q"], w["metric"], W)
        floor = w["tau_min"] * topo.h ** w["dim"]

        def bad(xh, elems):
            s_q, _ = cctx.target_sizes_w3(torch.from_numpy(xh).to(dev))
            detA = s_q.cpu().numpy() ** w["dim"]
            worst = np.where(np.isnan(detA), -np.inf, detA).min(axis=1)
            worst = worst if elems is None else worst[np.asarray(elems)]
            return np.flatnonzero(worst <= floor)
    mesh = meshgen.make_workload(name, bad_elements=bad)
    if W is None:
        W = mesh.h * np.eye(w["dim"])
    return w, mesh, W


def time_workload(T, torch, dev, name, steps, warmup, log, gpu_repair=False):
    """Builds the named workload and times its element operations in FP64
    and mixed FP32: seconds per step (energy + gradient, then the Hessian
    action), per-operation device time (HIP events on the library's stream)
    and per-launch kernel time."""
    w, mesh, W = build_mesh(T, torch, dev, name, gpu_repair)
    x = torch.from_numpy(mesh.x).to(dev)
    v = torch.from_numpy(meshgen.random_direction(mesh, w["seed"] + 100)).to(dev)
    log(f"# workload {name}: {mesh.n_elem} elements, {mesh.n_dof} DOFs, repair rounds "
        f"{mesh.info.get('repair_rounds', 0)}")
    results = {}
    # the mesh's default scatter beside the other one: 2D, the tiles beside the
    # colour launches; 3D, the colour launches and the element-vector scatter
    # (the default of 3D meshes with colours of at most 49,152 elements on
    # average, 131,072 in the mixed path, such as q2_cube_64, q2_cube_32 and
    # q3_cube_48)
    probe = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    main = probe.scatter
    probe.close()
    names = {T.TMOP_SCATTER_TILES: "tiles", T.TMOP_SCATTER_COLOURS: "colours", T.TMOP_SCATTER_ELEMENTS: "elements"}
    if w["dim"] == 2:
        other = T.TMOP_SCATTER_COLOURS if main == T.TMOP_SCATTER_TILES else T.TMOP_SCATTER_TILES
    else:
        other = T.TMOP_SCATTER_ELEMENTS if main == T.TMOP_SCATTER_COLOURS else T.TMOP_SCATTER_COLOURS
    oname = names[other]
    log(f"# {name}: default scatter {names[main]}, also timed: {oname}")
    variants = [(T.TMOP_FP64, "f64", main), (T.TMOP_MIXED_FP32, "mixed", main),
                (T.TMOP_FP64, f"f64_{oname}", other), (T.TMOP_MIXED_FP32, f"mixed_{oname}", other)]
    for prec, pname, scatter in variants:
        t_set = time.perf_counter()   # set-up on the host: tables, colouring, 2D tiles, uploads
        ctx = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W,
                        fixed=mesh.fixed, precision=prec)
        t_set = time.perf_counter() - t_set
        ctx.set_scatter(scatter)
        F, md, st = ctx.energy(x)
        if st != 0 or not md > 0:
            raise SystemExit(f"{name}: inverted input mesh (min det A = {md})")
        g = torch.empty_like(x)
        Hv = torch.empty_like(x)

        def step():
            ctx.energy_gradient(x, g)
            ctx.hessian_apply(x, v, Hv)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps

        # per-operation device time, HIP events on the stream the library uses
        stream = torch.cuda.current_stream()
        ops = {}
        for oname, fn in (("energy", lambda: ctx.energy(x)), ("gradient", lambda: ctx.gradient(x, g)),
                          ("energy_gradient", lambda: ctx.energy_gradient(x, g)),
                          ("hessian", lambda: ctx.hessian_apply(x, v, Hv)),
                          ("hessian_diagonal", lambda: ctx.hessian_diagonal(x, Hv))):
            ts = []
            for _ in range(max(steps, 5)):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            ops[oname] = float(np.median(ts))
        # per-launch device time of the element kernels over K steps
        ctx.timing_enable(True)
        for _ in range(steps):
            ctx.energy(x)
            ctx.gradient(x, g)
            ctx.hessian_diagonal(x, Hv)
            step()
        launch = {}
        for op, oname in enumerate(("energy", "gradient", "hessian", "energy_gradient", "hessian_diagonal")):
            tot_ms, n = ctx.timing_read(op)
            launch[oname] = dict(launches=n, us_per_launch=tot_ms * 1e3 / n, us_per_op=tot_ms * 1e3 / steps)
        ctx.timing_enable(False)
        results[pname] = dict(ms_per_step=ms, value=mesh.n_dof / (ms * 1e-3), ops=ops, F=F, ctx=ctx,
                              launch=launch, scatter=names[scatter])
        results[pname]["setup_s"] = t_set
        log(f"# {pname}: {ms:.3f} ms/step, E {ops['energy']*1e6:.1f} us, G {ops['gradient']*1e6:.1f} us, "
            f"E+G {ops['energy_gradient']*1e6:.1f} us, Hv {ops['hessian']*1e6:.1f} us, "
            f"diag {ops['hessian_diagonal']*1e6:.1f} us; per launch "
            + ", ".join(f"{k} {v['us_per_launch']:.1f}" for k, v in launch.items()))
    # "cold" operation times: a 512 MiB buffer is rewritten before each call,
    # evicting x, v and the outputs from the 256 MB Infinity Cache and the L2s
    flush = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for pname in ("f64", "mixed"):
        ctx = results[pname]["ctx"]
        cold = {}
        g = torch.empty_like(x)
        Hv = torch.empty_like(x)
        for oname, fn in (("energy_gradient", lambda: ctx.energy_gradient(x, g)),
                          ("hessian", lambda: ctx.hessian_apply(x, v, Hv))):
            ts = []
            for _ in range(max(steps // 2, 3)):
                flush.fill_(1.0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            cold[oname] = float(np.median(ts))
        results[pname]["cold"] = cold
        log(f"# {pname} cold (caches flushed before each call): E+G {cold['energy_gradient']*1e6:.1f} us, "
            f"Hv {cold['hessian']*1e6:.1f} us")
    del flush
    # error of the mixed path against the FP64 path (itself within 1e-12 of
    # the FP64 oracle in the parity tests), per result
    vals = {}
    for pname in ("f64", "mixed"):
        ctx = results[pname]["ctx"]
        F, _, _, g = ctx.energy_gradient(x)
        vals[pname] = (F, g, ctx.hessian_apply(x, v))
    (F64, g64, h64), (F32, g32, h32) = vals["f64"], vals["mixed"]
    gn64 = float(torch.linalg.vector_norm(g64))
    results["mixed"]["rel_err_vs_f64"] = {
        "F": abs(F32 - F64) / abs(F64),
        "grad_norm": abs(float(torch.linalg.vector_norm(g32)) - gn64) / gn64,
        "grad_max": float((g32 - g64).abs().max() / g64.abs().max()),
        "hessian_action_max": float((h32 - h64).abs().max() / h64.abs().max())}
    log(f"# mixed vs f64: " + ", ".join(f"{k} {e:.2e}" for k, e in results["mixed"]["rel_err_vs_f64"].items()))
    del vals, g64, g32, h64, h32
    return w, mesh, x, v, W, results


def op_times(torch, ctx, x, v, reps):
    """Median device time (s) of energy, energy + gradient, Hessian action
    and Hessian diagonal: HIP events on the stream the library uses."""
    stream = torch.cuda.current_stream()
    g, Hv = torch.empty_like(x), torch.empty_like(x)
    out = {}
    for oname, fn in (("energy", lambda: ctx.energy(x)), ("energy_gradient", lambda: ctx.energy_gradient(x, g)),
                      ("hessian", lambda: ctx.hessian_apply(x, v, Hv)),
                      ("hessian_diagonal", lambda: ctx.hessian_diagonal(x, Hv))):
        fn()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        out[oname] = float(np.median(ts))
    return out


def targets(T, torch, dev, args, w, mesh, x, v, W, log):
    """Per-point targets and sliding boundaries on the main workload.
    W_3 (Section 3.1: W_q = (det A(x_0))^(1/d) I at every point, from the
    input mesh itself): FP64 operation times and the Hessian launch (of the
    mesh's default scatter) against the constant target W = h I.  Sliding (Section 4.1: only the
    normal component of a boundary node is fixed): Newton with the
    inexact-Newton forcing from the same mesh, against the fixed
    boundary."""
    reps = max(args.steps, 5)
    us = lambda d: {k: round(t * 1e6, 2) for k, t in d.items()}

    def hess_launch(ctx):
        Hv = torch.empty_like(x)
        ctx.hessian_apply(x, v, Hv)
        ctx.timing_enable(True)
        for _ in range(reps):
            ctx.hessian_apply(x, v, Hv)
        ms, n = ctx.timing_read(T.TIMING_HESS)
        ctx.timing_enable(False)
        return ms * 1e3 / n

    ctx = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    const = op_times(torch, ctx, x, v, reps)
    const_l = hess_launch(ctx)
    sizes, st = ctx.target_sizes_w3(x)
    ctx.close()
    cq = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], None, fixed=mesh.fixed,
                   target_sizes=sizes.cpu().numpy())
    w3 = op_times(torch, cq, x, v, reps)
    w3_l = hess_launch(cq)
    cq.close()
    log(f"# targets W_3 on {args.workload}: Hv {const['hessian']*1e6:.1f} -> {w3['hessian']*1e6:.1f} us "
        f"(Hessian launch {const_l:.1f} -> {w3_l:.1f} us), E+G {const['energy_gradient']*1e6:.1f} -> "
        f"{w3['energy_gradient']*1e6:.1f} us")
    newton = {}
    for key, slide in (("fixed", False), ("sliding", True)):
        fixed = meshgen.box_mesh(w["dim"], w["n"], w["p"], slide=slide).fixed
        cs = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=fixed)
        xn = x.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rep = cs.newton_solve(xn, max_it=50, cg_forcing=1)
        torch.cuda.synchronize()
        newton[key] = dict(status=st, iters=rep["iters"], cg_iters=rep["cg_iters"],
                           wall_s=round(time.perf_counter() - t0, 4), F0=rep["F0"], F=rep["F"],
                           free_dofs=int(fixed.size - np.count_nonzero(fixed)))
        cs.close()
        log(f"# targets newton {key} boundary: {rep['iters']} it, {rep['cg_iters']} CG, {newton[key]['wall_s']} s, "
            f"F {rep['F0']:.4e} -> {rep['F']:.4e}, {newton[key]['free_dofs']} free DOFs")
    return {"workload": args.workload,
            "w3": {"ops_us_constant_W": us(const), "ops_us_w3": us(w3),
                   "hessian_launch_us_constant_W": round(const_l, 2), "hessian_launch_us_w3": round(w3_l, 2)},
            "newton_inexact_f64": newton}


def section4(T, torch, dev, args, w, mesh, x, v, W, log):
    """Cost of the Section 4 objectives.  Displacement penalty (eq. 4.2) on
    the main workload: FP64 operation times with and without it (fused into
    the element kernels), the separate penalty kernels' per-launch time in
    the mixed-precision Hessian action against the HBM peak (they move 3
    fields per unique node: v in, out read and written), and
    Newton with the penalty; the replication composite (Section 4.3.2,
    gamma = 1/2) on the main workload.  Second metric term (eq. 4.1, mu_77
    with W_2 = 0.7 h I and per-point weights) and replication composite on a
    2D workload: operation times."""
    reps = max(args.steps, 5)
    us = lambda d: {k: round(t * 1e6, 2) for k, t in d.items()}
    out = {}
    ctx = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    plain = op_times(torch, ctx, x, v, reps)
    delta = 1.0e3
    ctx.set_restriction(delta, x)
    pen = op_times(torch, ctx, x, v, reps)
    # the penalty's own kernels (they run separately in the mixed-precision
    # context; the FP64 3D kernels fuse the penalty into the element passes)
    cm = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed,
                   precision=T.TMOP_MIXED_FP32)
    cm.set_restriction(delta, x)
    Hv = torch.empty_like(x)
    cm.hessian_apply(x, v, Hv)
    cm.timing_enable(True)
    for _ in range(reps):
        cm.hessian_apply(x, v, Hv)
    ms, n = cm.timing_read(T.TIMING_PENALTY)
    cm.timing_enable(False)
    cm.close()
    per_op = n / reps
    t_l = ms * 1e-3 / n
    _, nbytes = algorithmic(w)
    gbps = nbytes[2] * mesh.n_elem / per_op / t_l / 1e9
    newton = {}
    for key, d in (("plain", 0.0), ("penalty", delta)):
        ctx.set_restriction(d, x)
        xn = x.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rep = ctx.newton_solve(xn, max_it=50, cg_forcing=1)
        torch.cuda.synchronize()
        newton[key] = dict(status=st, iters=rep["iters"], cg_iters=rep["cg_iters"],
                           wall_s=round(time.perf_counter() - t0, 4), F0=rep["F0"], F=rep["F"],
                           max_displacement_over_h=float((xn - x).abs().max()) / mesh.h)
        log(f"# section 4 newton {key}: {rep['iters']} it, {rep['cg_iters']} CG, {newton[key]['wall_s']} s, "
            f"F {rep['F0']:.4e} -> {rep['F']:.4e}, max |x - x_init| / h {newton[key]['max_displacement_over_h']:.3e}")
    # replication composite on the main workload (W_0 = A(x) per point)
    ctx.set_restriction(0.0)
    ctx.set_replication(0.5, x)
    repl = op_times(torch, ctx, x, v, reps)
    ctx.close()
    out["replication_main"] = {"workload": args.workload, "ops_us_plain": us(plain), "ops_us_replication": us(repl)}
    log(f"# section 4 replication on {args.workload}: Hv {plain['hessian']*1e6:.1f} -> {repl['hessian']*1e6:.1f} us, "
        f"E+G {plain['energy_gradient']*1e6:.1f} -> {repl['energy_gradient']*1e6:.1f} us")
    out["penalty"] = {"workload": args.workload, "delta": delta, "ops_us_plain": us(plain), "ops_us_penalty": us(pen),
                      "separate_kernel_hessian_launch_us": round(t_l * 1e6, 2), "launches_per_op": per_op,
                      "algorithmic_bytes_per_element": nbytes[2], "algorithmic_GBps": round(gbps, 1),
                      "frac_hbm_peak": round(gbps * 1e9 / HBM_PEAK, 4), "newton_inexact_f64": newton}
    log(f"# section 4 penalty on {args.workload}: Hv {plain['hessian']*1e6:.1f} -> {pen['hessian']*1e6:.1f} us, "
        f"E+G {plain['energy_gradient']*1e6:.1f} -> {pen['energy_gradient']*1e6:.1f} us (FP64, fused); separate penalty "
        f"kernel (mixed context) {t_l*1e6:.2f} us per launch, {gbps:.0f} GB/s algorithmic")
    # 2D: second metric term and replication composite
    name2 = args.section4_2d
    w2, mesh2, W2 = build_mesh(T, torch, dev, name2, gpu_repair=True)
    x2 = torch.from_numpy(mesh2.x).to(dev)
    v2 = torch.from_numpy(meshgen.random_direction(mesh2, w2["seed"] + 100)).to(dev)
    c2 = T.Context(2, w2["p"], mesh2.elem_node, mesh2.n_node, w2["Q"], w2["metric"], W2, fixed=mesh2.fixed)
    p2 = op_times(torch, c2, x2, v2, reps)
    eta_q = np.random.default_rng(7).uniform(0.2, 1.2, (mesh2.n_elem, w2["Q"] ** 2))
    c2.set_combo(77, 0.7 * mesh2.h * np.eye(2), 1.0, 1.0, eta_q)
    cb = op_times(torch, c2, x2, v2, reps)
    c2.set_replication(0.5, x2)
    rp = op_times(torch, c2, x2, v2, reps)
    c2.close()
    out["second_term"] = {"workload": name2, "elements": mesh2.n_elem, "ops_us_plain": us(p2),
                          "ops_us_combo_mu77": us(cb), "ops_us_replication": us(rp)}
    log(f"# section 4 on {name2}: Hv plain {p2['hessian']*1e6:.1f}, + mu_77 term {cb['hessian']*1e6:.1f}, "
        f"replication {rp['hessian']*1e6:.1f} us")
    return out


def dfo(T, torch, dev, args, w, mesh, x, W, log):
    """Derivative-free solver (Section 3.4): one sweep over the main
    workload (node moves per second), and the full solve on the 8x8 Q2
    workload against Newton's wall time to the same mesh."""
    out = {}
    ctx = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    xs = x.clone()
    ctx.dfo_sweep(xs.clone(), max_evals=4)                     # builds the node colouring
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mv = ctx.dfo_sweep(xs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    F0, F1 = ctx.energy(x)[0], ctx.energy(xs)[0]
    ctx.close()
    out["sweep"] = {"workload": args.workload, "nodes": mesh.n_node, "seconds": round(dt, 4),
                    "node_moves_per_s": mesh.n_node / dt, "F0": F0, "F_after": F1, "max_move_over_h": mv / mesh.h}
    log(f"# dfo: one sweep over {args.workload} in {dt:.3f} s ({mesh.n_node / dt:.3e} nodes/s), "
        f"F {F0:.4e} -> {F1:.4e}")
    w8, m8, W8 = build_mesh(T, torch, dev, "q2_square_8", gpu_repair=True)
    c8 = T.Context(2, w8["p"], m8.elem_node, m8.n_node, w8["Q"], w8["metric"], W8, fixed=m8.fixed)
    x8 = torch.from_numpy(m8.x).to(dev)
    xd = x8.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep = c8.dfo_solve(xd)
    torch.cuda.synchronize()
    t_dfo = time.perf_counter() - t0
    xn = x8.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_n, rn = c8.newton_solve(xn)
    torch.cuda.synchronize()
    t_newton = time.perf_counter() - t0
    diff = float((xd - xn).abs().max()) / m8.h
    c8.close()
    out["solve_q2_square_8"] = {"status": st, "sweeps": rep["sweeps"], "seconds": round(t_dfo, 4), "F0": rep["F0"],
                                "F": rep["F"], "newton_seconds": round(t_newton, 4), "newton_F": rn["F"],
                                "max_diff_to_newton_over_h": diff}
    log(f"# dfo: q2_square_8 solve {rep['sweeps']} sweeps {t_dfo:.3f} s, F {rep['F0']:.4e} -> {rep['F']:.4e}; "
        f"Newton {t_newton:.3f} s, F {rn['F']:.4e}; max |x_dfo - x_newton| / h {diff:.2e}")
    return out


def small_newton(T, torch, dev, log):
    """The 8x8 Q2 mu_2 workload's setting, 10 Newton iterations with the
    default inner solver (cg_rtol 1e-10): the library on the GPU against the
    FP64 oracle's Newton (same rules) on the host."""
    from oracle import tmop_oracle as O
    w = meshgen.WORKLOADS["q2_square_8"]
    mesh = meshgen.box_mesh(2, w["n"], w["p"])
    W = mesh.h * np.eye(2)
    prob = O.Problem(2, w["p"], w["Q"], mesh.elem_node, w["metric"], W)
    x0 = meshgen.perturb(mesh, w["noise"], w["seed"], bad_elements=prob.bad_elements)
    t0 = time.perf_counter()
    xo, rep_o = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=10, cg_rtol=1e-10))
    t_cpu = time.perf_counter() - t0
    ctx = T.Context(2, w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    xd = torch.from_numpy(x0).to(dev)
    ctx.newton_solve(xd.clone(), max_it=10, cg_rtol=1e-10)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep = ctx.newton_solve(xd, max_it=10, cg_rtol=1e-10)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    ctx.close()
    F_o = [h[0] for h in rep_o.history]
    out = dict(iters=rep["iters"], gpu_s=round(t_gpu, 4), oracle_s=round(t_cpu, 3), F_gpu=rep["history_F"],
               F_oracle=F_o, max_rel_F_diff=max(abs(a - b) / a for a, b in zip(F_o, rep["history_F"]) if a > 1e-8 * F_o[0]),
               dist_to_grid_over_h=float(np.max(np.abs(xd.cpu().numpy() - mesh.x_grid)) / mesh.h))
    log(f"# newton q2_square_8, 10 iterations: GPU {t_gpu:.4f} s, oracle {t_cpu:.2f} s, F {F_o[0]:.4e} -> "
        f"{rep['F']:.4e} (oracle {rep_o.F:.4e})")
    return out


def cg_iteration_cost(T, torch, dev, log, name="q2_square_512"):
    """Device time of one inner-solver iteration (a Hessian action plus the
    solver's vector kernels and device-side scalars, with its occasional
    host checks) against the Hessian action alone, on the learned-guess
    evaluation workload: one Newton iteration whose inner solve runs to its
    iteration cap (tolerance 1e-30), at two caps; the difference over the
    difference in iterations is the cost of one."""
    w, mesh, W = build_mesh(T, torch, dev, name, True)
    x0 = torch.from_numpy(mesh.x).to(dev)
    v = torch.from_numpy(meshgen.random_direction(mesh, w["seed"] + 100)).to(dev)
    out = {"workload": name}
    for prec, pname in ((T.TMOP_FP64, "f64"), (T.TMOP_MIXED_FP32, "mixed")):
        ctx = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W,
                        fixed=mesh.fixed, precision=prec)
        hess = op_times(torch, ctx, x0, v, 20)["hessian"]
        res = {"hessian_us": round(hess * 1e6, 2)}
        for inner, iname in ((T.TMOP_INNER_SHIFTED_CG, "shifted_cg"), (T.TMOP_INNER_CG, "cg"),
                             (T.TMOP_INNER_MINRES, "minres")):
            pts = []
            for cap in (40, 40, 140):   # the first run warms up
                x = x0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, rep = ctx.newton_solve(x, max_it=1, cg_rtol=1e-30, cg_max_it=cap, inner=inner)
                torch.cuda.synchronize()
                pts.append((rep["cg_iters"], time.perf_counter() - t0))
            (n1, t1), (n2, t2) = pts[1], pts[2]
            per = (t2 - t1) / (n2 - n1) if n2 > n1 else None
            res[iname] = {"iterations": [n1, n2], "us_per_iteration": round(per * 1e6, 2) if per else None,
                          "ratio_to_hessian": round(per / hess, 3) if per else None}
        ctx.close()
        out[pname] = res
        log(f"# inner iteration cost {name} {pname}: Hv {res['hessian_us']} us; "
            + ", ".join(f"{k} {res[k]['us_per_iteration']} us ({res[k]['ratio_to_hessian']}x)"
                        for k in ("shifted_cg", "cg", "minres")))
    return out


def workload_summary(w, mesh, results):
    """Per-operation rates of one workload against the FP64 VALU and HBM
    peaks (algorithmic flops and unique L-vector bytes per element)."""
    flops, nbytes = algorithmic(w)
    out = {"elements": mesh.n_elem, "dofs": mesh.n_dof}
    for pname, r in results.items():
        d = {"ms_per_step": round(r["ms_per_step"], 4), "dof_iterations_per_s": r["value"]}
        for k, (op, key) in enumerate((("energy", "energy"), ("gradient", "gradient"), ("hessian", "hessian"))):
            t = r["ops"][op]
            d[key] = {"us": round(t * 1e6, 2),
                      "tflops": round(flops[k] * mesh.n_elem / t / 1e12, 3),
                      "frac_fp64_peak": round(flops[k] * mesh.n_elem / t / FP64_PEAK, 4),
                      "algorithmic_GBps": round(nbytes[k] * mesh.n_elem / t / 1e9, 1),
                      "frac_hbm_peak": round(nbytes[k] * mesh.n_elem / t / HBM_PEAK, 4)}
        if "rel_err_vs_f64" in r:
            d["rel_err_vs_f64"] = r["rel_err_vs_f64"]
        if "setup_s" in r:
            d["setup_s"] = round(r["setup_s"], 3)
        out[pname] = d
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process and has no multi-GPU path; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_1807_09807_amd import tmop as T
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    T.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        copy_calibration(torch, dev)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    w, mesh, x, v, W, results = time_workload(T, torch, dev, args.workload, args.steps, args.warmup, log,
                                              gpu_repair=True)
    x_np = mesh.x
    v_np = v.cpu().numpy()
    flops, nbytes = algorithmic(w)

    # Newton wall time to F_tol = F_ref + 1e-8 F0, F_ref = F at the workload's known minimizer, the
    # unperturbed grid (T = I at every point, so F = 0 up to rounding)
    newton = None
    if not args.no_newton:
        newton = {}

        def solve(pname, **kw):
            ctx = results[pname]["ctx"]
            xn = x.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, rep = ctx.newton_solve(xn, max_it=50, **kw)
            torch.cuda.synchronize()
            rep["wall_s"] = time.perf_counter() - t0
            return st, rep

        c64 = results["f64"]["ctx"]
        F_ref = c64.energy(torch.from_numpy(mesh.x_grid).to(dev))[0]
        F_tol = F_ref + 1e-8 * c64.energy(x)[0]
        newton["F_ref"], newton["F_tol"] = F_ref, F_tol
        J, MR, TC = T.TMOP_PREC_JACOBI, T.TMOP_INNER_MINRES, T.TMOP_INNER_CG
        # default: CG on the Hessian shifted to positive definiteness; truncated CG (Steihaug) and MINRES beside it
        variants = (("f64", "f64", dict()), ("f64_inexact", "f64", dict(cg_forcing=1)),
                    ("mixed", "mixed", dict()), ("mixed_inexact", "mixed", dict(cg_forcing=1)),
                    ("f64_jacobi", "f64", dict(precond=J)),
                    ("f64_truncated_cg", "f64", dict(inner=TC)), ("f64_truncated_cg_inexact", "f64", dict(inner=TC, cg_forcing=1)),
                    ("f64_minres_inexact", "f64", dict(inner=MR, cg_forcing=1)),
                    ("f64_minres_jacobi", "f64", dict(inner=MR, precond=J)))
        for key, pname, kw in variants:
            st, rep = solve(pname, ftarget=F_tol, **kw)
            reached = next((k for k, f in enumerate(rep["history_F"]) if f <= F_tol), None)
            newton[key] = dict(status=st, reached_F_tol=reached is not None,
                               wall_s_to_F_tol=rep["history_time"][reached] if reached is not None else None,
                               iters=rep["iters"], cg_iters=rep["cg_iters"], neg_curv=rep["neg_curv"], F=rep["F"])
            print(f"# newton {key}: status {st}, {rep['iters']} it, {rep['cg_iters']} CG, {rep['neg_curv']} "
                  f"negative-curvature exits or CG restarts, {rep['wall_s']:.2f} s, F {rep['F0']:.4e} -> "
                  f"{rep['F']:.4e}", file=sys.stderr, flush=True)
        newton["q2_square_8"] = small_newton(T, torch, dev, lambda m: print(m, file=sys.stderr, flush=True))
        newton["inner_iteration_cost"] = cg_iteration_cost(T, torch, dev,
                                                           lambda m: print(m, file=sys.stderr, flush=True))

    tgt = None
    if not args.no_targets:
        tgt = targets(T, torch, dev, args, w, mesh, x, v, W, lambda m: print(m, file=sys.stderr, flush=True))

    sec4 = None
    if not args.no_section4:
        sec4 = section4(T, torch, dev, args, w, mesh, x, v, W, lambda m: print(m, file=sys.stderr, flush=True))

    dfo_res = None
    if not args.no_dfo:
        dfo_res = dfo(T, torch, dev, args, w, mesh, x, W, lambda m: print(m, file=sys.stderr, flush=True))

    learned = None
    if not args.no_learned:
        learned = learned_guess(args, lambda m: print(m, file=sys.stderr, flush=True))

    others = {}
    for name in [n for n in args.other_workloads.split(",") if n and n != args.workload]:
        wo, mo, xo, vo, Wo, ro = time_workload(T, torch, dev, name, args.steps, args.warmup, log, gpu_repair=True)
        others[name] = workload_summary(wo, mo, ro)
        for r in ro.values():
            r["ctx"].close()
        del xo, vo

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, mesh, x_np, v_np, min(args.cpu_elems, mesh.n_elem))

    r64 = results["f64"]
    hl = r64["launch"]["hessian"]
    per_op = hl["launches"] / args.steps                      # launches per Hessian action
    t_l = hl["us_per_launch"] * 1e-6
    fl = flops[2] * mesh.n_elem / per_op                     # algorithmic flops per launch
    scatter = r64["scatter"]
    traffic = measured_traffic(args.workload, scatter)
    kernel_label = ("Hessian-action element kernel (FP64), one colour launch" if scatter == "colours" else
                    "Hessian-action element kernel (FP64), one element-vector launch over every element")
    line = {
        "metric": "DOF-iterations/s of energy+grad+Hv (FP64 vs FP32), Newton wall-s to F tol",
        "value": r64["value"],
        "unit": "DOF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": w["dim"], "order": w["p"], "elements": mesh.n_elem,
                   "dofs": mesh.n_dof, "quadrature": f"{w['Q']}^{w['dim']} Gauss-Legendre",
                   "metric": f"mu_{w['metric']}", "target": "W = h I"},
        "roofline": {"kernel": kernel_label, "scatter": scatter,
                     "bound": "alu", "achieved": fl / t_l / 1e12, "peak": FP64_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": fl / t_l / FP64_PEAK, "traffic": traffic,
                     "launch_us": hl["us_per_launch"], "launches_per_op": per_op,
                     "elements_per_launch": mesh.n_elem / per_op,
                     "flops_per_element": flops[2], "algorithmic_bytes_per_element": nbytes[2],
                     "algorithmic_GBps": nbytes[2] * mesh.n_elem / per_op / t_l / 1e9,
                     "traffic_GBps": traffic / t_l / 1e9 if traffic else None},
        "launch_us": {p: {k: round(v["us_per_launch"], 2) for k, v in results[p]["launch"].items()}
                      for p in ("f64", "mixed")},
        "ops_us": {k: round(t * 1e6, 2) for k, t in r64["ops"].items()},
        "cold_ops_us": {p: {k: round(t * 1e6, 2) for k, t in results[p]["cold"].items()} for p in ("f64", "mixed")},
        "mixed_fp32": {"value": results["mixed"]["value"], "ms_per_step": results["mixed"]["ms_per_step"],
                       "ops_us": {k: round(t * 1e6, 2) for k, t in results["mixed"]["ops"].items()},
                       "rel_err_vs_f64": results["mixed"]["rel_err_vs_f64"]},
        "workloads": {args.workload: workload_summary(w, mesh, {k: r for k, r in results.items()}), **others},
        "newton": newton,
        "targets": tgt,
        "section4": sec4,
        "derivative_free": dfo_res,
        "learned_guess": learned,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
