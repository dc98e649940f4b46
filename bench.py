"""Throughput of the hybrid NS-LES / Euler DGSEM residual on one MI355X.

A step is one time step of the three-stage low-storage RK: three hybrid
residual evaluations with the RK update fused into the residual kernels.
Workload: extruded NACA0012 O-grid, 96 x 48 x 8 quadratic hexahedra, P = 4
(4,608,000 nodes, 18.4M DOF with 4 fields), Re = 1e4, alpha = 20 deg, about
29% of the elements flagged viscous (wall band + wake wedge), FP64.

Prints one JSON line: DOF-residual evaluations per second (nodes x 4 fields
x residuals / s), the roofline of the dominant kernel measured with HIP
events inside the timed region, and the FP64 CPU oracle timed on this
host's cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF-residual evals/s (mixed NS-LES/Euler DG), plain vs batched FP32; p99 latency"
HBM_PEAK_GBS = 8000.0
# FETCH_SIZE / WRITE_SIZE summary of the benchmark's kernels (rocprofv3 --pmc)
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "traffic_naca0012_ogrid_96x48x8_P4.txt")
# VALU instruction counts of the same kernels (rocprofv3 --pmc SQ_INSTS_VALU_*)
FLOPS_SUMMARY = os.path.join(ROOT, "profiles", "flops_naca0012_ogrid_96x48x8_P4.txt")
# FETCH_SIZE / WRITE_SIZE summary of the mixed-order airfoil's kernels
MIXED_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "traffic_naca0012_ogrid_192x96x16_mixedP2-6.txt")


def algorithmic_bytes(n_elem: int, N: int, fused_rk: bool, f32: bool = False, first_stage: bool = False) -> float:
    """Algorithmic bytes of one hybrid residual evaluation over the whole mesh
    (the operator's inputs and outputs, each moved once): state q 32 B/node
    (FP64 in both precision forms), metric terms 1/J + 9 Ja 80 B/node (40 in
    FP32), the owned face geometry (unit normal and surface scale, 32 B per
    face node, 16 in FP32, three faces per element), and the output: R 32
    B/node (16 in FP32), or for a fused RK stage the register dq read 32 (not
    in the first stage, whose coefficient A is zero) and written 32 plus the
    next state 32.  The viscous kernel's intermediates (viscous part and face
    traces, written and read back) are a property of this implementation and
    are not counted; ``intermediate_bytes`` gives them."""
    N3, N2 = N ** 3, N ** 2
    met, fg = (40, 16) if f32 else (80, 32)
    out = ((64 if first_stage else 96) if fused_rk else (16 if f32 else 32))
    return float(n_elem * ((32 + met + out) * N3 + 3 * N2 * fg))


def shared_metric_saving(n_elem: int, blocks: int, N: int, f32: bool = False) -> float:
    """Metric bytes of one whole-mesh evaluation that a mesh whose translated
    elements share one metric block does not move: the algorithmic count
    reads 1/J and Ja once per element, the library once per block."""
    return float((n_elem - blocks) * (40 if f32 else 80) * N ** 3)


def with_shared_metrics(alg_bytes: float, saving: float, seconds: float) -> dict:
    """The same time against the bytes left once shared metric blocks are read
    once: above 1 of peak on the algorithmic count only means that reuse."""
    b = alg_bytes - saving
    return {"bytes": b, "achieved": b / seconds / 1e9, "frac": b / seconds / 1e9 / HBM_PEAK_GBS}


def intermediate_bytes(n_visc: int, N: int, f32: bool = False) -> float:
    """Bytes of the viscous kernel's outputs that the residual kernel reads back,
    per stage (flagged elements): the viscous part of the divergence 24 B/node
    (12 in FP32) and both sides' viscous face traces, 24 B (12) per face node
    and side on six faces.  Written once and read once."""
    N3, N2 = N ** 3, N ** 2
    tv = 12 if f32 else 24
    return float(n_visc * (tv * N3 + 6 * N2 * tv))


def viscous_kernel_bytes(n_visc: int, N: int, f32: bool = False) -> float:
    """Bytes the viscous kernel moves at least: velocity 24 B/node and metric
    terms in, the viscous part per node and six faces of traces out."""
    N3, N2 = N ** 3, N ** 2
    met, tv = (40, 12) if f32 else (80, 24)
    return float(n_visc * ((24 + met + tv) * N3 + 6 * N2 * tv))


def kernel_symbol(kind: int, N: int, f32: bool, block: int, persistent: bool, fused_rk: bool = True) -> str:
    t = "float" if f32 else "double"
    p = "true" if persistent else "false"
    return f"k_viscous<{t}, {N}, {block}, {p}>" if kind == 0 else \
        f"k_residual<{t}, {1 if fused_rk else 0}, {N}, {block}, {p}>"


def fp32_residual_error(mesh, q, torch, hdg) -> dict:
    """Per-field relative error of the FP32 residual at state q against this
    library's FP64 residual (itself within 1e-12 of the FP64 oracle in the
    parity tests), in the mass-weighted L2 norm and the max norm, each
    floored at 1e-3 of the largest field's norm (the parity norm).  The
    pressure row of a nearly divergence-free field is a small difference of
    terms of size c0^2 |grad u|, which an FP32 evaluation cannot beat; its
    error against its own (floored) norm is reported as is."""
    r64 = torch.empty_like(q)
    r32 = torch.empty(q.shape, dtype=torch.float32, device=q.device)
    hdg.hdg_residual(mesh, q, r64)
    hdg.hdg_residual(mesh, q, r32, prec=hdg.HDG_F32)
    ref = hdg.hdg_reduce(mesh, r64)
    d = r32.double() - r64
    err = hdg.hdg_reduce(mesh, d)
    out = {"reference": "FP64 path of this library", "norm": "per field, floored at 1e-3 of the largest"}
    for key in ("l2", "max"):
        den = np.maximum(ref[key], 1e-3 * ref[key].max())
        out[key] = [float(x) for x in err[key] / den]
        out[key + "_unfloored"] = [float(x) for x in err[key] / np.maximum(ref[key], 1e-300)]
    out["fields"] = ["p", "u", "v", "w"]
    del r64, r32, d
    return out


def cpu_baseline(w, q0, budget_s: float = 12.0) -> dict:
    import oracle
    om = oracle.OracleMesh(w.mesh, w.P, w.flag)
    prm = oracle.make_params(**w.params)
    nodes = w.mesh.n_elem * (w.P + 1) ** 3
    t0 = time.perf_counter()
    evals = 0
    while True:
        om.residual(prm, q0)
        evals += 1
        el = time.perf_counter() - t0
        if el >= budget_s or evals >= 1000:
            break
    threads = oracle.get_threads()
    # the same on one core, a few evaluations
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        evals1 = 0
        while True:
            om.residual(prm, q0)
            evals1 += 1
            el1 = time.perf_counter() - t0
            if el1 >= budget_s / 3 or evals1 >= 100:
                break
    finally:
        oracle.set_threads(threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": nodes * 4 * evals / el, "unit": "DOF-residual evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{evals} full residual evaluations of the same workload ({nodes} nodes), {el:.1f} s",
            "value_1core": nodes * 4 * evals1 / el1, "sample_1core": f"{evals1} evaluations, {el1:.1f} s",
            "cpu_model": model, "host_cpus": os.cpu_count()}


def mixed_leg(ctx, args, torch, hdg) -> dict:
    """Mixed-order form: the airfoil O-grid refined twice (192 x 96 x 16,
    quadratic) with per-element orders 2..6 (higher where viscous), faces
    between orders coupled through mortars; every order's tiles and the
    mortar kernels of an RK stage replayed from one captured graph."""
    from paper_2403_05463_amd import workloads as W
    t0 = time.perf_counter()
    w = W.naca_mixed()
    q0 = W.initial_state(w, None)
    t1 = time.perf_counter()
    mesh = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    t2 = time.perf_counter()
    nodes = mesh.nodes
    P = np.asarray(w.P)
    nonconf = int(((w.mesh.nbr >= 0) & (P[np.maximum(w.mesh.nbr, 0)] != P[:, None])).sum() // 2)
    print(f"[bench] {w.name}: {nodes} nodes, {nonconf} mortar faces, set-up {t2 - t1:.1f} s",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    q = torch.from_numpy(q0).cuda()
    dq = torch.empty_like(q)
    hdg.hdg_mesh_autotune(mesh, q, reps=2, stream=stream)
    res = {"config": {"workload": w.name, "elements": w.mesh.n_elem, "nodes": nodes, "dof": 4 * nodes,
                      "orders": {int(k): int(v) for k, v in zip(*np.unique(P, return_counts=True))},
                      "viscous_fraction": float(np.mean(w.flag)), "mortar_faces": nonconf, "geometry": "quadratic",
                      "dt": w.dt, "host_generation_s": t1 - t0, "mesh_create_s": t2 - t1}}
    steps = args.mixed_steps
    orders, counts = np.unique(P, return_counts=True)

    def bytes_per_step(f32):
        # the operator's algorithmic bytes, each element at its own order;
        # the mortars' intermediates are this implementation's, not counted
        return sum(algorithmic_bytes(int(c), int(o) + 1, fused_rk=True, f32=f32, first_stage=(st == 0))
                   for o, c in zip(orders, counts) for st in range(3))

    for prec, tag in ((hdg.HDG_F64, "f64"), (hdg.HDG_F32, "f32")):
        q.copy_(torch.from_numpy(q0))
        hdg.hdg_rk3_steps(mesh, q, dq, w.dt, 6, prec=prec, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        hdg.hdg_rk3_steps(mesh, q, dq, w.dt, steps, prec=prec, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        hdg.hdg_timing_enable(mesh, True)
        hdg.hdg_rk3_steps(mesh, q, dq, w.dt, steps, prec=prec, stream=stream)
        kern = {name: hdg.hdg_timing_read(mesh, k) for k, name in hdg.KERNEL_NAMES.items()}
        hdg.hdg_timing_enable(mesh, False)
        red = hdg.hdg_reduce(mesh, q, allow_nonfinite=True)
        bps = bytes_per_step(prec == hdg.HDG_F32)
        res[tag] = {"value": nodes * 4 * 3 * steps / (ms / 1e3), "unit": "DOF-residual evals/s",
                    "ms_per_step": ms / steps, "state_finite": bool(red["finite"]),
                    "stage_roofline": {"bytes_per_step": bps, "achieved": bps / (ms / steps * 1e-3) / 1e9,
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": bps / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS},
                    "kernel_ms_per_step": {k: v[0] / steps for k, v in kern.items()},
                    "launches_per_step": {k: v[1] / steps for k, v in kern.items()}}
        tps = mixed_traffic_per_step(mesh, hdg, w.mesh, P, np.asarray(w.flag), prec == hdg.HDG_F32)
        res[tag]["traffic_roofline"] = None if tps is None else {
            "bytes_per_step": tps, "achieved": tps / (ms / steps * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": tps / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "source": os.path.relpath(MIXED_TRAFFIC_SUMMARY, ROOT)}
    del q, dq, mesh
    return res


def mixed_traffic_per_step(mesh, hdg, mesh_desc, P, flag, f32: bool):
    """Measured HBM traffic of one RK step on a mesh of mixed order: the
    per-dispatch FETCH_SIZE + WRITE_SIZE bytes of the profile summary, summed
    over the kernels a stage launches (each order's viscous and residual
    kernel in the launch shape the mesh uses, each pair's mortar lift kernel
    where a side is flagged and flux kernel), times three stages; None when
    the summary is missing or the kernel sources changed since it was taken."""
    from paper_2403_05463_amd.profiling import traffic_for
    prec = hdg.HDG_F32 if f32 else hdg.HDG_F64
    t = "float" if f32 else "double"
    nb = mesh_desc.nbr
    e_idx = np.repeat(np.arange(len(P)), 6).reshape(-1, 6)
    hi = (nb >= 0) & (P[np.maximum(nb, 0)] < P[:, None])
    nl, nh = P[np.maximum(nb, 0)][hi] + 1, P[e_idx][hi] + 1
    vis = (flag[np.maximum(nb, 0)][hi] != 0) | (flag[e_idx][hi] != 0)
    syms = []
    for N in np.unique(P + 1):
        for kind in (hdg.HDG_KERNEL_VISCOUS, hdg.HDG_KERNEL_RESIDUAL):
            if kind == hdg.HDG_KERNEL_VISCOUS and not np.any(flag[P + 1 == N]):
                continue
            lc = hdg.hdg_mesh_get_launch(mesh, kind, prec, int(N))
            syms.append(kernel_symbol(kind, int(N), f32, lc["block"], lc["persistent"]))
    for a, b in sorted(set(zip(nl.tolist(), nh.tolist()))):
        syms.append(f"k_mortar_flux<{a}, {b}, {t}>")
        if np.any(vis[(nl == a) & (nh == b)]):
            syms.append(f"k_mortar_lift<{a}, {b}, {t}>")
    total = 0.0
    for sym in syms:
        v = traffic_for(MIXED_TRAFFIC_SUMMARY, sym)
        if v is None:
            return None
        total += v
    return 3.0 * total


def secondary_leg(ctx, args, torch, hdg) -> dict:
    """Secondary roofline: the fused FP64 RK stage on the periodic 32^3-element
    P = 5 Taylor-Green box (7.08M nodes, half the elements flagged), the same
    graph-replayed steps and per-launch event timing as the primary workload."""
    from paper_2403_05463_amd import workloads as W
    w = W.tgv_box_precision()
    mesh = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    q0 = W.initial_state(w, hdg.hdg_mesh_node_coords(mesh))
    N, nodes = w.P + 1, mesh.nodes
    n_visc = int(np.count_nonzero(w.flag))
    print(f"[bench] {w.name}: {nodes} nodes, {n_visc} viscous of {w.mesh.n_elem} elements",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    q = torch.from_numpy(q0).cuda()
    dq = torch.empty_like(q)
    hdg.hdg_mesh_autotune(mesh, q, reps=2, stream=stream)
    steps = max(args.steps // 2, 5)
    hdg.hdg_rk3_steps(mesh, q, dq, w.dt, 2, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    hdg.hdg_rk3_steps(mesh, q, dq, w.dt, steps, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    hdg.hdg_timing_enable(mesh, True)
    hdg.hdg_rk3_steps(mesh, q, dq, w.dt, steps, stream=stream)
    us = hdg.hdg_timing_samples(mesh, hdg.HDG_KERNEL_RESIDUAL)
    hdg.hdg_timing_enable(mesh, False)
    red = hdg.hdg_reduce(mesh, q, allow_nonfinite=True)
    # the precision form on the same box: FP32 residual, FP64 state (the
    # graph-replayed step, and the residual's per-field error in the floored
    # norms against this library's FP64 path at the initial state)
    q.copy_(torch.from_numpy(q0))
    f32_err = fp32_residual_error(mesh, q, torch, hdg)
    hdg.hdg_rk3_steps(mesh, q, dq, w.dt, 2, prec=hdg.HDG_F32, stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    hdg.hdg_rk3_steps(mesh, q, dq, w.dt, steps, prec=hdg.HDG_F32, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1)
    per_step = sum(algorithmic_bytes(w.mesh.n_elem, N, fused_rk=True, first_stage=(st == 0)) for st in range(3))
    avg_us = float(np.mean(us))
    launches_per_step = len(us) / steps
    achieved = per_step / launches_per_step / (avg_us * 1e-6) / 1e9
    cfg = hdg.hdg_mesh_get_launch(mesh, hdg.HDG_KERNEL_RESIDUAL, hdg.HDG_F64, N)
    blocks = hdg.hdg_mesh_metric_blocks(mesh)
    saving = 3 * shared_metric_saving(w.mesh.n_elem, blocks, N)        # per step
    del q, dq, mesh
    return {"workload": w.name, "nodes": nodes, "viscous_elements": n_visc, "steps": steps,
            "value": nodes * 4 * 3 * steps / (ms / 1e3), "unit": "DOF-residual evals/s",
            "ms_per_step": ms / steps, "state_finite": bool(red["finite"]),
            "metric_blocks": blocks,
            "fp32": {"ms_per_step": ms32 / steps, "value": nodes * 4 * 3 * steps / (ms32 / 1e3),
                     "residual_error": f32_err},
            "stage_roofline": {"achieved": per_step / (ms / steps * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": per_step / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "with_shared_metrics": with_shared_metrics(per_step, saving, ms / steps * 1e-3)},
            "roofline": {"kernel": kernel_symbol(1, N, False, cfg["block"], cfg["persistent"]), "bound": "hbm",
                         "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "avg_launch_us": avg_us,
                         "algorithmic_bytes_per_launch": per_step / launches_per_step,
                         "with_shared_metrics": with_shared_metrics(per_step / launches_per_step,
                                                                    saving / launches_per_step, avg_us * 1e-6),
                         "launch_us_p10_p50_p90": [float(np.percentile(us, p)) for p in (10, 50, 90)]}}


def clustering_leg(w, mesh, args, torch, hdg, ms_step: float) -> dict:
    """Clustering on the benchmark mesh (Sec. 2.1): node features of the
    developed-flow stand-in, a two-component mixture fitted by EM, element
    regions.  The EM cost per iteration is the difference of two fits."""
    from paper_2403_05463_amd import workloads as W
    X = hdg.hdg_mesh_node_coords(mesh)
    q = torch.from_numpy(W.developed_airfoil_state(X)).cuda()
    nodes = mesh.nodes
    F = torch.empty(3 * nodes, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    hdg.hdg_cluster_features(mesh, q, F, stream=stream)
    hdg.hdg_cluster_fit(mesh, F, 5, 1e-6, stream=stream)
    torch.cuda.synchronize()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        hdg.hdg_cluster_features(mesh, q, F, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    feat_ms = e0.elapsed_time(e1) / reps

    def fit_ms(k):
        t0 = time.perf_counter()
        res, flags = hdg.hdg_cluster_fit(mesh, F, k, 1e-6, stream=stream)
        return 1e3 * (time.perf_counter() - t0), res, flags

    lo, hi = 20, 100
    t_lo = min(fit_ms(lo)[0] for _ in range(3))
    runs = [fit_ms(hi) for _ in range(3)]
    t_hi = min(r[0] for r in runs)
    _, res, flags = runs[0]
    it_us = 1e3 * (t_hi - t_lo) / (hi - lo)
    em_bytes = 24.0 * nodes
    # a fit ended by the convergence test on the device (change of the mean
    # log-likelihood below 1e-4), as a dynamic clustering step would run it
    t0 = time.perf_counter()
    rt, ft = hdg.hdg_cluster_fit(mesh, F, 500, 1e-6, stream=stream, tol=1e-4)
    tol_ms = 1e3 * (time.perf_counter() - t0)
    return {"workload": f"{w.name} developed-flow stand-in", "nodes": nodes,
            "features_ms": feat_ms, "fit_ms": t_hi, "em_iterations": hi, "em_iteration_us": it_us,
            "em_pass_GBps": em_bytes / (it_us * 1e-6) / 1e9, "em_pass_bytes": em_bytes,
            "clustering_ms": feat_ms + t_hi, "clustering_over_rk_step": (feat_ms + t_hi) / ms_step,
            "tol_1e-4": {"iterations": rt["iterations"], "converged": rt["converged"], "fit_ms": tol_ms,
                         "clustering_over_rk_step": (feat_ms + tol_ms) / ms_step,
                         "viscous_fraction": float(ft.mean())},
            "viscous_fraction": float(flags.mean()), "geometric_mask_fraction": float(np.mean(w.flag)),
            "agreement_with_geometric_mask": float(np.mean(flags == w.flag)),
            "log_likelihood": res["log_likelihood"], "weights": [float(x) for x in res["weight"]]}


def serving_leg(ctx, args, torch, hdg) -> dict:
    """Request stream: Poisson arrivals of independent periodic-box solves (n^3
    elements, n uniform in 4..24, P uniform in 2..6, 20-80 % viscous, nu in
    [1e-4, 1e-2], 50 RK steps each, FP32 residual with FP64 state), admitted by
    device footprint into one continuously refilled batch.  Then, on a fixed
    set of those solves, batched stepping against stepping each mesh on its
    own (plain) for the same RK steps."""
    from paper_2403_05463_amd import serving as S
    reqs = S.make_requests(args.serve_requests, rate=args.serve_rate, seed=0)
    budget = int(args.serve_budget_gb * (1 << 30))
    print(f"[bench] serving {len(reqs)} requests at {args.serve_rate}/s", file=sys.stderr, flush=True)
    be = S.HdgBackend(ctx, max_members=64, prec=hdg.HDG_F32, torch=torch)
    st = S.serve(reqs, be, mem_budget=budget, max_members=64, max_steps_per_call=10, setup_workers=8)
    res = st.summary()
    res.update({"all_finite": all(bool(r.result) for r in st.requests),
                "config": {"requests": len(reqs), "rate_per_s": args.serve_rate, "n": "U{4..24}", "P": "U{2..6}",
                           "viscous_fraction": "U[0.2, 0.8]", "nu": "U[1e-4, 1e-2]", "rk_steps": 50,
                           "memory_budget_bytes": budget, "slots": 64, "steps_per_batch_call": 10,
                           "prec": "f32 residual, f64 state"}})
    del be, st
    # batched vs plain on a fixed set of solves (already resident)
    fixed = S.make_requests(32, rate=1.0, seed=1)
    be = S.HdgBackend(ctx, max_members=32, prec=hdg.HDG_F32, torch=torch)
    solves = [be.make_alone(r) for r in fixed]
    nodes = sum(m.n_elem * m.N3 for (m, _, _, _) in solves)
    steps = 10
    stream = torch.cuda.current_stream()
    for (m, q, dq, dt) in solves:
        hdg.hdg_rk3_steps(m, q, dq, dt, 2, prec=hdg.HDG_F32, stream=stream)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for (m, q, dq, dt) in solves:
        hdg.hdg_rk3_steps(m, q, dq, dt, steps, prec=hdg.HDG_F32, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    plain_ms = t0.elapsed_time(t1)
    b = hdg.hdg_batch_create(ctx, len(solves))
    for (m, q, dq, dt) in solves:
        hdg.hdg_batch_add(b, m, q, dq, dt)
    hdg.hdg_batch_autotune(b, reps=2, stream=stream)
    hdg.hdg_batch_rk3_steps(b, 2, prec=hdg.HDG_F32, stream=stream)
    torch.cuda.synchronize()
    t0.record(stream)
    hdg.hdg_batch_rk3_steps(b, steps, prec=hdg.HDG_F32, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    batch_ms = t0.elapsed_time(t1)
    dof = nodes * 4 * 3 * steps
    res["batched_vs_plain"] = {"solves": len(solves), "nodes": nodes, "rk_steps": steps,
                               "plain_f32_value": dof / (plain_ms / 1e3), "batched_f32_value": dof / (batch_ms / 1e3),
                               "speedup": plain_ms / batch_ms, "unit": "DOF-residual evals/s"}
    return res


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-mb", type=int, default=1024, help="size of the stream-copy probe")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-order airfoil leg")
    ap.add_argument("--no-cluster", action="store_true", help="skip the clustering leg")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 32^3 P = 5 TGV roofline leg")
    ap.add_argument("--mixed-only", action="store_true",
                    help="profiling aid: run only the mixed-order leg and print its JSON")
    ap.add_argument("--mixed-steps", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    args = ap.parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU element partition is designed but not implemented", file=sys.stderr)
        return 2

    import torch
    from paper_2403_05463_amd import hdg, workloads as W
    from paper_2403_05463_amd.profiling import flops_for, traffic_for

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.mixed_only:
        ctx = hdg.hdg_init(0)
        # one plain copy of known size first, the calibration of a traffic profile
        src = torch.empty((args.copy_mb << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        hdg.hdg_stream_copy(ctx, dst, src, args.copy_mb << 20, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        del src, dst
        print(json.dumps({"mixed_order": mixed_leg(ctx, args, torch, hdg)}), flush=True)
        return 0
    w = W.naca_working()
    q0 = W.initial_state(w, None)
    dt = w.dt
    N = w.P + 1
    nodes = w.mesh.n_elem * N ** 3
    ctx = hdg.hdg_init(0)
    mesh = hdg.hdg_mesh_create(ctx, w.mesh, w.P, w.flag, hdg.make_params(**w.params))
    info = hdg.hdg_mesh_info(mesh)
    q = torch.from_numpy(q0).cuda()
    dq = torch.empty_like(q)
    stream = torch.cuda.current_stream()
    print(f"[bench] {w.name}: {nodes} nodes, {info['n_viscous']} viscous of {w.mesh.n_elem} elements, "
          f"dt={dt:.3e}, warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    # launch shapes chosen by the library's autotuner on this mesh (set-up, untimed)
    hdg.hdg_mesh_autotune(mesh, q, reps=3, stream=stream)
    tuned = {f"{hdg.KERNEL_NAMES[k]}_{'f32' if p else 'f64'}": hdg.hdg_mesh_get_launch(mesh, k, p, N)
             for p in (hdg.HDG_F64, hdg.HDG_F32) for k in (hdg.HDG_KERNEL_VISCOUS, hdg.HDG_KERNEL_RESIDUAL)}
    print(f"[bench] autotuned launch shapes: {tuned}", file=sys.stderr, flush=True)

    def timed_run(prec):
        """K timed RK steps after W warm-up steps, replayed from the library's
        captured HIP graph; then K more steps launched eagerly with per-launch
        HIP events, for the per-kernel durations."""
        hdg.hdg_rk3_steps(mesh, q, dq, dt, max(args.warmup, 2), prec=prec, stream=stream)
        torch.cuda.synchronize()
        t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_start.record(stream)
        hdg.hdg_rk3_steps(mesh, q, dq, dt, args.steps, prec=prec, stream=stream)
        t_end.record(stream)
        torch.cuda.synchronize()
        hdg.hdg_timing_enable(mesh, True)
        hdg.hdg_rk3_steps(mesh, q, dq, dt, args.steps, prec=prec, stream=stream)
        kern = {name: hdg.hdg_timing_read(mesh, k) for k, name in hdg.KERNEL_NAMES.items()}
        samples = {name: hdg.hdg_timing_samples(mesh, k) for k, name in hdg.KERNEL_NAMES.items()}
        hdg.hdg_timing_enable(mesh, False)
        return t_start.elapsed_time(t_end), kern, samples

    ms, kern, samples = timed_run(hdg.HDG_F64)
    red = hdg.hdg_reduce(mesh, q, allow_nonfinite=True)

    # plain copy kernel of known size: attainable HBM bandwidth, and the
    # reference dispatch that calibrates the FETCH_SIZE / WRITE_SIZE counters
    copy_bytes = args.copy_mb << 20
    src = torch.empty(copy_bytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    hdg.hdg_stream_copy(ctx, dst, src, copy_bytes, stream=stream)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        hdg.hdg_stream_copy(ctx, dst, src, copy_bytes, stream=stream)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * copy_bytes * 5 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst

    n_visc = info["n_viscous"]
    metric_blocks = hdg.hdg_mesh_metric_blocks(mesh)
    kinds = {name: k for k, name in hdg.KERNEL_NAMES.items()}
    evals = 3 * args.steps

    def roofline(kern, f32, samples):
        """The residual kernel (the dominant class): the operator's algorithmic
        bytes per launch over its mean event-timed duration."""
        dom = "residual"
        assert max(kern, key=lambda k: kern[k][0]) == dom, kern
        tot, n = kern[dom]
        avg_s = tot / max(n, 1) / 1e3
        # every stage runs the residual kernel once over every element; the
        # first of the three stages does not read the RK register
        per_step = sum(algorithmic_bytes(w.mesh.n_elem, N, fused_rk=True, f32=f32, first_stage=(st == 0))
                       for st in range(3))
        bytes_launch = per_step * args.steps / max(n, 1)
        achieved = bytes_launch / avg_s / 1e9
        # per launch, like the bytes: the intermediates and the shared metric
        # blocks' saving are per stage, and a stage may take several launches
        inter = 3 * intermediate_bytes(n_visc, N, f32) * args.steps / max(n, 1)
        saving = 3 * shared_metric_saving(w.mesh.n_elem, metric_blocks, N, f32) * args.steps / max(n, 1)
        cfg = tuned[f"{dom}_{'f32' if f32 else 'f64'}"]
        sym = kernel_symbol(kinds[dom], N, f32, cfg["block"], cfg["persistent"])
        sm = samples.get(dom) or [avg_s * 1e6]
        return {"kernel": sym, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(TRAFFIC_SUMMARY, sym),
                "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_launch,
                "with_viscous_intermediates": {"bytes_per_launch": bytes_launch + inter,
                                               "achieved": (bytes_launch + inter) / avg_s / 1e9},
                "with_shared_metrics": with_shared_metrics(bytes_launch, saving, avg_s),
                "flops": flops_for(FLOPS_SUMMARY, sym, avg_s),
                "launches_timed": len(sm),
                "launch_us_p10_p50_p90": [float(np.percentile(sm, p)) for p in (10, 50, 90)]}

    def stage_roofline(ms_step, f32):
        """The whole stage (viscous and residual kernels, and mortars if any):
        the operator's algorithmic bytes of the three stages of a step over
        the graph-replayed time per step."""
        per_step = sum(algorithmic_bytes(w.mesh.n_elem, N, fused_rk=True, f32=f32, first_stage=(st == 0))
                       for st in range(3))
        achieved = per_step / (ms_step * 1e-3) / 1e9
        saving = 3 * shared_metric_saving(w.mesh.n_elem, metric_blocks, N, f32)
        return {"bound": "hbm", "bytes_per_step": per_step, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "target_ms_per_step_at_half_peak": per_step / (0.5 * HBM_PEAK_GBS * 1e9) * 1e3,
                "with_shared_metrics": with_shared_metrics(per_step, saving, ms_step * 1e-3)}

    roof = roofline(kern, False, samples)
    achieved = roof["achieved"]
    out = {
        "metric": METRIC,
        "value": nodes * 4 * evals / (ms / 1e3),
        "unit": "DOF-residual evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "form": "plain FP64", "elements": w.mesh.n_elem, "P": w.P,
                   "nodes": nodes, "dof": nodes * 4, "viscous_elements": n_visc,
                   "residuals_per_step": 3, "dt": dt, "rk": "3-stage low-storage (2N)"},
        "roofline": roof,
        "stage_roofline": stage_roofline(ms / args.steps, False),
        "kernels_us_per_launch": {k: (v[0] / max(v[1], 1) * 1e3) for k, v in kern.items()},
        "node_evals_per_s": nodes * evals / (ms / 1e3),
        "metric_blocks": metric_blocks,
        "state_finite": bool(red["finite"]),
        "launch_shapes": tuned,
        "hip_graph": "RK steps replayed from a captured graph (2 steps per replay)",
        "stream_copy_GBps": copy_gbs,
        "frac_of_stream_copy": achieved / copy_gbs,
    }
    # precision form on the same workload and state: FP32 contractions and
    # fluxes, FP64 state and RK accumulation
    q.copy_(torch.from_numpy(q0))
    fp32_err = fp32_residual_error(mesh, q, torch, hdg)
    ms32, kern32, samples32 = timed_run(hdg.HDG_F32)
    red32 = hdg.hdg_reduce(mesh, q, allow_nonfinite=True)
    out["fp32_plain"] = {"value": nodes * 4 * evals / (ms32 / 1e3), "ms_per_step": ms32 / args.steps,
                         "speedup_vs_fp64": ms / ms32, "state_finite": bool(red32["finite"]),
                         "kernels_us_per_launch": {k: (v[0] / max(v[1], 1) * 1e3) for k, v in kern32.items()},
                         "roofline": roofline(kern32, True, samples32),
                         "stage_roofline": stage_roofline(ms32 / args.steps, True),
                         "residual_error": fp32_err,
                         "dtype": "f32 residual, f64 state"}
    del q, dq
    if not args.no_cluster:
        print("[bench] clustering", file=sys.stderr, flush=True)
        out["clustering"] = clustering_leg(w, mesh, args, torch, hdg, ms / args.steps)
    if not args.no_secondary:
        out["secondary_roofline"] = secondary_leg(ctx, args, torch, hdg)
    if not args.no_mixed:
        out["mixed_order"] = mixed_leg(ctx, args, torch, hdg)
    if not args.no_serving:
        out["serving"] = serving_leg(ctx, args, torch, hdg)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, q0, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
