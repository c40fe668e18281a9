#!/usr/bin/env python3
"""Throughput of the batched Mooney-Rivlin tetrahedral force path on one GPU.

Workload: 4,096 cells of uneven size (ellipsoids with semi-axes
U[0.7, 1.3] R, 500-20,000 tetrahedra each, ~42 M tetrahedra in total), each
with its own compression + shear, node noise and (mu, kappa, w); synthetic,
seeded (synth.configs.uneven_batch).

One step = one hot-path pass over the whole batch for the loss
L = sum_i v_i . f_i + sum_c ebar_c E_c (seeded v, ebar): forces and energies,
the Hessian-vector product ybar and the parameter gradient, computed by the
fused forward + backward tile pass (cm_forces_and_backward, whose outputs are
bitwise those of the separate passes; the step checks that) and replayed as
one captured HIP graph.  The reported value is tetrahedra per second of that
step.  Also reported: the same step as separate forward and backward passes
(the route of a loss whose cotangents depend on the forces, e.g. through
autograd), forward-only throughput, the passes as one launch per cell
(single-cell baseline), per-kernel device times from HIP events, a roofline
entry for the dominant kernel, parity against the FP64 oracle (64 sampled
cells, and every cell through the oracle's OpenMP build), and the oracle
timed on the host (CPU baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("tets/sec (fwd; fwd+bwd) and % of HBM roofline, batched vs "
          "single-cell, at 1e-5 rel err")
HBM_PEAK_GBS = 8000.0
# Vector FMA issue rate with packed FP32 disabled: 256 CUs x 4 SIMDs x 16
# lanes x 2 flops x 2.4 GHz (FP32 and FP64 alike).
ALU_PEAK_TFLOPS = 78.6
# Algorithmic flops per tetrahedron, counted on the method's operations:
# forward ~350 (deformation gradient, invariants, closed-form stress, P B^T),
# backward ~900 (the same plus the stress derivative along the direction and
# the parameter terms, ~2.5x the forward).
FWD_FLOPS, BWD_FLOPS = 350, 900
# The fused pass shares the deformation gradient, invariants and cofactor
# matrix: the backward's operations plus the forward-only ones (stress
# assembly ~78, P B^T 54, energy and float64 coefficients ~28).
FUSED_FLOPS = BWD_FLOPS + 160
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# Algorithmic bytes per tetrahedron and per node (int32 indices, float32
# inverse edge matrix and volume, float32 SoA node arrays), per pass.
FWD_BYTES = (56, 24)    # 16 idx + 36 B + 4 V0 per tet; y in + f out per node
BWD_BYTES = (56, 36)    # same tet stream; y, fbar in + ybar out per node
FUSED_BYTES = (56, 48)  # one tet stream; y, fbar in + f, ybar out per node
# Bytes per tetrahedron of the stored chunk format (uint16 tile-local
# indices: 8 + 36 + 4), the other denominator reported beside the canonical.
STORED_TET_BYTES = 48
F_TOL, E_TOL, G_TOL = 1e-5, 1e-6, 1e-5
TILE_KERNEL_SOURCES = ("kernels.hip", "backward.hip", "fused.hip",
                       "device_util.h", "finalize.h", "kernels.h", "layout.h",
                       "mr_tet.h", "prep.cpp", "util.hip")


def kernel_source_hash():
    """sha256 of the sources of the forward and backward kernels (their .hip
    files and the headers they include) and of the host code that lays out
    their data (prep.cpp: tiles, slots, chunks), and of the reference copy
    kernel the counters are scaled by (util.hip); a stored counter record
    applies only to the kernels and layout it was measured on.  The other
    host code and the auxiliary kernels (plates, quasi-static, shape) are
    not part of it."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2003_03130_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn in TILE_KERNEL_SOURCES:
            with open(os.path.join(csrc, fn), "rb") as fh:
                h.update(fn.encode() + fh.read())
    return h.hexdigest()


def measured_traffic(kernel, info):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    records (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration;
    one record per layout of the workload that was profiled: tiles, slots,
    chunks), or None if absent, taken on other kernel sources or on no
    record of this layout."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    for r in rec.get("records", []):
        lay = r.get("layout", {})
        if lay and all(info.get(k) == v for k, v in lay.items()):
            k = r.get("kernels", {}).get(kernel)
            return None if k is None else k.get("bytes")
    return None


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr,
          flush=True)


def time_graph(cb, stream, steps, warmup, ramp_s=0.0):
    """ms per replay of the captured graph over `steps` timed replays, after
    `warmup` untimed ones (and, if ramp_s > 0, untimed replays for about
    ramp_s seconds first, so that clocks reach their loaded state)."""
    import torch
    t_end = time.time() + ramp_s
    while time.time() < t_end:
        for _ in range(10):
            cb.graph_launch(stream=stream)
        torch.cuda.synchronize()
    for _ in range(warmup):
        cb.graph_launch(stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        cb.graph_launch(stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def replay_stats(cb, stream, reps):
    """Median, min and max ms of `reps` replays of the captured graph, each
    bracketed by its own pair of events (after the timed run, clocks loaded)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(stream)
        cb.graph_launch(stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return {"median": float(np.median(t)), "min": float(t.min()),
            "max": float(t.max()), "replays": reps}


def kernel_times(cb, stream, y, f, E, fbar, ebar, ybar, tb, reps=20):
    """Average device time of each kernel (cm_profile_kernels: HIP events on
    the launch stream around `reps` back-to-back launches), taken after
    about 0.3 s of replays of the captured step so that clocks are in their
    loaded state."""
    import torch
    t_end = time.time() + 0.3
    while time.time() < t_end:
        for _ in range(10):
            cb.graph_launch(stream=stream)
        torch.cuda.synchronize()
    return cb.profile_kernels(y, f, E, fbar, ebar, ybar, tb, reps=reps,
                              stream=stream)


def parity(cb, b, f, E, ybar, tb, vbar, ebar, cells):
    """Max errors of sampled cells against the oracle (forward + backward)."""
    import oracle
    if not cells:
        return {"cells_checked": 0, "ok": None}
    fh, yh = cb.to_host(f), cb.to_host(ybar)
    Eh, th = E.cpu().numpy(), tb.cpu().numpy().reshape(-1, 3)
    worst = {"force": 0.0, "energy": 0.0, "ybar": 0.0, "thetabar": 0.0}
    for c in cells:
        cell = b.cell(c)
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        m = oracle.OracleMesh(cell.x, cell.tets)
        y64 = cell.y.astype(np.float64)
        fo, Eo, _ = m.forces(y64, cell.theta)
        yo, to = m.backward(y64, cell.theta, vbar[n0:n1].astype(np.float64),
                            float(ebar[c]))
        worst["force"] = max(worst["force"], float(
            np.abs(fh[n0:n1] - fo).max() / np.abs(fo).max()))
        worst["energy"] = max(worst["energy"], abs(Eh[c] - Eo) / abs(Eo))
        worst["ybar"] = max(worst["ybar"], float(
            np.abs(yh[n0:n1] - yo).max() / np.abs(yo).max()))
        worst["thetabar"] = max(worst["thetabar"], float(
            np.abs(th[c] - to).max() / np.abs(to).max()))
    worst["ok"] = bool(worst["force"] <= F_TOL and worst["energy"] <= E_TOL
                       and worst["ybar"] <= G_TOL and worst["thetabar"] <= G_TOL)
    worst["cells_checked"] = len(cells)
    return worst


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build_oracle_omp():
    """The oracle's timing-mode build (-O3 -march=native -fopenmp) in a
    temporary file."""
    import tempfile

    import oracle
    so = os.path.join(tempfile.gettempdir(), f"cm_oracle_omp_{os.getpid()}.so")
    oracle.build_timing(so)
    return so


def parity_all_cells(b, dev, vbar, ebar, so, threads=None):
    """Every cell of the workload against the FP64 oracle (its OpenMP build):
    max-normalised force, ybar and thetabar errors and relative energy
    errors, worst over the cells.  dev = host (f, E, ybar, thetabar (n, 3)) of
    the benchmarked step.  thetabar's bar per cell is 1e-5 or twice the
    cell's sensitivity to float32 storage of B and V0 (the oracle run again
    on rounded B and V0)."""
    import oracle
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(
            16, os.cpu_count() or 1)
    t = time.time()
    ob = oracle.OracleBatch(b.node_off, b.tet_off, b.x, b.tets, lib_path=so)
    ob.threads(threads)
    y64, v64 = b.y.astype(np.float64), vbar.astype(np.float64)
    fo, Eo, yo, to = ob.fwd_bwd(y64, b.theta, v64, ebar)
    ob.B[:] = ob.B.astype(np.float32).astype(np.float64)
    ob.V0[:] = ob.V0.astype(np.float32).astype(np.float64)
    to32 = ob.fwd_bwd(y64, b.theta, v64, ebar)[3]
    fh, Eh, yh, th = dev
    start = b.node_off[:-1]

    def per_cell(g, o):
        num = np.maximum.reduceat(np.abs(g.astype(np.float64) - o).max(axis=1), start)
        return num / np.maximum.reduceat(np.abs(o).max(axis=1), start)

    ef, ey = per_cell(fh, fo), per_cell(yh, yo)
    eE = np.abs(Eh - Eo) / np.abs(Eo)
    sc = np.abs(to).max(axis=1)
    et = np.abs(th - to).max(axis=1) / sc
    sens = np.abs(to32 - to).max(axis=1) / sc
    over = np.flatnonzero(et > G_TOL)
    return {"cells": int(b.n_cells), "force": float(ef.max()),
            "energy": float(eE.max()), "ybar": float(ey.max()),
            "thetabar": float(et.max()),
            "thetabar_above_1e-5": [{"cell": int(c), "err": float(et[c]),
                                     "float32_input_sensitivity": float(sens[c])}
                                    for c in over],
            "ok": bool(ef.max() <= F_TOL and eE.max() <= E_TOL
                       and ey.max() <= G_TOL
                       and np.all(et <= np.maximum(G_TOL, 2.0 * sens))),
            "s": round(time.time() - t, 1)}


def cpu_baseline(b, vbar, ebar, seconds, so, threads=None, reps=5):
    """The FP64 oracle (forward by the derivative-table path + backward by
    dual-number JVPs, unchanged) in its timing mode: built with -O3
    -march=native -fopenmp for this host, OpenMP over the cells of the
    workload (OMP_PROC_BIND=close), preparation (B, V0) outside the timed
    calls.  A one-thread calibration sizes the samples; the reported value
    is the median of `reps` runs on `threads` threads (OMP_NUM_THREADS, else
    the GPU's host share of 16 cores) over a prefix of the workload's cells
    of about seconds / (reps + 3) each, beside the median of 3 one-thread
    runs on a shorter prefix."""
    import oracle
    os.environ.setdefault("OMP_PROC_BIND", "close")
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(
            16, os.cpu_count() or 1)
    tets = np.diff(b.tet_off)

    def prefix(n_tets):
        return int(min(b.n_cells, max(1, np.searchsorted(np.cumsum(tets), n_tets) + 1)))

    # the sample cells (a prefix) with their FP64 reference data
    per_run = seconds / (reps + 3)
    cal = prefix(2e5)
    ob = oracle.OracleBatch(b.node_off[:cal + 1], b.tet_off[:cal + 1],
                            b.x[:b.node_off[cal]], b.tets[:b.tet_off[cal]],
                            lib_path=so)
    th = b.theta[:cal]
    ob.threads(1)
    t0 = time.perf_counter()
    ob.fwd_bwd(b.y[:b.node_off[cal]], th, vbar[:b.node_off[cal]], ebar[:cal])
    rate1 = b.tet_off[cal] / (time.perf_counter() - t0)
    n1 = prefix(rate1 * per_run)
    nm = prefix(rate1 * per_run * threads * 0.8)
    c_max = max(n1, nm)
    ob = oracle.OracleBatch(b.node_off[:c_max + 1], b.tet_off[:c_max + 1],
                            b.x[:b.node_off[c_max]], b.tets[:b.tet_off[c_max]],
                            lib_path=so)
    y = b.y[:b.node_off[c_max]]
    v = vbar[:b.node_off[c_max]]

    def timed(nthreads, c1, n_reps):
        used = ob.threads(nthreads)
        ts = []
        for _ in range(n_reps):
            t0 = time.perf_counter()
            ob.fwd_bwd(y, b.theta[:c_max], v, ebar[:c_max], 0, c1)
            ts.append(time.perf_counter() - t0)
        return used, float(np.median(ts)), ts

    _, t1, _ = timed(1, n1, 3)
    used, tm, all_t = timed(threads, nm, reps)
    return {"value": float(b.tet_off[nm] / tm), "unit": "tets/s",
            "cores": int(used), "kind": "oracle",
            "single_thread_value": float(b.tet_off[n1] / t1),
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"FP64 oracle forward (derivative-table path) + backward "
                      f"(dual-number JVPs), g++ -O3 -march=native -fopenmp, "
                      f"OpenMP over cells (OMP_PROC_BIND=close): median of "
                      f"{reps} runs on {used} threads over cells 0..{nm - 1} "
                      f"({int(b.tet_off[nm])} tets, {tm:.2f} s each, runs "
                      f"{', '.join(f'{t:.2f}' for t in all_t)} s); one thread: "
                      f"median of 3 runs over cells 0..{n1 - 1} "
                      f"({int(b.tet_off[n1])} tets, {t1:.2f} s)"}


def run_relax(args):
    """Plate compression of 256 cells x ~51k tets over 200 steps: forward
    sweep and checkpointed reverse-mode gradient (dL/d(mu, kappa, w))."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.relax import PlateCompression
    from synth.configs import (DRAG, K_PLATE, STOKES_DT, compression_batch,
                               plate_schedule)
    t = time.time()
    b = compression_batch(args.relax_cells, 9000, 5000, n_meshes=8)
    log(f"relax workload: {b.n_cells} cells, {b.n_tets} tets "
        f"({time.time() - t:.1f} s)")
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets,
                   tile_tets=args.tile_tets)
    top, bot = plate_schedule(args.relax_steps, compression=0.2)
    pc = PlateCompression(cb, top, bot, K_PLATE, STOKES_DT / DRAG,
                          checkpoint=20)
    pc.set_theta(b.info["theta0"])
    # calibration targets: the oracle's FP64 replay of the same scheme at the
    # hidden theta* (written by tests/golden/make_relax_targets.py for the
    # 256-cell, 200-step workload; cells are generated in the same order for
    # any prefix of that batch)
    tgt = np.load(os.path.join(ROOT, "tests", "golden", "relax_targets.npy"))
    if args.relax_steps != tgt.shape[0] or b.n_cells > tgt.shape[1]:
        raise SystemExit(f"relax targets cover {tgt.shape[1]} cells x "
                         f"{tgt.shape[0]} steps; run with --relax-steps "
                         f"{tgt.shape[0]} and at most {tgt.shape[1]} cells")
    Ft = torch.from_numpy(np.ascontiguousarray(tgt[:, :b.n_cells])).to(cb.device)
    y0 = cb.to_device(b.y)
    scale = 1.0 / (args.relax_steps * b.n_cells)
    pc.forward(y0)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    F, yN, _ = pc.forward(y0)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    pc.gradient(y0, Ft, scale)  # warm-up (allocations)
    torch.cuda.synchronize()
    t = time.perf_counter()
    loss, g, _ = pc.gradient(y0, Ft, scale)
    torch.cuda.synchronize()
    t_bptt = time.perf_counter() - t
    # the same gradient with every state kept (no recomputation; the states
    # of this workload take a few GB of the 288 GB of HBM)
    pc_all = PlateCompression(cb, top, bot, K_PLATE, STOKES_DT / DRAG,
                              checkpoint=args.relax_steps)
    pc_all.gradient(y0, Ft, scale)  # warm-up (allocations)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, g_all, _ = pc_all.gradient(y0, Ft, scale)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t
    # the two-call route (forces, then the plate step as a pass of its own)
    pc_two = PlateCompression(cb, top, bot, K_PLATE, STOKES_DT / DRAG,
                              checkpoint=20, fused=False)
    pc_two.set_theta(b.info["theta0"])
    pc_two.gradient(y0, Ft, scale)  # warm-up (allocations)
    torch.cuda.synchronize()
    t = time.perf_counter()
    F_two, _, _ = pc_two.forward(y0)
    torch.cuda.synchronize()
    t_fwd_two = time.perf_counter() - t
    t = time.perf_counter()
    _, g_two, _ = pc_two.gradient(y0, Ft, scale)
    torch.cuda.synchronize()
    t_bptt_two = time.perf_counter() - t
    # the loss at the hidden parameters (targets reproduced by the device)
    pc.set_theta(b.info["theta_star"])
    F_star, _, _ = pc.forward(y0)
    loss_star = float(scale * ((F_star - Ft) ** 2).sum())
    target_err = float((F_star - Ft).abs().max() / Ft.abs().max())
    pc.set_theta(b.info["theta0"])
    M, N, S = b.n_tets, b.n_nodes, args.relax_steps
    # a fused step moves the tet stream, reads y and writes y_next
    step_bytes = FWD_BYTES[0] * M + FWD_BYTES[1] * N
    out = {
        "workload": f"{b.n_cells} spheres, {M} tets, {N} nodes, {S} steps, "
                    f"plates to 20% compression, checkpoint every 20",
        "fwd_s": t_fwd, "bptt_s": t_bptt,
        "fwd_tet_steps_per_s": M * S / t_fwd,
        "bptt_tet_steps_per_s": M * S / t_bptt,
        "bptt_all_states_s": t_all,
        "bptt_all_states_GB": S * 12 * N / 1e9,
        "bptt_all_states_same_gradient": bool(torch.equal(g_all, g)),
        "two_call_fwd_s": t_fwd_two, "two_call_bptt_s": t_bptt_two,
        "two_call_max_rel_diff": {
            "plate_force": float(((F_two - F).abs().max() / F.abs().max())),
            "gradient": float(((g_two - g).abs().max() / g.abs().max()))},
        "fwd_step_hbm_frac": step_bytes * S / t_fwd / (HBM_PEAK_GBS * 1e9),
        "loss": loss, "loss_at_theta_star": loss_star,
        "targets_vs_device_at_theta_star": target_err,
        "grad_finite": bool(torch.isfinite(g).all()),
        "max_plate_force": float(F.max()),
        "targets": "oracle FP64 replay of the same 200 steps at the hidden "
                   "(mu, kappa, w) of every cell (tests/golden/relax_targets.npy)",
        "compression": "20 % (explicit steps invert tetrahedra at 40-80 % "
                       "within 200 steps; 80 % is served by the quasi-static "
                       "and calibration legs)",
    }
    log(f"relax: {out}")
    return out


def run_template(args):
    """Shared-mesh batch: args.template_cells copies of one ~10k-tet sphere,
    each with its own deformation and parameters (cm_template_create).  The
    tet stream is stored once, so a step moves the per-node arrays and one
    copy of the tet data."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from synth.configs import cotangent, template_batch
    t = time.time()
    b = template_batch(args.template_cells, args.template_nodes, args.seed + 7)
    n1, m1 = b.info["template_nodes"], b.info["template_tets"]
    log(f"template workload: {b.n_cells} x ({n1} nodes, {m1} tets) "
        f"({time.time() - t:.1f} s)")
    cb = CellBatch.template(b.n_cells, b.x[:n1], b.tets[:m1],
                            tile_tets=args.tile_tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    dev = cb.device
    y = cb.to_device(b.y)
    vbar = cotangent(b.n_nodes, args.seed + 8)
    fbar = cb.to_device(vbar)
    ebar_h = np.full(b.n_cells, 0.5)
    ebar = torch.tensor(ebar_h, dtype=torch.float64, device=dev)
    f, ybar = cb.empty_nodes(), cb.empty_nodes()
    E = torch.empty(b.n_cells, dtype=torch.float64, device=dev)
    tb = torch.empty(3 * b.n_cells, dtype=torch.float64, device=dev)
    if args.launch:
        cb.set_launch(*(int(v) for v in args.launch.split(",")))
    elif not args.no_autotune:
        cb.autotune(y)
    cb.forces(y, f, E)
    cb.backward(y, fbar, ebar, ybar, tb)
    torch.cuda.synchronize()
    sample = [0, b.n_cells // 2, b.n_cells - 1] if args.parity_cells else []
    par = parity(cb, b, f, E, ybar, tb, vbar, ebar_h, sample)
    s = torch.cuda.Stream()
    res = {}
    for name, mode in (("fwd", 0), ("fwd_bwd", 1), ("fwd_bwd_fused", 6)):
        with torch.cuda.stream(s):
            cb.graph_capture(mode, y, f, E, None, fbar, ebar, ybar, tb,
                             stream=s)
        res[name] = time_graph(cb, s, args.steps, args.warmup, ramp_s=0.5)
    ms = kernel_times(cb, s, y, f, E, fbar, ebar, ybar, tb)
    M, N = b.n_tets, b.n_nodes
    fwd_b = FWD_BYTES[0] * m1 + FWD_BYTES[1] * N
    bwd_b = BWD_BYTES[0] * m1 + BWD_BYTES[1] * N
    out = {
        "workload": f"{b.n_cells} copies of one sphere mesh ({n1} nodes, "
                    f"{m1} tets), {M} tets, {N} nodes, per-cell deformation "
                    f"and parameters",
        "launch": list(cb.get_launch()),
        "fwd_bwd_tets_per_s": M / (res["fwd_bwd"] * 1e-3),
        "fwd_bwd_fused_tets_per_s": M / (res["fwd_bwd_fused"] * 1e-3),
        "fwd_tets_per_s": M / (res["fwd"] * 1e-3),
        "ms": {k: round(v, 5) for k, v in res.items()},
        "kernel_ms": [round(v, 5) for v in ms],
        "hbm_frac_fwd_bwd": (fwd_b + bwd_b) / (res["fwd_bwd"] * 1e-3)
        / (HBM_PEAK_GBS * 1e9),
        "alu_frac_fwd_bwd": (FWD_FLOPS + BWD_FLOPS) * M
        / (res["fwd_bwd"] * 1e-3) / (ALU_PEAK_TFLOPS * 1e12),
        "parity": par,
    }
    log(f"template: {out}")
    return out


def run_shape(args, cb, b, y):
    """Shape diagnostics (Taylor deformation D, semi-axes, cell strain) of
    every cell of the main workload: ms per cm_shape call (moments over all
    tetrahedra, the largest node distance of every cell, per-cell eigen-solve)."""
    import torch
    from oracle import shape as oshape
    d_ref = torch.full((b.n_cells,), 2.0, dtype=torch.float64, device=cb.device)
    out = cb.shape(y, d_ref)
    torch.cuda.synchronize()
    worst = {"volume": 0.0, "axes": 0.0, "D": 0.0, "d_max": 0.0}
    oh = out.cpu().numpy()
    for c in (0, b.n_cells // 2, b.n_cells - 1) if args.parity_cells else ():
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        t0, t1 = b.tet_off[c], b.tet_off[c + 1]
        ref = oshape.cell_shape(b.x[n0:n1], b.y[n0:n1].astype(np.float64),
                                b.tets[t0:t1], 2.0)
        worst["volume"] = max(worst["volume"],
                              abs(oh[c, 0] - ref["volume"]) / ref["volume"])
        worst["axes"] = max(worst["axes"], float(
            np.abs(oh[c, 4:7] - ref["axes"]).max() / ref["axes"].max()))
        worst["D"] = max(worst["D"], abs(oh[c, 7] - ref["D"]))
        worst["d_max"] = max(worst["d_max"],
                             abs(oh[c, 8] - ref["d_max"]) / ref["d_max"])
    worst["ok"] = bool(worst["volume"] <= 1e-12 and worst["axes"] <= 1e-10
                       and worst["D"] <= 1e-10 and worst["d_max"] <= 1e-12)
    for _ in range(3):
        cb.shape(y, d_ref, out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(5, args.steps // 5)
    e0.record()
    for _ in range(reps):
        cb.shape(y, d_ref, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res = {"workload": "main workload, every cell", "ms": ms,
           "tets_per_s": b.n_tets / (ms * 1e-3),
           "mean_D": float(oh[:, 7].mean()), "parity": worst}
    log(f"shape: {res}")
    return res


def run_quasistatic(args):
    """Quasi-static force-indentation curves: oblate cells (~2k nodes,
    ~11k tets each) between plates closing from first contact to 80 % of
    each cell's height in args.qs_steps positions, every position brought to
    equilibrium by Newton-CG on the device (inexact Newton, Hessian-vector
    products only for the cells still in CG, line search that never inverts
    a tetrahedron); reports wall time, Newton/CG counts, time per CG
    iteration, the mean curve, the deepest compression of the cells' own
    height, the plate balance, and the mean curves of the same cells with w
    set to 0.25, 0.5 and 1 (the paper's fitted values); then the same cells
    indented by a sphere (the colloidal-probe setup) to 40 % of their height,
    with its curve, balance, held centroids and small-depth exponent."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    from synth.configs import K_PLATE, oblate_batch
    t = time.time()
    b = oblate_batch(args.qs_cells, 2000, 7000)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, tile_tets=args.qs_tile_tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    top0 = np.array([b.x[b.node_off[c]:b.node_off[c + 1], 2].max()
                     for c in range(b.n_cells)])
    bot = np.array([b.x[b.node_off[c]:b.node_off[c + 1], 2].min()
                    for c in range(b.n_cells)])
    H = top0 - bot
    frac = np.linspace(0.04, 0.8, args.qs_steps)
    tops = top0[None, :] - frac[:, None] * H[None, :]
    log(f"quasi-static workload: {b.n_cells} cells, {b.n_tets} tets "
        f"({time.time() - t:.1f} s)")
    qs = QuasiStaticCompression(cb, K_PLATE)
    y0 = cb.to_device(b.y)
    torch.cuda.synchronize()
    t = time.perf_counter()
    Ft, Fb, ok, y = qs.curve(y0, tops, bot)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    hvp = qs.stats["cg"]
    ninv = torch.zeros(b.n_cells, dtype=torch.int32, device=cb.device)
    cb.forces(y, n_inverted=ninv)
    yh = cb.to_host(y)
    comp = np.array([1.0 - np.ptp(yh[b.node_off[c]:b.node_off[c + 1], 2]) / H[c]
                     for c in range(b.n_cells)])
    # the same cells with w = 0.25, 0.5, 1 (mu, kappa kept)
    w_curves = {}
    for w in (0.25, 0.5, 1.0):
        cb.set_params(b.theta[:, 0], b.theta[:, 1], np.full(b.n_cells, w))
        qw = QuasiStaticCompression(cb, K_PLATE)
        Fw, _, okw, _ = qw.curve(y0, tops, bot)
        w_curves[str(w)] = {"mean_force": [round(float(v), 6) for v in Fw.mean(axis=1)],
                            "converged": bool(okw.all())}
    # the colloidal-probe setup: a sphere of 0.66 times the cell radius (the
    # paper's probe-to-particle ratio) on each cell's axis, the cell on the
    # bottom plate with its centroid held laterally; Poisson ratio 0.48 (kappa
    # = 24.7 mu) and w = 1, the paper's choices for that comparison
    sphere_fr = np.linspace(0.02, 0.4, 10)
    kappa_s = b.theta[:, 0] * 2.0 * 1.48 / (3.0 * (1.0 - 2.0 * 0.48))
    cb.set_params(b.theta[:, 0], kappa_s, np.ones(b.n_cells))
    tops_s = top0[None, :] - sphere_fr[:, None] * H[None, :]
    qsph = QuasiStaticCompression(cb, K_PLATE, sphere_radius=0.66)
    torch.cuda.synchronize()
    t = time.perf_counter()
    Fs, Fsb, oks, ys = qsph.curve(y0, tops_s, bot)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t
    cb.forces(ys, n_inverted=ninv)
    start_c = qsph.cell_centroids(y0).cpu().numpy()
    sphere = {
        "setup": "sphere radius 0.66 on each cell's axis (centroid held laterally), "
                 "nu = 0.48 (kappa = 24.7 mu), w = 1",
        "indentation_fraction_of_height": [round(float(v), 4) for v in sphere_fr],
        "wall_s": wall_s, "newton": qsph.stats["newton"], "cg": qsph.stats["cg"],
        "ms_per_cg_iteration": 1e3 * wall_s / max(qsph.stats["cg"], 1),
        "converged_steps": int(oks.sum()), "steps": len(oks),
        "mean_force": [round(float(v), 6) for v in Fs.mean(axis=1)],
        "balance_max_by_step": [float(v) for v in
                                (np.abs(Fs - Fsb) / np.maximum(Fs, 1e-30)).max(axis=1)],
        "centroid_drift_max": float(np.abs(qsph.cell_centroids(ys).cpu().numpy()
                                           - start_c).max()),
        "inverted_tets_final": int(ninv.sum().item()),
        "loglog_slope_first_half": float(np.median(
            np.log(Fs[4] / Fs[1]) / np.log(sphere_fr[4] / sphere_fr[1]))),
    }
    out = {
        "workload": f"{b.n_cells} oblate cells, {b.n_tets} tets, plates "
                    f"closing from first contact to 80 % of each cell's height "
                    f"in {args.qs_steps} positions, {args.qs_tile_tets}-tet tiles",
        "wall_s": wall, "newton": qs.stats["newton"], "cg": hvp,
        "converged_steps": int(ok.sum()), "steps": len(ok),
        "unconverged_cells_last": int((qs.state[:, 11] > 0).sum().item()),
        "ms_per_cg_iteration": 1e3 * wall / max(hvp, 1),
        "eta_max": qs.eta_max,
        "plate_travel": [round(float(v), 4) for v in frac],
        "mean_force": [round(float(v), 6) for v in Ft.mean(axis=1)],
        "deepest_plate_travel": float(frac[-1]),
        "height_compression_mean": float(comp.mean()),
        "height_compression_min": float(comp.min()),
        "inverted_tets_final": int(ninv.sum().item()),
        "plate_balance_max_by_step": [float(v) for v in
                                      (np.abs(Ft - Fb) / np.maximum(Ft, 1e-30)).max(axis=1)],
        "upturn_loglog_slope_40_80": float(np.median(
            np.log(Ft[-1] / Ft[np.argmin(np.abs(frac - 0.4))]) / np.log(0.8 / 0.4))),
        "w_curves": w_curves,
        "sphere_indenter": sphere,
    }
    log(f"quasi-static: {out}")
    cb.close()
    return out


def run_latency(args):
    """Single-cell latency: the 1k-node sphere (~5.3k tets) and the
    paper-size 20k-node sphere (~115k tets) of the parity configurations, one
    cell per handle, tile size and launch tuned for the cell.  Per call
    (HIP events on the launch stream around each call, mean of the calls):
    forward, forward + backward as two calls, and as one fused call
    (cm_forces_and_backward), warm (back-to-back) and, for the 20k
    sphere, cold (a 1 GiB buffer written between calls, so that neither L2
    nor the MALL holds the cell's data)."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from synth.configs import cotangent, paper_sphere_case, small_sphere_case
    dev = torch.device("cuda", torch.cuda.current_device())
    flush = torch.empty(2 ** 28, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    out = {}
    for name, case in (("sphere_1k", small_sphere_case(1000)),
                       ("sphere_20k", paper_sphere_case(2000))):
        cb = CellBatch.tuned([0, len(case.x)], [0, len(case.tets)], case.x, case.tets,
                             tile_candidates=[128, 256, 384, 512, 768])
        cb.set_params(*case.theta)
        y = cb.to_device(case.y)
        fbar = cb.to_device(cotangent(case.n_nodes, 7))
        ebar = torch.full((1,), 0.5, dtype=torch.float64, device=dev)
        f, ybar = cb.empty_nodes(), cb.empty_nodes()
        E = torch.empty(1, dtype=torch.float64, device=dev)
        tb = torch.empty(3, dtype=torch.float64, device=dev)

        def fwd():
            cb.forces(y, f, E, stream=s)

        def fwd_bwd():
            cb.forces(y, f, E, stream=s)
            cb.backward(y, fbar, ebar, ybar, tb, stream=s)

        def fwd_bwd_fused():
            cb.forces_and_backward(y, fbar, ebar, f=f, energy=E, ybar=ybar,
                                   thetabar=tb, stream=s)

        def per_call(fn, reps, cold):
            ev = [(torch.cuda.Event(enable_timing=True),
                   torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            with torch.cuda.stream(s):
                for _ in range(20):
                    fn()
                for e0, e1 in ev:
                    if cold:
                        flush.fill_(0.0)
                    e0.record(s)
                    fn()
                    e1.record(s)
            torch.cuda.synchronize()
            return 1e3 * float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))

        rec = {"tets": cb.n_tets, "nodes": cb.n_nodes,
               "tile_tets": int(cb.info["tile_tets"]), "launch": list(cb.get_launch()),
               "fwd_us_warm": per_call(fwd, 200, False),
               "fwd_bwd_us_warm": per_call(fwd_bwd, 200, False),
               "fwd_bwd_fused_us_warm": per_call(fwd_bwd_fused, 200, False)}
        if name == "sphere_20k":
            rec["fwd_us_cold"] = per_call(fwd, 20, True)
            rec["fwd_bwd_us_cold"] = per_call(fwd_bwd, 20, True)
            rec["fwd_bwd_fused_us_cold"] = per_call(fwd_bwd_fused, 20, True)
        out[name] = rec
        cb.close()
    del flush
    log(f"latency: {out}")
    return out


def run_calibration(args):
    """Calibration at 80 % compression by the quasi-static route: oblate
    cells (~2k nodes) with hidden (mu, kappa, w); their force-indentation
    curves (10 plate positions, 8 % to 80 % of the height) come from the FP64
    oracle (tests/golden/qs_targets.npy, written by make_qs_targets.py).  From
    a start drawn like the hidden values, Levenberg-Marquardt per cell with
    dF/d(mu, kappa, w) from the adjoint of every equilibrium (one more CG
    solve on the device per position).  Reports the loss and the parameter
    errors per iteration and the time per iteration."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.calibrate import fit_curves
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    from synth.configs import K_PLATE, calibration_batch, qs_fractions
    tgt = np.load(os.path.join(ROOT, "tests", "golden", "qs_targets.npy"))
    n = tgt.shape[1]
    t = time.time()
    b = calibration_batch(n, 2000, 7100)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, tile_tets=args.qs_tile_tets)
    theta0, theta_star = b.info["theta0"], b.info["theta_star"]
    cb.set_params(theta0[:, 0], theta0[:, 1], theta0[:, 2])
    top0 = np.array([b.x[b.node_off[c]:b.node_off[c + 1], 2].max() for c in range(n)])
    bot = np.array([b.x[b.node_off[c]:b.node_off[c + 1], 2].min() for c in range(n)])
    tops = top0[None, :] - qs_fractions()[:, None] * (top0 - bot)[None, :]
    log(f"calibration workload: {n} cells, {b.n_tets} tets ({time.time() - t:.1f} s)")
    qs = QuasiStaticCompression(cb, K_PLATE)
    y0 = cb.to_device(b.y)
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = fit_curves(qs, y0, tops, bot, tgt, theta0, iters=args.calib_iters,
                     log=log)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    hist = res["history"]

    def errs(th):
        rel = np.abs(th - theta_star)
        rel[:, :2] /= theta_star[:, :2]
        return {"mu_rel_max": float(rel[:, 0].max()), "kappa_rel_max": float(rel[:, 1].max()),
                "w_abs_max": float(rel[:, 2].max()),
                "mu_rel_median": float(np.median(rel[:, 0])),
                "kappa_rel_median": float(np.median(rel[:, 1])),
                "w_abs_median": float(np.median(rel[:, 2]))}

    out = {
        "workload": f"{n} oblate cells, {b.n_tets} tets, 10 plate positions to 80 % of "
                    f"the height, hidden (mu, kappa, w) per cell",
        "targets": "FP64 oracle equilibria at the hidden parameters "
                   "(tests/golden/qs_targets.npy)",
        "iterations": args.calib_iters, "wall_s": wall,
        "s_per_iteration": wall / max(args.calib_iters, 1),
        "loss_by_iteration": [float(h["loss"].sum()) for h in hist],
        "errors_start": errs(hist[0]["theta"]), "errors_end": errs(res["theta"]),
        "newton": qs.stats["newton"], "cg": qs.stats["cg"],
        "adjoint_cg": qs.stats.get("adjoint_cg", 0),
        "accepted_by_iteration": [int(h["accepted"].sum()) for h in hist[1:]],
        "unconverged_trials": int(sum((~h["converged"]).sum() for h in hist)),
    }
    log(f"calibration: {out}")
    cb.close()
    return out


def run_regions(args, b):
    """The main workload with three material regions per cell (nucleus,
    cytoplasm, cortex shell by reference radius), each (cell, region) with
    its own parameters: one step = forward + backward, as the main value."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from synth.configs import cotangent, radial_regions, random_theta
    R = 3
    t = time.time()
    reg = np.concatenate([
        radial_regions(b.x[b.node_off[c]:b.node_off[c + 1]],
                       b.tets[b.tet_off[c]:b.tet_off[c + 1]])
        for c in range(b.n_cells)])
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets,
                   tile_tets=args.tile_tets, regions=reg, n_regions=R)
    rng = np.random.default_rng(args.seed + 9)
    th = np.array([random_theta(rng) for _ in range(cb.n_mat)])
    cb.set_params(th[:, 0], th[:, 1], th[:, 2])
    log(f"regions workload prepared in {time.time() - t:.1f} s: "
        f"{cb.info['n_tiles']} tiles")
    dev = cb.device
    y = cb.to_device(b.y)
    vbar = cotangent(b.n_nodes, args.seed + 1)
    fbar = cb.to_device(vbar)
    ebar_h = np.full(b.n_cells, 0.5)
    ebar = torch.tensor(ebar_h, dtype=torch.float64, device=dev)
    f, ybar = cb.empty_nodes(), cb.empty_nodes()
    E = torch.empty(b.n_cells, dtype=torch.float64, device=dev)
    tb = torch.empty(3 * cb.n_mat, dtype=torch.float64, device=dev)
    if args.launch:
        cb.set_launch(*(int(v) for v in args.launch.split(",")))
    elif not args.no_autotune:
        cb.autotune(y)
    cb.forces(y, f, E)
    cb.backward(y, fbar, ebar, ybar, tb)
    torch.cuda.synchronize()
    # parity: three cells against the oracle's region composition
    import oracle
    fh, yh = cb.to_host(f), cb.to_host(ybar)
    th_h = tb.cpu().numpy().reshape(-1, 3)
    worst = {"force": 0.0, "ybar": 0.0, "thetabar": 0.0}
    for c in (0, b.n_cells // 2, b.n_cells - 1) if args.parity_cells else ():
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        t0, t1 = b.tet_off[c], b.tet_off[c + 1]
        rm = oracle.RegionMesh(b.x[n0:n1], b.tets[t0:t1], reg[t0:t1], R)
        y64 = b.y[n0:n1].astype(np.float64)
        fo, _, _ = rm.forces(y64, th[c * R:(c + 1) * R])
        yo, to = rm.backward(y64, th[c * R:(c + 1) * R],
                             vbar[n0:n1].astype(np.float64), ebar_h[c])
        worst["force"] = max(worst["force"], float(
            np.abs(fh[n0:n1] - fo).max() / np.abs(fo).max()))
        worst["ybar"] = max(worst["ybar"], float(
            np.abs(yh[n0:n1] - yo).max() / np.abs(yo).max()))
        worst["thetabar"] = max(worst["thetabar"], float(
            np.abs(th_h[c * R:(c + 1) * R] - to).max() / np.abs(to).max()))
    worst["ok"] = bool(max(worst["force"], worst["ybar"], worst["thetabar"])
                       <= F_TOL)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        cb.graph_capture(1, y, f, E, None, fbar, ebar, ybar, tb, stream=s)
    step = time_graph(cb, s, args.steps, args.warmup, ramp_s=0.5)
    with torch.cuda.stream(s):
        cb.graph_capture(6, y, f, E, None, fbar, ebar, ybar, tb, stream=s)
    step_fused = time_graph(cb, s, args.steps, args.warmup, ramp_s=0.5)
    out = {
        "workload": f"main workload, {R} material regions per cell "
                    f"(nucleus, cytoplasm, cortex by reference radius), "
                    f"{cb.n_mat} parameter sets",
        "n_tiles": cb.info["n_tiles"], "launch": list(cb.get_launch()),
        "ms_per_step": step, "fwd_bwd_tets_per_s": b.n_tets / (step * 1e-3),
        "ms_per_step_fused": step_fused,
        "fwd_bwd_fused_tets_per_s": b.n_tets / (step_fused * 1e-3),
        "parity": worst,
    }
    log(f"regions: {out}")
    cb.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cells", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--tile-tets", type=int, default=None,
                    help="fixed tile size (default: chosen with the launch by "
                         "cm_batch_create_tuned over 512..1024)")
    ap.add_argument("--order", type=int, default=None,
                    help="tile order (0 input, 1 RCM, 2 Morton, 3 bisection; "
                         "default: the library's)")
    ap.add_argument("--parity-cells", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity-all", action="store_true",
                    help="skip the every-cell oracle check of the main workload")
    ap.add_argument("--no-percell", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch", type=str, default=None,
                    help="fixed launch 'waves,blocks_per_cu' (skips autotune)")
    ap.add_argument("--relax-cells", type=int, default=256)
    ap.add_argument("--relax-steps", type=int, default=200)
    ap.add_argument("--no-relax", action="store_true")
    ap.add_argument("--template-cells", type=int, default=4096)
    ap.add_argument("--template-nodes", type=int, default=1930,
                    help="node target of the shared sphere mesh (~10k tets)")
    ap.add_argument("--no-template", action="store_true")
    ap.add_argument("--no-regions", action="store_true")
    ap.add_argument("--no-shape", action="store_true")
    ap.add_argument("--qs-cells", type=int, default=256)
    ap.add_argument("--qs-tile-tets", type=int, default=512,
                    help="tile size of the quasi-static leg (its masked "
                         "Hessian-vector products are bound by the latency "
                         "of single tiles once few cells are left in CG)")
    ap.add_argument("--no-qs", action="store_true")
    ap.add_argument("--qs-steps", type=int, default=20)
    ap.add_argument("--calib-iters", type=int, default=8)
    ap.add_argument("--no-calibration", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB "
                         "(reference kernel for the HBM byte counters)")
    ap.add_argument("--only", choices=["relax", "qs", "template", "shape",
                                       "regions", "calibration", "latency"],
                    default=None,
                    help="run one leg alone (for profiling it) and print its "
                         "JSON line; shape and regions build the main "
                         "workload first")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the batched cell-force path "
              "has no multi-GPU mode (cells are independent, so a batch would "
              "shard by cell, one process per GPU). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    from paper_2003_03130_amd import CellBatch
    from synth.configs import cotangent, uneven_batch

    if args.only in ("relax", "qs", "template", "calibration", "latency"):
        leg = {"relax": run_relax, "qs": run_quasistatic,
               "template": run_template, "calibration": run_calibration,
               "latency": run_latency}[args.only](args)
        print(json.dumps({"leg": args.only, **leg}), flush=True)
        return

    t = time.time()
    b = uneven_batch(n_cells=args.cells, seed=args.seed)
    log(f"workload: {b.n_cells} cells, {b.n_tets} tets, {b.n_nodes} nodes "
        f"({time.time() - t:.1f} s)")
    t = time.time()
    tuning = None
    if args.tile_tets is None and not args.launch and not args.no_autotune:
        cand = [512, 640, 768, 896, 1024]
        cb = CellBatch.tuned(b.node_off, b.tet_off, b.x, b.tets,
                             tile_candidates=cand, order=args.order)
        tuning = {"tile_candidates": cand,
                  "candidate_ms_fwd_bwd": [round(float(v), 5) for v in cb.candidate_ms],
                  "tile_tets": int(cb.info["tile_tets"]),
                  "launch": list(cb.get_launch()),
                  "persistent": bool(cb.get_launch()[1] > 0), "s": round(time.time() - t, 1)}
        log(f"tuned creation (tile size and launch) in {time.time() - t:.1f} s: "
            f"{tuning}")
    else:
        cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets,
                       tile_tets=args.tile_tets or 768, order=args.order)
    log(f"prepared + uploaded in {time.time() - t:.1f} s: {cb.info}")
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    dev = cb.device
    y = cb.to_device(b.y)
    if args.only:
        leg = run_shape(args, cb, b, y) if args.only == "shape" else run_regions(args, b)
        print(json.dumps({"leg": args.only, **leg}), flush=True)
        return
    vbar = cotangent(b.n_nodes, args.seed + 1)
    fbar = cb.to_device(vbar)
    ebar_h = np.random.default_rng(args.seed + 2).uniform(0.0, 1.0, b.n_cells)
    ebar = torch.tensor(ebar_h, dtype=torch.float64, device=dev)
    f, ybar = cb.empty_nodes(), cb.empty_nodes()
    E = torch.empty(b.n_cells, dtype=torch.float64, device=dev)
    tb = torch.empty(3 * b.n_cells, dtype=torch.float64, device=dev)
    ninv = torch.empty(b.n_cells, dtype=torch.int32, device=dev)

    # device-to-device copy bandwidth (context for the HBM roof): 1 GiB
    # read + 1 GiB written, best of 5
    src = torch.empty(2 ** 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    copy_ms = []
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_ms.append(e0.elapsed_time(e1))
    copy_gbps = 2 * src.numel() * 4 / min(copy_ms) / 1e6
    del src, dst
    log(f"device copy: {copy_gbps:.0f} GB/s")

    if args.calibrate_copy:
        # the library's plain copy kernel (stream_copy_kernel): the reference
        # of known traffic for the byte counters
        nf = args.calibrate_copy * 2 ** 20 // 4
        src = torch.ones(nf, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        from paper_2003_03130_amd import _native as nat
        from paper_2003_03130_amd.cells import _ptr, _stream
        nat.check(nat.lib().cm_stream_copy(_ptr(src), _ptr(dst), nf, _stream(None)))
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy} MiB read + written")
        del src, dst
    if args.launch:
        w_, b_ = (int(v) for v in args.launch.split(","))
        cb.set_launch(w_, b_)
    elif not args.no_autotune and tuning is None:
        t = time.time()
        launch = cb.autotune(y)
        log(f"autotuned launch (waves/block, blocks/CU) = {launch} in "
            f"{time.time() - t:.1f} s")
    launch = cb.get_launch()

    # eager pass for the parity gate
    cb.forces(y, f, E, ninv)
    cb.backward(y, fbar, ebar, ybar, tb)
    torch.cuda.synchronize()
    sample = sorted(set(np.linspace(0, b.n_cells - 1,
                                    args.parity_cells).astype(int).tolist())
                    ) if args.parity_cells > 0 else []
    t = time.time()
    par = parity(cb, b, f, E, ybar, tb, vbar, ebar_h, sample)
    log(f"parity on {len(sample)} cells ({time.time() - t:.1f} s): {par}")
    n_inverted = int(ninv.sum().item())
    dev_out = (cb.to_host(f), E.cpu().numpy(), cb.to_host(ybar),
               tb.cpu().numpy().reshape(-1, 3))

    # the fused pass must reproduce the separate passes bit for bit (the
    # oracle parity above then holds for it too)
    eager = [t.clone() for t in (f, E, ninv, ybar, tb)]
    for t in (f, ybar):
        t.fill_(float("nan"))
    cb.forces_and_backward(y, fbar, ebar, f=f, energy=E, n_inverted=ninv,
                           ybar=ybar, thetabar=tb)
    torch.cuda.synchronize()
    fused_bitwise = all(torch.equal(a, c) for a, c in
                        zip((f, E, ninv, ybar, tb), eager))
    log(f"fused pass bitwise equal to the separate passes: {fused_bitwise}")
    if not fused_bitwise:
        raise SystemExit("fused forward + backward differs from the separate "
                         "passes")

    s = torch.cuda.Stream()
    M, N = b.n_tets, b.n_nodes
    res = {}
    replays = {}
    for name, mode in (("fwd", 0), ("fwd_bwd", 1), ("fwd_bwd_fused", 6)):
        with torch.cuda.stream(s):
            cb.graph_capture(mode, y, f, E, ninv, fbar, ebar, ybar, tb,
                             stream=s)
        res[name] = time_graph(cb, s, args.steps, args.warmup, ramp_s=0.5)
        replays[name] = replay_stats(cb, s, args.steps)
        log(f"batched {name}: {res[name]:.4f} ms/step, replays "
            f"{replays[name]}")
    step_ms = res["fwd_bwd_fused"]
    # per-kernel event times right after the step timing, clocks loaded
    ms = kernel_times(cb, s, y, f, E, fbar, ebar, ybar, tb)
    log(f"kernel ms (fwd tile, fwd finalize, bwd tile, bwd finalize, "
        f"fused tile, fused finalize): {np.round(ms, 4).tolist()}")
    if not args.no_percell:
        psteps = max(2, args.steps // 4)
        for name, mode in (("percell_fwd_bwd", 3), ("percell_fwd", 2)):
            t = time.time()
            with torch.cuda.stream(s):
                cb.graph_capture(mode, y, f, E, ninv, fbar, ebar, ybar, tb,
                                 stream=s)
            res[name] = time_graph(cb, s, psteps, 1)
            log(f"single-cell launches {name}: {res[name]:.3f} ms/step "
                f"(capture {time.time() - t:.1f} s)")

    fwd_b = FWD_BYTES[0] * M + FWD_BYTES[1] * N
    bwd_b = BWD_BYTES[0] * M + BWD_BYTES[1] * N
    fused_b = FUSED_BYTES[0] * M + FUSED_BYTES[1] * N
    def views(ms_k, nbytes, flops):
        return {"ms": ms_k, "bytes": nbytes, "GBps": nbytes / ms_k / 1e6,
                "hbm_frac": nbytes / ms_k / 1e6 / HBM_PEAK_GBS,
                "flops": flops, "TFLOPs": flops / ms_k / 1e9,
                "alu_frac": flops / ms_k / 1e9 / ALU_PEAK_TFLOPS}
    kern = {
        "forward_tile": views(ms[0], fwd_b, FWD_FLOPS * M),
        "backward_tile": views(ms[2], bwd_b, BWD_FLOPS * M),
        "fused_tile": views(ms[4], fused_b, FUSED_FLOPS * M),
        "forward_finalize_ms": ms[1], "backward_finalize_ms": ms[3],
        "fused_finalize_ms": ms[5],
    }
    # the step's dominant kernel: the fused tile kernel
    dom = "fused_tile"
    kd = kern[dom]
    traffic = measured_traffic(dom, cb.info)
    if kd["alu_frac"] > kd["hbm_frac"]:
        roofline = {"bound": "alu", "kernel": dom,
                    "achieved": round(kd["TFLOPs"], 2),
                    "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(kd["alu_frac"], 4), "traffic": traffic,
                    "hbm_frac": round(kd["hbm_frac"], 4)}
    else:
        roofline = {"bound": "hbm", "kernel": dom,
                    "achieved": round(kd["GBps"], 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(kd["hbm_frac"], 4),
                    "traffic": traffic, "alu_frac": round(kd["alu_frac"], 4)}

    shape = None
    if not args.no_shape:
        shape = run_shape(args, cb, b, y)
    relax = None
    if not args.no_relax:
        relax = run_relax(args)
    template = None
    if not args.no_template:
        template = run_template(args)
    regions = None
    if not args.no_regions:
        regions = run_regions(args, b)
    quasistatic = None
    if not args.no_qs:
        quasistatic = run_quasistatic(args)
    calibration = None
    if not args.no_calibration:
        calibration = run_calibration(args)
    latency = None
    if not args.no_latency:
        latency = run_latency(args)

    cpu = par_all = None
    if not args.no_cpu_baseline or not args.no_parity_all:
        os.environ.setdefault("OMP_PROC_BIND", "close")
        so = build_oracle_omp()
        if not args.no_parity_all:
            par_all = parity_all_cells(b, dev_out, vbar, ebar_h, so)
            log(f"parity on every cell: {par_all}")
        if not args.no_cpu_baseline:
            cpu = cpu_baseline(b, vbar, ebar_h, args.cpu_seconds, so)
            log(f"cpu baseline: {cpu}")
        try:
            os.remove(so)
        except OSError:
            pass

    out = {
        "metric": METRIC,
        "value": M / (step_ms * 1e-3),
        "unit": "tets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{b.n_cells} uneven ellipsoid cells, {M} tets, "
                        f"{N} nodes; one step = batched forward + backward "
                        f"(fused pass; separate passes in ms.fwd_bwd)",
            "step": "cm_forces_and_backward: forces, energies, ybar and "
                    "thetabar of L = sum v.f + sum ebar E in one pass, "
                    "bitwise the separate passes",
            "n_cells": b.n_cells, "n_tets": M, "n_nodes": N,
            "tile_tets": cb.info["tile_tets"], "launch": list(launch),
            "layout": {k: int(cb.info[k]) for k in ("n_tiles", "n_chunks",
                                                    "n_slots", "n_shared",
                                                    "max_tile_nodes")},
            # launch = (tiles per workgroup, workgroups per CU); 0 workgroups
            # per CU is one workgroup per group of tiles (not persistent)
            "persistent": bool(launch[1] > 0),
            "tile_order": {0: "input", 1: "rcm", 2: "morton", 3: "bisection",
                           None: "bisection"}[args.order],
            "parallelism": "single GPU",
        },
        "fwd_tets_per_s": M / (res["fwd"] * 1e-3),
        "fwd_bwd_tets_per_s": M / (step_ms * 1e-3),
        "fwd_bwd_separate_tets_per_s": M / (res["fwd_bwd"] * 1e-3),
        "fused_bitwise_equal": fused_bitwise,
        "hbm_copy_GBps": copy_gbps,
        "hbm_frac_fwd": fwd_b / (res["fwd"] * 1e-3) / (HBM_PEAK_GBS * 1e9),
        # separate passes: both passes' algorithmic bytes over their step
        "hbm_frac_fwd_bwd": (fwd_b + bwd_b) / (res["fwd_bwd"] * 1e-3)
        / (HBM_PEAK_GBS * 1e9),
        # fused pass: its own algorithmic bytes (one tet stream) over its step
        "hbm_frac_fwd_bwd_fused": fused_b / (step_ms * 1e-3)
        / (HBM_PEAK_GBS * 1e9),
        # the separate passes' canonical bytes over the fused step: the
        # fraction of the HBM roof at which a forward + backward that moves
        # both passes' bytes would have to run to match the fused throughput
        "hbm_frac_fwd_bwd_effective": (fwd_b + bwd_b) / (step_ms * 1e-3)
        / (HBM_PEAK_GBS * 1e9),
        # the same fractions with the stored chunk bytes per tetrahedron
        "hbm_frac_fwd_stored": (fwd_b - (FWD_BYTES[0] - STORED_TET_BYTES) * M)
        / (res["fwd"] * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "hbm_frac_fwd_bwd_stored": (fwd_b + bwd_b - (FWD_BYTES[0] + BWD_BYTES[0]
                                                     - 2 * STORED_TET_BYTES) * M)
        / (res["fwd_bwd"] * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "ms": {k: round(v, 5) for k, v in res.items()},
        # each replay timed on its own (after the timed run): median, min, max
        "replay_ms": replays,
        "autotune": tuning,
        "kernels": kern,
        "roofline": roofline,
        "parity": par,
        "parity_all_cells": par_all,
        "n_inverted": n_inverted,
        "cpu_baseline": cpu,
        "relax": relax,
        "template": template,
        "regions": regions,
        "shape": shape,
        "quasistatic": quasistatic,
        "calibration": calibration,
        "latency": latency,
    }
    if not args.no_percell:
        out["percell_fwd_tets_per_s"] = M / (res["percell_fwd"] * 1e-3)
        out["percell_fwd_bwd_tets_per_s"] = M / (res["percell_fwd_bwd"] * 1e-3)
        out["batched_speedup_fwd_bwd"] = res["percell_fwd_bwd"] / res["fwd_bwd"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
