"""Benchmark of the sparse-grid MPM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload landslide|collapse_3d]

Prints ONE JSON line.  A step is one pass of the whole hot path -- active-node
indexing (bin, radix sort, hash insert, compaction), P2G, grid update and G2P --
over the workload's particles, all resident in HBM before timing starts.

* value      particle-steps/s of the sparse step (N_p x K / wall time of K steps,
             HIP events on the compute stream, bracketed by synchronisation);
* dense      the same step with the dense background grid (every block of the
             potential domain cleared and updated each step), same kernels;
* roofline   the dominant kernel's algorithmic bytes per launch over its
             average event-timed duration, against the 8 TB/s HBM peak;
* cpu_baseline  the FP64 oracle on a bounded sample of the same workload on the
             host (one thread).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s (sparse vs dense, 1 GPU); adjoint/forward step time ratio"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="landslide", choices=["landslide", "collapse_3d"])
    ap.add_argument("--dense-steps", type=int, default=10)
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--block-capacity", type=int, default=0)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-resolution", action="store_true",
                    help="skip the landslide at dx = 4 m and 2 m (sparse and dense steps, device memory; "
                         "--no-dense skips it too)")
    ap.add_argument("--no-configs", action="store_true", help="skip the column collapse and sliding-block legs")
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=200)
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle on the whole 2D collapse (200 steps), the 1/8-volume 3D "
                         "collapse (20 steps) and one 2D collapse per host core at once (minutes of CPU time)")
    ap.add_argument("--no-builders", action="store_true",
                    help="skip the hash vs scan-based build comparison")
    ap.add_argument("--late-steps", default="1000,2500,5000",
                    help="comma-separated steps from the release at which the landslide is timed again "
                         "(sparse and dense); empty to skip")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of this many MiB (a kernel of known traffic "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2605_28525_amd import workloads as wl
    if name == "landslide":
        return wl.landslide()
    return wl.collapse_3d()


def time_steps(sim, steps, stream, phases=True):
    """Time `steps` full steps on `stream` with HIP events: one event pair around
    the whole run (wall time) and, with ``phases``, events between the four calls
    of every step (per-call durations, which for P2G, grid update and G2P are
    single-kernel launches).  Returns (seconds, {phase: mean ms})."""
    import torch
    from paper_2605_28525_amd import mpm as M
    torch.cuda.synchronize()
    if not phases:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(steps, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3, {}
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    for k in range(steps):
        a, b = sim.a.view(sim.carry_id), sim.b.view(sim.carry_id)
        e = ev[k]
        e[0].record(stream)
        M.mpm_sparse_build(sim.ctx, a, stream)
        e[1].record(stream)
        M.mpm_p2g(sim.ctx, a, stream)
        e[2].record(stream)
        M.mpm_grid_update(sim.ctx, stream)
        e[3].record(stream)
        M.mpm_g2p(sim.ctx, a, b, stream)
        e[4].record(stream)
        sim.a, sim.b = sim.b, sim.a
    torch.cuda.synchronize()
    t = np.array([[ev[k][i].elapsed_time(ev[k][i + 1]) for i in range(4)] for k in range(steps)])
    total = ev[0][0].elapsed_time(ev[-1][4]) / 1e3
    return total, dict(zip(["build", "p2g", "grid_update", "g2p"], t.mean(axis=0).tolist()))


def adjoint_ratio(steps, checkpoint=50):
    """Calibration workload (262,144 particles).  rollout_ratio: wall time of
    the checkpointed backward pass (each segment recomputed on the tape, then
    the reverse sweep over it) over the forward rollout.  step_ratio: one
    stand-alone adjoint step (mpm_step_adj: rebuild, P2G and grid update of the
    input state, then the reverse kernels) over one forward step (mpm_step) on
    the same input state.  tape_step_ratio: per step of a segment, the reverse
    sweep over the tape (mpm_tape_adjoint) over the forward step."""
    import torch
    from paper_2605_28525_amd import autograd as AG
    from paper_2605_28525_amd import mpm as M
    from paper_2605_28525_amd import workloads as wl
    w = wl.differentiable_3d()
    n = w.n
    roll = AG.Rollout(w, steps=steps, checkpoint=checkpoint)
    try:
        v0 = torch.from_numpy(wl.calibration_target_velocity(n, seed=1003)).cuda()
        # warm-up (code objects, allocator)
        final = roll.run_forward(v0, w.E, w.friction_deg)
        roll.backward(roll.checkpoints, final.id, torch.zeros_like(final.x), w.E, w.friction_deg)
        torch.cuda.synchronize()
        fwds, bwds = [], []
        for _ in range(3):  # median of three rollouts
            t0 = time.perf_counter()
            final = roll.run_forward(v0, w.E, w.friction_deg)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x_bar = (final.x - final.x.mean()) / n
            gE, gphi, gv0 = roll.backward(roll.checkpoints, final.id, x_bar, w.E, w.friction_deg)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            fwds.append(t1 - t0)
            bwds.append(t2 - t1)
        # mpm_step reads a and writes b; mpm_step_adj reads a and the output
        # adjoint and writes the input adjoint: both leave a unchanged
        reps = 20
        a = final
        b = M.ParticleSet(w.dim, n, zero=False)
        ob = M.ParticleSet(w.dim, n)
        ob.x.copy_(x_bar)
        ib = M.ParticleSet(w.dim, n, zero=False)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        for _ in range(2):
            M.mpm_step(roll.ctx, a.view(), b.view(), 1)
            M.mpm_step_adj(roll.ctx, a.view(), ob.view(), ib.view(), roll.param_bar)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            M.mpm_step(roll.ctx, a.view(), b.view(), 1)
        ev[1].record()
        for _ in range(reps):
            M.mpm_step_adj(roll.ctx, a.view(), ob.view(), ib.view(), roll.param_bar)
        ev[2].record()
        torch.cuda.synchronize()
        t_step = ev[0].elapsed_time(ev[1]) / reps
        t_adj = ev[1].elapsed_time(ev[2]) / reps
        # one segment on the tape: recorded forward, then the reverse sweep
        K = roll.K
        views = [st.view() for st in roll._pool[:K + 1]]
        tb, ts = M.ParticleSet(w.dim, n), M.ParticleSet(w.dim, n, zero=False)
        tb.x.copy_(x_bar)
        M.mpm_tape_forward(roll.ctx, views)
        M.mpm_tape_adjoint(roll.ctx, views, tb.view(), ts.view(), roll.param_bar)
        torch.cuda.synchronize()
        ev[0].record()
        M.mpm_tape_forward(roll.ctx, views)
        ev[1].record()
        M.mpm_tape_adjoint(roll.ctx, views, tb.view(), ts.view(), roll.param_bar)
        ev[2].record()
        torch.cuda.synchronize()
        t_tape_fwd = ev[0].elapsed_time(ev[1]) / K
        t_tape_adj = ev[1].elapsed_time(ev[2]) / K
    finally:
        roll.close()
    fwd, bwd = float(np.median(fwds)), float(np.median(bwds))
    return {"workload": w.name, "particles": n, "steps": steps, "checkpoint_every": checkpoint,
            "step_ms": t_step, "adjoint_step_ms": t_adj, "step_ratio": t_adj / t_step,
            "tape_forward_step_ms": t_tape_fwd, "tape_adjoint_step_ms": t_tape_adj,
            "tape_step_ratio": t_tape_adj / t_step,
            "rollout_forward_ms": 1e3 * fwd, "rollout_backward_ms": 1e3 * bwd, "rollout_ratio": bwd / fwd,
            "grad_finite": bool(np.isfinite(gE) and np.isfinite(gphi) and torch.isfinite(gv0).all().item())}


def ensemble_leg(steps, stream):
    """64 uneven column collapses (about 19.5 M particles): autotuned, a graph
    of 10 captured steps replayed, against the same instances run one after
    another as 64 stand-alone simulations (eager steps)."""
    import torch
    from paper_2605_28525_amd import mpm as M
    from paper_2605_28525_amd import workloads as wl
    steps += steps & 1
    ens = wl.ensemble()
    n = ens.n
    log(f"bench: ensemble of {ens.n_instances} instances, {n} particles")
    sim = M.Simulation(ens)
    chosen = M.mpm_autotune(sim.ctx, sim.a.view(), sim.b.view(), stream)
    log(f"bench: ensemble autotune -> chunk {chosen[0]}, g2p block {chosen[1]}, p2g wgs {chosen[2]}, "
        f"g2p wgs {chosen[3]}")
    # a graph of 10 steps (inside one capture G2P bins for the next step)
    cap = 10
    steps = max(cap, steps - steps % cap)
    M.mpm_graph_capture(sim.ctx, sim.a.view(), sim.b.view(), cap, stream)
    M.mpm_graph_launch(sim.ctx, 1, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    M.mpm_graph_launch(sim.ctx, steps // cap, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / 1e3
    rc, flags = sim.status()
    if rc != 0:
        raise SystemExit(f"ensemble status: {rc} flags={flags}")
    nb, _ = M.mpm_active_count(sim.ctx)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    log("bench: ensemble, 64 stand-alone runs")
    sims = [M.Simulation(m) for m in ens.members]
    for s_ in sims:
        s_.step(2, stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for s_ in sims:
        s_.step(steps, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1) / 1e3
    for s_ in sims:
        rc, flags = s_.status()
        if rc != 0:
            raise SystemExit(f"ensemble member status: {rc} flags={flags}")
        s_.close()
    del sims
    torch.cuda.empty_cache()
    return {"workload": ens.name, "instances": ens.n_instances, "particles": n,
            "particles_min": min(m.n for m in ens.members), "particles_max": max(m.n for m in ens.members),
            "steps": steps, "active_blocks": nb, "tuning": {"chunk": chosen[0], "g2p_block": chosen[1],
                                                             "p2g_workgroups": chosen[2], "g2p_workgroups": chosen[3]},
            "batched": {"value": n * steps / t_batch, "ms_per_step": 1e3 * t_batch / steps, "graph": True},
            "sequential": {"value": n * steps / t_seq, "ms_per_step": 1e3 * t_seq / steps, "graph": False},
            "speedup": t_seq / t_batch, "unit": "particle-steps/s"}


def config_leg(name, steps, stream, dense=False):
    """A smaller configuration beside the headline one: the sparse step eager
    (phase-timed) and replayed from a graph, the build time, the step's byte
    model against the HBM peak, and with ``dense`` the dense-grid step."""
    import torch
    from paper_2605_28525_amd import mpm as M
    from paper_2605_28525_amd import workloads as wl
    w = {"collapse_2d": wl.collapse_2d, "collapse_3d": wl.collapse_3d,
         "sliding_block_30": lambda: wl.sliding_block(30.0)}[name]()
    n, d = w.n, w.dim
    sim = M.Simulation(w)
    try:
        sim.step(10, stream=stream)
        t, ph = time_steps(sim, steps, stream)
        t_graph = time_graph(sim, steps, stream)
        rc, flags = sim.status()
        if rc != 0:
            raise SystemExit(f"{name}: device status {rc} flags={flags}")
        nb, _ = M.mpm_active_count(sim.ctx)
    finally:
        sim.close()
    n_slot = nb * 4 ** d
    step_bytes = (276 if d == 3 else 148) * n + (72 if d == 3 else 52) * n_slot
    best = min(t / steps, t_graph)
    out = {"workload": name, "particles": n, "cells": list(w.cells[:d]), "steps": steps,
           "value": n * steps / t, "ms_per_step": 1e3 * t / steps, "phases_ms": ph,
           "graph": {"value": n / t_graph, "ms_per_step": 1e3 * t_graph},
           "build_ms_per_step": ph["build"], "active_blocks": nb,
           "step_roofline_frac": step_bytes / best / 1e9 / HBM_PEAK_GBS}
    if dense:
        simd = M.Simulation(w, grid_mode=M.MPM_GRID_DENSE)
        try:
            simd.step(2, stream=stream)
            td, _ = time_steps(simd, steps, stream, phases=False)
            rc, flags = simd.status()
            if rc != 0:
                raise SystemExit(f"{name} dense: device status {rc} flags={flags}")
        finally:
            simd.close()
        out["dense"] = {"value": n * steps / td, "ms_per_step": 1e3 * td / steps}
        out["speedup_vs_dense"] = td / t
    torch.cuda.empty_cache()
    return out


def device_bytes_of(make):
    """The object make() returns and the device memory it took (free memory
    before minus after; torch's cache is emptied first, so the figure holds the
    particle arrays and the context's own allocations)."""
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    f0 = torch.cuda.mem_get_info()[0]
    obj = make()
    torch.cuda.synchronize()
    return obj, f0 - torch.cuda.mem_get_info()[0]


def resolution_leg(h, steps, stream):
    """The landslide coarsened to dx = h metres (same terrain and release):
    whole sparse and dense steps (events around `steps` steps after 10) and
    the device memory of each (particles included)."""
    import torch
    from paper_2605_28525_amd import mpm as M
    from paper_2605_28525_amd import workloads as wl
    w = wl.landslide(h=h)
    n = w.n
    out = {"workload": w.name, "dx_m": float(h), "particles": n, "cells": list(w.cells), "steps": steps}
    for mode, name in ((M.MPM_GRID_SPARSE, "sparse"), (M.MPM_GRID_DENSE, "dense")):
        sim, nbytes = device_bytes_of(lambda: M.Simulation(w, grid_mode=mode))
        try:
            sim.step(10, stream=stream)
            t, _ = time_steps(sim, steps, stream, phases=False)
            rc, flags = sim.status()
            if rc != 0:
                raise SystemExit(f"{w.name} {name}: device status {rc} flags={flags}")
            if mode == M.MPM_GRID_SPARSE:
                out["active_blocks"] = M.mpm_active_count(sim.ctx)[0]
        finally:
            sim.close()
            del sim
            torch.cuda.empty_cache()
        out[name] = {"value": n * steps / t, "ms_per_step": 1e3 * t / steps, "device_bytes": nbytes}
    out["speedup_vs_dense"] = out["dense"]["ms_per_step"] / out["sparse"]["ms_per_step"]
    out["memory_reduction"] = out["dense"]["device_bytes"] / out["sparse"]["device_bytes"]
    return out


def copy_state(dst, src):
    """Device copy of src's current particle state (ids included) into dst.a."""
    dst.a.copy_(src.a)
    dst.a.id.copy_(src.a.id)


def builder_leg(w, src, cap, steps, stream):
    """The active-node construction compared at equal footing on the live
    state of `src`: the hash build (Algorithms 5-6) and the scan-based build
    (Algorithms 1-4), both sorting from scratch every step, plus the default
    hash build with the incremental re-sort (the headline).  Whole steps
    through mpm_step and the build phase alone, events on the stream, median
    of three runs of `steps` steps each; and the scan-based active-set query
    (mpm_scan_active, synchronous) per call."""
    import torch
    from paper_2605_28525_amd import mpm as M
    out = {"steps": steps}
    dummy = torch.empty(1, dtype=torch.int64, device="cuda")
    for name, flags in (("hash_resort", 0), ("hash_full_sort", M.MPM_FLAG_FULL_SORT),
                        ("scan_full_sort", M.MPM_FLAG_SCAN_BUILD)):
        sim = M.Simulation(w, block_capacity=cap, flags=flags)
        sim.carry_id = src.carry_id
        try:
            copy_state(sim, src)
            sim.step(2, stream=stream)
            whole = [time_steps(sim, steps, stream, phases=False)[0] for _ in range(3)]
            _, ph = time_steps(sim, steps, stream)
            rc, flags_ = sim.status()
            if rc != 0:
                raise SystemExit(f"builder leg {name}: device status {rc} flags={flags_}")
            rec = {"ms_per_step": 1e3 * float(np.median(whole)) / steps, "build_ms": ph["build"],
                   "active_blocks": M.mpm_active_count(sim.ctx)[0]}
            if flags == M.MPM_FLAG_SCAN_BUILD:
                M.mpm_scan_active(sim.ctx, sim.a.view(), dummy, dummy, 0, stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(5):
                    M.mpm_scan_active(sim.ctx, sim.a.view(), dummy, dummy, 0, stream)
                rec["query_ms_per_call"] = 1e3 * (time.perf_counter() - t0) / 5
            out[name] = rec
        finally:
            sim.close()
            del sim
            torch.cuda.empty_cache()
    out["scan_over_hash_step"] = out["scan_full_sort"]["ms_per_step"] / out["hash_full_sort"]["ms_per_step"]
    out["scan_over_hash_build"] = out["scan_full_sort"]["build_ms"] / out["hash_full_sort"]["build_ms"]
    return out


def late_state_leg(sim, simd, steps_done, targets, steps, dense_steps, stream):
    """The run continued from the headline state to each step in `targets`
    (counted from the release): there, `steps` sparse steps timed three times
    (median), the active blocks, and the dense step on a copy of that state.
    Returns (records, steps_done)."""
    from paper_2605_28525_amd import mpm as M
    recs = []
    for tgt in targets:
        if tgt > steps_done:
            sim.step(tgt - steps_done, stream=stream)
            steps_done = tgt
        runs = [time_steps(sim, steps, stream, phases=False)[0] for _ in range(3)]
        steps_done += 3 * steps
        rc, flags = sim.status()
        if rc != 0:
            raise SystemExit(f"late state {tgt}: device status {rc} flags={flags}")
        nb, nt = M.mpm_active_count(sim.ctx)
        ms = 1e3 * float(np.median(runs)) / steps
        rec = {"step": tgt, "ms_per_step": ms, "value": sim.a.n * 1e3 / ms, "active_blocks": nb,
               "runs_ms_per_step": [1e3 * r / steps for r in runs]}
        if simd is not None:
            copy_state(simd, sim)
            td, _ = time_steps(simd, dense_steps, stream, phases=False)
            rc, flags = simd.status()
            if rc != 0:
                raise SystemExit(f"late state {tgt} dense: device status {rc} flags={flags}")
            rec["dense_ms_per_step"] = 1e3 * td / dense_steps
            rec["speedup_vs_dense"] = rec["dense_ms_per_step"] / ms
        log(f"bench: step {tgt}: {ms:.3f} ms/step, {nb} active blocks"
            + (f", dense {rec['dense_ms_per_step']:.2f} ms" if simd is not None else ""))
        recs.append(rec)
    return recs, steps_done


def graph_len(steps):
    """Steps captured in one graph: as many as one timed run (even, so that the
    state returns to sim.a), so that its steps bin in G2P like mpm_step's."""
    return max(2, steps - steps % 2)


def time_graph(sim, steps, stream):
    """The same steps replayed from a HIP graph of graph_len(steps) captured
    steps (`mpm_graph_capture`), one replay after a warm-up replay, timed with
    events.  Returns seconds per step."""
    import torch
    from paper_2605_28525_amd import mpm as M
    n_cap = graph_len(steps)
    M.mpm_graph_capture(sim.ctx, sim.a.view(sim.carry_id), sim.b.view(sim.carry_id), n_cap, stream)
    try:
        M.mpm_graph_launch(sim.ctx, 1, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        M.mpm_graph_launch(sim.ctx, 1, stream)
        e1.record(stream)
        torch.cuda.synchronize()
    finally:
        M.mpm_graph_release(sim.ctx)
    return e0.elapsed_time(e1) / 1e3 / n_cap


def graph_steps(steps):
    """Steps that time_graph advances the state by."""
    return 2 * graph_len(steps)


def measured_copy_gbs(mib=2048, reps=5):
    """Device-to-device copy bandwidth of this GPU (read + write bytes / time),
    the measured counterpart of the 8 TB/s spec peak."""
    import torch
    a = torch.empty(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def src_digest(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2605_28525_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, digest):
    """HBM traffic per launch from a committed rocprofv3 --pmc summary, only if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("src_digest") != digest:
        return None
    return rec.get("bytes_per_launch")


def all_src_digest():
    names = sorted(f for f in os.listdir(os.path.join(ROOT, "paper_2605_28525_amd", "csrc"))
                   if f.endswith((".hip", ".h")))
    return src_digest(*names)


def profile_counters(workload, digest_unused=None):
    """Per-step counter figures from a committed rocprofv3 summary
    (profiles/counters_<workload>.json: VALU busy fraction of the transfer
    kernels, the HBM traffic of one whole step and of its sort / re-sort
    kernels), used only if it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("src_digest") != all_src_digest():
        return None
    rec = dict(rec)
    rec.pop("src_digest", None)
    return rec


def host_info():
    """CPU model, core counts and the BLAS thread pools numpy would use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    info = {"cpu_model": model, "cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        from threadpoolctl import threadpool_info
        info["blas"] = [{"api": t.get("internal_api"), "threads": t.get("num_threads")} for t in threadpool_info()]
    except Exception:  # pragma: no cover
        info["blas"] = None
    return info


def _oracle_steps(name, steps, progress=False):
    """Runs the FP64 oracle `steps` steps of a workload on one thread; returns
    (particles, seconds).  Top-level so that spawned worker processes can run it."""
    from threadpoolctl import threadpool_limits
    from oracle import mpm as om
    from paper_2605_28525_amd import workloads as wl
    w = {"collapse_2d": wl.collapse_2d, "collapse_3d_1of8": lambda: wl.collapse_3d(scale=2),
         "landslide_window": wl.landslide_crop}[name]()
    with threadpool_limits(1):
        p = om.Params.from_workload(w)
        st = om.state_from_soa(w.state(), w.dim)
        t0 = time.perf_counter()
        for k in range(steps):
            st = om.step(st, p)
            if progress and (k + 1) % 5 == 0:
                log(f"bench: oracle {name} step {k + 1}/{steps}, {time.perf_counter() - t0:.1f} s")
        return w.n, time.perf_counter() - t0


def cpu_baseline(w_name, budget_s):
    """FP64 oracle on a bounded sample of the workload, single thread."""
    from threadpoolctl import threadpool_limits
    from oracle import mpm as om
    from paper_2605_28525_amd import workloads as wl
    if w_name == "landslide":
        w = wl.landslide_crop()
        sample = "landslide window 64x64x256 cells (same terrain, dx = 1 m), 16,384 particles"
    else:
        w = wl.collapse_3d(scale=2)
        sample = "3D collapse at 1/8 volume, 262,144 particles"
    with threadpool_limits(1):
        p = om.Params.from_workload(w)
        st = om.state_from_soa(w.state(), w.dim)
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            st = om.step(st, p)
            steps += 1
        dt = time.perf_counter() - t0
    host = host_info()
    # the oracle on the smaller configurations too: the whole 2D collapse, and
    # three steps of the 1/8-volume 3D collapse (all 20 with --cpu-full)
    n2, t2 = _oracle_steps("collapse_2d", 200)
    n3, t3 = _oracle_steps("collapse_3d_1of8", 3)
    return {"value": w.n * steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}, {steps} steps in {dt:.1f} s, float64 numpy, one thread "
                      f"(1 of {host['affinity']} usable host cores)",
            "configs": {"collapse_2d": {"particles": n2, "steps": 200, "seconds": t2, "value": n2 * 200 / t2},
                        "collapse_3d_1of8": {"particles": n3, "steps": 3, "seconds": t3, "value": n3 * 3 / t3}},
            "host": host}


def cpu_full_runs():
    """The oracle on whole configurations: the 2D collapse over its 200 steps,
    the 1/8-volume 3D collapse over 20 steps (one thread each), and the 2D
    collapse run by one process per usable core at once (aggregate rate)."""
    import multiprocessing as mp
    out = {}
    n, t = _oracle_steps("collapse_2d", 200)
    out["collapse_2d_200_steps"] = {"particles": n, "seconds": t, "value": n * 200 / t}
    log(f"bench: oracle collapse_2d 200 steps {t:.1f} s")
    n, t = _oracle_steps("collapse_3d_1of8", 20, progress=True)
    out["collapse_3d_1of8_20_steps"] = {"particles": n, "seconds": t, "value": n * 20 / t}
    log(f"bench: oracle collapse_3d 1/8 20 steps {t:.1f} s")
    procs = min(16, len(os.sched_getaffinity(0)))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.starmap(_oracle_steps, [("collapse_2d", 50)] * procs)
    wall = time.perf_counter() - t0
    out["collapse_2d_aggregate"] = {"processes": procs, "steps_each": 50,
                                    "value": sum(r[0] * 50 for r in res) / wall, "wall_seconds": wall}
    out["host"] = host_info()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU only: sharding it over several GPUs is "
                                   "designed but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2605_28525_amd import mpm as M

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        a = torch.ones(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copy probe of {args.copy_probe} MiB done")
        del a, b
    log(f"bench: generating {args.workload}")
    w = make_workload(args.workload)
    n = w.n
    d = w.dim
    log(f"bench: {w.name} n={n} cells={w.cells}")
    cap = args.block_capacity or (1 << 18 if args.workload == "landslide" else 1 << 16)
    sim, sparse_bytes = device_bytes_of(lambda: M.Simulation(w, block_capacity=cap))
    # The particle id that may travel with each particle is bookkeeping for the
    # caller, not the method's work: the headline runs without it, and one run
    # with it is timed beside.
    sim.carry_id = False
    log("bench: warmup")
    steps_done = 0
    if args.warmup:
        sim.step(args.warmup, stream=stream)
        steps_done += args.warmup
    rc, flags = sim.status()
    if rc != 0:
        raise SystemExit(f"device status after warmup: {rc} flags={flags}")
    tuning = None
    if not args.no_autotune:
        # leaves the state unchanged
        chosen = M.mpm_autotune(sim.ctx, sim.a.view(), sim.b.view(), stream)
        tuning = dict(zip(("chunk", "g2p_block", "p2g_workgroups", "g2p_workgroups"), chosen))
        log(f"bench: autotune -> {tuning}")
    nb, nt = M.mpm_active_count(sim.ctx)
    log(f"bench: timed {args.steps} steps (active blocks {nb})")
    # the headline: exactly K steps through mpm_step (one call), then the same
    # twice more for the spread
    t, _ = time_steps(sim, args.steps, stream, phases=False)
    runs = [t] + [time_steps(sim, args.steps, stream, phases=False)[0] for _ in range(2)]
    steps_done += 3 * args.steps
    rc, flags = sim.status()
    if rc != 0:
        raise SystemExit(f"device status after timing: {rc} flags={flags}")
    # a separate instrumented run: events between the four calls of each step
    _, ph = time_steps(sim, args.steps, stream)
    steps_done += args.steps
    t_graph = time_graph(sim, args.steps, stream)
    steps_done += graph_steps(args.steps)
    sim.carry_id = True
    t_id, _ = time_steps(sim, args.steps, stream, phases=False)
    steps_done += args.steps
    sim.carry_id = False
    rc, flags = sim.status()
    if rc != 0:
        raise SystemExit(f"device status after graph replays: {rc} flags={flags}")
    log(f"bench: {1e3 * t / args.steps:.3f} ms/step (runs "
        f"{', '.join(f'{1e3 * r / args.steps:.3f}' for r in runs)}), graph replay {1e3 * t_graph:.3f} ms/step")
    value = n * args.steps / t
    ms_per_step = 1e3 * t / args.steps
    nb, nt = M.mpm_active_count(sim.ctx)
    npb = 4 ** d
    n_slot = nb * npb
    n_dense_nodes = int(np.prod([c + 1 for c in w.cells[:d]]))
    n_tau = 3 if d == 2 else 6
    # algorithmic bytes per launch, counted once per field the method needs:
    # G2P reads x, F and the particle's source index and the nodal velocity of
    # each active node slot, and writes x, v, C, F, tau; P2G reads x, v, C, tau
    # and the index and writes mass and momentum of each slot
    g2p_bytes = n * (4 * d + 4 * d * d + 4 + 4 * (d + d + d * d + d * d + n_tau)) + 4 * d * n_slot
    g2p_id_bytes = 8 * n   # the optional particle id read and written beside the state
    p2g_bytes = n * (4 * (d + d + d * d + n_tau) + 4) + 16 * n_slot
    kernels = {"g2p": (g2p_bytes, ph["g2p"]), "p2g": (p2g_bytes, ph["p2g"])}
    dom = max(kernels, key=lambda k: kernels[k][1])
    dom_bytes, dom_ms = kernels[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    digest = src_digest("transfer.hip", "particle.h", "internal.h")
    traffic = measured_traffic(dom, args.workload, digest)
    build_bytes = n * 16 + 24 * (1 << max(10, int(np.ceil(np.log2(2 * cap))))) + 16 * nb
    step_bytes = (276 if d == 3 else 148) * n + (72 if d == 3 else 52) * n_slot
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "particles": n, "cells": list(w.cells[:d]), "dx_m": w.dx,
                   "block": "4^3", "grid": "sparse"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": dom_bytes, "ms_per_launch": dom_ms,
                     "time_source": "HIP events around the single-kernel mpm_g2p / mpm_p2g call"},
        "runs_ms_per_step": [1e3 * r / args.steps for r in runs],
        "median_ms_per_step": 1e3 * float(np.median(runs)) / args.steps,
        "phases_ms": ph,
        "g2p_id_carry_bytes": g2p_id_bytes,
        "graph": {"ms_per_step": 1e3 * t_graph, "value": n / t_graph},
        "with_id": {"ms_per_step": 1e3 * t_id / args.steps, "value": n * args.steps / t_id},
        "tuning": tuning,
        "build_ms_per_step": ph["build"],
        "build_roofline_frac": build_bytes / (ph["build"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_bytes_model": step_bytes,
        "step_roofline_frac": step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        # against the bytes a step with G2P and the next P2G fused would move (192 B per particle)
        "fused_bound_roofline_frac": 192.0 * n / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "measured_copy_GBps": measured_copy_gbs(),
        "active_blocks": nb,
        "block_capacity": cap,
        "active_fraction": n_slot / n_dense_nodes,
    }
    counters = profile_counters(args.workload, digest)
    if counters:
        out["counters"] = counters
    if not args.no_builders and args.workload == "landslide":
        log("bench: hash and scan-based builds")
        out["builders"] = builder_leg(w, sim, cap, args.steps, stream)
    simd = None
    if not args.no_dense:
        log("bench: dense baseline")
        simd, dense_bytes = device_bytes_of(lambda: M.Simulation(w, grid_mode=M.MPM_GRID_DENSE))
        simd.carry_id = False
        simd.step(2, stream=stream)
        td, _ = time_steps(simd, args.dense_steps, stream, phases=False)
        rc, flags = simd.status()
        if rc != 0:
            raise SystemExit(f"dense status: {rc} flags={flags}")
        dense_value = n * args.dense_steps / td
        out["dense"] = {"value": dense_value, "ms_per_step": 1e3 * td / args.dense_steps,
                        "steps": args.dense_steps}
        out["speedup_vs_dense"] = value / dense_value
        # device memory, particle arrays included (the same in both)
        out["memory"] = {"sparse_bytes": sparse_bytes, "dense_bytes": dense_bytes,
                         "reduction": dense_bytes / sparse_bytes}
    if args.late_steps and args.workload == "landslide":
        log("bench: the run continued to later states")
        targets = [int(v) for v in args.late_steps.split(",") if v]
        out["late_states"], steps_done = late_state_leg(sim, simd, steps_done, targets, 20, 5, stream)
    if simd is not None:
        simd.close()
        del simd
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not args.no_configs:
        log("bench: 2D and 3D column collapse")
        out["configs"] = [config_leg("collapse_2d", args.steps, stream),
                          config_leg("collapse_3d", args.steps, stream, dense=True),
                          config_leg("sliding_block_30", args.steps, stream, dense=True)]
    if not (args.no_resolution or args.no_dense) and args.workload == "landslide":
        log("bench: landslide at dx = 4 m and 2 m")
        out["resolution"] = [resolution_leg(h, args.steps, stream) for h in (4, 2)]
    if not args.no_adjoint:
        log("bench: adjoint/forward ratio")
        out["adjoint"] = adjoint_ratio(args.adjoint_steps)
        # the adjoint's cost including the checkpoint recompute
        out["adjoint_forward_ratio"] = out["adjoint"]["rollout_ratio"]
    if not args.no_ensemble:
        log("bench: ensemble")
        out["ensemble"] = ensemble_leg(args.ensemble_steps, stream)
    if not args.no_cpu:
        log("bench: cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    if args.cpu_full:
        log("bench: oracle on whole configurations")
        out["cpu_full"] = cpu_full_runs()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
