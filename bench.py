"""Benchmark of the electronic-temperature hot path on one MI355X.

One step = one pass of the whole path over the 4,000,000-atom jittered FCC
system (100^3 cells, cut-off 1.2a): cell binning and neighbour sets, the
Eq. 4 lattice temperature from velocities with the kinetic-energy gate,
parameters, T_e, 10,000 FP32C sub-steps of Eq. 2 in the tuned launch (one
LDS-brick launch per sub-step, the sub-steps of an advance captured in one
hipGraph), and the FP64 energy ledger.  Inputs are resident in HBM before the
timed region starts.

Also reported:
  * roofline of the dominant kernel (the FP32C sub-step launch), from HIP events
    on the library's stream, against 8 TB/s HBM, with the algorithmic bytes
    20 + 2 n_mean (brick form) or 20 + 4 n_mean (global gathers) per
    atom-substep, the HBM traffic rocprofv3 measured for it (and that traffic
    over the live launch time), and a 1 GiB device copy on the same GPU;
  * the same system in the plain FP64 form (a bounded sample of sub-steps);
  * the batched FP32C form vs the plain FP64 form on the 256-system laser batch
    (same sub-step count for both);
  * the lattice side on the same system: sub-step cost with the per-atom energy
    record off and on, the Eq. 8 coupling coefficient and one Eq. 5 velocity
    step, against HBM bandwidth;
  * the sub-step cost with a shell of held electronic temperatures and the
    mean-field parameter refresh at every advance;
  * the batch of two-temperature 1D bars (FP64, electrons and lattice);
  * the recorded forward and the adjoint on the differentiation workload
    (64 systems of 32,000 atoms, 2,000 sub-steps, checkpoints every 100);
  * the FP64 CPU oracle on the host cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
XGMI_LINK_GBS = 153.0   # one xGMI link of an MI355X, each direction (AMD public figure)
# L2T_OPT_GRAPH of every context the bench makes: None leaves the library's
# default (the FP32C advance times direct launches against graph replays in the
# autotuner); 0 launches every sub-step directly (rocprofv3 counter passes),
# 1 replays captured hipGraphs
GRAPH = None
# (option, value) pairs set on every FP32C context the bench makes, from the
# launch-form options (--kernel, --block, --brick-edge, --sweep,
# --table-stream).  Counter passes pin the form the timed run chose: the
# build's and the autotuner's timings are perturbed under the counters.
FP32C_PINS = []


def new_context(L, systems, prec, **kw):
    ctx = L.Context(systems, prec, **kw)
    if GRAPH is not None:
        L.l2t_set_option(ctx.h, L.L2T_OPT_GRAPH, GRAPH)
    if prec == L.L2T_FP32C:
        for opt, value in FP32C_PINS:
            L.l2t_set_option(ctx.h, opt, value)
    return ctx


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def library_source_hash() -> str:
    """sha256 over the sources the sub-step kernels are compiled from (their
    translation unit, the device helpers, the state encoding, the internal and
    the C header) and over the layout builder, whose brick order sets the
    kernel's L2 reuse and so its traffic."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1810_12357_amd", "csrc")
    files = [os.path.join(csrc, f) for f in ("k_step.hip", "step_device.h", "state_fp32c.h",
                                             "l2t_internal.h", "k_geometry.hip")]
    files.append(os.path.join(ROOT, "include", "l2t.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, n_atoms: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the summary is missing, covers another kernel or size, or was
    taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_c3_4M_traffic.md")
    if n_atoms != 4_000_000 or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", "|", "`")):
                k, _, v = line.partition(":")
                vals[k.strip()] = v.strip()
    if vals.get("kernel") != kernel or vals.get("csrc_sha256") != library_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def setup_system(L, ctx_h, sy, dev):
    """Device copies of the inputs of one system."""
    import torch
    return dict(pos=torch.from_numpy(np.ascontiguousarray(sy.pos.reshape(-1))).to(dev),
                vel=torch.from_numpy(np.ascontiguousarray(sy.vel.reshape(-1))).to(dev),
                mass=torch.from_numpy(np.ascontiguousarray(sy.mass)).to(dev),
                Te=torch.from_numpy(np.ascontiguousarray(sy.T_e0)).to(dev))


def one_pass(L, h, sy, d, r_cut, n_sub, timer):
    """A1..A6 of the path for one system; returns the advance duration (ms)."""
    L.l2t_set_positions(h, 0, d["pos"])
    mx, mean = L.l2t_build_neighbors(h, r_cut)
    L.l2t_set_params(h, 0, sy.params)
    L.l2t_set_field(h, 0, L.L2T_FIELD_TE, d["Te"])
    L.l2t_set_velocities(h, 0, d["vel"], d["mass"])
    timer[0].record()
    L.l2t_advance(h, n_sub)
    timer[1].record()
    e = L.l2t_energies(h, 0)
    e["max_nbrs"], e["mean_nbrs"] = mx, mean
    return e


def bench_c4_speedup(L, torch, n_sub, n_full, only_fp32c=False):
    """Batched FP32C (one tuned launch per sub-step for all systems) vs plain
    FP64 on the 256-system batch.  The plain form runs the systems one after
    another, one launch per sub-step and system; the batched FP64 form (all
    systems in one launch per sub-step) is timed beside it.  Every form runs
    the first n_sub sub-steps from t = 0 (the pulse peaks at 150 fs, sub-step
    3,000), where the speedup is taken; the batched FP32C form also runs the
    whole n_full sub-steps of the workload.  only_fp32c times the batched
    FP32C form alone (for profiling that kernel; no speedup is reported)."""
    import workloads as W
    w = W.c4()
    n_atoms = w.n_atoms
    out = {}
    info = {}
    forms = (("fp32c_batched", L.L2T_FP32C, 0), ("fp64_plain", L.L2T_FP64, 0),
             ("fp64_batched", L.L2T_FP64, 1))
    if only_fp32c:
        forms = forms[:1]
    for name, prec, batch in forms:
        ctx = new_context(L, w.systems, prec)
        if batch:
            L.l2t_set_option(ctx.h, L.L2T_OPT_BATCH_FP64, 1)
            L.l2t_set_option(ctx.h, L.L2T_OPT_RESIDENT_MAX, -1)
        _, mean, _ = ctx.setup(w.r_cut)
        ctx.advance(2)                 # warm-up (autotune, graph capture)
        runs = [n_sub] + ([n_full] if prec == L.L2T_FP32C and n_full > n_sub else [])
        for n in runs:
            for s, sy in enumerate(w.systems):
                L.l2t_set_field(ctx.h, s, L.L2T_FIELD_TE, sy.T_e0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.advance(n)
            L.l2t_sync(ctx.h)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            key = name if n == n_sub else name + "_full"
            out[key] = n_atoms * n / dt
            log(f"  C4 {key}: {n_atoms} atoms x {n} sub-steps in {dt:.3f} s")
        kernel = L.l2t_get_option(ctx.h, L.L2T_OPT_KERNEL)
        # algorithmic bytes per atom-substep: the state read and written (FP32C
        # hi and its 16-bit low part: 12; FP64: 16), T_lat (4 / 8), the source
        # weight of the laser (4 / 8), a row offset (4) and one index per
        # neighbour (2 B in the brick forms, 4 B through the global-slot table)
        per_nbr = 2.0 if kernel == 1 else 4.0
        fixed = 24.0 if prec == L.L2T_FP32C else 36.0
        info[name] = dict(kernel=["global-gather", "lds-brick"][kernel], mean_neighbors=mean,
                          bytes_per_atom_substep=fixed + per_nbr * mean,
                          brick_edge=L.l2t_get_option(ctx.h, L.L2T_OPT_BRICK_EDGE),
                          block=L.l2t_get_option(ctx.h, L.L2T_OPT_BLOCK),
                          sweep=["fixed", "alternating"][
                              L.l2t_get_option(ctx.h, L.L2T_OPT_SWEEP) - 1],
                          table_loads=["cached", "streamed"][
                              L.l2t_get_option(ctx.h, L.L2T_OPT_TABLE_STREAM) - 1],
                          launches=["direct", "graph replays"][
                              L.l2t_get_option(ctx.h, L.L2T_OPT_GRAPH)])
        ctx.close()
    if only_fp32c:
        res = dict(workload=f"c4 batch of {len(w.systems)} laser slabs, {n_atoms} atoms, "
                            f"batched FP32C only", substeps=n_sub,
                   fp32c_batched_atom_substeps_per_s=out["fp32c_batched"],
                   fp32c_batched_form=info["fp32c_batched"])
        if "fp32c_batched_full" in out:
            res["fp32c_batched_full_run_atom_substeps_per_s"] = out["fp32c_batched_full"]
        return res
    res = dict(workload=f"c4 batch of {len(w.systems)} laser slabs, {n_atoms} atoms; the speedup "
                        f"over the first {n_sub} sub-steps (pulse centre at sub-step 3000), "
                        f"batched FP32C also over all {n_full}",
               speedup_substeps=n_sub,
               fp32c_batched_atom_substeps_per_s=out["fp32c_batched"],
               fp64_plain_atom_substeps_per_s=out["fp64_plain"],
               fp64_batched_atom_substeps_per_s=out["fp64_batched"],
               speedup=out["fp32c_batched"] / out["fp64_plain"],
               speedup_vs_fp64_batched=out["fp32c_batched"] / out["fp64_batched"],
               brick_edge=info["fp32c_batched"]["brick_edge"])
    if "fp32c_batched_full" in out:
        res["fp32c_batched_full_run_atom_substeps_per_s"] = out["fp32c_batched_full"]
    for name in ("fp32c_batched", "fp64_plain", "fp64_batched"):
        gbps = info[name]["bytes_per_atom_substep"] * out[name] / 1e9
        res[name + "_form"] = dict(info[name], algorithmic_GBps=gbps, frac=gbps / HBM_PEAK_GBS)
    return res


def bench_shard(L, torch, w, parts=(2, 4, 8), n_sub=2000, reps=3):
    """One GPU's share of the 4M-atom system when it is cut into x-slabs over
    N GPUs (a design study on one GPU): the slab's own atoms plus ghost layers
    of width r_c from both neighbours, held at their T_e (L2T_FIELD_FIXED)
    where a multi-GPU run would have the neighbours' exchange write them.
    The sub-step time of the share is measured with HIP events on the
    library's stream (median of reps advances of n_sub sub-steps); the
    exchange (the hi of each ghost face, 4 B per ghost atom, one face per
    xGMI link) is estimated, not run."""
    import workloads as W
    res = {}
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for n in parts:
        sh, ghost = W.c3_shard(w, n)
        ctx = new_context(L, [sh], L.L2T_FP32C, stream=torch.cuda.current_stream().cuda_stream)
        _, mean, _ = ctx.setup(w.r_cut)
        L.l2t_set_field(ctx.h, 0, L.L2T_FIELD_FIXED, ghost)
        ctx.advance(2)                     # warm-up (autotune, graph capture)
        times = []
        for _ in range(reps):
            a, b = ev(), ev()
            a.record()
            ctx.advance(n_sub)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        ms = float(np.median(times))
        n_ghost = int(ghost.sum())
        n_own = sh.n - n_ghost
        face_bytes = 4.0 * n_ghost / 2.0
        res[f"n{n}"] = dict(own_atoms=n_own, ghost_atoms=n_ghost, substeps=n_sub,
                            substep_us=ms * 1e3 / n_sub,
                            own_atom_substeps_per_s=n_own * n_sub / (ms * 1e-3),
                            kernel=["global-gather", "lds-brick"][
                                L.l2t_get_option(ctx.h, L.L2T_OPT_KERNEL)],
                            brick_edge=L.l2t_get_option(ctx.h, L.L2T_OPT_BRICK_EDGE),
                            block=L.l2t_get_option(ctx.h, L.L2T_OPT_BLOCK),
                            mean_neighbors=mean,
                            exchange_bytes_per_face=face_bytes,
                            exchange_us_per_link_est=face_bytes / XGMI_LINK_GBS / 1e3)
        log(f"  shard of {n}: {n_own} own + {n_ghost} ghost atoms, "
            f"{res[f'n{n}']['substep_us']:.2f} us per sub-step")
        ctx.close()
    return dict(workload="one x-slab of the 4M-atom system cut over N GPUs, with ghost layers "
                         "of width r_c held (exchange not run)", xgmi_link_GBps=XGMI_LINK_GBS,
                **res)


def bench_md_coupling(L, torch, h, sy, d, n_sub=10, reps=20):
    """Lattice side on the same system: one MD step of n_sub sub-steps with the
    per-atom energy record off and on, then the Eq. 8 coupling coefficient
    (ledger mode) and one Eq. 5 velocity step on device arrays, each timed
    with HIP events on the library's stream."""
    dev = d["vel"].device
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        for _ in range(10):                     # warm-up (graph capture, autotune, clocks)
            fn()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for _ in range(k):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k * 1e3      # us per call

    out = {}
    for on in (0, 1):
        L.l2t_set_option(h, L.L2T_OPT_ATOM_LEDGER, on)
        out["substep_us_record_" + ("on" if on else "off")] = \
            timed(lambda: L.l2t_advance(h, n_sub), 40) / n_sub
    dt_md = n_sub * sy.params["dt"]
    xi = torch.empty(sy.n, dtype=torch.float64, device=dev)
    v = d["vel"].clone()
    cu = timed(lambda: L.l2t_coupling(h, 0, L.L2T_XI_LEDGER, dt_md, d["vel"], d["mass"], xi), reps)
    du = timed(lambda: L.l2t_damping_step(h, 0, dt_md, xi, None, d["mass"], v), reps)
    L.l2t_set_option(h, L.L2T_OPT_ATOM_LEDGER, 0)
    # algorithmic bytes per atom: coupling reads the slot map (4), v (24), m (8),
    # T_lat (4) and the record (8) and writes xi (8); the velocity step reads
    # xi (8), m (8) and v (24) and writes v (24)
    bc, bd = 56.0, 64.0
    out.update(coupling_us=cu, damping_step_us=du,
               coupling_GBps=bc * sy.n / (cu * 1e-6) / 1e9,
               damping_step_GBps=bd * sy.n / (du * 1e-6) / 1e9)
    out["coupling_frac"] = out["coupling_GBps"] / HBM_PEAK_GBS
    out["damping_step_frac"] = out["damping_step_GBps"] / HBM_PEAK_GBS
    out["record_overhead"] = out["substep_us_record_on"] / out["substep_us_record_off"] - 1.0
    log(f"  MD coupling: sub-step {out['substep_us_record_off']:.1f} us (record off), "
        f"{out['substep_us_record_on']:.1f} us (on); xi {cu:.1f} us, velocity step {du:.1f} us")
    return out


def bench_boundary_mean_field(L, torch, h, sy, n_sub=10, reps=40):
    """Held electronic temperatures on a spherical shell (Section 4 boundary)
    and the Section 2 mean-field refresh at the start of every advance, on the
    same system: cost per sub-step against the plain advance."""
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def per_substep():
        for _ in range(10):                     # warm-up (graph capture, clocks)
            L.l2t_advance(h, n_sub)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            L.l2t_advance(h, n_sub)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e3 / (reps * n_sub)

    plain = per_substep()
    r2 = ((sy.pos - (sy.box_len / 2)[:, None]) ** 2).sum(0)
    held = ((r2 > 60.0 ** 2) & (r2 < 64.0 ** 2)).astype(np.float64)
    lam_atom = 1065.0 * (sy.params["v_atom"] * 1e-30) / 1.602176634e-19
    k_coef = 2 * 3 * 91.0 / (1065.0 * 12 * (3.61e-10) ** 2) * 1e-15
    L.l2t_set_field(h, 0, L.L2T_FIELD_FIXED, held)
    held_only = per_substep()
    L.l2t_set_mean_field(h, 0, True, lam_atom, k_coef)
    both = per_substep()
    L.l2t_set_field(h, 0, L.L2T_FIELD_FIXED, np.zeros(sy.n))
    mf_only = per_substep()
    L.l2t_set_mean_field(h, 0, False)
    log(f"  per sub-step: plain {plain:.1f} us, held shell {held_only:.1f} us, mean field "
        f"{mf_only:.1f} us, both {both:.1f} us")
    return dict(substeps_per_advance=n_sub, held_atoms=int(held.sum()), substep_us_plain=plain,
                substep_us_held=held_only, substep_us_mean_field=mf_only,
                substep_us_held_and_mean_field=both,
                mean_field_refresh_us_per_advance=(mf_only - plain) * n_sub)


def bench_adjoint(L, torch):
    """Differentiation workload (64 FCC systems of 32,000 atoms, 2,000 FP32C
    sub-steps, a checkpoint every 100): the recorded forward, then the adjoint
    (recomputation between checkpoints and the reverse sub-steps) of the MSE
    loss against targets run with each system's perturbed K and g.  Inputs
    and dL/dT^N are device-resident; both calls end synchronised and are timed
    on the wall clock after one untimed round."""
    import workloads as W
    w = W.c5()
    n, ck = w.n_substeps, w.checkpoint_every
    dev = torch.device("cuda:0")
    tw = W.c5()
    for s, sy in enumerate(tw.systems):
        K, g = tw.extra["target_params"][s]
        sy.params = dict(sy.params, K=K, g=g)
    ctx_t = new_context(L, tw.systems, L.L2T_FP32C)
    ctx_t.setup(tw.r_cut)
    ctx_t.advance(n)
    tgt = np.concatenate([ctx_t.get(s) for s in range(len(tw.systems))])
    ctx_t.close()
    ctx = new_context(L, w.systems, L.L2T_FP32C, stream=torch.cuda.current_stream().cuda_stream)
    _, mean, _ = ctx.setup(w.r_cut)
    h, S = ctx.h, len(w.systems)
    N = w.n_atoms
    T0 = [torch.from_numpy(np.ascontiguousarray(sy.T_e0)).to(dev) for sy in w.systems]
    times = []
    for rep in range(2):
        for s in range(S):
            L.l2t_set_field(h, s, L.L2T_FIELD_TE, T0[s])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.l2t_advance_recorded(h, n, ck)
        L.l2t_sync(h)
        t1 = time.perf_counter()
        TN = np.concatenate([ctx.get(s) for s in range(S)])
        dL = torch.from_numpy(2.0 * (TN - tgt) / N).to(dev)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        dK, dg = L.l2t_adjoint(h, dL, S)
        t3 = time.perf_counter()
        times.append((t1 - t0, t3 - t2))
    kernel = L.l2t_get_option(h, L.L2T_OPT_KERNEL)
    ctx.close()
    fwd, adj = times[-1]
    # algorithmic bytes per atom-substep, 2 B per neighbour index in the brick
    # form and 4 B in the global-gather form.  Forward: hi and the 16-bit low
    # part read and written (12), T_lat (4), row offset (4).  Reverse: T hi (4),
    # lambda hi+lo read and write (16), T_lat (4), row offset (4).  The
    # recomputation runs the forward on all but one sub-step per checkpoint
    # (the global-gather form also copies the low part into the next state of
    # the segment, 4 B).
    per_nbr = 2.0 if kernel == 1 else 4.0
    fb = 20.0 + per_nbr * mean
    ab = (28.0 + per_nbr * mean) + (fb + (0.0 if kernel == 1 else 4.0)) * (ck - 1) / ck
    out = dict(workload=f"c5: {S} FCC systems of {w.systems[0].n} atoms, {n} FP32C sub-steps, "
                        f"checkpoint every {ck}",
               kernel=["global-gather", "lds-brick"][kernel], mean_neighbors=mean,
               forward_recorded_atom_substeps_per_s=N * n / fwd,
               adjoint_atom_substeps_per_s=N * n / adj,
               adjoint_over_forward=adj / fwd,
               forward_GBps=fb * N * n / fwd / 1e9,
               adjoint_GBps=ab * N * n / adj / 1e9,
               loss=float(np.mean((TN - tgt) ** 2)),
               dL_dK_sys0=float(dK[0]), dL_dg_sys0=float(dg[0]))
    out["adjoint_frac"] = out["adjoint_GBps"] / HBM_PEAK_GBS
    log(f"  adjoint: forward {fwd * 1e3:.1f} ms, adjoint {adj * 1e3:.1f} ms "
        f"({N} atoms x {n} sub-steps)")
    return out


def bench_bar_batch(L, torch, n_sub=30000):
    """Two-temperature bars of Section 3.1: 2048 periodic 141-node Ni bars,
    electrons by Eq. 2 and lattice by the three-point Fourier law, FP64, one
    launch per sub-step for the whole batch, 3 ps at dt = 0.1 fs."""
    import workloads as W
    w = W.c6(n_substeps=n_sub)
    ctx = new_context(L, w.systems, L.L2T_FP64)
    ctx.setup(w.r_cut)
    L.l2t_set_option(ctx.h, L.L2T_OPT_BATCH_FP64, 1)
    for s in range(len(w.systems)):
        L.l2t_set_lattice_fd(ctx.h, s, True, W.K_L_BAR, W.C_L_BAR)
    ctx.advance(100)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    ctx.advance(n_sub)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    nodes = sum(sy.n for sy in w.systems)
    ctx.close()
    log(f"  bars: {len(w.systems)} x {w.systems[0].n} nodes, {n_sub} sub-steps in {ms:.1f} ms")
    # algorithmic bytes per node-substep: T_e and T_lat read and written (32)
    # and two int32 neighbour indices (8)
    per = 40.0
    return dict(workload=f"c6: {len(w.systems)} two-temperature Ni bars of {w.systems[0].n} nodes, "
                         f"{n_sub} FP64 sub-steps (3 ps)",
                node_substeps_per_s=nodes * n_sub / (ms * 1e-3), substep_us=ms * 1e3 / n_sub,
                algorithmic_GBps=per * nodes * n_sub / (ms * 1e-3) / 1e9)


def copy_rate(torch, dev, reps=5):
    """STREAM-style copy of 1 GiB on the device (read + write bytes per second),
    the practical bandwidth denominator next to the 8 TB/s peak."""
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2.0 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbps


def bench_c3_fp64(L, torch, w, n_sub=100, kernel="auto"):
    """The same 4M-atom system in the plain FP64 form (one launch per
    sub-step): a bounded sample of sub-steps timed with HIP events, for the
    FP32C / FP64 ratio on this system.  kernel pins the FP64 launch form as
    --kernel does for FP32C."""
    sy = w.systems[0]
    ctx = new_context(L, w.systems, L.L2T_FP64, stream=torch.cuda.current_stream().cuda_stream)
    if kernel != "auto":
        L.l2t_set_option(ctx.h, L.L2T_OPT_KERNEL, 1 if kernel == "brick" else 0)
    _, mean, _ = ctx.setup(w.r_cut)
    ctx.advance(4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.advance(n_sub)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / n_sub
    log(f"  C3 FP64 plain: {us:.1f} us per sub-step")
    # per atom-substep: T read and write (16), T_lat (8), row offset (4), one
    # index per neighbour (2 B brick-local in k_brick_fp64, the form a launch
    # of this many bricks takes; 4 B in the global-gather k_step_fp64)
    brick = L.l2t_get_option(ctx.h, L.L2T_OPT_KERNEL) == 1
    ctx.close()
    bytes_per = 28.0 + (2.0 if brick else 4.0) * mean
    gbps = bytes_per * sy.n / (us * 1e-6) / 1e9
    return dict(substeps=n_sub, substep_us=us, atom_substeps_per_s=sy.n / (us * 1e-6),
                kernel="k_brick_fp64" if brick else "k_step_fp64",
                algorithmic_bytes_per_atom_substep=bytes_per,
                achieved_GBps=gbps, frac=gbps / HBM_PEAK_GBS,
                bound="vector work: one FP64 exponential and one division per pair of the literal pair term"
                      if brick else "latency of the neighbour gathers")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.partition(":")[2].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(L, torch, w, n_steps, checkpoints, n_single):
    """The FP64 oracle on the host cores: timed over the first n_steps
    sub-steps of the 4M-atom system on all OpenMP threads (the reported
    value) and over n_single sub-steps on one thread; then continued to each
    sub-step count in checkpoints, where the FP32C library's T_e (a fresh
    context advanced from the same initial state) is compared with it on
    every atom."""
    import oracle
    sy = w.systems[0]
    row, col = oracle.neighbors(sy.pos, sy.box_lo, sy.box_len, sy.periodic, w.r_cut)
    Tl, gated = oracle.lattice_temperature(row, col, sy.vel, sy.mass, sy.params["ke_eps"])
    cores = oracle.threads()
    single = None
    if n_single > 0:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.run(row, col, sy.T_e0, Tl, sy.params, n_single, gated=gated)
        dt1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        single = dict(value=sy.n * n_single / dt1, threads=1,
                      sample=f"{n_single} sub-steps ({dt1:.1f} s)")
        log(f"  oracle on one thread: {sy.n * n_single / dt1 / 1e6:.2f} M atom-substeps/s")
    t0 = time.perf_counter()
    T_ref, _, _ = oracle.run(row, col, sy.T_e0, Tl, sy.params, n_steps, gated=gated)
    dt = time.perf_counter() - t0
    ctx = new_context(L, w.systems, L.L2T_FP32C, stream=torch.cuda.current_stream().cuda_stream)
    ctx.setup(w.r_cut)
    parity = []
    step = 0
    for c in sorted(set([n_steps] + [c for c in checkpoints if c > n_steps])):
        if c > n_steps:
            T_ref, _, _ = oracle.run(row, col, T_ref, Tl, sy.params, c - max(step, n_steps),
                                     step0=max(step, n_steps), gated=gated)
        ctx.advance(c - step)
        step = c
        T = ctx.get(0)
        rel = np.abs(T - T_ref) / np.abs(T_ref)
        parity.append(dict(substeps=c, max_rel_err=float(rel.max()),
                           mean_rel_err=float(rel.mean()),
                           T_e_changed_max=float(np.max(np.abs(T_ref - sy.T_e0)))))
        log(f"  FP32C vs FP64 oracle after {c} sub-steps, all {sy.n} atoms: max rel "
            f"{rel.max():.2e}")
    ctx.close()
    return dict(value=sy.n * n_steps / dt, unit="atom-substeps/s", cores=cores, kind="oracle",
                cpu=cpu_model(), logical_cpus=os.cpu_count(),
                sample=f"FP64 oracle, same 4,000,000-atom system, {n_steps} sub-steps "
                       f"({dt:.1f} s) on {cores} OpenMP threads, neighbour build not timed",
                single_thread=single,
                fp32c_vs_oracle=dict(tolerance=1e-5, checkpoints=parity,
                                     max_rel_err=max(p["max_rel_err"] for p in parity)))


def make_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--substeps", type=int, default=10000)
    ap.add_argument("--cells", type=int, default=100)
    ap.add_argument("--c4-substeps", type=int, default=600)
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=200,
                    help="oracle sub-steps timed on all host threads")
    ap.add_argument("--cpu-checkpoints", type=str, default="500,1000",
                    help="further sub-step counts at which every atom is compared with the oracle")
    ap.add_argument("--cpu-single-steps", type=int, default=5,
                    help="oracle sub-steps timed on one thread (0 = skip)")
    ap.add_argument("--c4-full-substeps", type=int, default=6000)
    ap.add_argument("--c4-fp32c-only", action="store_true",
                    help="C4: time the batched FP32C form alone (profiling; no speedup)")
    ap.add_argument("--table-stream", type=int, choices=[0, 1, 2], default=0,
                    help="table loads of the FP32C brick kernels: 0 = measured at the build, "
                         "1 = cached, 2 = streamed (every FP32C context; counter passes)")
    ap.add_argument("--sweep", type=int, choices=[0, 1, 2], default=0,
                    help="brick order of the FP32C brick kernels: 0 = measured at the build, "
                         "1 = fixed, 2 = reversed every other sub-step (every FP32C context)")
    ap.add_argument("--graph", type=int, choices=[0, 1], default=None,
                    help="0 = launch sub-steps directly (rocprofv3 counter passes), 1 = replay "
                         "captured hipGraphs (default: the FP32C autotuner times both)")
    ap.add_argument("--only", choices=["all", "c3", "c4", "md", "bars", "adjoint", "fp64",
                                       "shard"],
                    default="all", help="run one section only (profiling)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-shard", action="store_true",
                    help="skip the per-GPU share of the 4M-atom system over 2, 4, 8 GPUs")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 sample on the 4M-atom system")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the recorded forward and adjoint timing")
    ap.add_argument("--no-md", action="store_true", help="skip the lattice-side (Eq. 5, 8) timing")
    ap.add_argument("--kernel", choices=["auto", "global", "brick"], default="auto",
                    help="pin the sub-step launch form (every FP32C context and the FP64 sample)")
    ap.add_argument("--brick-edge", type=int, default=0,
                    help="brick edge in cells of every FP32C context (0 = measured at the build)")
    ap.add_argument("--block", type=int, default=0,
                    help="threads per workgroup of the FP32C sub-step kernel (0 = autotuned)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration)")
    return ap


def main():
    args = make_parser().parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; splitting the systems over "
                                   "several GPUs is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1810_12357_amd import l2t as L
    global GRAPH
    GRAPH = args.graph
    if args.brick_edge:
        FP32C_PINS.append((L.L2T_OPT_BRICK_EDGE, args.brick_edge))
    if args.kernel != "auto":
        FP32C_PINS.append((L.L2T_OPT_KERNEL, 1 if args.kernel == "brick" else 0))
    if args.block:
        FP32C_PINS.append((L.L2T_OPT_BLOCK, args.block))
    if args.sweep:
        FP32C_PINS.append((L.L2T_OPT_SWEEP, args.sweep))
    if args.table_stream:
        FP32C_PINS.append((L.L2T_OPT_TABLE_STREAM, args.table_stream))

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)     # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "copies": 3}))
        return
    w = W.c3(n_cells=args.cells, n_substeps=args.substeps)
    sy = w.systems[0]
    want = lambda sec: args.only in ("all", sec)
    out = {}
    if want("c3") or want("md"):
        log(f"C3: {sy.n} atoms, r_c = {w.r_cut:.4f} A, {args.substeps} sub-steps per step")
        ctx = new_context(L, w.systems, L.L2T_FP32C,
                          stream=torch.cuda.current_stream().cuda_stream)
        h = ctx.h
        d = setup_system(L, h, sy, dev)
        torch.cuda.synchronize()
        timer = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        if not want("c3"):
            one_pass(L, h, sy, d, w.r_cut, 1, timer)
    if want("c3"):
        for k in range(args.warmup):
            one_pass(L, h, sy, d, w.r_cut, args.substeps, timer)
            log(f"warm-up {k + 1}/{args.warmup} done")
        torch.cuda.synchronize()
        adv_ms = []
        t0 = time.perf_counter()
        for k in range(args.steps):
            e = one_pass(L, h, sy, d, w.r_cut, args.substeps, timer)
            torch.cuda.synchronize()
            adv_ms.append(timer[0].elapsed_time(timer[1]))
            log(f"step {k + 1}/{args.steps}: advance {adv_ms[-1]:.1f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n_atom_steps = sy.n * args.substeps * args.steps
        value = n_atom_steps / wall
        mx, mean = e["max_nbrs"], e["mean_nbrs"]
        persistent = L.l2t_get_option(h, L.L2T_OPT_PERSISTENT)
        block = L.l2t_get_option(h, L.L2T_OPT_BLOCK)
        kernel = L.l2t_get_option(h, L.L2T_OPT_KERNEL)
        adv = float(np.mean(adv_ms))
        # algorithmic bytes per atom-substep: hi and its 16-bit low part read
        # and written (12), T_lat (4), row offset (4) and one index per
        # neighbour (4 B global, 2 B brick-local)
        bytes_per = 20.0 + (2.0 if kernel == 1 else 4.0) * mean
        if kernel == 1:
            launch_ms, units, kname = adv / args.substeps, sy.n, "k_brick_fp32c"
        elif persistent:
            launch_ms, units, kname = adv, sy.n * args.substeps, "k_persistent_fp32c"
        else:
            launch_ms, units, kname = adv / args.substeps, sy.n, "k_step_fp32c"
        achieved = bytes_per * units / (launch_ms * 1e-3) / 1e9
        traffic = measured_traffic(kname, sy.n) if units == sy.n else None
        copy_gbps = copy_rate(torch, dev)
        roof = dict(bound="hbm", kernel=kname, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                    traffic_unit="bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                 "copy-calibrated)",
                    algorithmic_bytes_per_atom_substep=bytes_per,
                    launch_ms=launch_ms, units_per_launch=units,
                    # measured HBM bytes over the live launch time (the gate's reading)
                    measured_GBps=None if traffic is None else traffic / (launch_ms * 1e-3) / 1e9,
                    measured_frac=None if traffic is None else
                    traffic / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    # a 1 GiB device copy on the same GPU: the practical denominator
                    copy_GBps=copy_gbps, frac_of_copy=achieved / copy_gbps)
        # value: the atom-substeps/s half of the metric; the batched-FP32C over
        # plain-FP64 speedup half is c4_speedup.speedup
        out = dict(metric="electron atom-substeps/s, 4M-atom FCC; batched FP32 vs plain FP64 "
                          "speedup",
                   value=value,
                   unit="atom-substeps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                   ms_per_step=wall / args.steps * 1e3, higher_is_better=True, scaling="weak",
                   vs_baseline=None, dtype="f32", data="synthetic",
                   config=dict(workload=f"c3: FCC {args.cells}^3 cells ({sy.n} atoms), jittered "
                                        f"0.05 A, r_c 1.2a, {args.substeps} FP32C sub-steps per "
                                        f"step",
                               n_atoms=sy.n, substeps=args.substeps, mean_neighbors=mean,
                               max_neighbors=mx, kernel=["global-gather", "lds-brick"][kernel],
                               brick_edge=L.l2t_get_option(h, L.L2T_OPT_BRICK_EDGE),
                               sweep=["fixed", "alternating"][
                                   L.l2t_get_option(h, L.L2T_OPT_SWEEP) - 1],
                               table_loads=["cached", "streamed"][
                                   L.l2t_get_option(h, L.L2T_OPT_TABLE_STREAM) - 1],
                               launches=["direct", "graph replays"][
                                   L.l2t_get_option(h, L.L2T_OPT_GRAPH)],
                               persistent=persistent, block=block),
                   advance_only_atom_substeps_per_s=sy.n * args.substeps / (adv * 1e-3),
                   advance_ms_median=float(np.median(adv_ms)),
                   roofline=roof,
                   energy=dict(E_e=e["E_e"], sum_T=e["sum_T"],
                               T_ledger=e["sum_T"] + e["T_ledger_acc"], T_max=e["T_max_atom"]))
    if want("md") and not args.no_md:
        log("MD coupling (Eq. 5, Eq. 8) ...")
        out["md_coupling"] = bench_md_coupling(L, torch, h, sy, d)
        log("held atoms and mean-field refresh ...")
        out["boundary_mean_field"] = bench_boundary_mean_field(L, torch, h, sy)
    if want("c3") or want("md"):
        ctx.close()
    if want("fp64") and not args.no_fp64:
        log("C3 in plain FP64 ...")
        f64 = bench_c3_fp64(L, torch, w, kernel=args.kernel)
        if "advance_only_atom_substeps_per_s" in out:
            f64["fp32c_over_fp64"] = (out["advance_only_atom_substeps_per_s"] /
                                      f64["atom_substeps_per_s"])
        out["c3_fp64"] = f64
    if want("c4") and not args.no_c4:
        log("C4 batched vs plain ...")
        out["c4_speedup"] = bench_c4_speedup(L, torch, args.c4_substeps, args.c4_full_substeps,
                                             only_fp32c=args.c4_fp32c_only)
    if want("shard") and not args.no_shard:
        log("one GPU's share of the 4M-atom system over N GPUs ...")
        out["c3_shard"] = bench_shard(L, torch, w)
    if want("bars") and not args.no_md:
        log("two-temperature bars (Section 3.1) ...")
        out["bar_batch"] = bench_bar_batch(L, torch)
    if want("adjoint") and not args.no_adjoint:
        log("adjoint (differentiation workload) ...")
        out["adjoint"] = bench_adjoint(L, torch)
    if args.only == "all" and not args.no_cpu:
        log("CPU oracle baseline ...")
        cps = [int(c) for c in args.cpu_checkpoints.split(",") if c.strip()]
        out["cpu_baseline"] = cpu_baseline(L, torch, w, args.cpu_steps, cps,
                                           args.cpu_single_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
