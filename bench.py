#!/usr/bin/env python
"""Benchmark of the P3MaZe long-range mesh step on one MI355X.

python bench.py [--steps K] [--warmup W] [--workload water-3000|nacl-batch64|...] [--gpus 1]

One "step" is one velocity-Verlet MD step that drives one mesh step (bin,
spread, smoothing, warm-started multigrid constraint solve, field update,
gather) plus the short-range pairs and the non-electrostatic terms.  The
default workload is the largest single-GPU system (7,999,998 atoms, 512^3
mesh, order 5).  The headline value is the mesh-step time per atom (spread +
smoothing + solve + gather, from HIP events around those stages) in the
mixed32 mode (FP32 charge source and V-cycle; FP64 sigma_p, outer residual,
projections, coarsest solve and updates); the mixed (FP64 charge source) and
plain FP64 modes are measured the same way and reported beside it.  Inputs
are seeded synthetic systems generated on the host and resident in HBM
before the timed region.

Extra fields of the JSON line:
  roofline      the dominant kernel family's algorithmic bytes per launch over
                its average launch duration (HIP events around each of its
                finest-level launches in MD steps of the same run, launched
                kernel by kernel), against the 8 TB/s HBM peak; plus the
                whole mesh step's and the multigrid sweeps' fractions
  cpu_baseline  the CPU FP64 oracle timed on this host on a bounded sample
                (first mesh steps along the initial velocities)
  parity        both GPU modes against the oracle on that sample
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "mesh-step ns/atom (spread+MG+gather) & HBM GB/s vs roofline, mixed vs FP64"


T0 = time.perf_counter()
PHASES = {}   # wall seconds of each part of the run, for the time budget


def log(*a):
    print(f"[{time.perf_counter() - T0:7.1f}s]", *a, file=sys.stderr, flush=True)


def phase(name, t_start):
    PHASES[name] = round(PHASES.get(name, 0.0) + time.perf_counter() - t_start, 2)


def md_terms(P, kind):
    t = P.p3mz_mdterms()
    t.force_to_acc = 1.0 / 103.6427
    t.mv2_to_energy = 103.6427
    if kind == "nacl":
        t.model, t.bm_a, t.bm_rho = 1, 4000.0, 0.317
    else:
        kc = 0.0433641
        t.model = 2
        t.lj_eps, t.lj_sigma = 0.1554253 * kc, 3.165492
        t.k_bond, t.r0 = 1059.162 * kc, 1.012
        t.k_angle, t.theta0 = 75.90 * kc, math.radians(113.24)
    return t


def make_params(P, w, precision):
    return P.make_params(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, predictor=w.predictor,
                         precision=precision, coulomb_k=14.3996454784, nu_pre=2, nu_post=2,
                         excl_group=w.excl_group)


def source_digest() -> str:
    """SHA-256 over the HIP sources: a changed kernel invalidates stored counters."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_31379_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, mode):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary for this workload (FETCH_SIZE and WRITE_SIZE passes, each scaled
    by the same counter's reading for a copy of known size), or None when
    there is no summary or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}_{mode}.md")
    if not os.path.exists(path):
        return None, f"no counter summary {os.path.relpath(path, ROOT)}"
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ln.startswith("- ") and ": " in ln:
                k, v = ln[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != source_digest():
        return None, f"{os.path.relpath(path, ROOT)} predates the current kernels"
    return float(vals["hbm_bytes_per_launch"]), os.path.relpath(path, ROOT)


def mg_sweep_roofline(fam):
    """Bandwidth of the finest-level multigrid sweep kernels together
    (red-black half-sweeps, the first sweep from zero, fused legs)."""
    ms = sum(fam[k]["avg_active_launch_us"] * fam[k]["active_launches"] for k in
             ("halfsweep", "sweep0", "fused_down", "fused_up") if fam.get(k) and fam[k]["active_launches"])
    by = sum(fam[k]["bytes_per_active_launch"] * fam[k]["active_launches"] for k in
             ("halfsweep", "sweep0", "fused_down", "fused_up") if fam.get(k) and fam[k]["active_launches"])
    if ms <= 0:
        return None
    gbps = by / (ms * 1e-6) / 1e9
    return dict(achieved=gbps, frac=gbps / HBM_PEAK_GBPS, kernels="halfsweep+sweep0+fused legs, finest level")


def copy_ceiling_gbps(torch, nbytes=1 << 30, reps=10):
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def autotune_schedule(torch, P, w, system, precision, warmup, n_frames=8):
    """Autotuner run: after `warmup` MD steps, the next `n_frames` MD
    positions are the tuning frames; every candidate schedule restarts from
    the history at the start of those frames."""
    import numpy as np
    dev = torch.device("cuda")
    ctx = P.p3mz_create(make_params(P, w, precision), system.charges)
    try:
        pos = torch.from_numpy(np.ascontiguousarray(system.pos)).to(dev)
        vel = torch.from_numpy(np.ascontiguousarray(system.vel)).to(dev)
        mass = torch.from_numpy(np.ascontiguousarray(system.masses)).to(dev)
        terms = md_terms(P, w.kind)
        stream = torch.cuda.current_stream().cuda_stream
        P.p3mz_md_run(ctx, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), terms, w.dt_fs, max(warmup, 4), None,
                      None, stream)
        blob = P.p3mz_save_state(ctx)
        frames = torch.zeros((n_frames, system.n, 3), dtype=torch.float64, device=dev)
        for k in range(n_frames):
            P.p3mz_md_run(ctx, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), terms, w.dt_fs, 1, None, None,
                          stream)
            frames[k].copy_(pos)
        P.p3mz_load_state(ctx, blob)
        r = P.p3mz_autotune(ctx, frames.data_ptr(), n_frames, stream)
        cands = [dict(nu_pre=r.cand_nu_pre[k], nu_post=r.cand_nu_post[k], ms=r.cand_ms[k],
                      cycles=r.cand_cycles[k], ms_cycle=r.cand_ms_cycle[k], cycles_frac=r.cand_cycles_frac[k],
                      expected_ms=r.cand_expected_ms[k]) for k in range(r.n_candidates)]
        return dict(nu_pre=r.nu_pre, nu_post=r.nu_post, smooth_tile=r.smooth_tile, ms_best=r.ms_best,
                    ms_default=r.ms_default, ms_smooth=r.ms_smooth, frames=n_frames, candidates=cands)
    finally:
        P.p3mz_destroy(ctx)


K_B_EV = 8.617333262e-5   # Boltzmann constant, eV/K


def run_mode(torch, P, w, system, precision, warmup, steps, kernel, schedule=None, skin=None, gamma=None):
    """Warm up, pick the dominant kernel family, then time `steps` MD steps."""
    import numpy as np
    dev = torch.device("cuda")
    ctx = P.p3mz_create(make_params(P, w, precision), system.charges)
    try:
        if skin is not None:
            P.p3mz_set_neighbor_list(ctx, skin)
        if gamma:
            P.p3mz_set_thermostat(ctx, gamma, K_B_EV * w.temp_k, w.seed)
        if schedule:
            P.p3mz_set_schedule(ctx, schedule["nu_pre"], schedule["nu_post"], schedule["smooth_tile"])
        pos = torch.from_numpy(np.ascontiguousarray(system.pos)).to(dev)
        vel = torch.from_numpy(np.ascontiguousarray(system.vel)).to(dev)
        mass = torch.from_numpy(np.ascontiguousarray(system.masses)).to(dev)
        elog = torch.zeros((max(steps, 1), 6), dtype=torch.float64, device=dev)
        clog = torch.zeros(max(steps, 1), dtype=torch.int32, device=dev)
        terms = md_terms(P, w.kind)
        stream = torch.cuda.current_stream().cuda_stream
        dt = w.dt_fs

        def md(n, with_logs=False, offset=0):
            for k in range(n):
                P.p3mz_md_run(ctx, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), terms, dt, 1,
                              elog[offset + k].data_ptr() if with_logs else None,
                              clog[offset + k].data_ptr() if with_logs else None, stream)

        md(warmup)
        # Per-family kernel time: `probe` MD steps launched kernel by kernel
        # with HIP events around every finest-level launch of one family (on
        # the library's stream).  Launches that found the solve converged (a
        # speculative cycle beyond the step's count, a field update enqueued
        # before the last cycle) return at once; they are counted apart as
        # idle (below a quarter of the family's longest launch).
        shares, fam = {}, {}
        P.p3mz_set_timing(ctx, True)
        probe = max(2, min(5, steps))
        for name, kid in P.KERNELS.items():
            P.p3mz_set_kernel_timer(ctx, kid)
            md(probe)
            ms_l, by_l = P.p3mz_get_kernel_launches(ctx)
            shares[name] = sum(ms_l) / probe
            top = max(ms_l) if ms_l else 0.0
            act = [(m, b) for m, b in zip(ms_l, by_l) if m >= 0.25 * top and m > 0]
            a_ms = sum(m for m, _ in act)
            a_by = sum(b for _, b in act)
            fam[name] = dict(ms_per_step=shares[name], launches=len(ms_l), active_launches=len(act),
                             avg_active_launch_us=1e3 * a_ms / len(act) if act else None,
                             bytes_per_active_launch=a_by / len(act) if act else None,
                             active_bytes_per_step=a_by / probe,
                             gbps=a_by / (a_ms * 1e-3) / 1e9 if a_ms > 0 else None)
        P.p3mz_set_kernel_timer(ctx, -1)
        # the dominant family of the mesh step (the short-range pair kernel is
        # outside the measured metric), by its share of the step
        mesh_shares = {k: v for k, v in shares.items() if k != "sr"}
        dominant = kernel if kernel != "auto" else max(mesh_shares, key=mesh_shares.get)
        log(f"[{('fp64', 'mixed', 'mixed32')[precision]}] kernel ms/step: "
            + ", ".join(f"{k}={v:.4f}" for k, v in sorted(shares.items(), key=lambda x: -x[1])))
        P.p3mz_set_kernel_timer(ctx, -1)      # the headline region runs with captured graphs
        mesh_ms_tot, sr_ms_tot, graphs = 0.0, 0.0, 1
        builds0 = P.p3mz_get_neighbor_stats(ctx)[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            md(1, with_logs=True, offset=k)
            st = P.p3mz_get_stats(ctx)
            mesh_ms_tot += st.ms_mesh
            sr_ms_tot += st.ms_short_range
            graphs &= st.graphs
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        builds, over, cap = P.p3mz_get_neighbor_stats(ctx)
        cycles = clog.cpu().numpy()[:steps]
        energies = elog.cpu().numpy()[:steps]
        # Back-to-back launches of the dominant family's finest-level kernel
        # on the live buffers of the last timed step (a cross-check of the
        # in-step durations above).
        burst_ok = dominant in ("halfsweep", "sweep0", "restrict", "prolong", "tail", "fused_down", "fused_up",
                                "smooth", "outer", "sigma",
                                "spread", "gather")
        reps = 20 if system.n > 1_000_000 else 200
        bms, _ = P.p3mz_kernel_bench(ctx, P.KERNELS[dominant], reps, stream) if burst_ok else (float("nan"), 0.0)
        mesh_ms = mesh_ms_tot / steps
        d = fam[dominant]
        step_bytes = sum(f["active_bytes_per_step"] for k, f in fam.items() if k != "sr")
        out = dict(
            ns_per_atom=mesh_ms * 1e6 / system.n,
            mesh_ms_per_step=mesh_ms,
            md_ms_per_step=wall * 1e3 / steps,
            short_range_ms_per_step=sr_ms_tot / steps, graphs=bool(graphs),
            neighbor_lists=dict(capacity=cap, builds_per_step=(builds - builds0) / steps, over_capacity_atoms=over),
            kinetic_temperature_k=[float(2.0 * e / (3.0 * system.n * K_B_EV)) for e in
                                   (energies[0, 4], energies[-1, 4])] if steps > 0 else None,
            thermostat=dict(gamma_per_fs=gamma, kt_ev=K_B_EV * w.temp_k) if gamma else None,
            vcycles_per_step=float(cycles.mean()), vcycles_min=int(cycles.min()), vcycles_max=int(cycles.max()),
            energy_drift_per_step=float(np.polyfit(np.arange(steps), energies[:, 5], 1)[0]) if steps > 2 else None,
            kernel_ms_per_step=shares, kernel_families=fam, dominant=dominant,
            dominant_share=shares[dominant] / max(sum(mesh_shares.values()), 1e-12),
            dominant_avg_launch_us=d["avg_active_launch_us"], dominant_launches=d["active_launches"],
            dominant_idle_launches=d["launches"] - d["active_launches"],
            dominant_bytes_per_launch=d["bytes_per_active_launch"], dominant_gbps=d["gbps"],
            dominant_burst_avg_launch_us=bms * 1e3 if burst_ok else None,
            # finest-level algorithmic bytes of every mesh kernel per step over
            # the mesh-step time (coarse levels add at most 1/7 of the V-cycle's)
            whole_step=dict(finest_level_bytes=step_bytes, mesh_ms=mesh_ms,
                            gbps=step_bytes / (mesh_ms * 1e-3) / 1e9,
                            frac=step_bytes / (mesh_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS),
            schedule=dict(nu_pre=P.p3mz_get_stats(ctx).nu_pre, nu_post=P.p3mz_get_stats(ctx).nu_post,
                          smooth_tile=schedule["smooth_tile"] if schedule else 0),
        )
        return out
    finally:
        P.p3mz_destroy(ctx)


def oracle_sample(w, system, traj, nu_pre, nu_post, targets, min_time_s=0.0, max_reps=200):
    """Oracle forces and cycle counts on `traj` (a cold step, then warm
    steps); with min_time_s the sequence is run again from a cold start
    (timing only) until the warm mesh steps add up to that many seconds, so
    the timed steps keep the sample's mix of V-cycle counts."""
    import numpy as np
    from oracle import oracle as O
    op = O.make_params(w.box, w.alpha, w.r_cut, w.mesh, w.order, tol=w.tol, predictor=w.predictor,
                       coulomb_k=14.3996454784, nu_pre=nu_pre, nu_post=nu_post, excl_group=w.excl_group)
    ref, cyc_ref, t_mesh = [], [], []
    rep = 0
    while rep == 0 or (sum(t_mesh) < min_time_s and rep < max_reps):
        orc = O.Oracle(op, system.charges)
        if targets is not None:
            orc.set_sr_targets(targets)
        for k, x in enumerate(traj):
            f, e, _ = orc.compute(x)
            st = orc.stats()
            if rep == 0:
                ref.append(f if targets is None else f[targets])
                cyc_ref.append(st.cycles)
                log(f"[oracle nu=({nu_pre},{nu_post})] step {k} cycles={st.cycles} "
                    f"mesh_s={st.t_spread + st.t_solve + st.t_gather:.3f}")
            if k > 0:
                t_mesh.append(st.t_spread + st.t_solve + st.t_gather)
        orc.close()
        rep += 1
    return ref, cyc_ref, t_mesh


def parity_and_baseline(torch, P, w, system, sample_steps, schedules):
    """Oracle on a bounded sample (cold solve + warm steps along the initial
    velocities) with each mode's V-cycle schedule, the GPU modes on the same
    positions, and the oracle's time (with the headline mode's schedule)."""
    import numpy as np
    traj = [system.pos + k * w.dt_fs * system.vel for k in range(sample_steps)]
    # large systems: the oracle's all-pairs short-range sum only for a seeded
    # sample of atoms, forces compared on that sample
    targets = None
    if system.n > 20000:
        rng = np.random.Generator(np.random.PCG64(w.seed + 17))
        targets = np.sort(rng.choice(system.n, size=1000 if system.n > 2_000_000 else 512, replace=False))
    runs = {}
    out = {}
    dev = torch.device("cuda")
    head = schedules.get("mixed32") or schedules.get("mixed") or schedules.get("fp64")
    head_key = (head["nu_pre"], head["nu_post"])
    for precision, name in ((0, "fp64"), (1, "mixed"), (2, "mixed32")):
        sch = schedules.get(name)
        if sch is None:
            continue
        key = (sch["nu_pre"], sch["nu_post"])
        if key not in runs:
            # the headline schedule's run also times the oracle: at least
            # ~10 s of warm mesh steps
            runs[key] = oracle_sample(w, system, traj, *key, targets, min_time_s=10.0 if key == head_key else 0.0)
        ref, cyc_ref, t_mesh = runs[key]
        ctx = P.p3mz_create(make_params(P, w, precision), system.charges)
        try:
            P.p3mz_set_schedule(ctx, sch["nu_pre"], sch["nu_post"], sch["smooth_tile"])
            pos = torch.zeros((system.n, 3), dtype=torch.float64, device=dev)
            frc = torch.zeros_like(pos)
            errs, cyc = [], []
            for k, x in enumerate(traj):
                pos.copy_(torch.from_numpy(np.ascontiguousarray(x)))
                P.p3mz_compute(ctx, pos.data_ptr(), frc.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
                torch.cuda.synchronize()
                fg = frc.cpu().numpy()
                if targets is not None:
                    fg = fg[targets]
                errs.append(float(np.sqrt(((fg - ref[k]) ** 2).sum() / (ref[k] ** 2).sum())))
                cyc.append(P.p3mz_get_stats(ctx).cycles)
            out[name] = dict(max_rel_rms_force_err=max(errs), vcycles_gpu=cyc, vcycles_oracle=cyc_ref,
                             vcycles_equal=cyc == cyc_ref, schedule=[sch["nu_pre"], sch["nu_post"]],
                             force_atoms="all" if targets is None else f"{len(targets)} seeded atoms")
        finally:
            P.p3mz_destroy(ctx)
    t_mesh = runs[head_key][2]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    mean_s = float(np.mean(t_mesh)) if t_mesh else float("nan")
    baseline = dict(value=mean_s * 1e9 / system.n, unit="ns/atom/step", cores=cores, kind="oracle",
                    sample=f"{len(t_mesh)} warm mesh steps of {w.name} ({sum(t_mesh):.1f} s of oracle time): "
                           f"{sample_steps}-step runs along the initial velocities (dt {w.dt_fs} fs), each from a "
                           f"cold step that is not timed, repeated to at least 10 s, V-cycle schedule "
                           f"({head['nu_pre']},{head['nu_post']}); spread+smoothing+solve+gather only")
    return out, baseline


def batch_params(P, w, r, precision):
    return P.make_params(r.box, w.alpha, w.r_cut, r.mesh, w.order, tol=w.tol, predictor=w.predictor,
                         precision=precision, coulomb_k=14.3996454784, nu_pre=2, nu_post=2)


def run_batch_mode(torch, P, w, systems, precision, warmup, steps):
    """All replicas advanced together: each MD step is one batched step
    (every kernel launched once for all replicas, captured in graphs)."""
    import numpy as np
    dev = torch.device("cuda")
    n = [s.n for s in systems]
    b = P.p3mz_batch_create([batch_params(P, w, r, precision) for r in w.replicas], n,
                            np.ascontiguousarray(np.concatenate([s.charges for s in systems])))
    try:
        cat = lambda key: torch.from_numpy(np.ascontiguousarray(np.concatenate([getattr(s, key) for s in systems]))).to(dev)
        pos, vel, mass = cat("pos"), cat("vel"), cat("masses")
        terms = md_terms(P, "nacl")
        stream = torch.cuda.current_stream().cuda_stream
        clog = torch.zeros((len(n), 1), dtype=torch.int32, device=dev)

        def step():
            P.p3mz_batch_md_run(b, pos.data_ptr(), vel.data_ptr(), mass.data_ptr(), terms, w.dt_fs, 1, None,
                                clog.data_ptr(), stream)

        for _ in range(warmup):
            step()
        P.p3mz_batch_set_timing(b, True)
        mesh_ms, sr_ms, graphs, cyc = 0.0, 0.0, 1, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
            m, sr, g = P.p3mz_batch_get_timing(b)
            mesh_ms += m
            sr_ms += sr
            graphs &= g
            cyc.append(clog[:, 0].cpu().numpy().copy())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        P.p3mz_batch_set_timing(b, False)
        reps = 100
        kms, kbytes = P.p3mz_batch_kernel_bench(b, P.KERNELS["halfsweep"], reps, stream)
        # the same half-sweeps in one persistent launch with per-system device barriers
        pms, _ = P.p3mz_batch_kernel_bench(b, P.PERSIST_HALFSWEEP, reps, stream)
        cyc = np.array(cyc)
        total = sum(n)
        return dict(ns_per_atom=mesh_ms / steps * 1e6 / total, mesh_ms_per_step=mesh_ms / steps,
                    md_ms_per_step=wall * 1e3 / steps, short_range_ms_per_step=sr_ms / steps, graphs=bool(graphs),
                    vcycles_mean=float(cyc.mean()), vcycles_max_per_step=float(cyc.max(axis=1).mean()),
                    dominant="halfsweep", dominant_avg_launch_us=kms * 1e3, dominant_launches=reps,
                    dominant_bytes_per_launch=kbytes, dominant_gbps=kbytes / (kms * 1e-3) / 1e9,
                    persistent_halfsweep_us=pms * 1e3, persistent_halfsweep_gbps=kbytes / (pms * 1e-3) / 1e9)
    finally:
        P.p3mz_batch_destroy(b)


def run_unbatched(torch, P, w, systems, precision, warmup, steps):
    """The same replicas one context each, stepped one after another."""
    import numpy as np
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    terms = md_terms(P, "nacl")
    ctxs, bufs = [], []
    try:
        for r, s in zip(w.replicas, systems):
            ctxs.append(P.p3mz_create(batch_params(P, w, r, precision), s.charges))
            P.p3mz_set_timing(ctxs[-1], True)
            bufs.append([torch.from_numpy(np.ascontiguousarray(getattr(s, k))).to(dev) for k in ("pos", "vel", "masses")])
        def step():
            ms = 0.0
            for h, (p_, v_, m_) in zip(ctxs, bufs):
                P.p3mz_md_run(h, p_.data_ptr(), v_.data_ptr(), m_.data_ptr(), terms, w.dt_fs, 1, None, None, stream)
                ms += P.p3mz_get_stats(h).ms_mesh
            return ms
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mesh_ms = sum(step() for _ in range(steps))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        total = sum(s.n for s in systems)
        return dict(ns_per_atom=mesh_ms / steps * 1e6 / total, mesh_ms_per_step=mesh_ms / steps,
                    md_ms_per_step=wall * 1e3 / steps)
    finally:
        for h in ctxs:
            P.p3mz_destroy(h)


def batch_parity_and_baseline(torch, P, w, systems, sample_atoms=64):
    """Every replica: cold step + one warm step along its velocities on the
    oracle (pair term only for `sample_atoms` seeded atoms per replica, so the
    all-pairs sum stays bounded) and through the batched GPU path; forces
    compared on the sampled atoms, V-cycle counts on every replica.  The
    oracle's warm mesh-step time over all replicas is the CPU baseline."""
    import numpy as np
    from oracle import oracle as O
    rng = np.random.Generator(np.random.PCG64(77))
    dev = torch.device("cuda")
    n = [s.n for s in systems]
    trajs = [[s.pos, s.pos + w.dt_fs * s.vel] for s in systems]
    targets = [np.sort(rng.choice(s.n, size=min(sample_atoms, s.n), replace=False)) for s in systems]
    ref, cyc_ref, t_mesh = [], [], 0.0
    for r, s, tr, tg in zip(w.replicas, systems, trajs, targets):
        o = O.Oracle(O.make_params(r.box, w.alpha, w.r_cut, r.mesh, w.order, tol=w.tol, predictor=w.predictor,
                                   coulomb_k=14.3996454784, nu_pre=2, nu_post=2), s.charges)
        o.set_sr_targets(tg)
        fr, cr = [], []
        for k, x in enumerate(tr):
            f, _, _ = o.compute(x)
            st = o.stats()
            fr.append(f[tg])
            cr.append(st.cycles)
            if k == 1:
                t_mesh += st.t_spread + st.t_solve + st.t_gather
        o.close()
        ref.append(fr)
        cyc_ref.append(cr)
    log(f"[oracle] {len(systems)} replicas, warm mesh step total {t_mesh:.3f} s")
    out = {}
    for precision, name in ((0, "fp64"), (1, "mixed")):
        b = P.p3mz_batch_create([batch_params(P, w, r, precision) for r in w.replicas], n,
                                np.ascontiguousarray(np.concatenate([s.charges for s in systems])))
        try:
            pos = torch.zeros((sum(n), 3), dtype=torch.float64, device=dev)
            frc = torch.zeros_like(pos)
            errs, equal = [], True
            for k in range(2):
                pos.copy_(torch.from_numpy(np.ascontiguousarray(np.concatenate([tr[k] for tr in trajs]))))
                P.p3mz_batch_compute(b, pos.data_ptr(), frc.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
                torch.cuda.synchronize()
                fg = frc.cpu().numpy()
                off = 0
                for i, s in enumerate(systems):
                    a, rf = fg[off:off + s.n][targets[i]], ref[i][k]
                    errs.append(float(np.sqrt(((a - rf) ** 2).sum() / (rf ** 2).sum())))
                    equal &= P.p3mz_batch_get_stats(b, i).cycles == cyc_ref[i][k]
                    off += s.n
            out[name] = dict(max_rel_rms_force_err=max(errs), vcycles_equal=bool(equal),
                             sampled_atoms_per_replica=sample_atoms)
        finally:
            P.p3mz_batch_destroy(b)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    baseline = dict(value=t_mesh * 1e9 / sum(n), unit="ns/atom/step", cores=cores, kind="oracle",
                    sample=f"one warm mesh step (after the cold solve) of each of the {len(systems)} replicas, "
                           f"one after another; spread+smoothing+solve+gather only")
    return out, baseline


def main_batch(args, torch, P, w):
    import numpy as np
    log(f"workload {w.name}: generating {len(w.replicas)} replicas")
    systems = w.systems()
    log(f"atoms {sum(s.n for s in systems)}; meshes " +
        ", ".join(f"{m}^3 x{sum(r.mesh == m for r in w.replicas)}" for m in sorted({r.mesh for r in w.replicas})))
    ceiling = copy_ceiling_gbps(torch)
    res = {}
    for precision, name in ((0, "fp64"), (1, "mixed")):
        if name not in args.modes.split(","):
            continue
        res[name] = run_batch_mode(torch, P, w, systems, precision, args.warmup, args.steps)
        log(f"[batch {name}] {json.dumps(res[name])}")
    unb = run_unbatched(torch, P, w, systems, 1, 2, max(3, min(args.steps, 10)))
    log(f"[unbatched mixed] {json.dumps(unb)}")
    parity, baseline = None, None
    if not args.no_cpu_baseline:
        parity, baseline = batch_parity_and_baseline(torch, P, w, systems)
    m, f = res.get("mixed"), res.get("fp64")
    head = m if m is not None else f
    traffic, traffic_note = measured_traffic("halfsweep", w.name, "mixed" if m is not None else "fp64")
    roof = dict(bound="hbm", kernel="halfsweep (one batched launch over every replica's finest level)",
                achieved=head["dominant_gbps"], peak=HBM_PEAK_GBPS, unit="GB/s",
                frac=head["dominant_gbps"] / HBM_PEAK_GBPS, traffic=traffic,
                traffic_source=traffic_note,
                avg_launch_us=head["dominant_avg_launch_us"], alg_bytes_per_launch=head["dominant_bytes_per_launch"],
                launches=head["dominant_launches"], copy_ceiling_GBps=ceiling)
    line = dict(
        metric=METRIC, value=head["ns_per_atom"], unit="ns/atom/step", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=head["md_ms_per_step"], higher_is_better=False, scaling="weak",
        vs_baseline=None, dtype="f32+f64" if m is not None else "f64", data="synthetic",
        config=dict(workload=w.name, n_systems=len(systems), n_atoms=sum(s.n for s in systems), order=w.order,
                    alpha=w.alpha, r_cut=w.r_cut, tol=w.tol, predictor=w.predictor, dt_fs=w.dt_fs,
                    meshes=sorted({r.mesh for r in w.replicas}), precision="mixed" if m is not None else "fp64"),
        mixed=m, fp64=f, unbatched_mixed=unb,
        speedup_mixed_vs_fp64=(f["mesh_ms_per_step"] / m["mesh_ms_per_step"]) if (m and f) else None,
        speedup_batched_vs_unbatched=unb["mesh_ms_per_step"] / head["mesh_ms_per_step"],
        roofline=roof, cpu_baseline=baseline, parity=parity,
    )
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="water-7999998")
    ap.add_argument("--kernel", default="auto", help="kernel family for the roofline (default: dominant)")
    ap.add_argument("--cpu-sample-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--modes", default="fp64,mixed,mixed32",
                    help="precision modes to run: fp64, mixed (FP32 V-cycle and gather), mixed32 (also an FP32 "
                         "charge source)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default (2,2) V-cycle schedule")
    ap.add_argument("--schedule", default=None,
                    help="NU_PRE,NU_POST: run this V-cycle schedule in every mode instead of autotuning")
    ap.add_argument("--gamma", type=float, default=None,
                    help="OVRVO thermostat friction in 1/fs at the workload's temperature (default: none)")
    ap.add_argument("--skin", type=float, default=None,
                    help="neighbour-list skin in box units (0: scan the cells every step; default: 0.1 r_cut)")
    ap.add_argument("--predictor", type=int, default=None,
                    help="multiplier predictor order 0..3 (0: no warm start, the plain real-space P3M solve; "
                         "default: the workload's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(domain decomposition is design-only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2606_31379_amd import configs
    from paper_2606_31379_amd import p3maze as P
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "nacl-batch64":
        return main_batch(args, torch, P, configs.nacl_batch_64())
    w = configs.WORKLOADS[args.workload]()
    if args.predictor is not None:
        import dataclasses
        w = dataclasses.replace(w, predictor=args.predictor)
    PHASES["startup"] = round(time.perf_counter() - T0, 2)
    log(f"workload {w.name}: generating inputs")
    t = time.perf_counter()
    system = w.system(progress=lambda msg: log(f"[inputs] {msg}"))
    phase("inputs", t)
    log(f"atoms {system.n} box {system.box} mesh {w.mesh}^3 order {w.order} tol {w.tol}")
    ceiling = copy_ceiling_gbps(torch)
    log(f"device copy ceiling {ceiling:.0f} GB/s")
    res, tune, schedules = {}, {}, {}
    modes = args.modes.split(",")
    fixed = None
    if args.schedule:
        a, b = (int(v) for v in args.schedule.split(","))
        fixed = dict(nu_pre=a, nu_post=b, smooth_tile=0)
    elif args.no_tune:
        fixed = dict(nu_pre=2, nu_post=2, smooth_tile=0)
    if fixed is None and not os.environ.get("P3MZ_TUNE_CACHE"):
        import tempfile
        os.environ["P3MZ_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="p3mz_tune_"), "tune.json")
    for precision, name in ((0, "fp64"), (1, "mixed"), (2, "mixed32")):
        if name not in modes:
            continue
        if fixed is not None:
            schedules[name] = dict(fixed)
        else:
            t = time.perf_counter()
            tune[name] = autotune_schedule(torch, P, w, system, precision, args.warmup)
            phase("autotune", t)
            schedules[name] = {k: tune[name][k] for k in ("nu_pre", "nu_post", "smooth_tile")}
            log(f"[{name}] autotune: {json.dumps({k: v for k, v in tune[name].items() if k != 'candidates'})}")
        log(f"[{name}] warmup {args.warmup}, timed {args.steps}")
        t = time.perf_counter()
        res[name] = run_mode(torch, P, w, system, precision, args.warmup, args.steps, args.kernel, schedules[name],
                             args.skin, args.gamma)
        phase("gpu_runs", t)
        log(f"[{name}] {json.dumps({k: v for k, v in res[name].items() if k not in ('kernel_ms_per_step', 'kernel_families')})}")
    parity, baseline = None, None
    if not args.no_cpu_baseline:
        sample = args.cpu_sample_steps or (8 if system.n <= 4000 else 3 if system.n <= 2_000_000 else 2)
        t = time.perf_counter()
        parity, baseline = parity_and_baseline(torch, P, w, system, sample, schedules)
        phase("oracle_parity_and_baseline", t)
    # the headline is the fastest form of the benchmark spec's precision split
    # that is run: FP32 charge source and V-cycle (mixed32), else mixed,
    # else FP64; every mode's parity is reported beside it
    m32, m, f = res.get("mixed32"), res.get("mixed"), res.get("fp64")
    head_name = "mixed32" if m32 is not None else "mixed" if m is not None else "fp64"
    head = res[head_name]
    traffic, traffic_note = measured_traffic(head["dominant"], w.name, head_name)
    roof = dict(bound="hbm", kernel=head["dominant"], achieved=head["dominant_gbps"], peak=HBM_PEAK_GBPS,
                unit="GB/s", frac=(head["dominant_gbps"] / HBM_PEAK_GBPS) if head["dominant_gbps"] else None,
                traffic=traffic, traffic_source=traffic_note, avg_launch_us=head["dominant_avg_launch_us"],
                alg_bytes_per_launch=head["dominant_bytes_per_launch"], launches=head["dominant_launches"],
                idle_launches=head["dominant_idle_launches"], share_of_mesh_step=head["dominant_share"],
                burst_avg_launch_us=head["dominant_burst_avg_launch_us"],
                whole_step_frac=head["whole_step"]["frac"],
                mg_sweeps=mg_sweep_roofline(head["kernel_families"]),
                copy_ceiling_GBps=ceiling)
    line = dict(
        metric=METRIC, value=head["ns_per_atom"], unit="ns/atom/step", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=head["md_ms_per_step"], higher_is_better=False, scaling="weak",
        vs_baseline=None, dtype="f32+f64" if head_name != "fp64" else "f64", data="synthetic",
        config=dict(workload=w.name, n_atoms=system.n, box=w.box, mesh=w.mesh, order=w.order,
                    alpha=w.alpha, r_cut=w.r_cut, tol=w.tol, predictor=w.predictor, dt_fs=w.dt_fs,
                    precision=head_name),
        mixed32=m32, mixed=m, fp64=f, autotune=tune or None,
        speedup_mixed_vs_fp64=(f["mesh_ms_per_step"] / m["mesh_ms_per_step"]) if (m and f) else None,
        speedup_mixed32_vs_fp64=(f["mesh_ms_per_step"] / m32["mesh_ms_per_step"]) if (m32 and f) else None,
        roofline=roof, cpu_baseline=baseline, parity=parity,
    )
    PHASES["total"] = round(time.perf_counter() - T0, 2)
    line["phase_s"] = PHASES
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
