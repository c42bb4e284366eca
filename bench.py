#!/usr/bin/env python
"""Benchmark of the merged implicit r-z PIC/MC step on one MI355X.

Workload: 129x65 mesh (R = 4 cm, L = 2 cm), 2M electrons + 2M Ar+ ions
(seeded Maxwellian init, weights proportional to r), 200 V 13.56 MHz drive,
3 V(0,1) cycles per step; the headline runs the mixed form (FP32 particles and
smoothing, FP64 residual / defect correction and int64 deposit), and the same
workload runs in plain FP64 beside it.

Prints one JSON line: particle-steps/s of the mixed form (`value`), the FP64
rate, V-cycle times and the cycles each form needs for a fixed phi error,
the roofline of the fused particle pass (HIP events on the library's stream
over the timed region), and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec + multigrid V-cycle ms, mixed vs FP64 GPU at fixed phi err"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one particle through the fused pass: read the 8 real
# fields + 8-byte id, write 7 real fields (the weight is only read).
BYTES_PER_PARTICLE = {"mixed": 8 * 4 + 8 + 7 * 4, "fp64": 8 * 8 + 8 + 7 * 8}


def measured_traffic(name, shape=None):
    """HBM bytes per particle of the fused pass from a committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None when
    the kernel sources have changed since the counters were taken, or when
    `shape` (threads, particles per block) is not the launch shape they were
    taken with."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", name)
    try:
        text = open(path).read()
    except OSError:
        return None
    t = re.search(r"^traffic_bytes_per_particle: ([0-9.]+)$", text, re.M)
    hs = re.search(r"^kernel_sources_sha256: ([0-9a-f]{64})$", text, re.M)
    if not t or not hs:
        return None
    sh = re.search(r"^pass_shape: ([0-9]+) ([0-9]+)$", text, re.M)
    if shape is not None and (not sh or (int(sh.group(1)), int(sh.group(2))) != tuple(shape)):
        return None
    h = hashlib.sha256()
    for f in ("particles.hip", "device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1001_2969_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return float(t.group(1)) if h.hexdigest() == hs.group(1) else None


def run_gpu(w, precision, steps, warmup, timing_steps=50, capacity_factor=1.25, tune=False,
            shape=None, graph=False, pipeline=True):
    """Throughput over `steps` merged steps with nothing else on the stream,
    then `timing_steps` more with the library's HIP events around each phase
    (per-phase device times; every event costs the stream a few microseconds,
    which is why the throughput run records none; those steps run directly).
    tune: the library's autotuner picks the pass's launch shape first (its
    steps precede the warm-up); shape: (threads, particles per block) set
    instead.  graph: after the timed steps, `timing_steps` more captured and
    replayed as HIP graphs (rzpic_set_step_graph, on a stream of the
    context's own) are timed too.  pipeline: the timed steps pipelined
    (rzpic_set_step_pipeline: each step prepares the next step's grid in its
    list maintenance launches, same results bit for bit); as many
    unpipelined steps are timed after them for comparison."""
    import torch

    from paper_1001_2969_amd import rzpic

    ctx = rzpic.make_context(w, precision=precision, capacity_factor=capacity_factor)
    ctx.init_particles(0, w.n_per_species, w.n0, w.Te_eV, 0)
    ctx.init_particles(1, w.n_per_species, w.n0, w.Ti_eV, 0)
    ctx.prologue()
    if w.sort_every:
        # tile-sorted from the start (the steps then re-sort every sort_every)
        for s in (0, 1):
            ctx.sort(s)
    n = 0
    tuning_steps = 0
    if tune:
        shape, table, n = ctx.autotune(5, 0)
        tuning_steps = n
    elif shape is not None:
        ctx.set_pass_shape(*shape)
    ctx.set_step_pipeline(pipeline)
    for _ in range(warmup):
        ctx.step(n)
        n += 1
    ctx.sync()
    d0 = ctx.diag()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(n)
        n += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d1 = ctx.diag()
    direct_ms = None
    if pipeline:
        ctx.set_step_pipeline(False)
        for _ in range(5):
            ctx.step(n)
            n += 1
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(steps):
            ctx.step(n)
            n += 1
        torch.cuda.synchronize()
        direct_ms = 1e3 * (time.perf_counter() - t2) / steps
    graph_ms = None
    if graph:
        ctx.use_stream(torch.cuda.Stream())
        ctx.set_step_graph(True)
        for _ in range(5):
            ctx.step(n)
            n += 1
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(timing_steps):
            ctx.step(n)
            n += 1
        torch.cuda.synchronize()
        graph_ms = 1e3 * (time.perf_counter() - t2) / timing_steps
        ctx.set_step_graph(False)
    ctx.set_step_pipeline(pipeline)
    ctx.set_timing(True)
    ctx.timing()  # reset accumulators
    for _ in range(timing_steps):
        ctx.step(n)
        n += 1
    ctx.sync()
    tim = ctx.timing()
    ctx.set_timing(False)
    psteps = sum(d1["particle_steps"]) - sum(d0["particle_steps"])
    dt = t1 - t0
    return ctx, {
        "value": psteps / dt, "ms_per_step": 1e3 * dt / steps, "particle_steps": psteps,
        "timing": tim, "count": d1["count"], "events_last_step": d1["events"],
        "pass_shape": None if shape is None else {"threads": shape[0],
                                                  "particles_per_block": shape[1]},
        "tuning_steps": tuning_steps, "graph_ms_per_step": graph_ms,
        "pipelined": pipeline, "unpipelined_ms_per_step": direct_ms,
    }


def vcycle_study(w, rho, chi, phi0):
    """Solver level, identical (rho, chi): cycles each form needs to bring the
    L-inf error of phi below 1e-8 of |phi| (reference: the FP64 solve to a
    1e-12 residual), and device time per V-cycle on the benchmark mesh."""
    import numpy as np
    import torch

    from paper_1001_2969_amd import rzpic

    out = {}
    ref_ctx = rzpic.Context(w, precision="fp64", mg_fixed_cycles=0, mg_tol=1e-12,
                            mg_max_cycles=200)
    for g, a in ((rzpic.G_RHO, rho), (rzpic.G_CHI, chi), (rzpic.G_PHI, phi0)):
        ref_ctx.set_grid(g, a)
    t_ref = 1e-9
    ref_ctx.solve(t_ref)
    phi_ref = ref_ctx.grid(rzpic.G_PHI)
    scale = np.abs(phi_ref).max()
    for prec in ("fp64", "mixed"):
        ctx = rzpic.Context(w, precision=prec, mg_fixed_cycles=1)
        errs = []
        for k in range(1, 41):
            ctx.set_mg(fixed_cycles=k)
            for g, a in ((rzpic.G_RHO, rho), (rzpic.G_CHI, chi), (rzpic.G_PHI, phi0)):
                ctx.set_grid(g, a)
            ctx.solve(t_ref, want=False)
            e = float(np.abs(ctx.grid(rzpic.G_PHI) - phi_ref).max() / scale)
            errs.append(e)
            if e <= 1e-8:
                break
        k_need = len(errs) if errs[-1] <= 1e-8 else None
        # device time per cycle: (T(1 + m cycles) - T(1 cycle)) / m
        times = {}
        for k in (1, 21):
            ctx.set_mg(fixed_cycles=k)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            best = math.inf
            for _ in range(5):
                ctx.stream.synchronize()
                ev0.record(ctx.stream)
                ctx.solve(t_ref, want=False)
                ev1.record(ctx.stream)
                ev1.synchronize()
                best = min(best, ev0.elapsed_time(ev1))
            times[k] = best
        out[prec] = {"vcycle_ms": (times[21] - times[1]) / 20.0, "cycles_to_1e-8": k_need,
                     "err_after_3_cycles": errs[2] if len(errs) >= 3 else errs[-1],
                     "solve_ms_at_1e-8": (times[1] + (times[21] - times[1]) / 20.0 *
                                          ((k_need or 41) - 1))}
    return out


# Algorithmic bytes per fine node of one V(0,1) cycle on the long-line path
# (two half-sweeps per level): the down leg reads phi, f, eps (FP64) and
# writes the restricted right-hand sides of the coarser levels; each level's
# up leg reads eps, f, the neighbour lines and the coarse correction and
# writes its unknowns (coarser levels add half, a quarter, ... of the
# finest); the mixed form adds phi += correction.
VCYCLE_BYTES_PER_NODE = {"fp64": 32 + 2 * 44, "mixed": 32 + 2 * 22 + 20}


def vcycle_time(w, precision):
    """Device time of one V(0,1) cycle on w's mesh: (T(6) - T(1)) / 5 for
    fixed-cycle solves of a smooth rho, chi ~ 1 (best of 7 each: the
    difference of two short event-timed solves is noisy), and the path."""
    import numpy as np
    import torch

    from paper_1001_2969_amd import rzpic, workloads as wl

    ctx = rzpic.Context(w, precision=precision, mg_fixed_cycles=1)
    rho, chi = wl.smooth_rho(w, 5, 2e-4), wl.smooth_chi(w, 1.0)
    ctx.set_grid(rzpic.G_RHO, rho)
    ctx.set_grid(rzpic.G_CHI, chi)
    ctx.set_grid(rzpic.G_PHI, np.zeros((w.nz, w.nr)))
    del rho, chi
    times = {}
    for k in (1, 6):
        ctx.set_mg(fixed_cycles=k)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = math.inf
        for _ in range(7):
            ctx.stream.synchronize()
            ev0.record(ctx.stream)
            ctx.solve(1e-9, want=False)
            ev1.record(ctx.stream)
            ev1.synchronize()
            best = min(best, ev0.elapsed_time(ev1))
        times[k] = best
    ctx.close()
    return (times[6] - times[1]) / 5.0


def vcycle_by_mesh():
    """V-cycle device time on every workload mesh, and on a synthetic
    8193 x 2049 grid (square cells, 16.8M nodes: a working set far above the
    256 MB last-level cache) where the smoother's bandwidth means something."""
    from paper_1001_2969_amd import workloads as wl

    meshes = [wl.small_fp64(), wl.rf_129x65(), wl.large_513x129(),
              wl.Workload(name="synthetic_8193x2049_vcycle", nr=8193, nz=2049, R=0.16, L=0.04,
                          n_per_species=1, steps=1, V_dc=35.0)]
    out = {}
    for w in meshes:
        row = {}
        for prec in ("mixed", "fp64"):
            ms = vcycle_time(w, prec)
            row[prec] = {"vcycle_ms": ms}
            if w.nr * w.nz > 1 << 24:
                b = VCYCLE_BYTES_PER_NODE[prec] * w.nr * w.nz
                row[prec]["algorithmic_GBps"] = b / (ms * 1e-3) / 1e9
                row[prec]["bytes_per_node"] = VCYCLE_BYTES_PER_NODE[prec]
        out[f"{w.nr}x{w.nz}"] = row
        print(f"# V-cycle {w.nr}x{w.nz}: {json.dumps(row)}", file=sys.stderr, flush=True)
    return out


def host_info():
    """The host the CPU baseline ran on: CPUs this process may use, the
    machine's count and the processor model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "model": model}


def cpu_threads():
    """All-core thread count: the CPUs this process may use, at most 16 (the
    host share of one GPU)."""
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def cpu_leg(o, n0, steps, threads):
    """`steps` merged steps from step n0 of the OpenMP timing build of the
    oracle on `threads` threads: particle-steps/s, particle and solve time
    per step, V-cycle time."""
    from oracle import rzo

    rzo.Oracle.set_threads(threads)
    ps = 0
    tp = ts = 0.0
    cycles = 0
    t0 = time.perf_counter()
    for n in range(n0, n0 + steps):
        ps += o.count(0) + o.count(1)
        st, a, b, k = o.step_omp(n, with_cycles=True)
        if st != 0:
            raise RuntimeError(f"oracle step {n} failed ({st})")
        tp += a
        ts += b
        cycles += k
    wall = time.perf_counter() - t0
    return {"threads": threads, "steps": steps, "particle_steps_per_s": ps / wall,
            "particle_ms_per_step": 1e3 * tp / steps, "solve_ms_per_step": 1e3 * ts / steps,
            "vcycles_per_step": cycles / steps,
            "vcycle_ms": 1e3 * ts / cycles if cycles else None, "seconds": wall}


def cpu_oracle(w):
    from oracle import rzo

    o = rzo.Oracle(w.replace(precision="fp64"), omp=True)
    o.init_particles(0, w.n_per_species, w.n0, w.Te_eV, 0)
    o.init_particles(1, w.n_per_species, w.n0, w.Ti_eV, 0)
    o.prologue()
    return o


def cpu_baseline(study=False):
    """The FP64 CPU oracle on this host, in its OpenMP timing build (the
    oracle's own functions, particle loops on threads; tested equal to the
    serial oracle): one thread and all cores, particle and multigrid time
    apart.  Default (bounded): the 129x65 workload (10 steps on one thread,
    then 30 on all cores), the 33x33 workload in full (10 steps, each
    thread count), and 20 steps of the 513x129 workload on all cores.
    study: the 129x65 workload's 200 steps on all cores and 20 of them on one
    thread, and the 513x129 workload's 20 steps on one thread as well."""
    from paper_1001_2969_amd import workloads as wl

    nt = cpu_threads()
    legs = {}
    w1 = wl.rf_129x65()
    o = cpu_oracle(w1)
    single = cpu_leg(o, 0, 20 if study else 10, 1)
    allc = cpu_leg(o, single["steps"], 200 if study else 30, nt)
    legs[w1.name] = {"single_thread": single, "all_cores": allc}
    del o
    w0 = wl.small_fp64()
    o = cpu_oracle(w0)
    s0 = cpu_leg(o, 0, w0.steps, 1)
    o = cpu_oracle(w0)
    a0 = cpu_leg(o, 0, w0.steps, nt)
    legs[w0.name] = {"single_thread": s0, "all_cores": a0, "note": "in full (10 steps)"}
    del o
    w2 = wl.large_513x129()
    o = cpu_oracle(w2)
    big = {"note": "20 of its 1000 steps (steps 0-19)"}
    big["all_cores"] = cpu_leg(o, 0, 20, nt)
    if study:
        o = cpu_oracle(w2)
        big["single_thread"] = cpu_leg(o, 0, 20, 1)
    legs[w2.name] = big
    del o
    return {"value": allc["particle_steps_per_s"], "unit": "particle-steps/s", "cores": nt,
            "kind": "oracle",
            "sample": f"{w1.name}: steps {single['steps']}..{single['steps'] + allc['steps'] - 1} "
                      f"on {nt} threads (FP64 oracle, OpenMP timing build), "
                      f"{allc['seconds']:.1f} s",
            "single_thread": {k: single[k] for k in ("particle_steps_per_s", "steps", "seconds")},
            "host": host_info(), "legs": legs}


def large_mesh(steps, warmup):
    """The 513x129 / 16M-per-species workload (R >> L, weight split every 100
    steps, tile sort every 20), mixed and FP64: throughput and per-phase
    device times, for context beside the headline workload.  Capacity 2x:
    the split at step 99 clones every particle that drifted inward of the
    radius its weight was set for (about half of them)."""
    from paper_1001_2969_amd import workloads as wl

    w = wl.large_513x129()
    out = {"workload": w.name, "mesh": f"{w.nr}x{w.nz}", "particles_per_species": w.n_per_species,
           "sort_every": w.sort_every, "resize_every": w.resize_every}
    for prec in ("mixed", "fp64"):
        ctx, r = run_gpu(w, prec, steps, warmup, timing_steps=min(steps, 40), capacity_factor=2.0)
        ctx.close()
        tm = r["timing"]
        out[prec] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                     "breakdown_ms_per_step": {k: tm[k] for k in
                                               ("step_ms", "solve_ms", "pass_ms", "collide_ms",
                                                "grid_ms", "lists_ms", "resize_ms", "sort_ms")},
                     "pass_GBps": BYTES_PER_PARTICLE[prec] * (tm["n0"] + tm["n1"]) /
                     (1e-3 * tm["pass_ms"]) / 1e9}
    tpp = measured_traffic("k_pass2_hbm_traffic_513x129.md")
    if tpp is not None:
        out["mixed"]["pass_traffic_over_algorithmic"] = tpp / BYTES_PER_PARTICLE["mixed"]
    return out


def batch_run(steps, warmup, tune_steps=2):
    """64 independent discharges (meshes 65x33 / 129x65 / 257x129, 1e5-2e6
    particles per species, log-uniform, seeded; 94M particles in all), mixed
    and FP64, stepped as one batch (rzpic_batch_step, graph replay on):
    first in the default pass configuration, then the batch autotuner picks
    each mesh group's launch shape, deposit form and tile shape
    (rzpic_batch_autotune), and the same contexts are stepped one by one on
    the stream and as the batch.  Particle-steps/s of each; the timed steps
    include the tile sorts (every 20 steps)."""
    import torch

    from paper_1001_2969_amd import rzpic, workloads as wl

    ws = wl.batch_64()
    out = {"discharges": len(ws), "particles": 2 * sum(w.n_per_species for w in ws),
           "meshes": sorted({f"{w.nr}x{w.nz}" for w in ws})}
    for prec in ("mixed", "fp64"):
        ctxs = []
        for w in ws:
            c = rzpic.make_context(w, precision=prec, capacity_factor=1.3)
            c.init_particles(0, w.n_per_species, w.n0, w.Te_eV, 0)
            c.init_particles(1, w.n_per_species, w.n0, w.Ti_eV, 0)
            c.prologue()
            for s in (0, 1):
                c.sort(s)
            ctxs.append(c)

        def psteps():
            return sum(sum(c.diag()["particle_steps"]) for c in ctxs)

        b = rzpic.Batch(ctxs, stream=torch.cuda.Stream())
        b.set_graph(True)  # steps replayed from captured graphs
        n = 0

        def batched(k):
            nonlocal n
            torch.cuda.synchronize()
            p0, t0 = psteps(), time.perf_counter()
            for _ in range(k):
                b.step(n)
                n += 1
            torch.cuda.synchronize()
            return time.perf_counter() - t0, psteps() - p0

        batched(warmup)
        t_u, p_u = batched(steps)  # default configuration
        rows, n = b.autotune(tune_steps, n)
        chosen = {}
        for k, c in enumerate(ctxs):
            chosen.setdefault(f"{ws[k].nr}x{ws[k].nz}", c.pass_config())
        torch.cuda.synchronize()
        for _ in range(warmup):
            for c in ctxs:
                c.step(n)
            n += 1
        torch.cuda.synchronize()
        p0, t0 = psteps(), time.perf_counter()
        for _ in range(steps):
            for c in ctxs:
                c.step(n)
            n += 1
        torch.cuda.synchronize()
        t_seq, p_seq = time.perf_counter() - t0, psteps() - p0
        batched(warmup)
        t_b, p_b = batched(steps)
        out[prec] = {"batched_value": p_b / t_b, "batched_ms_per_step": 1e3 * t_b / steps,
                     "one_by_one_value": p_seq / t_seq,
                     "one_by_one_ms_per_step": 1e3 * t_seq / steps,
                     "speedup": (p_b / t_b) / (p_seq / t_seq), "launches": b.stats(),
                     "untuned_batched_value": p_u / t_u,
                     "untuned_batched_ms_per_step": 1e3 * t_u / steps,
                     "tuned_over_untuned": (p_b / t_b) / (p_u / t_u),
                     "autotune": {"configurations_timed": len(rows), "chosen": chosen}}
        b.close()
        for c in ctxs:
            c.close()
        del ctxs
        torch.cuda.empty_cache()
    out["mixed_over_fp64_batched"] = out["mixed"]["batched_value"] / out["fp64"]["batched_value"]
    return out


def adjoint_run(reps=2):
    """The gradient window: 257x129 mesh, 4M particles per species, 50
    collision-free FP64 steps with converged solves, checkpointed every 10,
    particles sorted by tile after the prologue and every 10 steps.
    Wall time of the forward window (the steps plus the objective) and of the
    backward pass (segment recompute, reverse particle passes, adjoint
    solves), the last of `reps` repetitions; the context steps on from each
    window's end."""
    import torch

    from paper_1001_2969_amd import rzpic, workloads as wl

    w = wl.adjoint_257x129()
    ctx = rzpic.make_context(w, precision="fp64", with_xsec=False, capacity_factor=1.25)
    for s, T in ((0, w.Te_eV), (1, w.Ti_eV)):
        ctx.init_particles(s, w.n_per_species, w.n0, T, 0)
    ctx.prologue()
    for s in (0, 1):
        ctx.sort(s)
    adj = rzpic.Adjoint(ctx, w.steps, checkpoint_every=10, delta=2 * w.L / (w.nz - 1))
    out = {"workload": w.name, "mesh": f"{w.nr}x{w.nz}", "particles_per_species": w.n_per_species,
           "window_steps": w.steps, "checkpoint_every": 10, "mg_tol": w.mg_tol}
    step0 = 0
    for _ in range(reps):
        p0 = sum(ctx.diag()["particle_steps"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = adj.forward(step0)
        t1 = time.perf_counter()
        p1 = sum(ctx.diag()["particle_steps"])
        dvdc, dvrf, _, _ = adj.backward(density=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        step0 += w.steps
        out.update({"J": J, "dJ_dV_rf": dvrf, "dJ_dV_dc": dvdc,
                    "forward_ms": 1e3 * (t1 - t0), "backward_ms": 1e3 * (t2 - t1),
                    "gradient_ms": 1e3 * (t2 - t0),
                    "backward_over_forward": (t2 - t1) / (t1 - t0),
                    "forward_particle_steps_per_s": (p1 - p0) / (t1 - t0)})
    adj.close()
    ctx.close()
    torch.cuda.empty_cache()
    return out


def circuit_and_subcycle(steps, warmup):
    """The headline workload (129x65, 2M + 2M, mixed, 3 V-cycles per solve)
    with a 10 pF blocking capacitor between the rf source and the electrode
    (two solves per step, the circuit update), with the ions subcycled every
    4 steps, and with both: ms per step against the plain form measured the
    same way.  Particle-steps count the particles a step moves (ions only in
    their steps), so ms per simulated step is the comparison."""
    from paper_1001_2969_amd import workloads as wl

    base = wl.rf_129x65()
    forms = {"plain": base, "circuit_10pF": base.replace(circuit_C=1e-11),
             "ions_every_4": base.replace(ion_subcycle=4),
             "circuit_and_ions_every_4": base.replace(circuit_C=1e-11, ion_subcycle=4)}
    out = {"workload": base.name, "precision": "mixed"}
    for name, w in forms.items():
        ctx, r = run_gpu(w, "mixed", steps, warmup, timing_steps=20)
        tm = r["timing"]
        out[name] = {"ms_per_step": r["ms_per_step"], "value": r["value"],
                     "solve_ms": tm["solve_ms"], "pass_ms": tm["pass_ms"]}
        if w.circuit_C > 0:
            out[name]["circuit"] = ctx.circuit()
        ctx.close()
    for name in forms:
        out[name]["step_time_over_plain"] = out[name]["ms_per_step"] / out["plain"]["ms_per_step"]
    return out


def calibration_copy():
    """The device copy that calibrates the byte counters: 1 GiB, read from a
    buffer written before another 1 GiB was written (so that the copy's reads
    come from HBM, not from the 256 MB last-level cache).  Returns the bytes
    copied each way."""
    import torch

    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    evict = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del evict
    return nbytes


def pmc_run(steps, workload, shape=None):
    """Short run for hardware-counter passes: a few merged steps of the mixed
    workload, then a plain device copy of known size (the calibration of the
    byte counters: its algorithmic traffic is exactly the bytes read and
    written)."""
    import torch

    from paper_1001_2969_amd import workloads as wl

    w = {"rf_129x65": wl.rf_129x65, "large_513x129": wl.large_513x129}[workload]()
    # the pass shape the benchmark's autotuner picked (timings under a
    # counter run are not the benchmark's, so no tuning here)
    ctx, res = run_gpu(w, "mixed", steps, 3, timing_steps=steps, capacity_factor=2.0,
                       shape=shape)
    ctx.close()
    nbytes = calibration_copy()
    print(json.dumps({"pmc_run": True, "workload": w.name, "steps": steps, "particles_per_pass":
                      [res["timing"]["n0"], res["timing"]["n1"]],
                      "bytes_per_particle": BYTES_PER_PARTICLE["mixed"],
                      "copy_bytes_each_way": nbytes,
                      "pass_shape": list(shape) if shape else [512, 8192]}), flush=True)


def pmc_vcycle(mesh, precision, solves=3, cycles=2):
    """Short run for counter passes on the multigrid: `solves` fixed-cycle
    solves of `cycles` V(0,1) cycles on the mesh (smooth rho, chi ~ 1), then
    the device copy that calibrates the byte counters (calibration_copy)."""
    import numpy as np
    import torch

    from paper_1001_2969_amd import rzpic, workloads as wl

    if mesh == "129x65":
        w = wl.rf_129x65()
    else:
        w = wl.Workload(name="synthetic_8193x2049_vcycle", nr=8193, nz=2049, R=0.16, L=0.04,
                        n_per_species=1, steps=1, V_dc=35.0)
    ctx = rzpic.Context(w, precision=precision, mg_fixed_cycles=cycles)
    ctx.set_grid(rzpic.G_RHO, wl.smooth_rho(w, 5, 2e-4))
    ctx.set_grid(rzpic.G_CHI, wl.smooth_chi(w, 1.0))
    ctx.set_grid(rzpic.G_PHI, np.zeros((w.nz, w.nr)))
    for _ in range(solves):
        ctx.solve(1e-9, want=False)
    ctx.sync()
    ctx.close()
    nbytes = calibration_copy()
    print(json.dumps({"pmc_vcycle": True, "mesh": f"{w.nr}x{w.nz}", "precision": precision,
                      "solves": solves, "cycles_per_solve": cycles,
                      "copy_bytes_each_way": nbytes}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-study", action="store_true",
                    help="only the CPU oracle study (longer legs), printed as JSON")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-vcycle-study", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 513x129 / 16M-per-species context measurement")
    ap.add_argument("--large-steps", type=int, default=60)
    ap.add_argument("--no-vcycle-meshes", action="store_true",
                    help="skip the V-cycle timing on every mesh and the synthetic grid")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-discharge batch measurement")
    ap.add_argument("--batch-steps", type=int, default=40)
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the 257x129 / 4M-per-species gradient window")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default pass launch shape (no autotuning)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the graph-replayed steps timed after the headline steps")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="time unpipelined steps (no rzpic_set_step_pipeline) as the headline")
    ap.add_argument("--no-circuit", action="store_true",
                    help="skip the external-circuit and ion-subcycling forms")
    ap.add_argument("--pmc-run", type=int, default=0, metavar="STEPS",
                    help="only a short mixed run plus a copy calibration (for counter passes)")
    ap.add_argument("--pmc-workload", default="rf_129x65", choices=["rf_129x65", "large_513x129"])
    ap.add_argument("--pmc-shape", default=None, metavar="THREADS,PARTICLES",
                    help="pass launch shape of the counter run (default 512,8192)")
    ap.add_argument("--pmc-vcycle", default=None, metavar="MESH,PRECISION",
                    help="only fixed-cycle solves on 129x65 or 8193x2049, mixed or fp64, "
                         "plus the copy calibration (for counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU form is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1001_2969_amd import rzpic, workloads as wl

    if args.cpu_study:
        print(json.dumps(cpu_baseline(study=True)), flush=True)
        return
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.pmc_vcycle:
        mesh, prec = args.pmc_vcycle.split(",")
        pmc_vcycle(mesh, prec)
        return
    if args.pmc_run:
        pmc_run(args.pmc_run, args.pmc_workload,
                None if args.pmc_shape is None else tuple(int(x) for x in args.pmc_shape.split(",")))
        return
    w = wl.rf_129x65()
    print(f"# workload {w.name}: warmup {args.warmup}, timed {args.steps} steps", file=sys.stderr,
          flush=True)
    ctx_m, mixed = run_gpu(w, "mixed", args.steps, args.warmup, tune=not args.no_tune,
                           graph=not args.no_graph, pipeline=not args.no_pipeline)
    print(f"# mixed: {mixed['value']:.4g} particle-steps/s, {mixed['ms_per_step']:.4f} ms/step",
          file=sys.stderr, flush=True)
    fp64 = None
    rho = chi = phi = None
    if not args.no_fp64:
        ctx_d, fp64 = run_gpu(w, "fp64", args.steps, args.warmup, tune=not args.no_tune,
                              graph=not args.no_graph, pipeline=not args.no_pipeline)
        print(f"# fp64: {fp64['value']:.4g} particle-steps/s, {fp64['ms_per_step']:.4f} ms/step",
              file=sys.stderr, flush=True)
        rho, chi, phi = (ctx_d.grid(g) for g in (rzpic.G_RHO, rzpic.G_CHI, rzpic.G_PHI))
        ctx_d.close()
    vstudy = None
    if not args.no_vcycle_study:
        if rho is None:
            rho, chi, phi = (ctx_m.grid(g) for g in (rzpic.G_RHO, rzpic.G_CHI, rzpic.G_PHI))
        phi0 = np.zeros_like(phi)
        vstudy = vcycle_study(w, rho, chi, phi0)
        print(f"# V-cycle study: {json.dumps(vstudy)}", file=sys.stderr, flush=True)
    ctx_m.close()
    vmesh = None if args.no_vcycle_meshes else vcycle_by_mesh()
    batch = None
    if not args.no_batch:
        batch = batch_run(args.batch_steps, 3)
        print(f"# batch: {json.dumps(batch)}", file=sys.stderr, flush=True)
    circ = None
    if not args.no_circuit:
        circ = circuit_and_subcycle(100, 5)
        print(f"# circuit/subcycle: {json.dumps(circ)}", file=sys.stderr, flush=True)
    adjoint = None
    if not args.no_adjoint:
        adjoint = adjoint_run()
        print(f"# adjoint: {json.dumps(adjoint)}", file=sys.stderr, flush=True)
    large = None
    if not args.no_large:
        large = large_mesh(args.large_steps, 5)
        print(f"# large mesh: {json.dumps(large)}", file=sys.stderr, flush=True)

    tm = mixed["timing"]
    # one launch of the fused pass moves both species
    n_launch = tm["n0"] + tm["n1"]
    t_launch_ms = tm["pass_ms"]
    bpp = BYTES_PER_PARTICLE["mixed"]
    achieved = bpp * n_launch / (t_launch_ms * 1e-3) / 1e9 if t_launch_ms > 0 else None
    roofline = {"kernel": "k_one<pass2_body<float, 111>> (fused pass, whole-grid LDS deposit)",
                "bound": "hbm",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS if achieved else None,
                "traffic": None,
                "bytes_per_particle": bpp, "particles_per_launch": n_launch,
                "avg_launch_ms": t_launch_ms}
    ps = mixed["pass_shape"]
    tpp = measured_traffic("k_pass2_hbm_traffic_rf129x65.md",
                           None if ps is None else (ps["threads"], ps["particles_per_block"]))
    if tpp is not None:
        # counter bytes per particle (profile run) times this launch's particles
        roofline["traffic"] = tpp * n_launch
        roofline["traffic_over_algorithmic"] = tpp / bpp

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()
        print(f"# cpu baseline: {json.dumps(cpu)}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": mixed["value"], "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 particles / f64 residual / int64 deposit", "data": "synthetic",
        "config": {"workload": w.name, "mesh": f"{w.nr}x{w.nz}", "R_m": w.R, "L_m": w.L,
                   "particles_per_species": w.n_per_species, "precision": "mixed",
                   "v_cycles_per_step": w.mg_fixed_cycles, "V_rf": w.V_rf, "f_rf": w.f_rf,
                   "pass_shape": mixed["pass_shape"],
                   "autotune_steps": mixed["tuning_steps"]},
        "graph_ms_per_step": mixed["graph_ms_per_step"],
        "pipelined": mixed["pipelined"],
        "unpipelined_ms_per_step": mixed["unpipelined_ms_per_step"],
        "breakdown_ms_per_step": {k: tm[k] for k in ("step_ms", "solve_ms", "pass_ms",
                                                     "collide_ms", "grid_ms", "lists_ms",
                                                     "resize_ms", "sort_ms")},
        "vcycle_ms": {"mixed": tm["solve_ms"] / max(tm["vcycles"], 1)},
        "fp64": None if fp64 is None else {
            "value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
            "graph_ms_per_step": fp64["graph_ms_per_step"],
            "unpipelined_ms_per_step": fp64["unpipelined_ms_per_step"],
            "breakdown_ms_per_step": {k: fp64["timing"][k] for k in
                                      ("step_ms", "solve_ms", "pass_ms", "collide_ms")},
            "pass_GBps": BYTES_PER_PARTICLE["fp64"] * (fp64["timing"]["n0"] +
                                                      fp64["timing"]["n1"]) /
            (1e-3 * fp64["timing"]["pass_ms"]) / 1e9},
        "mixed_over_fp64": None if fp64 is None else mixed["value"] / fp64["value"],
        "fixed_phi_err": vstudy,
        "large_mesh": large,
        "vcycle_by_mesh": vmesh,
        "batch_64": batch,
        "adjoint_window": adjoint,
        "circuit_and_subcycling": circ,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if fp64 is not None:
        line["vcycle_ms"]["fp64"] = fp64["timing"]["solve_ms"] / max(fp64["timing"]["vcycles"], 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
