#!/usr/bin/env python3
"""Benchmark: scattering events per second of the deviational phonon Monte Carlo
hot path on one MI355X.

Workload (one step): the silicon-like frequency-dependent material (1000
frequency bins per branch, LA + doubly degenerate TA, sine dispersion,
tau^-1 = A w^4 + B w^2 T exp(-C/T)) in 12 cross-plane films of thicknesses
log-spaced 10 nm - 10 um between isothermal walls at T_eq +- 0.5 K, 1e8
particles per film, 20 temperature / heat-flux bins, FP32 flight with FP64
tallies, all 12 films in ONE persistent launch.  Inputs (material tables,
job descriptors) are resident on the device before timing starts; every
particle is generated on the device from (seed, pid).

Printed JSON line: metric/value (scattering events/s), the plain form
(one FP64 launch per film, one thread per particle, global tables, direct
FP64 atomics) timed on a subsample of the same workload, the ALU roofline of
the trajectory kernel from HIP-event timing, and the FP64 CPU oracle timed on a
bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU work, counted in full-rate VALU issue slots per lane (the
# MI355X issues 64 lane-slots per CU per clock).  The costs of the operations
# that are not one slot each (a Philox4x32-10 block: 20 32x32->64 multiply-adds
# and 20 three-input xors, with the key schedule on the scalar unit since a
# wave's particles share a seed; the transcendental and reciprocal
# instructions; FP64 adds) are measured live by the library's instruction-cost
# probe (dmc_debug_op_cost, op_costs() below; figures in profiles/op_costs.md).
# Every other item is one full-rate instruction per slot.  The counts are the
# cheapest form of each step found so far: a kernel change that removes work
# from the minimum lowers them, so the fraction does not flatter an older,
# costlier kernel.
def philox_cost(c):
    """A Philox4x32-10 block in the cheaper of its two measured forms: the key
    schedule in scalar registers, or held per lane in vector registers (the
    trajectory kernels' form)."""
    return min(c["philox_uniform_key"], c["philox_lane_key"])


def slab_items(c):
    """One flight of the cross-plane slab path (persistent FP32 slab kernel).
    The start bin of a segment is the end bin of the previous one, so one bin
    index per flight is the minimum; the signed length through a bin depends
    only on a trajectory's end points, so it costs nothing per flight; a slab
    needs only the z direction cosine after a scattering event (no azimuth)."""
    return [
        ("Philox4x32-10 block", philox_cost(c)),
        ("uniform u for the flight (funnel shift, subtract)", 2),
        ("mu = 2u - 1 from a second word (funnel shift, FMA, add)", 3),
        ("flight time -tau ln2 log2 u: log2, one multiply", c["log"] + 1),
        ("wall distance through the reciprocal of the axial speed, hit test, segment select", 7 + c["rcp"]),
        ("position update", 2),
        ("end-of-segment bin index (scale, truncate, 2 clamps), compare with the start bin", 6),
        ("two FP64 tally sums, time and time/tau (1 FP32 product, 2 converts, 2 adds)", 3 + 2 * c["f64_add"]),
        ("gain alias draw (shift, mask, compare, select) + state fetch address", 6),
        ("flight / scatter counters and the flight-cap test", 4),
        ("sign and select logic of the boundary / scatter outcome", 2),
    ]


def half_items(c):
    """One flight of the transient half-space path (heated spot, snapshot
    estimator only): nearly every flight ends in a scattering event (the surface
    is met on few flights), and a snapshot crossing (50 per particle over about
    2744 flights) costs a cell index (3 axes: subtract, scale, floor, convert, 2
    compares) and one FP64 atomic, about 25 slots, i.e. 0.46 per flight."""
    return [
        ("Philox4x32-10 block", philox_cost(c)),
        ("flight time: uniform (2), log2, one multiply", 3 + c["log"]),
        ("surface distance through the reciprocal of v Omega_z, hit test, select", 4 + c["rcp"]),
        ("segment end time t + seg in FP64 (convert, add), next-sample and final-time compares",
         3 + c["f64_add"]),
        ("position update (v seg, 3 FMAs)", 4),
        ("gain alias draw + state fetch address", 6),
        ("isotropic direction: mu (3), azimuth uniform (2), sin, cos, sqrt(1 - mu^2) (1 + sqrt), 2 products",
         8 + c["sin"] + c["cos"] + c["sqrt"]),
        ("flight / scatter counters and the flight-cap test", 3),
        ("outcome select", 2),
        ("snapshot crossings, amortised", 0.46),
    ]


def grad_unit_costs(c):
    """Per-event algorithmic costs of the in-plane film and pore-cell path under
    the gradient source (GEOM_GRAD kernel): a flight draws one Philox block; each
    segment searches the surfaces and adds its algebraic z length (and H_j);
    segments end in a scattering event, a wall or pore-surface interaction, or a
    periodic face crossing (the flight continues with its remaining time)."""
    search_film = 5 + c["rcp"]  # one candidate plane by the sign of the axial speed
    # two periodic face pairs (each: speed, sign tests, distance through the reciprocal) and
    # the pore's quadratic: offsets (2), a, b, c (7), discriminant (2), sqrt, root through the
    # reciprocal of a (2 + rcp), time through the reciprocal of v (1 + rcp), selects (4)
    search_pore = 2 * (5 + c["rcp"]) + 18 + c["sqrt"] + 2 * c["rcp"]
    seg_common = (2  # outcome compare, select
                  + 4  # position update
                  + 3 + 2 * c["f64_add"]  # s v Omega_z seg to FP64, added to L_z and H_j
                  + 3)  # segment counter, cap test, continuation test
    return {
        "flight": philox_cost(c) + 3 + c["log"],
        "segment_film": search_film + seg_common,
        "segment_pore": search_pore + seg_common,
        "scatter": 6 + 8 + c["sin"] + c["cos"] + c["sqrt"] + 1 + 2 * c["f64_add"],  # alias, isotropic, H_j flush
        # specular test (2) + Lambertian about the wall normal: mu = sqrt(u) (2 + sqrt), azimuth
        # (2 + sin + cos), sqrt(1 - mu^2) (1 + sqrt), 3 components
        "wall_hit": 10 + 2 * c["sqrt"] + c["sin"] + c["cos"],
        # the pore normal (2 offsets, norm: 2 + sqrt, 2 products through its reciprocal) and the
        # cosine law about it in the tangent frame (6 components)
        "pore_hit": 8 + c["sqrt"] + c["rcp"] + 2 + 3 + 2 * c["sqrt"] + c["sin"] + c["cos"] + 6,
        "periodic": 4,  # wrap the coordinate, remaining time, resting face
    }


OP_COST_ITERS = {"fma": 200_000, "philox_uniform_key": 4_000, "philox_lane_key": 3_000, "log": 60_000,
                 "sin": 60_000, "cos": 60_000, "sqrt": 60_000, "rcp": 60_000, "f64_add": 100_000}


def op_costs(b):
    """VALU issue slots per lane of each operation the counts use, from the
    library's instruction-cost probe at full occupancy."""
    out = {}
    for op, iters in OP_COST_ITERS.items():
        ms, n = b.debug_op_cost(op, iters)
        out[op] = ms * 1e-3 * PEAK_LANE_OPS / n
    return out


# HBM traffic of one launch of the timed workload from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs (profiles/), scaled by the same counters' reading for a plain
# device copy of known size (bench.py --copy-probe); valid only for the kernel
# source it was measured on.
TRAFFIC = {"kernel_sha1": "4adf109c3c2fedfd353c3657fb61159a4fa0fa08", "bytes": 54574142}  # profiles/persistent_kernel_slab_12films_counters.md
CU, LANES_PER_CU_CLK, CLOCK = 256, 64, 2.4e9
PEAK_LANE_OPS = CU * LANES_PER_CU_CLK * CLOCK  # 3.93e13 full-rate VALU lane-ops/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(jobs, target_s=15.0):
    """The FP64 oracle on a bounded sample of every film, on the host cores."""
    import oracle

    threads = os.cpu_count() or 1
    if "OMP_NUM_THREADS" in os.environ:
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))

    def run(n, nt):
        ev = 0
        t0 = time.perf_counter()
        for j in jobs:
            _, cnt, _ = oracle.run_raw(j, 0, n, threads=nt)
            ev += cnt["scatters"]
        return ev, time.perf_counter() - t0

    def grow(nt, goal):
        n = 256
        ev, dt = run(n, nt)
        # heavy-tailed trajectory lengths make small samples noisy: grow until the
        # sample itself takes at least a third of the goal
        while dt < goal / 3 and n < 4_000_000:
            n = int(n * min(8.0, max(2.0, goal / max(dt, 1e-3))))
            ev, dt = run(n, nt)
        return n, ev, dt

    n, ev, dt = grow(threads, target_s)
    n1, ev1, dt1 = grow(1, target_s / 3)  # one core, for the per-core rate
    return {"value": ev / dt, "unit": "scattering events/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} particles of each of the 12 films ({ev} scattering events, {dt:.1f} s)",
            "cpu": host_cpu(),
            "single_core": {"value": ev1 / dt1, "sample": f"first {n1} particles of each film ({ev1} events, {dt1:.1f} s)"}}


def host_cpu():
    """The host's processor model and logical CPU count (/proc/cpuinfo, os.cpu_count)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def launch_params(jobs, mat, precision="fp32", stream=None, overrides=None, tune=True):
    """Launch parameters of the timed configuration: the library's autotuner on
    this batch (cached per process and batch signature), or the library's
    defaults when tune is False, then any explicit non-zero overrides."""
    from paper_1206_3316_amd import binding as b

    if tune:
        params, trials = b.autotune(jobs, material=mat, precision=precision, stream=stream)
        if trials:
            launch_params.trials = trials
    else:
        params = {"block": 0, "chunk": 0, "refill_min": 0, "lds_tally": 1}
    for k, v in (overrides or {}).items():
        if v:
            params[k] = v
    return params


def grad_roofline(jobs, st, ms, costs):
    """Algorithmic VALU work of a gradient-source launch (films and pore cells)
    from its per-job event counts: flights (Philox blocks), segments, scattering
    events, wall / pore-surface interactions and periodic face crossings
    (segments - flights), each at its unit cost (grad_unit_costs)."""
    u = grad_unit_costs(costs)
    tot = {"flight": 0.0, "segment": 0.0, "scatter": 0.0, "hit": 0.0, "periodic": 0.0}
    for j, s in zip(jobs, st):
        pore = j.geometry.kind == "pore_cell_xz"
        periodic = s.iterations - s.flights
        hits = s.boundary - periodic
        tot["flight"] += s.flights * u["flight"]
        tot["segment"] += s.iterations * (u["segment_pore"] if pore else u["segment_film"])
        tot["scatter"] += s.scatters * u["scatter"]
        tot["hit"] += hits * (u["pore_hit"] if pore else u["wall_hit"])
        tot["periodic"] += periodic * u["periodic"]
    ops = sum(tot.values())
    achieved = ops / (ms / 1e3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "T VALU lane-ops/s",
            "frac": achieved / PEAK_LANE_OPS, "kernel": "persistent_kernel<float, GEOM_GRAD>",
            "ops_per_launch": ops, "ops_by_event": {k: v for k, v in tot.items()},
            "unit_costs_slots": {k: round(v, 3) for k, v in u.items()}}


def other_workloads(b, di, mat, mat_in, stream, costs):
    """One autotuned launch each of the transient heated spot (1e9 particles,
    64^3 grid x 50 times; alone, and with the windowed tally in a 10 um x 5 nm
    surface cylinder like a thermoreflectance probe), of the 64 batched
    nanostructures (1e6-1e8 particles each, K_max = 40), and of the same batch
    with first-event termination for its 24 films (exact for films), after the
    tuner's trials have loaded the kernels, each with the ALU roofline of its
    kernel.  Reported beside the headline, not in it."""
    res = {}
    for name, jobs in (("heated_spot_1e9_64cube_50times", [di.heated_spot(material=mat_in)]),
                       ("heated_spot_1e9_64cube_50times_ttr_probe",
                        [di.heated_spot(material=mat_in, probe=di.TTR_PROBE)]),
                       ("nanostructures_64_instances", di.batched_nanostructures(material=mat_in)),
                       ("nanostructures_64_instances_first_event_films",
                        di.batched_nanostructures(material=mat_in, first_event_films=True))):
        t0 = time.perf_counter()
        params = launch_params(jobs, mat, stream=stream)
        tune_s = time.perf_counter() - t0
        r = b.simulate(jobs, material=mat, stream=stream, **params)
        st = [r.stats(i) for i in range(len(jobs))]
        ms = st[0].kernel_ms
        sc = sum(s.scatters for s in st)
        fl = sum(s.iterations for s in st)
        parts = sum(s.particles for s in st)
        if jobs[0].tally.region is not None:
            T, Tse = r.read(0, b.Q_REGION_T)
            res["ttr_probe_T_windows_10_20_30_40_49"] = [[float(T[i]), float(Tse[i])] for i in (10, 20, 30, 40, 49)]
        res[name] = {"scattering_events_per_s": sc / (ms / 1e3), "particles_per_s": parts / (ms / 1e3),
                     "flights_per_s": fl / (ms / 1e3), "kernel_ms": ms, "particles": parts, "scattering_events": sc,
                     "capped": sum(s.capped for s in st), "launch": params, "autotune_s": tune_s}
        if name == "heated_spot_1e9_64cube_50times":
            items = half_items(costs)
            per = sum(v for _, v in items)
            ach = per * fl / (ms / 1e3)
            res[name]["roofline"] = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                                     "unit": "T VALU lane-ops/s", "frac": ach / PEAK_LANE_OPS,
                                     "kernel": "persistent_kernel<float, GEOM_HALF>", "ops_per_flight": per,
                                     "ops_items": [[k, round(v, 3)] for k, v in items]}
        elif name.startswith("nanostructures"):
            res[name]["roofline"] = grad_roofline(jobs, st, ms, costs)
        if "roofline" in res[name]:
            log(f"{name}: roofline fraction {res[name]['roofline']['frac']:.3f}")
        log(f"{name}: {sc:.3e} scatters in {ms:.1f} ms ({sc / (ms / 1e3):.3e} /s), params {params}")
        r.close()
    # the steady temperature and heat-flux fields of a pore cell (16 x 16 cells privatised in
    # LDS, 32 x 32 in global memory), against the same cell with only its conductivity
    # tallied; the nanostructure batch's launch parameters
    fr = {}
    for tag, field in (("kappa_only", None), ("field_16x16", (16, 16)), ("field_32x32", (32, 32))):
        jobs = [di.pore_cell(100e-9, 0.3, 20_000_000, seed=1108, material=mat_in, kmax=40, n_hj=0, field=field)]
        params = {"block": 0, "chunk": 1024, "refill_min": 16, "lds_tally": 1}
        r = b.simulate(jobs, material=mat, stream=stream, **params)
        st = r.stats(0)
        fr[tag] = {"kernel_ms": st.kernel_ms, "flights_per_s": st.iterations / (st.kernel_ms / 1e3), "launch": params}
        r.close()
    res["pore_cell_100nm_phi0.3_2e7_fields"] = fr
    log(f"pore cell fields: 16x16 {fr['field_16x16']['kernel_ms']:.1f} ms, 32x32 {fr['field_32x32']['kernel_ms']:.1f} ms, "
        f"without {fr['kappa_only']['kernel_ms']:.1f} ms")
    # the same 64 instances with K_max planned per instance from a pilot run
    # (tail of <H_j> cut where its fitted sum is below 0.2 standard errors)
    jobs = di.batched_nanostructures(material=mat_in)
    t0 = time.perf_counter()
    ks = []
    for j in jobs:
        plan = b.plan_truncation(j, material=mat, stream=stream)
        j.tally.kmax = int(plan["kmax"])
        j.tally.n_hj = min(j.tally.n_hj, j.tally.kmax)
        ks.append(j.tally.kmax)
    plan_s = time.perf_counter() - t0
    params = launch_params(jobs, mat, stream=stream)
    r = b.simulate(jobs, material=mat, stream=stream, **params)
    st = [r.stats(i) for i in range(len(jobs))]
    ms = st[0].kernel_ms
    sc = sum(s.scatters for s in st)
    res["nanostructures_64_instances_planned_kmax"] = {
        "scattering_events_per_s": sc / (ms / 1e3), "kernel_ms": ms, "scattering_events": sc,
        "flights": sum(s.iterations for s in st), "planning_s": plan_s, "launch": params,
        "kmax_films": sorted(set(ks[:24])), "kmax_pores_min": min(ks[24:]),
        "kmax_pores_median": sorted(ks[24:])[20], "kmax_pores_max": max(ks[24:])}
    log(f"planned K_max: films {sorted(set(ks[:24]))}, pores {ks[24:]}; "
        f"{sc:.3e} scatters in {ms:.1f} ms (planning {plan_s:.1f} s)")
    r.close()
    return res


def plain_vs_persistent(b, di, mat, mat_in, stream, n):
    """The plain form (one FP64 launch per film, one thread per particle run to
    completion, global tables, direct FP64 atomics) against the persistent
    FP32-flight / FP64-tally batched form on the same 12 films at the same
    particle count per film, i.e. at equal error (the persistent form in FP64 too,
    to separate the precision from the form).  Kernel time from HIP events."""
    pjobs = di.cross_plane_films(n_per_film=n, material=mat_in)
    rp = b.simulate(pjobs, material=mat, precision="fp64", form="plain", stream=stream)
    sp = rp.stats(-1)
    rp.close()
    log(f"plain form, {n:.0e} per film: {sp.scatters:.3e} scatters in {sp.kernel_ms:.1f} ms")
    params = launch_params(pjobs, mat, stream=stream)
    rq = b.simulate(pjobs, material=mat, precision="fp32", form="persistent", stream=stream, **params)
    sq = rq.stats(-1)
    rq.close()
    p64 = launch_params(pjobs, mat, precision="fp64", stream=stream)
    r64 = b.simulate(pjobs, material=mat, precision="fp64", form="persistent", stream=stream, **p64)
    s64 = r64.stats(-1)
    r64.close()
    plain = sp.scatters / (sp.kernel_ms / 1e3)
    pers = sq.scatters / (sq.kernel_ms / 1e3)
    log(f"persistent, {n:.0e} per film: fp32 {sq.kernel_ms:.1f} ms, fp64 {s64.kernel_ms:.1f} ms; "
        f"fp32 / plain = {pers / plain:.1f}")
    return {"particles_per_film": n, "plain_fp64_events_per_s": plain, "plain_kernel_ms": sp.kernel_ms,
            "persistent_fp32_events_per_s": pers, "persistent_fp32_kernel_ms": sq.kernel_ms,
            "persistent_fp64_events_per_s": s64.scatters / (s64.kernel_ms / 1e3),
            "persistent_fp64_kernel_ms": s64.kernel_ms, "persistent_fp32_over_plain": pers / plain,
            "persistent_fp64_over_plain": (s64.scatters / (s64.kernel_ms / 1e3)) / plain,
            "target_20x_met": bool(pers / plain >= 20.0), "launch_fp32": params, "launch_fp64": p64}


def flights_per_particle(job, sums):
    C_tot, G_tau, G_v = sums
    if job.source.kind == "walls":
        return 2.0 * job.geometry.length * G_tau / G_v + 1.0
    if job.source.kind == "gaussian":
        return job.tally.times[-1] * G_tau / C_tot + 1.0
    return 1.5 * job.tally.kmax + 1.0


def mix_capacity(b, di, mat, reqs, stream, args, n_sample=64, n_epochs=24):
    """Device throughput of the request mix when saturated: the first n_sample
    requests submitted at once to a server, flights / kernel time over epochs
    3 .. n_epochs (the mix runs the generic kernel in time-bounded epochs)."""
    free, _ = torch_free_bytes()
    srv = b.Server(mat, int(min(0.8 * free, 64 << 30)), max_active=32, epoch_flights=args.epoch_flights,
                   stream=stream, refill_min=4, class_epochs=args.serve_class_epochs)
    for _, j in reqs[:n_sample]:
        srv.submit(j)
    f0 = k0 = 0.0
    for e in range(n_epochs):
        srv.step()
        if e == 1:
            t = srv.totals()
            f0, k0 = float(t.iterations), float(t.kernel_ms)
    t = srv.totals()
    srv.close()
    return (float(t.iterations) - f0) / ((float(t.kernel_ms) - k0) / 1e3)


def torch_free_bytes():
    import torch
    return torch.cuda.mem_get_info()


def serve(b, di, torch, mat, mat_in, stream, n_requests, args):
    """Poisson stream of mixed requests (films, heated spots, pore cells) on the
    continuous-batching server at 0.8 x the mix's measured capacity; p50/p99
    latency."""
    _, sums = mat.info()
    reqs = di.serving_stream(n_requests, material=mat_in)
    work = [j.n_particles * flights_per_particle(j, sums) for _, j in reqs]
    capacity = mix_capacity(b, di, mat, reqs, stream, args)
    rate = args.serve_rate or 0.8 * capacity / (sum(work) / len(work))
    log(f"serving: mix capacity {capacity:.3e} flights/s, arrival rate {rate:.2f} requests/s")
    arrivals = di.poisson_arrivals(n_requests, rate)
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(0.8 * free, 64 << 30))
    srv = b.Server(mat, budget, max_active=32, epoch_flights=args.epoch_flights, stream=stream, refill_min=4,
                   class_epochs=args.serve_class_epochs)
    lat, kinds, rel_se, kept, scat = [], [], [], {}, 0
    pending = {}
    i = 0
    epochs = 0
    epoch_s = 0.0
    t0 = time.perf_counter()
    last_log = 0.0
    while len(lat) < i or i < n_requests:
        now = time.perf_counter() - t0
        if now > args.serve_max_s and i < n_requests:
            log(f"serving: stopping arrivals after {now:.0f} s ({i} of {n_requests} requests submitted)")
            n_requests = i
            continue
        while i < n_requests and arrivals[i] <= now:
            pending[srv.submit(reqs[i][1])] = (i, arrivals[i])
            i += 1
        q, r = srv.load()
        if q + r > 0:
            te = time.perf_counter()
            srv.step()
            epochs += 1
            epoch_s += time.perf_counter() - te
            t_done = time.perf_counter() - t0
            for t in [t for t in pending if srv.done(t)]:
                k, ta = pending.pop(t)
                res = srv.collect(t)
                scat += res.stats(0).scatters
                lat.append(t_done - ta)
                kinds.append(reqs[k][0])
                rel_se.append(main_rel_se(b, res, reqs[k][0], reqs[k][1]))
                if k % 20 == 0:  # kept for the comparison with the same request run alone
                    kept[k] = res.raw(0)
                res.close()
        elif i < n_requests:
            time.sleep(max(0.0, min(arrivals[i] - now, 0.05)))
        if time.perf_counter() - t0 - last_log > 5.0:
            last_log = time.perf_counter() - t0
            log(f"serving t={last_log:.0f}s submitted {i} done {len(lat)} queued {q} running {r} "
                f"epochs {epochs} mean epoch {1e3 * epoch_s / max(epochs, 1):.1f} ms "
                f"events/s {scat / max(last_log, 1e-9):.3e}")
    wall = time.perf_counter() - t0
    srv.close()
    # each kept request (every 20th) alone, after the stream: the same tallies as in the mix
    worst = 0.0
    for k, a in kept.items():
        solo = b.simulate([reqs[k][1]], material=mat, stream=stream)
        c = solo.raw(0)
        worst = max(worst, float(abs(a - c).max() / max(abs(c).max(), 1e-300)))
        solo.close()

    def pct(vals, p):
        v = sorted(vals)
        return v[min(len(v) - 1, int(round(p / 100.0 * (len(v) - 1))))] if v else None

    at = [l for l, e in zip(lat, rel_se) if e <= 1e-3]
    by_kind = {}
    for kd in sorted(set(kinds)):
        e = [x for x, y in zip(rel_se, kinds) if y == kd]
        by_kind[kd] = {"requests": len(e), "median_rel_se": pct(e, 50), "max_rel_se": max(e),
                       "reached_1e-3": sum(1 for x in e if x <= 1e-3)}
    return {"requests": n_requests, "arrival_rate_per_s": rate, "mix_capacity_flights_per_s": capacity,
            "p50_latency_s": pct(lat, 50), "p99_latency_s": pct(lat, 99),
            "requests_at_1e-3_rel_se": len(at), "p50_latency_at_1e-3_s": pct(at, 50),
            "p99_latency_at_1e-3_s": pct(at, 99), "achieved_rel_se": by_kind,
            "rel_se_quantity": {"film": "heat flux q", "pore": "kappa",
                                "spot": "snapshot temperature of the hottest cell at the last time"},
            "scattering_events_per_s": scat / wall, "wall_s": wall, "epochs": epochs,
            "mean_epoch_ms": 1e3 * epoch_s / max(epochs, 1),
            "mix_vs_alone_checked": len(kept), "mix_vs_alone_max_rel_diff": worst,
            "mix": {k: kinds.count(k) for k in sorted(set(kinds))}}


def main_rel_se(b, res, kind, job):
    """Relative standard error of a served request's main quantity: the heat flux
    of a film (the same in every bin), the conductivity of a pore cell, the
    temperature of the hottest snapshot cell at the last time of a heated spot."""
    if kind == "film":
        m, se = res.read(0, b.Q_FLUX)
        return float(se[0] / max(abs(m[0]), 1e-300))
    if kind == "pore":
        m, se = res.read(0, b.Q_KAPPA)
        return float(se[0] / max(abs(m[0]), 1e-300))
    m, se = res.read(0, b.Q_SNAPSHOT, len(job.tally.times) - 1)
    i = int(abs(m).argmax())
    return float(se[i] / max(abs(m[i]), 1e-300))


def copy_probe():
    """A plain device copy of known size, for scaling the HBM traffic counters."""
    import torch
    n = 1 << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n}))


def kernel_sha1():
    """Hash of the device code with comments and layout removed (the kernel
    source and its private header): a comment edit keeps the counters valid,
    any code change invalidates them."""
    h = hashlib.sha1()
    for name in ("dmc_kernels.hip", "dmc_internal.h"):
        src = open(os.path.join(ROOT, "paper_1206_3316_amd", "csrc", name)).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=float, default=1e8, help="particles per film")
    ap.add_argument("--plain-n", type=float, default=1e7,
                    help="particles per film of the equal-N comparison with the plain form")
    ap.add_argument("--chunk", type=int, default=0, help="queue chunk (0: autotuned)")
    ap.add_argument("--refill-min", type=int, default=0, help="refill threshold (0: autotuned)")
    ap.add_argument("--block", type=int, default=0, help="workgroup size (0: autotuned)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (library defaults plus --block/--chunk/--refill-min); "
                         "profiles use it so that only the timed launches are traced")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--epoch-flights", type=float, default=2e10)
    ap.add_argument("--serve-max-s", type=float, default=120.0, help="stop admitting requests after this long")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="request arrival rate per second (default: 0.8 x the mix's measured capacity)")
    ap.add_argument("--serve-class-epochs", action="store_true",
                    help="epochs take one request class at a time, in that class's specialised kernel")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--op-costs", action="store_true",
                    help="print the instruction-cost probe's VALU slots per operation and exit")
    ap.add_argument("--only", choices=["spot", "nano"], default=None,
                    help="one launch of the heated spot (1e9, 64^3 x 50) or of the 64 nanostructures, "
                         "nothing else (for profiling those kernels)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the single-launch measurements of the heated spot and the batched nanostructures")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.op_costs:
        from paper_1206_3316_amd import binding as b
        c = op_costs(b)
        print(json.dumps({"op_costs_slots": c, "slab_ops_per_flight": sum(v for _, v in slab_items(c)),
                          "half_ops_per_flight": sum(v for _, v in half_items(c)),
                          "grad_unit_costs": grad_unit_costs(c)}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: run with --gpus 1 (sharding particle ranges across GPUs is not implemented)"}))
        sys.exit(2)

    import torch

    import dmc_inputs as di
    from paper_1206_3316_amd import binding as b

    torch.cuda.set_device(0)
    mat_in = di.silicon_like()
    jobs = di.cross_plane_films(n_per_film=int(args.n), material=mat_in)
    mat = b.Material(mat_in)
    stream = torch.cuda.current_stream()
    if args.only:
        ojobs = [di.heated_spot(material=mat_in)] if args.only == "spot" else di.batched_nanostructures(material=mat_in)
        params = launch_params(ojobs, mat, stream=stream,
                               overrides={"chunk": args.chunk, "refill_min": args.refill_min, "block": args.block},
                               tune=not args.no_tune)
        r = b.simulate(ojobs, material=mat, stream=stream, **params)
        st = [r.stats(i) for i in range(len(ojobs))]
        print(json.dumps({"workload": args.only, "launch": params, "kernel_ms": st[0].kernel_ms,
                          "flights": sum(x.iterations for x in st), "scattering_events": sum(x.scatters for x in st),
                          "particles": sum(x.particles for x in st)}))
        return
    nbytes = b.workspace_bytes(jobs, mat)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    t_tune = time.perf_counter()
    params = launch_params(jobs, mat, stream=stream,
                           overrides={"chunk": args.chunk, "refill_min": args.refill_min, "block": args.block},
                           tune=not args.no_tune)
    log(f"launch parameters {params} (autotuner {time.perf_counter() - t_tune:.1f} s, "
        f"{len(getattr(launch_params, 'trials', []))} trials)")

    def step():
        r = b.simulate(jobs, material=mat, precision="fp32", form="persistent", stream=stream, workspace=ws,
                       **params)
        return r, r.stats(-1)

    for i in range(args.warmup):
        r, st = step()
        log(f"warmup {i}: {st.scatters:.3e} scatters, kernel {st.kernel_ms:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scat = flights = parts = 0
    kms = []
    for i in range(args.steps):
        r, st = step()
        scat += st.scatters
        flights += st.iterations
        parts += st.particles
        kms.append(st.kernel_ms)
        log(f"step {i}: {st.scatters:.4e} scatters, {st.iterations:.4e} flights, kernel {st.kernel_ms:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    value = scat / wall
    kernel_s = sum(kms) / 1e3
    costs = op_costs(b)
    items = slab_items(costs)
    ops_per_flight = sum(v for _, v in items)
    achieved = ops_per_flight * flights / kernel_s
    out = {
        "metric": "scattering events/s", "value": value, "unit": "scattering events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 flight / f64 tally", "data": "synthetic",
        "config": {"workload": "12 silicon-like cross-plane films 10 nm - 10 um, 1e8 particles each "
                               "(1000 omega bins x LA+2TA, walls T_eq +- 0.5 K, 20 bins), one persistent launch",
                   "particles_per_step": parts // args.steps, "launch": params},
        "particles_per_s": parts / wall,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "T VALU lane-ops/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": TRAFFIC["bytes"] if TRAFFIC["kernel_sha1"] == kernel_sha1() else None,
                     "kernel": "persistent_kernel<float, GEOM_SLAB>", "ops_per_flight": ops_per_flight,
                     "ops_items": [[k, round(v, 3)] for k, v in items], "op_costs_slots": costs,
                     "flights_per_launch": flights / args.steps,
                     "kernel_ms_per_step": kernel_s * 1e3 / args.steps},
    }
    if not args.no_plain:
        out["plain_form"] = plain_vs_persistent(b, di, mat, mat_in, stream, int(args.plain_n))
        out["vs_plain"] = out["plain_form"]["persistent_fp32_over_plain"]
        out["plain_form"]["headline_over_plain_rate"] = value / out["plain_form"]["plain_fp64_events_per_s"]
    if args.serve_requests > 0:
        out["serving"] = serve(b, di, torch, mat, mat_in, stream, args.serve_requests, args)
        out["p50_latency_s"] = out["serving"]["p50_latency_s"]
        out["p99_latency_s"] = out["serving"]["p99_latency_s"]
        out["p50_latency_at_1e-3_rel_se_s"] = out["serving"]["p50_latency_at_1e-3_s"]
        out["p99_latency_at_1e-3_rel_se_s"] = out["serving"]["p99_latency_at_1e-3_s"]
    if not args.no_extra:
        out["other_workloads"] = other_workloads(b, di, mat, mat_in, stream, costs)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(jobs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
