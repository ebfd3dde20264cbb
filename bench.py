#!/usr/bin/env python3
"""Benchmark of the multigrid pressure solve on one MI355X.

Workload (the variable-density pressure-Poisson solve of the collapsing-column /
rising-bubble scheme, synthetic): 256^3 cells on the unit cube, rho = 1000 in a
sphere of radius 0.15 at the centre and 1 outside (two-cell ramp), k = 1/rho,
zero-normal-derivative walls, Gaussian right-hand side projected to zero mean.
One step = one solve from x = 0 to relative residual 1e-8 (FP64 throughout):
b-norm, the finest residual before each cycle, every sawtooth V(0,2) cycle and
the final projection.  The hierarchy (coefficient coarsening, coarsest inverse)
is built once before the timed region, as a time-stepping code keeps it
resident; its cost is reported separately.

Prints one JSON line: value = finest cells x V-cycles / second / 1e9
(Gcell-updates/s), the roofline figure of the dominant kernel from HIP events
recorded on the solve stream, and beside it: the FP32-smoothing / FP64-refinement
solve of the same workload, the flexible-CG outer iteration (time to the same
tolerance), the 64^3 constant-coefficient Dirichlet Poisson solve, the
256 x 256 x 512 rising-bubble solve with the FP16-stored coefficient (and its
difference from the FP64 solve of the same system), one two-phase time step on
a 128^3 collapsing column split into pressure solves and explicit stencils (and
the same step at 64^3 .. 256^3 with M_s and H_s of Eq. speed fitted), the
mass-conservation study of the i-j correction strategies over 1000 steps of a
reduced rising bubble (C(t)/C0), the served stream of 512 solves of uneven
sizes (solves/s, p50/p99 latency), and
the FP64 oracle timed on the host over a bounded sample of V-cycles of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# Algorithmic bytes per finest cell of each finest-level kernel class: every
# array the kernel needs is read once and every output written once.  With the
# default two post-sweeps, both run in one pass ("sweeps").  In FP64 that pass
# smooths x + P e_1 against b and writes the new iterate to a second buffer, so
# the residual kernel writes only the restricted residual; in mixed precision it
# smooths the FP32 correction against the FP32 residual the residual kernel
# writes out.
BYTES_PER_CELL = {
    "fp64": {"resid": 8 + 8 + 8 + 1,          # x, b, k; restricted residual (1/8 cell)
             "sweeps": 1 + 8 + 8 + 8 + 8,     # e_1 (1/8), x, b, k; x' written
             "sweep": 8 + 8 + 8 + 8},         # (nu_post != 2 only) y, b, k; x
    "mixed": {"resid": 8 + 8 + 8 + 4 + 0.5,   # x, b, k (FP64); r32, restricted r32
              "sweeps": 0.5 + 4 + 4 + 8 + 8,  # e_1 (FP32, 1/8), r32, k32; x64 read + write
              "sweep": 4 + 4 + 4 + 8 + 8},    # (nu_post != 2 only)
    "fp16": {"resid": 8 + 8 + 8 + 4 + 0.5,    # as mixed, smoothing with the FP16 copy of k
             "sweeps": 0.5 + 4 + 2 + 8 + 8,
             "sweep": 4 + 4 + 2 + 8 + 8},
    "fp64c": {"resid": 8 + 8 + 1,             # constant coefficient: no k
              "sweeps": 1 + 8 + 8 + 8,
              "sweep": 8 + 8 + 8},
}
# FP64 with the finest sweeps in the 8^3 block form (an autotuner choice on
# small grids): the correction is smoothed against the full residual r, which
# the residual kernel writes out, and added into x.
BYTES_PER_CELL_BLOCK = {
    "fp64": {"resid": 8 + 8 + 8 + 8 + 1,      # x, b, k; r, restricted residual
             "sweeps": 1 + 8 + 8 + 8 + 8,     # e_1, r, k; x read + write
             "sweep": 8 + 8 + 8 + 8},
    "fp64c": {"resid": 8 + 8 + 8 + 1,
              "sweeps": 1 + 8 + 8 + 8,
              "sweep": 8 + 8 + 8},
}


def fine_bytes(mode, res):
    """Bytes per finest cell of each kernel class in the run `res`."""
    tiles = res.get("tiles")
    if mode in BYTES_PER_CELL_BLOCK and tiles and list(tiles[0][1]) == [8, 8, 8]:
        return BYTES_PER_CELL_BLOCK[mode]
    return BYTES_PER_CELL[mode]
# bytes per cell of the coefficient on the coarse levels, per mode
COARSE_K_BYTES = {"fp64": 8, "mixed": 4, "fp16": 2, "fp64c": 0}
KCLASS = {"resid": 0, "sweeps": 1, "sweep": 2}

# HBM bytes per finest-level launch (256^3, FP64, nodal k) from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by what the same counters read for
# a plain 256 MiB device copy (fetch x2.0, write x1.0); the commands and raw
# counts are in profiles/dense_sphere_256_fp64_fine_kernels.md.  Each figure
# carries a hash of the kernel's source files and the algorithmic bytes per
# cell of the form it ran in (which outputs the launch writes), as profiled;
# once either differs, the figure no longer describes the kernel and traffic
# is null.
KERNEL_SOURCES = {"resid": ("mg_stencil.hip", "mg_device.h", "mg_internal.h"),
                  "sweeps": ("mg_fused.hip", "mg_device.h", "mg_internal.h")}
MEASURED_TRAFFIC_FP64_256 = {"resid": (430.9e6, "709d85d8a64f9915", 25),
                             "sweeps": (620.0e6, "e73c1377598a5410", 33)}


def kernel_source_hash(cls):
    import hashlib

    m = hashlib.sha256()
    for f in KERNEL_SOURCES[cls]:
        with open(os.path.join(ROOT, "paper_2401_06755_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_traffic(table, bytes_per_cell):
    """Counter-measured bytes per launch of each kernel class whose sources
    still hash to the profiled ones and that ran in the profiled form."""
    return {cls: val for cls, (val, hsh, bpc) in table.items()
            if kernel_source_hash(cls) == hsh and bytes_per_cell.get(cls) == bpc}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cycle_model_bytes(res, mode):
    """Algorithmic bytes of one V(0,2) cycle over all levels (finest kernels as
    above; coarse level l: restriction w + w/8 B, both sweeps in one pass
    reading e_{l+1} (w/8), b, k and writing e (3w); FP32 on coarse levels in
    mixed mode; no k with a constant coefficient)."""
    levels = res["levels"]
    w = 8 if mode in ("fp64", "fp64c") else 4
    kb = COARSE_K_BYTES[mode]
    n0 = levels[0][0] * levels[0][1] * levels[0][2]
    fb = fine_bytes(mode, res)
    tot = n0 * (fb["resid"] + fb["sweeps"])
    for l in range(1, len(levels) - 1):
        n = levels[l][0] * levels[l][1] * levels[l][2]
        tot += n * ((w + w / 8) + (w / 8 + 2 * w + kb))
    return tot


def run_solver(nn4mg, torch, work, precision, steps, warmup, rtol, autotune=True, outer=0, profile=True,
               keep_x=False):
    nx, ny, nz = work["shape"]
    n = nx * ny * nz
    nodal = work["k"] is not None
    cfg = nn4mg.config_default(nx, ny, nz, work["h"], bc=work["bc"],
                               coef_mode=nn4mg.COEF_NODAL if nodal else nn4mg.COEF_CONST,
                               precision=precision, outer=outer)
    kd = torch.from_numpy(work["k"].reshape(-1)).cuda() if nodal else None
    bd = torch.from_numpy(work["b"].reshape(-1)).cuda()
    xd = torch.zeros_like(bd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = nn4mg.Hierarchy(cfg, kd)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    update_ms = None
    if nodal:
        t0 = time.perf_counter()
        H.update_coef(kd)
        torch.cuda.synchronize()
        update_ms = (time.perf_counter() - t0) * 1e3
    tiles, tune_ms = None, 0.0
    if autotune:
        t0 = time.perf_counter()
        tiles = H.autotune(bd, xd)
        tune_ms = (time.perf_counter() - t0) * 1e3
        log(f"  autotuned tiles per level (resid, first sweep, sweep): {tiles}")
    info = None
    for w in range(warmup):
        xd.zero_()
        info = H.solve(bd, xd, rtol=rtol, max_cycles=2000)
        log(f"  warmup {w}: cycles {info.cycles} relres {info.relres:.3e} {info.solve_ms:.1f} ms")
    # timed region: K solves, no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = 0
    infos = []
    for s in range(steps):
        xd.zero_()
        info = H.solve(bd, xd, rtol=rtol, max_cycles=2000)
        cycles += info.cycles
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for s, inf in enumerate(infos):
        log(f"  step {s}: cycles {inf.cycles} relres {inf.relres:.3e} status {inf.status} {inf.solve_ms:.1f} ms")
    # the same K solves again with every finest-level launch bracketed by HIP
    # events on the solve stream (event records add a little host overhead,
    # so they are kept out of the timed region above)
    kern, dt_prof = {}, 0.0
    if profile:
        H.profile(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for s in range(steps):
            xd.zero_()
            H.solve(bd, xd, rtol=rtol, max_cycles=2000)
        torch.cuda.synchronize()
        dt_prof = time.perf_counter() - t1
        H.profile(False)
        for name, cls in KCLASS.items():
            cnt, ms = H.profile_read(cls)
            kern[name] = (cnt, ms)
    levels = H.levels()
    if keep_x:
        xd.zero_()
        H.solve(bd, xd, rtol=rtol, max_cycles=2000)
    H.close()
    return dict(n=n, dt=dt, dt_prof=dt_prof, cycles=cycles, info=infos[-1], kern=kern, levels=levels,
                x=xd if keep_x else None,
                setup_ms=setup_ms,
                update_ms=update_ms, tiles=tiles, tune_ms=tune_ms,
                all_converged=all(i.status == 0 for i in infos))


def roofline(res, mode, traffic=None):
    best = None
    for name, (cnt, ms) in res["kern"].items():
        if cnt == 0:
            continue
        if best is None or ms > res["kern"][best][1]:
            best = name
    cnt, ms = res["kern"][best]
    avg_s = ms / cnt / 1e3
    fb = fine_bytes(mode, res)
    bytes_per_launch = fb[best] * res["n"]
    achieved = bytes_per_launch / avg_s / 1e9
    per_kernel = {}
    for name, (c, m) in res["kern"].items():
        if c:
            a = fb[name] * res["n"] / (m / c / 1e3) / 1e9
            per_kernel[name] = {"launches": c, "avg_us": round(m / c * 1e3, 2), "GBps": round(a, 1),
                                "bytes_per_cell": fb[name]}
    tr = traffic.get(best) if traffic else None
    return best, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                  "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": tr}, per_kernel


def percentile(v, p):
    import numpy as np

    return float(np.percentile(np.asarray(v), p)) if len(v) else None


def serving_bench(nn4mg, torch, n_requests, budget_gib, slots, bound_budget_gib=1.0, seed_base=4000):
    """Served stream: n_requests variable-coefficient solves (cube edges drawn
    from {32, 48, 64, 96, 128}, random dense sphere, Neumann walls), FP32
    smoothing + FP64 refinement to rtol 1e-8, up to `slots` running at once
    (requests of one size run as copies of one batched group).  First closed
    loop (everything submitted at once) for the capacity, then open loop with
    Poisson arrivals at 0.7 x that capacity (latency = completion - arrival),
    then the closed loop again under an HBM budget small enough to bind
    (groups smaller, idle ones evicted)."""
    import numpy as np

    from paper_2401_06755_amd import inputs

    t0 = time.perf_counter()
    reqs = []
    for i in range(n_requests):
        w = inputs.served_request(i, base_seed=seed_base)
        n = w["edge"]
        cfg = nn4mg.config_default(n, n, n, w["h"], bc=w["bc"], coef_mode=nn4mg.COEF_NODAL,
                                   precision=nn4mg.PREC_FP32_SMOOTH)
        reqs.append((cfg, torch.from_numpy(w["k"].reshape(-1)).cuda(), torch.from_numpy(w["b"].reshape(-1)).cuda()))
    torch.cuda.synchronize()
    cells = sum(c.nx * c.ny * c.nz for c, _, _ in reqs)
    log(f"  generated {n_requests} requests ({cells / n_requests:.0f} cells mean) in {time.perf_counter() - t0:.1f} s")
    budget = int(budget_gib * 2 ** 30)

    def run(arrivals, bud):
        srv = nn4mg.Server(bud, slots)
        xs = [torch.zeros_like(b) for _, _, b in reqs]
        torch.cuda.synchronize()
        results = []
        start = time.perf_counter()
        nxt = 0
        last_log = start
        while len(results) < len(reqs):
            now = time.perf_counter() - start
            while nxt < len(reqs) and arrivals[nxt] <= now:
                cfg, k, b = reqs[nxt]
                srv.submit(cfg, b, xs[nxt], k=k, rtol=1e-8, max_cycles=2000, tag=nxt)
                nxt += 1
            results.extend(srv.poll())
            if time.perf_counter() - last_log > 20:
                log(f"    {len(results)}/{len(reqs)} served")
                last_log = time.perf_counter()
            if nxt < len(reqs) and arrivals[nxt] > now:
                time.sleep(min(5e-4, arrivals[nxt] - now))
            else:
                time.sleep(2e-4)
        wall = time.perf_counter() - start
        st = srv.stats()
        srv.close()
        lat = [r.t_done_ms - r.t_submit_ms for r in results]
        ok = sum(1 for r in results if r.info.status == 0)
        cyc = [r.info.cycles for r in results]
        return dict(wall=wall, lat=lat, ok=ok, cycles=cyc, peak=st["peak_bytes"])

    closed = run([0.0] * len(reqs), budget)
    capacity = len(reqs) / closed["wall"]
    rate = 0.7 * capacity
    rng = np.random.default_rng(seed_base)
    arrivals = list(np.cumsum(rng.exponential(1.0 / rate, size=len(reqs))))
    opened = run(arrivals, budget)
    bound = run([0.0] * len(reqs), int(bound_budget_gib * 2 ** 30))
    return {"requests": len(reqs), "mean_cells": round(cells / len(reqs)),
            "precision": "f32 smoothing + f64 residual/coarsest/refinement", "rtol": 1e-8,
            "hbm_budget_GiB": budget_gib, "slots": slots,
            "closed_loop": {"solves_per_s": round(capacity, 2), "wall_s": round(closed["wall"], 3),
                            "p50_ms": round(percentile(closed["lat"], 50), 2),
                            "p99_ms": round(percentile(closed["lat"], 99), 2), "converged": closed["ok"],
                            "peak_GiB": round(closed["peak"] / 2 ** 30, 3)},
            "open_loop": {"arrival_rate_per_s": round(rate, 2),
                          "solves_per_s": round(len(reqs) / opened["wall"], 2),
                          "p50_ms": round(percentile(opened["lat"], 50), 2),
                          "p99_ms": round(percentile(opened["lat"], 99), 2), "converged": opened["ok"],
                          "peak_GiB": round(opened["peak"] / 2 ** 30, 3)},
            "bound_budget": {"hbm_budget_GiB": bound_budget_gib,
                             "solves_per_s": round(len(reqs) / bound["wall"], 2),
                             "p99_ms": round(percentile(bound["lat"], 99), 2), "converged": bound["ok"],
                             "peak_GiB": round(bound["peak"] / 2 ** 30, 3)},
            "mean_cycles": round(float(np.mean(closed["cycles"])), 1),
            "gcell_updates_per_s_closed": round(sum(c.nx * c.ny * c.nz * cy for (c, _, _), cy in
                                                    zip(reqs, closed["cycles"])) / closed["wall"] / 1e9, 3)}


def step_bench(nn4mg, torch, n, steps, order=1):
    """One full two-phase time step (Sec. 2.4 Stages 1-4) on the n^3 collapsing
    water column (water/air, 20 cycles x 3 pressure solves), each timed step
    starting from the same initial state; device time from HIP events, split
    into the pressure solves (H) and the explicit momentum/volume-fraction
    stencils (M) like Eq. speed.  order 2: quadratic ConvFEM filters for the
    momentum, interface and volume-fraction advection terms."""
    import numpy as np

    from paper_2401_06755_amd import inputs

    h, st = inputs.water_block(n)
    init = {k: torch.from_numpy(np.ascontiguousarray(st[k]).reshape(-1)).cuda() for k in nn4mg.STEP_FIELDS}
    dev = {k: torch.empty_like(v) for k, v in init.items()}
    S = nn4mg.Stepper(n, n, n, h, nn4mg.step_params(order=order))
    tot, mg = [], []
    for i in range(steps + 1):
        for k in dev:
            dev[k].copy_(init[k])
        info = S.step(dev)
        if i > 0:
            tot.append(info.ms_total)
            mg.append(info.ms_mg)
    S.close()
    t, m = float(np.median(tot)), float(np.median(mg))
    cells = n ** 3
    p = nn4mg.step_params()
    cycles = p.mg_cycles * (1 + p.n_corr)
    return {"workload": f"collapsing water column {n}^3 (block [0,0.25]x[0,1]x[0,0.5]), water/air, "
                        f"dt 1e-4, {p.n_vel_iter} predictor iterations, {p.n_corr} corrections, "
                        f"{p.mg_cycles} cycles per pressure solve, "
                        + ("linear filters" if order != 2 else
                           "quadratic ConvFEM filters for momentum/interface/VOF advection (p = 2)"),
            "ms_per_step": round(t, 3), "ms_pressure_solves": round(m, 3), "ms_explicit": round(t - m, 3),
            "solve_share": round(m / t, 3), "steps_timed": steps,
            "p": 2 if order == 2 else 1,
            "M_s": (t - m) * 1e-3 / (cells * (2 if order == 2 else 1)), "H_s": m * 1e-3 / (cycles * cells),
            "relres": [info.relres[i] for i in range(info.solves)],
            "paper_context": {"M_s": 1.2e-8, "H_s": 1.1e-10, "hardware": "NVIDIA A10",
                              "note": "Eq. speed coefficients: seconds per node (times polynomial order p; here p = 1)"}}


def mass_study(nn4mg, torch, nx=32, steps=1000, ratio=2.0):
    """The mass-conservation study of Sec. 3.2 (Fig. Multigrid_iteration):
    C(t)/C0, C(t) = sum C^n h^3, over `steps` steps of a rising air bubble
    (radius H/2 at height H in a 3H x 3H x 6H water tank, 6 mm wide, nx x nx x
    2nx cells) for the i-j strategies (i corrections, j cycles per correction
    solve; the hydrostatic solve keeps 20).  The density ratio is 2, not the
    paper's water/air: the printed correction multiplies the light-phase
    interface speed by about (rho_l - rho_g) / (2 rho_g) per correction, which
    diverges within a few steps at a sharp interface once the ratio exceeds 3."""
    import numpy as np

    from paper_2401_06755_amd import inputs

    width = 6e-3
    _, st = inputs.bubble_state(nx)
    h = width / nx
    nz, ny = st["C"].shape[:2]
    out = {"workload": f"rising bubble {nx}x{nx}x{2 * nx}, tank 6 mm x 6 mm x 12 mm, bubble radius 1 mm at "
                       f"(3, 3, 2) mm, density ratio {ratio:g} (rho_l 1000), mu 1e-3/1.8e-5, sigma 0.07, "
                       f"dt 1e-5 s, {steps} steps, 2 predictor iterations, hydrostatic solve 20 cycles",
           "strategies": {}}
    sample = sorted(set([0] + list(range(0, steps + 1, max(1, steps // 10))) + [steps]))
    for i, j in ((1, 10), (2, 10), (1, 20), (2, 20)):
        dev = {k: torch.from_numpy(np.ascontiguousarray(st[k]).reshape(-1).copy()).cuda() for k in nn4mg.STEP_FIELDS}
        S = nn4mg.Stepper(nx, ny, nz, h, nn4mg.step_params(rho_g=1000.0 / ratio, dt=1e-5, n_corr=i, mg_cycles=20,
                                                           mg_cycles_nh=j))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vols, done, info = S.run(dev, steps, raise_on_breakdown=False)
        dt = time.perf_counter() - t0
        S.close()
        v = np.array(vols)
        ratio_t = v / v[0]
        out["strategies"][f"{i}-{j}"] = {
            "steps_done": done,
            "C_over_C0": {str(n): float(ratio_t[n]) for n in sample if n < len(ratio_t)},
            "max_abs_drift": float(np.max(np.abs(ratio_t - 1.0))),
            "final_drift": float(ratio_t[-1] - 1.0),
            "ms_per_step": round(dt / max(done, 1) * 1e3, 3)}
        log(f"  strategy {i}-{j}: {done} steps, C(t)/C0 - 1 = {ratio_t[-1] - 1.0:.3e}, "
            f"{dt / max(done, 1) * 1e3:.2f} ms/step")
    out["note"] = ("the paper gives this study only as a figure (no values), so the comparison is "
                   "qualitative: more corrections (i) and more cycles (j) should conserve better")
    return out


def eq_speed_fit(nn4mg, torch, sizes=(64, 96, 128, 192, 256), steps=2):
    """Eq. speed on this GPU: the collapsing-column step timed at several grid
    sizes, then M_s and H_s fitted by least squares, p = 1.  The headline fit
    is affine (explicit time = c_M + N M_s, pressure-solve time =
    c_H + N (N_h + N_I N_nh) H_s): the fixed terms are the launch-bound cost of
    the coarse levels and small kernels, which the paper's model (a line
    through the origin) has no room for and which dominates small grids here.
    The through-origin fit of the paper's form is reported beside it, with each
    size's deviation from both."""
    import numpy as np

    pts = []
    for n in sizes:
        r = step_bench(nn4mg, torch, n, steps)
        pts.append((n, n ** 3, r["ms_per_step"], r["ms_pressure_solves"], r["ms_explicit"]))
        log(f"  step {n}^3: {r['ms_per_step']:.3f} ms ({r['ms_pressure_solves']:.3f} ms in the solves)")
    p = nn4mg.step_params()
    cycles = p.mg_cycles * (1 + p.n_corr)
    N = np.array([q[1] for q in pts], dtype=np.float64)
    mg = np.array([q[3] for q in pts]) * 1e-3
    ex = np.array([q[4] for q in pts]) * 1e-3
    Ms = float(np.dot(N, ex) / np.dot(N, N))
    Hs = float(np.dot(N * cycles, mg) / np.dot(N * cycles, N * cycles))
    model = N * (Ms + cycles * Hs)
    meas = mg + ex
    # affine fits: a fixed per-step cost (launch-bound coarse levels, small grids) plus the per-node slope
    A = np.stack([np.ones_like(N), N], axis=1)
    (ex0, Ms_a), (mg0, mgs) = np.linalg.lstsq(A, ex, rcond=None)[0], np.linalg.lstsq(A, mg, rcond=None)[0]
    model_a = (ex0 + N * Ms_a) + (mg0 + N * mgs)
    return {"sizes": [q[0] for q in pts], "ms_per_step": [q[2] for q in pts],
            "ms_pressure_solves": [q[3] for q in pts], "ms_explicit": [q[4] for q in pts],
            "cycles_per_step": cycles,
            "M_s": float(Ms_a), "H_s": float(mgs / cycles),
            "explicit_fixed_ms": round(float(ex0) * 1e3, 3), "solves_fixed_ms": round(float(mg0) * 1e3, 3),
            "model_rel_error": [round(float(v), 3) for v in (model_a - meas) / meas],
            "fit": "affine least squares over the sizes listed (fixed per-step cost + per-node slope), p = 1",
            "through_origin": {"M_s": Ms, "H_s": Hs,
                               "model_rel_error": [round(float(v), 3) for v in (model - meas) / meas],
                               "fit": "least squares through the origin, the paper's form"},
            "paper_context": {"A10": {"M_s": 1.2e-8, "H_s": 1.1e-10}, "RTX A5000": {"M_s": 1.37e-8, "H_s": 1.3e-10}}}


def poisson64_bench(nn4mg, torch, inputs, steps, warmup, rtol):
    """64^3 constant-coefficient Poisson on the unit cube, zero Dirichlet walls,
    sine mode plus 1e-3 uniform noise, FP64 V(0,2) to rtol.  The grid (2 MiB per
    field) runs from the on-die caches, so this is a latency figure."""
    work = inputs.poisson_sine_noise(64, seed=1)
    r = run_solver(nn4mg, torch, work, nn4mg.PREC_FP64, steps, warmup, rtol)
    best, roof, pk = roofline(r, "fp64c")
    hist = r["info"].history()
    return {"workload": "64^3 constant-coefficient Poisson, zero Dirichlet, sin(pi x)sin(pi y)sin(pi z) "
                        "+ 1e-3 U[-1,1), FP64 V(0,2) to rtol 1e-8, 5 levels to 4^3",
            "value": round(r["n"] * r["cycles"] / r["dt"] / 1e9, 3), "unit": "Gcell-updates/s",
            "ms_per_solve": round(r["dt"] / steps * 1e3, 3), "cycles_per_solve": r["info"].cycles,
            "relres": r["info"].relres,
            "reduction_per_cycle": round((r["info"].relres / r["info"].relres0) ** (1.0 / r["info"].cycles), 4),
            "relres_history_first": [float(f"{v:.3e}") for v in hist[:6]],
            "all_converged": r["all_converged"], "fine_kernels": pk,
            "note": "all fields fit the 256 MB on-die cache; launch/latency-bound"}


def bubble_bench(nn4mg, torch, inputs, steps, rtol):
    """256 x 256 x 512 rising-bubble solve with the FP16-stored coefficient,
    FP32 smoothing and FP64 residual/refinement, autotuned tiles per level;
    its solution against the FP64 solve of the same system on the GPU."""
    work = inputs.rising_bubble(256, seed=5)
    r16 = run_solver(nn4mg, torch, work, nn4mg.PREC_FP16_COEF, steps, 1, rtol, keep_x=True)
    r64 = run_solver(nn4mg, torch, work, nn4mg.PREC_FP64, 1, 0, rtol, profile=False, keep_x=True)
    rf = run_solver(nn4mg, torch, work, nn4mg.PREC_FP16_COEF, 1, 1, rtol, outer=nn4mg.OUTER_FCG, profile=False)
    x16, x64 = r16["x"], r64["x"]
    err = float(torch.linalg.vector_norm(x16 - x64) / torch.linalg.vector_norm(x64))
    best, roof, pk = roofline(r16, "fp16")
    model = cycle_model_bytes(r16, "fp16")
    return {"workload": "rising bubble 256x256x512 on a 1x1x2 box, air sphere r=0.25 at (0.5,0.5,0.5) in water "
                        "(rho 1/1000), zero pressure on top, Neumann elsewhere, Gaussian RHS",
            "dtype": "f16-stored k, f32 smoothing, f64 residual/coarsest/refinement",
            "value": round(r16["n"] * r16["cycles"] / r16["dt"] / 1e9, 3), "unit": "Gcell-updates/s",
            "ms_per_solve": round(r16["dt"] / steps * 1e3, 3), "cycles_per_solve": r16["info"].cycles,
            "relres": r16["info"].relres, "all_converged": r16["all_converged"],
            "fp64_solve_ms": round(r64["dt"] * 1e3, 3), "fp64_cycles": r64["info"].cycles,
            "rel_diff_vs_fp64_solution": float(f"{err:.3e}"),
            "fcg": {"ms_per_solve": round(rf["dt"] * 1e3, 3), "iterations": rf["info"].cycles,
                    "relres": rf["info"].relres, "all_converged": rf["all_converged"]},
            "roofline": roof, "roofline_kernel": best, "fine_kernels": pk,
            "hbm_model_GBps": round(model * r16["cycles"] / r16["dt"] / 1e9, 1),
            "model_bytes_per_cell_cycle": round(model / r16["n"], 2),
            "tiles_per_level": r16["tiles"]}


def _cpu_leg(threads):
    """Runs in a child process: the oracle timed on `threads` host threads
    (1: the parity build; more: the OpenMP build of the same sources, chosen
    by the environment before the oracle is loaded).  Median of 5 runs of one
    V-cycle of the 256^3 dense-sphere workload and of the whole 64^3 Poisson
    solve to 1e-8, after one warm-up of each."""
    import statistics

    import numpy as np

    import oracle
    from paper_2401_06755_amd import inputs

    out = {"threads": threads}
    w = inputs.dense_sphere(256, seed=2)
    OH = oracle.Hierarchy(w["shape"], w["h"], w["bc"], k=w["k"])
    b = w["b"] - w["b"].mean()
    x = OH.vcycle(np.zeros_like(b), b)  # warm-up
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        x = OH.vcycle(x, b)
        ts.append(time.perf_counter() - t0)
    out["dense_sphere_256_s_per_cycle"] = statistics.median(ts)
    p = inputs.poisson_sine_noise(64, seed=1)
    P = oracle.Hierarchy(p["shape"], p["h"], p["bc"])
    _, hist, _ = P.solve(p["b"], rtol=1e-8, max_cycles=100)  # warm-up
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        P.solve(p["b"], rtol=1e-8, max_cycles=100)
        ts.append(time.perf_counter() - t0)
    out["poisson64_solve_s"] = statistics.median(ts)
    out["poisson64_cycles"] = len(hist) - 1
    return out


def _host_description():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(gpu_cycles_per_solve):
    """The FP64 oracle on the host, beside the GPU: one thread (the parity
    build as it stands) and every thread the process may use (the OpenMP
    build; OMP_NUM_THREADS if set, else the affinity mask).  Each leg runs in
    a child process (about 15 s on one thread); value is the all-threads
    figure in the benchmark's unit on the 256^3 workload's V-cycles, with the
    whole 256^3 solve projected from the median cycle time and the GPU's
    cycle count (a whole oracle solve there takes minutes)."""
    import subprocess

    import oracle

    oracle.build(force=False)
    oracle.build_timing()
    model, ncpu, avail = _host_description()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or avail
    legs = {}
    for name, t in (("one_thread", 1), ("all_threads", threads)):
        env = dict(os.environ, OMP_NUM_THREADS=str(t))
        if t > 1:
            env["NN4MG_ORACLE_OPENMP"] = "1"
        code = f"import json, bench; print(json.dumps(bench._cpu_leg({t})))"
        p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=600)
        if p.returncode != 0:
            raise RuntimeError(f"CPU baseline leg ({t} threads) failed: {p.stderr[-2000:]}")
        legs[name] = json.loads(p.stdout.strip().splitlines()[-1])
    n = 256 ** 3
    best = legs["all_threads"]
    for leg in legs.values():
        leg["dense_sphere_256_Gcell_updates_per_s"] = round(n / leg["dense_sphere_256_s_per_cycle"] / 1e9, 5)
        leg["dense_sphere_256_solve_s_projected"] = round(leg["dense_sphere_256_s_per_cycle"] * gpu_cycles_per_solve, 1)
    return {"value": best["dense_sphere_256_Gcell_updates_per_s"], "unit": "Gcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"median of 5 FP64 V(0,2) cycles of the 256^3 dense-sphere workload (and of 5 whole 64^3 "
                      f"Poisson solves to 1e-8) per leg, after a warm-up; OpenMP build on {threads} threads, "
                      f"parity build on 1",
            "host": {"cpu_model": model, "os_cpu_count": ncpu, "threads_available": avail},
            "legs": legs}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid edge (default 256)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-fcg", action="store_true", help="skip the flexible-CG outer iteration legs")
    ap.add_argument("--serve-requests", type=int, default=512, help="served-stream requests (0: skip)")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-bound-budget-gib", type=float, default=1.0)
    ap.add_argument("--step-n", type=int, default=128, help="time-step grid edge (0: skip)")
    ap.add_argument("--step-steps", type=int, default=3)
    ap.add_argument("--mass-steps", type=int, default=1000,
                    help="steps per strategy of the mass-conservation study (0: skip)")
    ap.add_argument("--no-poisson64", action="store_true", help="skip the 64^3 constant-coefficient leg")
    ap.add_argument("--no-bubble", action="store_true", help="skip the 256x256x512 FP16-coefficient leg")
    ap.add_argument("--no-eq-speed", action="store_true", help="skip the multi-size time-step fit of Eq. speed")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy first (reference for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2401_06755_amd import inputs, nn4mg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.ones(32 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"generating the {args.n}^3 dense-sphere workload")
    work = inputs.dense_sphere(args.n, seed=2)
    log("FP64 solve")
    r64 = run_solver(nn4mg, torch, work, nn4mg.PREC_FP64, args.steps, args.warmup, args.rtol,
                     autotune=not args.no_autotune)
    value = r64["n"] * r64["cycles"] / r64["dt"] / 1e9
    best, roof, per_kernel = roofline(r64, "fp64",
                                      measured_traffic(MEASURED_TRAFFIC_FP64_256, fine_bytes("fp64", r64))
                                      if args.n == 256 else None)
    model_bytes = cycle_model_bytes(r64, "fp64")
    out = {
        "metric": "V-cycle Gcell-updates/s (solve to relative residual 1e-8)",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["dt"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"variable-density pressure Poisson {args.n}^3, dense sphere r=0.15 "
                               "rho 1000/1 (k=1/rho), Neumann walls, zero-mean Gaussian RHS, "
                               "sawtooth V(0,2) to rtol 1e-8",
                   "grid": [args.n] * 3, "levels": len(r64["levels"]),
                   "cycles_per_solve": r64["info"].cycles, "precision": "fp64",
                   "relres": r64["info"].relres, "all_converged": r64["all_converged"]},
        "roofline": roof,
        "roofline_kernel": {"class": best, **per_kernel[best],
                            "timing": "HIP events on the solve stream over a second run of the same K steps"},
        "ms_per_step_profiled": round(r64["dt_prof"] / args.steps * 1e3, 3),
        "fine_kernels": per_kernel,
        "hbm_model_GBps": round(model_bytes * r64["cycles"] / r64["dt"] / 1e9, 1),
        "model_bytes_per_cell_cycle": round(model_bytes / r64["n"], 2),
        "setup_ms": round(r64["setup_ms"], 2),
        "autotune_ms": round(r64["tune_ms"], 1),
        "tiles_per_level": r64["tiles"],
        "update_coef_ms": round(r64["update_ms"], 2) if r64["update_ms"] is not None else None,
        "paper_context": {"metric": "1/H_s node-cycles/s (Eq. speed)", "value_G": 9.09,
                          "hardware": "NVIDIA A10", "precision": "not stated"},
    }
    if not args.no_mixed:
        log("mixed precision solve (FP32 smoothing, FP64 residual/refinement)")
        rm = run_solver(nn4mg, torch, work, nn4mg.PREC_FP32_SMOOTH, args.steps, args.warmup, args.rtol,
                        autotune=not args.no_autotune)
        bm, roofm, pkm = roofline(rm, "mixed")
        out["mixed"] = {"value": round(rm["n"] * rm["cycles"] / rm["dt"] / 1e9, 3),
                        "ms_per_step": round(rm["dt"] / args.steps * 1e3, 3),
                        "cycles_per_solve": rm["info"].cycles, "relres": rm["info"].relres,
                        "speedup_vs_fp64_solve": round(r64["dt"] / rm["dt"], 3),
                        "dtype": "f32 smoothing + f64 residual/coarsest/refinement",
                        "roofline": roofm, "roofline_kernel": bm, "fine_kernels": pkm}
    if not args.no_fcg:
        fcg = {}
        for name, prec in (("fp64", nn4mg.PREC_FP64), ("mixed", nn4mg.PREC_FP32_SMOOTH)):
            if name == "mixed" and args.no_mixed:
                continue
            log(f"flexible CG outer iteration, {name} cycle")
            rf = run_solver(nn4mg, torch, work, prec, args.steps, args.warmup, args.rtol,
                            autotune=not args.no_autotune, outer=nn4mg.OUTER_FCG, profile=False)
            ms = rf["dt"] / args.steps * 1e3
            fcg[name] = {"ms_per_solve": round(ms, 3), "iterations_per_solve": rf["info"].cycles,
                         "relres": rf["info"].relres, "all_converged": rf["all_converged"],
                         "speedup_vs_stationary_fp64": round(r64["dt"] / rf["dt"], 3)}
        out["fcg"] = fcg
    if not args.no_poisson64:
        log("64^3 constant-coefficient Poisson, zero Dirichlet walls, FP64")
        out["poisson64"] = poisson64_bench(nn4mg, torch, inputs, args.steps, args.warmup, args.rtol)
    if not args.no_bubble:
        log("rising bubble 256x256x512, FP16-stored coefficient")
        out["bubble"] = bubble_bench(nn4mg, torch, inputs, min(args.steps, 3), args.rtol)
    if args.serve_requests > 0:
        log(f"served stream: {args.serve_requests} requests")
        out["serving"] = serving_bench(nn4mg, torch, args.serve_requests, args.serve_budget_gib, args.serve_slots,
                                       args.serve_bound_budget_gib)
    if args.step_n > 0:
        log(f"time step: {args.step_n}^3 collapsing column")
        out["step"] = step_bench(nn4mg, torch, args.step_n, args.step_steps)
        log(f"time step with quadratic ConvFEM filters: {args.step_n}^3 collapsing column")
        out["step_quadratic"] = step_bench(nn4mg, torch, args.step_n, args.step_steps, order=2)
    if args.mass_steps > 0:
        log(f"mass-conservation study: {args.mass_steps} steps per strategy")
        out["mass_study"] = mass_study(nn4mg, torch, steps=args.mass_steps)
    if not args.no_eq_speed:
        log("Eq. speed fit: time step at 64^3 .. 256^3")
        out["eq_speed"] = eq_speed_fit(nn4mg, torch)
    if not args.no_cpu_baseline:
        log("CPU baseline: oracle on one and on all host threads")
        out["cpu_baseline"] = cpu_baseline(r64["info"].cycles)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
