"""Benchmark of the deforming-box pair-force path on one GPU.  Prints one JSON line.

Workloads (--workload):
  plain  (default) 1,048,576 LJ particles (r_c = 2.5, rho = 0.8) under
         uniaxial elongation (rate 0.5), cycling through 64 strain values
         t_k = k T / 64 that cross one lattice remap.  One step = set the
         lattice at t_k, bin into cells, sweep neighbourhoods for forces,
         energy and virial.  The line also carries the batched form on 512
         WCA replicas (N log-uniform in [2048, 65536]) against a loop of
         single-box calls over the same replicas, unless --no-batch.
  batch  the 512-replica batch alone as the headline.
  nemd   SLLOD steps (h = 0.002) of 64 LJ replicas, N log-uniform in
         [262144, 2097152], captured as one HIP graph per step.
  longrun the long-run neighbourhood experiment of Sec. 5.3 with measured
         candidate and pair counts (search efficiency of both lists).

value = pair interactions / s: interacting pairs (each unordered pair once)
summed over the timed steps, divided by the wall time of those steps.
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
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = VALU lane-instructions per
# second (one non-packed FP32/FP64 op per lane per cycle); HBM3E 8 TB/s.
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
HBM_PEAK_GBS = 8000.0
# algorithmic VALU lane-ops: 7 per candidate distance check (3 sub, mul,
# 2 fma, cmp) and 22 per in-range ordered pair in FP32 (rcp, LJ force and
# energy, 3 force fma, energy add, 6-component virial)
OPS_PER_CANDIDATE = 7
OPS_PER_PAIR = 22
# algorithmic HBM bytes per particle of one sweep launch: read the FP32
# offset (16), the FP64 position for the exact re-evaluations is not counted,
# perm (4), write F (12 in FP32) and cell_start (~4 per particle)
SWEEP_BYTES_PER_PARTICLE = 16 + 4 + 12 + 4
# algorithmic HBM bytes per particle of the cell build (bin pass): bin count
# (read x 24, write cell and rank 8, count atomic 8), scatter (read cell,
# rank, cell start 12, write perm 4), per-cell sort of perm (8), gather (read
# perm 4 and x 24, write FP64 position 32, FP32 offset 16 and residual 16)
BUILD_BYTES_PER_PARTICLE = 40 + 16 + 8 + 92

# HBM traffic of the sweep kernel per launch, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes over this benchmark (default arguments, 3 steps), each
# scaled by the reading of the same counter for a plain 1 GiB elementwise
# kernel in the same run; see profiles/sweep_particle_do_lj1M_traffic.md.
# Valid only while the sweep sources hash to src_sha (null otherwise).
SWEEP_TRAFFIC = {"bytes_per_launch": 114432646, "src_sha": "d06d77ac586d7dcf"}
SWEEP_SOURCES = ["paper_1412_3784_amd/csrc/sweep_common.hpp", "paper_1412_3784_amd/csrc/kernels.hip",
                 "paper_1412_3784_amd/csrc/kernels.hpp", "paper_1412_3784_amd/csrc/geometry.hpp"]


def sweep_src_sha() -> str:
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=64)
    p.add_argument("--warmup", type=int, default=4)
    p.add_argument("--workload", default="plain", choices=["plain", "batch", "nemd", "longrun"])
    p.add_argument("--n", type=int, default=1 << 20)
    p.add_argument("--variant", default="do", choices=["do", "ds"])
    p.add_argument("--precision", default="fp32", choices=["fp32", "fp32k", "fp64"])
    p.add_argument("--sweep", default="auto", choices=["tiled", "particle", "auto", "half"])
    p.add_argument("--deterministic", type=int, default=1, choices=[0, 1],
                   help="0: the autotuner may pick the half list (atomic sums)")
    p.add_argument("--replicas", type=int, default=None, help="batch/nemd: number of replicas")
    p.add_argument("--skin", type=float, default=0.0,
                   help="nemd: neighbour-list skin (0: cells rebuilt every step, graph-replayed)")
    p.add_argument("--no-batch", action="store_true", help="plain: skip the batched comparison")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-copy-probe", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=3, help="oracle evaluations in the CPU baseline")
    return p.parse_args()


def lattice_at(b: wl.Box, t: float) -> np.ndarray:
    """exp(tA) L0 for the diagonal flows of these workloads."""
    return np.exp(np.diag(b.A) * t)[:, None] * b.L0


def copy_probe():
    """A plain elementwise kernel over 1 GiB (reads 1 GiB, writes 1 GiB):
    the reference reading for the HBM byte counters of a profiled run."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y


def roofline_alu(tot_cands, tot_pairs, t_force, steps, kernel, n):
    ops = OPS_PER_CANDIDATE * tot_cands + OPS_PER_PAIR * 2 * tot_pairs
    achieved = ops / t_force / 1e9
    traffic = None
    if SWEEP_TRAFFIC["bytes_per_launch"] is not None and SWEEP_TRAFFIC["src_sha"] == sweep_src_sha():
        traffic = SWEEP_TRAFFIC["bytes_per_launch"]
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
            "frac": achieved / VALU_PEAK_GOPS, "traffic": traffic, "kernel": kernel,
            "ops_per_launch": ops / steps, "avg_launch_ms": 1e3 * t_force / steps,
            "hbm_algorithmic_GBs": SWEEP_BYTES_PER_PARTICLE * n / (t_force / steps) / 1e9,
            "hbm_algorithmic_frac": SWEEP_BYTES_PER_PARTICLE * n / (t_force / steps) / 1e9 / HBM_PEAK_GBS}


# ---------------------------------------------------------------------------
def run_plain(a, out):
    import torch
    from paper_1412_3784_amd import Handle
    from paper_1412_3784_amd import nemdcl as ncl

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    boxes = [wl.lj_uniaxial_strain(k=k, n=a.n) for k in range(64)]
    b0 = boxes[0]
    h = Handle(0, stream)
    h.set_potential(b0.pot)
    h.set_option(ncl.NCL_OPT_SWEEP, {"tiled": ncl.NCL_SWEEP_TILED, "particle": ncl.NCL_SWEEP_PARTICLE,
                                     "auto": ncl.NCL_SWEEP_AUTO, "half": ncl.NCL_SWEEP_HALF}[a.sweep])
    h.set_option(ncl.NCL_OPT_DETERMINISTIC, a.deterministic)
    # positions for every strain value: the fixed fractional configuration
    # carried by the flow, x_k = L(t_k) s, resident in HBM before timing
    s = torch.from_numpy(b0.frac).to(dev)
    xs = []
    for b in boxes:
        h.set_lattice(b.L0, b.A, b.t, [])          # no remap: L(t) = exp(tA) L0
        Lt, _, _ = h.get_lattice()
        xs.append((s @ torch.from_numpy(Lt).to(dev).T).contiguous())
    n = a.n
    F = torch.empty((n, 3), dtype=torch.float64 if a.precision == "fp64" else torch.float32, device=dev)
    U = torch.empty(1, dtype=torch.float64, device=dev)
    W = torch.empty(9, dtype=torch.float64, device=dev)

    def step(k, ev=None):
        b = boxes[k % 64]
        h.set_lattice(b.L0, b.A, b.t, b.automorphisms)
        if ev is not None:
            ev[0].record(stream)
        h.build_cells(a.variant, xs[k % 64], a.precision)
        if ev is not None:
            ev[1].record(stream)
        h.compute_forces(F, U, W)
        if ev is not None:
            ev[2].record(stream)

    # pair and candidate counts per strain value (untimed; the autotuner
    # settles the schedule of every strain's workload class here)
    pairs, cands, halfk = np.zeros(64), np.zeros(64), np.zeros(64, dtype=bool)
    sched = {}
    for k in range(64):
        step(k)
        st = h.stats()
        pairs[k], cands[k], halfk[k] = st["pairs"] / 2, st["candidates"], st["sweep"] == ncl.NCL_SWEEP_HALF
        key = {0: "tiled" + "x".join(map(str, st["brick"])), 1: "particle", 3: "half"}[st["sweep"]]
        sched[key] = sched.get(key, 0) + 1
    for k in range(a.warmup):
        step(k)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(k, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_build = sum(e[0].elapsed_time(e[1]) for e in evs) / 1e3
    t_force = sum(e[1].elapsed_time(e[2]) for e in evs) / 1e3
    ks = [k % 64 for k in range(a.steps)]
    tot_pairs = float(sum(pairs[k] for k in ks))
    tot_cands = float(sum(cands[k] for k in ks))
    # pair evaluations: twice per interacting pair for full lists, once for the half list
    tot_evals = float(sum(pairs[k] * (1 if halfk[k] else 2) for k in ks))
    out.update({
        "metric": "pair interactions/s (bin + force, FP32 offsets, 1e-5 force accuracy)",
        "value": tot_pairs / wall,
        "unit": "pairs/s",
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / a.steps,
        "ns_per_particle_step": 1e9 * wall / (a.steps * n),
        "dtype": {"fp32": "f32 (f64 lattice)", "fp32k": "f32+kahan (f64 lattice)", "fp64": "f64"}[a.precision],
        "config": {"workload": f"lj2.5_uniaxial_rho0.8_N{n}_64strains_{a.variant}", "n": n,
                   "variant": a.variant, "precision": a.precision, "sweep": a.sweep, "rate": 0.5,
                   "density": 0.8, "rc": 2.5},
        "breakdown_ms": {"build": 1e3 * t_build / a.steps, "force": 1e3 * t_force / a.steps},
        "schedule": sched,
        "bin_pass": {"bound": "hbm", "bytes_per_particle": BUILD_BYTES_PER_PARTICLE,
                     "achieved_GBs": BUILD_BYTES_PER_PARTICLE * n / (t_build / a.steps) / 1e9,
                     "peak_GBs": HBM_PEAK_GBS,
                     "frac": BUILD_BYTES_PER_PARTICLE * n / (t_build / a.steps) / 1e9 / HBM_PEAK_GBS},
        "candidates_per_particle": tot_cands / (a.steps * n),
        "search_efficiency": tot_evals / tot_cands,
        "deterministic": bool(a.deterministic) and a.sweep != "half",
        "roofline": roofline_alu(tot_cands, tot_evals / 2, t_force, a.steps,
                                 f"sweep[{a.sweep}]<{a.variant},{a.precision}>", n),
    })
    h.close()
    return boxes


# ---------------------------------------------------------------------------
def batch_measure(a, boxes, steps, loop_reps=3):
    """Batched bin + force over every replica per step, against a loop of
    single-box calls (one stream, then one stream per replica group)."""
    import torch
    from paper_1412_3784_amd import Batch, Handle

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    xs = [b.positions(lattice_at(b, b.t)) for b in boxes]
    ns = [len(v) for v in xs]
    ntot = sum(ns)
    x = torch.from_numpy(np.concatenate(xs)).to(dev)
    bt = Batch(ns, 0, stream)
    bt.set_potential(boxes[0].pot)
    bt.set_lattices(a.variant, [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    F = torch.empty((ntot, 3), dtype=torch.float32, device=dev)
    U = torch.empty(len(boxes), dtype=torch.float64, device=dev)
    W = torch.empty(9 * len(boxes), dtype=torch.float64, device=dev)
    bt.build_cells(x, "fp32")
    bt.compute_forces(F, U, W)
    st = bt.stats()
    for _ in range(2):
        bt.build_cells(x, "fp32")
        bt.compute_forces(F, U, W)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k][0].record(stream)
        bt.build_cells(x, "fp32")
        evs[k][1].record(stream)
        bt.compute_forces(F, U, W)
        evs[k][2].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    t_build = sum(e[0].elapsed_time(e[1]) for e in evs) / 1e3 / steps
    t_force = sum(e[1].elapsed_time(e[2]) for e in evs) / 1e3 / steps
    bt.close()
    pairs = st["pairs"] / 2
    res = {"value": pairs / wall, "unit": "pairs/s", "ms_per_step": 1e3 * wall,
           "ns_per_particle_step": 1e9 * wall / ntot, "replicas": len(boxes), "n_total": ntot,
           "breakdown_ms": {"build": 1e3 * t_build, "force": 1e3 * t_force},
           "candidates_per_particle": st["candidates"] / ntot, "pairs": pairs, "cands": st["candidates"],
           "t_force": t_force}
    # the same replicas through single-box calls, one after another on one stream
    hs = Handle(0, stream)
    hs.set_potential(boxes[0].pot)
    xr = [torch.from_numpy(v).to(dev) for v in xs]
    Fr = [torch.empty((len(v), 3), dtype=torch.float32, device=dev) for v in xs]

    def loop():
        for r, b in enumerate(boxes):
            hs.set_lattice(b.L0, b.A, b.t, b.automorphisms)
            hs.build_cells(a.variant, xr[r], "fp32")
            hs.compute_forces(Fr[r], U[r:r + 1], W[9 * r:9 * r + 9])

    loop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(loop_reps):
        loop()
    torch.cuda.synchronize()
    t_loop = (time.perf_counter() - t0) / loop_reps
    hs.close()
    # a fairer loop: replicas spread over 4 streams with a handle each
    nstr = 4
    strs = [torch.cuda.Stream(dev) for _ in range(nstr)]
    hl = [Handle(0, s_) for s_ in strs]
    for hh in hl:
        hh.set_potential(boxes[0].pot)

    def mloop():
        for r, b in enumerate(boxes):
            hh = hl[r % nstr]
            with torch.cuda.stream(strs[r % nstr]):
                hh.set_lattice(b.L0, b.A, b.t, b.automorphisms)
                hh.build_cells(a.variant, xr[r], "fp32")
                hh.compute_forces(Fr[r], U[r:r + 1], W[9 * r:9 * r + 9])

    torch.cuda.synchronize()
    mloop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(loop_reps):
        mloop()
    torch.cuda.synchronize()
    t_mloop = (time.perf_counter() - t0) / loop_reps
    for hh in hl:
        hh.close()
    res["loop"] = {"ms_per_step": 1e3 * t_loop, "value": pairs / t_loop, "speedup_batched": t_loop / wall}
    res["loop_4streams"] = {"ms_per_step": 1e3 * t_mloop, "value": pairs / t_mloop,
                            "speedup_batched": t_mloop / wall}
    return res


def run_batch(a, out):
    boxes = wl.wca_replica_batch(replicas=a.replicas or 512)
    r = batch_measure(a, boxes, a.steps)
    out.update({
        "metric": "pair interactions/s (batched bin + force over all replicas, FP32 offsets, 1e-5 force accuracy)",
        "value": r["value"], "unit": "pairs/s", "steps": a.steps, "warmup": 3,
        "ms_per_step": r["ms_per_step"], "ns_per_particle_step": r["ns_per_particle_step"],
        "dtype": "f32 (f64 lattice)",
        "config": {"workload": f"wca_rho0.8442_{len(boxes)}replicas_N{r['n_total']}_{a.variant}",
                   "replicas": len(boxes), "n_total": r["n_total"], "variant": a.variant},
        "breakdown_ms": r["breakdown_ms"], "candidates_per_particle": r["candidates_per_particle"],
        "loop": r["loop"], "loop_4streams": r["loop_4streams"],
        "roofline": roofline_alu(r["cands"], r["pairs"], r["t_force"], 1, f"kb_sweep<{a.variant},fp32>",
                                 r["n_total"]),
    })
    return boxes


def run_nemd(a, out):
    import torch
    from paper_1412_3784_amd import Batch

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    boxes = wl.lj_sllod_batch(replicas=a.replicas or 64)
    xs = [b.positions(lattice_at(b, b.t)) for b in boxes]
    ns = [len(v) for v in xs]
    ntot = sum(ns)
    x = torch.from_numpy(np.concatenate(xs)).to(dev)
    p = torch.from_numpy(np.concatenate([wl.maxwell_momenta(n_, 1.0, seed=5000 + r)
                                         for r, n_ in enumerate(ns)])).to(dev)
    del xs
    bt = Batch(ns, 0, stream)
    bt.set_potential(boxes[0].pot)
    if a.skin > 0:
        bt.set_option(5, a.skin)                  # NCL_OPT_SKIN: neighbour lists
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    bt.build_cells(x, "fp32")
    h = 0.002
    graph = a.skin == 0
    bt.sllod_run(x, p, h, 1.0, a.warmup, use_graph=graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F, U, W, hist = bt.sllod_run(x, p, h, 1.0, a.steps, use_graph=graph, history=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = bt.stats()
    bt.close()
    hist = hist.cpu().numpy()                     # (steps + 1, R, 8)
    # energy balance H(t) - H(0) + int sum_a A_aa (K_aa + W_aa) dt per replica
    adiag = np.array([np.diag(b.A) for b in boxes])               # (R, 3)
    H = 0.5 * hist[:, :, 5:8].sum(-1) + hist[:, :, 1]
    rate = (adiag[None] * (hist[:, :, 5:8] + hist[:, :, 2:5])).sum(-1)
    work = np.concatenate([np.zeros((1, len(boxes))), np.cumsum(0.5 * h * (rate[1:] + rate[:-1]), axis=0)])
    drift = np.abs(H - H[0] + work).max(axis=0) / np.abs(H[0])
    pairs = st["pairs"] / 2                       # pairs at the last step
    out.update({
        "metric": ("pair interactions/s (SLLOD step: bin + force + integrate, graph-replayed, FP32 forces)"
                   if graph else
                   f"pair interactions/s (SLLOD step: neighbour lists with skin {a.skin}, rebuilt when the "
                   "skin bound or a remap requires, + force + integrate, FP32 forces)"),
        "value": pairs * a.steps / wall, "unit": "pairs/s", "steps": a.steps,
        "ms_per_step": 1e3 * wall / a.steps, "ns_per_particle_step": 1e9 * wall / (a.steps * ntot),
        "dtype": "f32 forces, f64 state and lattice",
        "config": {"workload": f"lj2.5_rho0.8_{len(boxes)}replicas_N{ntot}_sllod_h0.002",
                   "replicas": len(boxes), "n_total": ntot, "h": h},
        "energy_balance_rel_drift": {"max": float(drift.max()), "median": float(np.median(drift))},
        "skin": a.skin, "list_rebuilds": st.get("list_rebuilds", 0),
        "pairs_note": "pairs/s uses the last step's pair count for every step",
    })
    return boxes


def longrun_measure(samples=200, periods=20, density=100.0, seed=0):
    """The long-run experiment of Sec. 5.3 with measured counts: a box of
    initial side 10 d_cut (d_cut = (3/4pi)^(1/3), sphere volume one) under
    uniaxial flow diag(0.05, -0.025, -0.025) with generalised KR remaps;
    uniform particles carried by the flow; at each sampled time the GPU
    lists count candidates and in-range pairs.  Returns the measured search
    efficiencies (in-range pairs / candidates over the run) of the
    dynamic-size list and of the dynamic-offset list with the paper's
    neighbourhood (grown by whole cells) and with the tight one (grown by
    d_cut), and the geometric efficiencies 1 / <neighbourhood volume> at the
    same times."""
    import torch
    from paper_1412_3784_amd import Handle
    from paper_1412_3784_amd import nemdcl as ncl
    dcut = (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)
    side = 10.0 * dcut
    n = int(round(density * side ** 3))
    box = wl.make_box("uniaxial", 0.05, n, side=side, t=0.0, seed=seed)
    ts = np.linspace(0.0, periods * box.period, samples, endpoint=False)
    dev = torch.device("cuda:0")
    s = torch.from_numpy(box.frac).to(dev)
    out = {}
    geo = {"ds": [], "do_paper": []}
    for name, variant, tight in (("ds", "ds", 1.0), ("do_paper", "do", 0.0), ("do_tight", "do", 1.0)):
        h = Handle(0)
        h.set_potential(eps=1.0, sigma=dcut / 2 ** (1 / 6), rc=dcut, shift=1)
        h.set_option(ncl.NCL_OPT_DO_TIGHT, tight)
        # the per-particle sweep visits exactly each particle's neighbourhood
        # (the tiled sweep's counts include its bricks' staging)
        h.set_option(ncl.NCL_OPT_SWEEP, ncl.NCL_SWEEP_PARTICLE)
        cand = pairs = 0
        for t in ts:
            h.set_lattice(box.L0, box.A, t, [])
            Lt, _, _ = h.get_lattice()
            x = (s @ torch.from_numpy(Lt).to(dev).T).contiguous()
            h.set_lattice(box.L0, box.A, t, box.automorphisms)
            h.build_cells(variant, x, "fp32")
            h.compute_forces()
            st = h.stats()
            cand += st["candidates"]
            pairs += st["pairs"]
            if name in geo:
                Lr, _, _ = h.get_lattice()
                V = abs(np.linalg.det(Lr))
                c = np.array(st["cells"], dtype=float)
                if variant == "ds":
                    geo[name].append(27.0 * V / c.prod())
                else:
                    geo[name].append((27.0 + 14.0 / c[2] + 6.0 / c[1] - 4.0 / (c[1] * c[2])) * V / c.prod())
        h.close()
        out[name] = pairs / cand
    out["geometric_ds"] = 1.0 / np.mean(geo["ds"])
    out["geometric_do_paper"] = 1.0 / np.mean(geo["do_paper"])
    out["n"] = n
    out["samples"] = samples
    out["periods"] = periods
    return out


def run_longrun(a, out):
    t0 = time.perf_counter()
    r = longrun_measure(samples=a.steps if a.steps != 64 else 200)
    wall = time.perf_counter() - t0
    out.update({
        "metric": "long-run search efficiency (in-range pairs / candidates), dynamic offset",
        "value": r["do_tight"], "unit": "ratio", "steps": r["samples"], "ms_per_step": 1e3 * wall / r["samples"],
        "dtype": "f32 (f64 lattice)",
        "config": {"workload": f"uniaxial_0.05_side10dcut_N{r['n']}_{r['periods']}periods", "n": r["n"]},
        "measured": {k: r[k] for k in ("ds", "do_paper", "do_tight")},
        "geometric": {"ds": r["geometric_ds"], "do_paper": r["geometric_do_paper"]},
        "paper": {"ds": 0.0688, "do": 0.123},
    })


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                          "(replicas or a slab decomposition would shard across GPUs)"}))
        sys.exit(2)
    out = {"metric": None, "value": None, "unit": None, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": None, "data": "synthetic", "config": {}}
    boxes = None
    if a.workload == "plain":
        boxes = run_plain(a, out)
        if not a.no_batch:
            r = batch_measure(a, wl.wca_replica_batch(replicas=a.replicas or 512), 20)
            out["batched"] = {k: v for k, v in r.items() if k not in ("pairs", "cands", "t_force")}
            out["batched"]["workload"] = f"wca_rho0.8442_{r['replicas']}replicas_N{r['n_total']}_{a.variant}"
    elif a.workload == "batch":
        boxes = run_batch(a, out)
    elif a.workload == "longrun":
        run_longrun(a, out)
    else:
        boxes = run_nemd(a, out)
    if not a.no_copy_probe:
        copy_probe()
    if not a.no_cpu_baseline and a.workload == "plain":
        out["cpu_baseline"] = cpu_baseline(boxes, a.cpu_sample)
    print(json.dumps(out), flush=True)


def cpu_baseline(boxes, nsample):
    """The FP64 oracle (plain dynamic-size cell list, all host threads) on a
    bounded sample of the same workload: nsample strain values at full N."""
    import oracle
    ks = [int(round(q * 63 / max(nsample - 1, 1))) for q in range(nsample)]
    tot_pairs, tot_t = 0.0, 0.0
    for k in ks:
        b = boxes[k]
        x = b.positions(oracle.lattice_at(b.L0, b.A, b.t))
        Lr, Mt, _ = oracle.reduce(b.L0, b.A, b.t, b.automorphisms)
        t0 = time.perf_counter()
        r = oracle.forces_cells(x, Lr, b.pot, want_hash=False)
        tot_t += time.perf_counter() - t0
        tot_pairs += r.stats[1] / 2
    return {"value": tot_pairs / tot_t, "unit": "pairs/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{len(ks)} strain values (k={ks}) of the same workload at full N, FP64 DS cell list",
            "seconds": tot_t}


if __name__ == "__main__":
    main()
