"""Benchmark of the deforming-box pair-force path on one GPU.  Prints one JSON line.

Default run (--workload plain): the headline is the 1,048,576-particle LJ
workload (r_c = 2.5, rho = 0.8, uniaxial elongation at rate 0.5) cycling
through 64 strain values t_k = k T / 64 that cross one lattice remap, timed
with the dynamic-offset list; one step = set the lattice at t_k, bin into
cells, sweep neighbourhoods for forces, energy and virial.  The same line
also carries, each under its own key:
  variants.ds   the same workload with the dynamic-size list;
  precision_16m 16,777,216 LJ particles on a jittered 256^3 grid (biaxial,
                rate 0.2, t = T/2), FP32 offsets with Kahan sums, both lists,
                with the force error of a sample of particles against the
                FP64 oracle;
  batched       512 WCA replicas (N log-uniform in [2048, 65536]) in one
                batched pass, against loops of single-box calls;
  nemd          1,000 graph-replayed SLLOD steps (h = 0.002) of 64 LJ
                replicas (N log-uniform in [262144, 2097152]), with the
                energy-balance drift, the pressure tensor of four replicas
                against the oracle on the GPU's own states every 100 steps,
                and the smallest replica against its FP64 oracle trajectory;
  cpu_baseline  the FP64 oracle on the host (all threads and one thread).
Legs can be skipped (--no-batch, --no-16m, --no-nemd, --no-cpu-baseline).
Other headlines: --workload batch | nemd | longrun (the long-run
neighbourhood experiment of Sec. 5.3 with measured counts).

value = pair interactions / s: interacting pairs (each unordered pair once)
summed over the timed steps, divided by the wall time of those steps.
"""
from __future__ import annotations

import argparse
import gc
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
# algorithmic VALU lane-ops of the sweep: 7 per candidate distance check
# (3 sub, mul, 2 fma, cmp) and 40 per evaluation of an in-range pair (rcp,
# LJ force and energy, force accumulation, 6-component virial, Kahan terms);
# a full list evaluates every interacting pair from both ends
OPS_PER_CANDIDATE = 7
OPS_PER_PAIR = 40
# algorithmic HBM bytes per particle of one sweep launch: read the FP32
# offset (16) and perm (4), write F (12 in FP32); cell starts are ~0.1-4 B
# per particle and not counted
SWEEP_BYTES_PER_PARTICLE = 16 + 4 + 12
# algorithmic HBM bytes per particle of the cell build (bin pass) of a
# counting sort: read x for the histogram (24) and again for the scatter
# (24), write the FP32 offset (16), perm (4) and the cell id (4), plus ~1 B
# of cell arrays per particle
BIN_BYTES_PER_PARTICLE = 24 + 24 + 16 + 4 + 4 + 1
# the bytes per particle of this build's own cell build by its own count:
# positions read twice, cell keys and indices through the radix sort, the
# sorted FP64 position and FP32 offset written (the FP32 offset's residual,
# 16 more, is written only when a tiled sweep may read it, which the timed
# steps of the per-particle schedule do not)
BUILD_DESIGN_BYTES_PER_PARTICLE = 140

# HBM traffic of the sweep kernel per launch, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes over this benchmark (default arguments, 3 steps), each
# scaled by the reading of the same counter for a plain 1 GiB elementwise
# kernel in the same run; see profiles/sweep_particle_do_lj1M_traffic.md.
# Valid only while the sweep sources hash to src_sha (null otherwise).
SWEEP_TRAFFIC = {"bytes_per_launch": 130033571, "src_sha": "7dffc170a59caa23"}
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
    p.add_argument("--no-16m", action="store_true", help="plain: skip the 16M precision-form leg")
    p.add_argument("--no-nemd", action="store_true", help="plain: skip the SLLOD leg")
    p.add_argument("--no-variants", action="store_true", help="plain: skip the other cell-list variant")
    p.add_argument("--nemd-steps", type=int, default=1000, help="plain: SLLOD steps of the nemd leg")
    p.add_argument("--nemd-traj", type=int, default=4,
                   help="plain: smallest replicas given their own 100-step FP64 oracle trajectory")
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


def roofline_alu(tot_cands, tot_evals, t_force, steps, kernel, n, measured=False):
    """the sweep against the VALU: algorithmic lane-ops (7 per candidate, 40
    per pair evaluation) over the force call's event time.  `measured`: the
    launch is the one SWEEP_TRAFFIC was counted on (1 M LJ, dynamic offset,
    FP32, per-particle sweep); other launches report no traffic."""
    ops = OPS_PER_CANDIDATE * tot_cands + OPS_PER_PAIR * tot_evals
    achieved = ops / t_force / 1e9
    traffic = None
    if (measured and SWEEP_TRAFFIC["bytes_per_launch"] is not None
            and SWEEP_TRAFFIC["src_sha"] == sweep_src_sha()):
        traffic = SWEEP_TRAFFIC["bytes_per_launch"]
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
            "frac": achieved / VALU_PEAK_GOPS, "traffic": traffic, "kernel": kernel,
            "ops_per_launch": ops / steps, "avg_launch_ms": 1e3 * t_force / steps,
            "ops_count": f"{OPS_PER_CANDIDATE} per candidate + {OPS_PER_PAIR} per pair evaluation",
            "hbm_algorithmic_GBs": SWEEP_BYTES_PER_PARTICLE * n / (t_force / steps) / 1e9,
            "hbm_algorithmic_frac": SWEEP_BYTES_PER_PARTICLE * n / (t_force / steps) / 1e9 / HBM_PEAK_GBS}


# ---------------------------------------------------------------------------
def bin_pass(t_build, n):
    """the cell build against HBM: algorithmic bytes of a counting-sort build
    per particle, and this build's own count beside it"""
    gbs = BIN_BYTES_PER_PARTICLE * n / t_build / 1e9
    own = BUILD_DESIGN_BYTES_PER_PARTICLE * n / t_build / 1e9
    return {"bound": "hbm", "bytes_per_particle": BIN_BYTES_PER_PARTICLE, "achieved_GBs": gbs,
            "peak_GBs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS,
            "design_bytes_per_particle": BUILD_DESIGN_BYTES_PER_PARTICLE, "design_GBs": own,
            "design_frac": own / HBM_PEAK_GBS, "avg_ms": 1e3 * t_build}


def plain_measure(a, variant, boxes, steps, warmup):
    """1 M LJ strain sweep with one cell-list variant: per-step lattice, bin
    and force, timed over `steps` steps after `warmup` untimed ones."""
    import torch
    from paper_1412_3784_amd import Handle
    from paper_1412_3784_amd import nemdcl as ncl

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
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
    del s
    n = len(b0.frac)
    F = torch.empty((n, 3), dtype=torch.float64 if a.precision == "fp64" else torch.float32, device=dev)
    U = torch.empty(1, dtype=torch.float64, device=dev)
    W = torch.empty(9, dtype=torch.float64, device=dev)

    def step(k, ev=None):
        b = boxes[k % 64]
        h.set_lattice(b.L0, b.A, b.t, b.automorphisms)
        if ev is not None:
            ev[0].record(stream)
        h.build_cells(variant, xs[k % 64], a.precision)
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
    for k in range(warmup):
        step(k)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_build = sum(e[0].elapsed_time(e[1]) for e in evs) / 1e3
    t_force = sum(e[1].elapsed_time(e[2]) for e in evs) / 1e3
    h.close()
    del xs, F
    torch.cuda.empty_cache()
    ks = [k % 64 for k in range(steps)]
    tot_pairs = float(sum(pairs[k] for k in ks))
    tot_cands = float(sum(cands[k] for k in ks))
    # pair evaluations: twice per interacting pair for full lists, once for the half list
    tot_evals = float(sum(pairs[k] * (1 if halfk[k] else 2) for k in ks))
    return {
        "value": tot_pairs / wall, "unit": "pairs/s", "ms_per_step": 1e3 * wall / steps,
        "ns_per_particle_step": 1e9 * wall / (steps * n),
        "breakdown_ms": {"build": 1e3 * t_build / steps, "force": 1e3 * t_force / steps},
        "schedule": sched, "bin_pass": bin_pass(t_build / steps, n),
        "candidates_per_particle": tot_cands / (steps * n), "search_efficiency": tot_evals / tot_cands,
        "deterministic": bool(a.deterministic) and a.sweep != "half",
        "roofline": roofline_alu(tot_cands, tot_evals, t_force, steps,
                                 f"sweep[{a.sweep}]<{variant},{a.precision}>", n,
                                 measured=(variant == "do" and a.precision == "fp32" and n == 1 << 20
                                           and set(sched) == {"particle"})),
    }


def run_plain(a, out):
    boxes = [wl.lj_uniaxial_strain(k=k, n=a.n) for k in range(64)]
    n = a.n
    r = plain_measure(a, a.variant, boxes, a.steps, a.warmup)
    out.update({
        "metric": "pair interactions/s (bin + force, FP32 offsets, 1e-5 force accuracy)",
        "value": r["value"],
        "unit": "pairs/s",
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "ns_per_particle_step": r["ns_per_particle_step"],
        "dtype": {"fp32": "f32 (f64 lattice)", "fp32k": "f32+kahan (f64 lattice)", "fp64": "f64"}[a.precision],
        "config": {"workload": f"lj2.5_uniaxial_rho0.8_N{n}_64strains_{a.variant}", "n": n,
                   "variant": a.variant, "precision": a.precision, "sweep": a.sweep, "rate": 0.5,
                   "density": 0.8, "rc": 2.5},
    })
    for k in ("breakdown_ms", "schedule", "bin_pass", "candidates_per_particle", "search_efficiency",
              "deterministic", "roofline"):
        out[k] = r[k]
    if not a.no_variants:
        other = "ds" if a.variant == "do" else "do"
        gc.collect()
        o = plain_measure(a, other, boxes, a.steps, a.warmup)
        o["roofline"] = {k: o["roofline"][k] for k in ("achieved", "frac", "avg_launch_ms", "kernel")}
        o["workload"] = f"lj2.5_uniaxial_rho0.8_N{n}_64strains_{other}"
        out["variants"] = {other: o}
    return boxes


# ---------------------------------------------------------------------------
def precision_measure(a, steps, nsample=2048):
    """16,777,216 LJ particles on a jittered grid (biaxial, t = T/2), FP32
    offsets with Kahan sums, both lists: bin + force timed over `steps`
    steps; the force error of a seeded sample of particles against the FP64
    oracle, relative to max(sum_j |f_ij|, eps/sigma) as the parity bound and
    to |F_i| for information."""
    import torch
    import oracle
    from paper_1412_3784_amd import Handle
    from paper_1412_3784_amd import nemdcl as ncl

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    box = wl.lj_biaxial_grid()
    x = box.positions(lattice_at(box, box.t))
    n = len(x)
    idx = np.sort(np.random.default_rng(77).choice(n, size=nsample, replace=False))
    Lr, Mt, _ = oracle.reduce(box.L0, box.A, box.t, box.automorphisms)
    ref = oracle.forces_cells(x, Lr, box.pot, Mkey=Mt, want_hash=False, subset=idx)
    xt = torch.from_numpy(x).to(dev)
    res = {"workload": f"lj2.5_biaxial_rho0.8_grid256_jitter0.05_N{n}_tHalfT_fp32k", "n": n}
    for variant in ("do", "ds"):
        h = Handle(0, stream)
        h.set_potential(box.pot)
        h.set_option(ncl.NCL_OPT_DETERMINISTIC, 1)
        h.set_lattice(box.L0, box.A, box.t, box.automorphisms)
        F = torch.empty((n, 3), dtype=torch.float32, device=dev)
        U = torch.empty(1, dtype=torch.float64, device=dev)
        W = torch.empty(9, dtype=torch.float64, device=dev)
        for _ in range(2):                         # autotuner and warm-up, untimed
            h.build_cells(variant, xt, "fp32k")
            h.compute_forces(F, U, W)
        st = h.stats()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            evs[k][0].record(stream)
            h.build_cells(variant, xt, "fp32k")
            evs[k][1].record(stream)
            h.compute_forces(F, U, W)
            evs[k][2].record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        t_build = sum(e[0].elapsed_time(e[1]) for e in evs) / 1e3 / steps
        t_force = sum(e[1].elapsed_time(e[2]) for e in evs) / 1e3 / steps
        Fs = F[torch.from_numpy(idx).to(dev)].double().cpu().numpy()
        h.close()
        del F
        dF = np.linalg.norm(Fs - ref.F, axis=1)
        cond = dF / np.maximum(ref.fmag, 1.0)
        Fn = np.linalg.norm(ref.F, axis=1)
        pairs = st["pairs"] / 2
        rf = roofline_alu(st["candidates"], st["pairs"], t_force, 1, f"sweep[auto]<{variant},fp32k>", n)
        res[variant] = {
            "value": pairs / wall, "unit": "pairs/s", "ms_per_step": 1e3 * wall,
            "ns_per_particle_step": 1e9 * wall / n,
            "breakdown_ms": {"build": 1e3 * t_build, "force": 1e3 * t_force},
            "candidates_per_particle": st["candidates"] / n, "pairs_per_particle": st["pairs"] / n,
            "sweep_valu_frac": rf["frac"], "sweep_hbm_algorithmic_frac": rf["hbm_algorithmic_frac"],
            "bin_pass": bin_pass(t_build, n),
            "bin_plus_sweep_hbm_algorithmic_frac":
                (BIN_BYTES_PER_PARTICLE + SWEEP_BYTES_PER_PARTICLE) * n / (t_build + t_force) / 1e9 / HBM_PEAK_GBS,
            "force_error": {"sample": nsample, "max_rel_to_sum_abs_fij": float(cond.max()),
                            "rms_rel_to_sum_abs_fij": float(np.sqrt(np.mean(cond ** 2))),
                            "max_rel_to_abs_Fi": float((dF / Fn).max()),
                            "rms_rel_to_abs_Fi": float(np.sqrt(np.mean((dF / Fn) ** 2)))},
        }
    del xt
    torch.cuda.empty_cache()
    return res


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
    bt.compute_forces(F, U, W)  # the batched autotuner times the staged and fused schedules here
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
           "t_force": t_force,
           "schedule": {1: "staged", 4: "fused"}.get(st["sweep"], str(st["sweep"])),
           "tune_ms": {"staged": st["tune_ms"][0], "fused": st["tune_ms"][1]}}
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
        "schedule": r["schedule"], "tune_ms": r["tune_ms"],
        "roofline": roofline_alu(r["cands"], 2 * r["pairs"], r["t_force"], 1, f"kb_sweep<{a.variant},fp32>",
                                 r["n_total"]),
    })
    return boxes


def energy_drift(hist, boxes, h):
    """energy balance H(t) - H(0) + int sum_a A_aa (K_aa + W_aa) dt per
    replica (zero along exact SLLOD solutions), relative to |H(0)|; hist has
    shape (steps + 1, R, 8) with rows (t, U, W diag, K diag)"""
    adiag = np.array([np.diag(b.A) for b in boxes])               # (R, 3)
    H = 0.5 * hist[:, :, 5:8].sum(-1) + hist[:, :, 1]
    rate = (adiag[None] * (hist[:, :, 5:8] + hist[:, :, 2:5])).sum(-1)
    work = np.concatenate([np.zeros((1, len(boxes))), np.cumsum(0.5 * h * (rate[1:] + rate[:-1]), axis=0)])
    return np.abs(H - H[0] + work).max(axis=0) / np.abs(H[0])


def nemd_measure(a, nsteps=1000, chunk=100, nshadow=4, traj_steps=100, skin=0.0, ntraj=4):
    """SLLOD run of the 64-replica LJ batch: nsteps steps in graph-replayed
    chunks of `chunk` steps (the time of each chunk's call is summed).  The
    oracle evaluates the forces of the `nshadow` smallest replicas on the
    GPU's own FP64 states at step 0 and after every chunk (shadow mode), and
    their pressure tensors P = (sum p p^T / m + W) / V are compared; the
    `ntraj` smallest replicas also run their own FP64 oracle trajectories
    for traj_steps steps, compared pointwise at their end and as time
    averages of the diagonal pressure over the steps.  Returns the result
    dict and the boxes."""
    import torch
    import oracle
    from paper_1412_3784_amd import Batch

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    boxes = wl.lj_sllod_batch(replicas=a.replicas or 64)
    R = len(boxes)
    xs = [b.positions(lattice_at(b, b.t)) for b in boxes]
    ns = [len(v) for v in xs]
    ntot = sum(ns)
    off = np.concatenate([[0], np.cumsum(ns)])
    ps = [wl.maxwell_momenta(n_, 1.0, seed=5000 + r) for r, n_ in enumerate(ns)]
    order = [int(r) for r in np.argsort(ns, kind="stable")]
    shadow = order[:nshadow] if nshadow > 0 else []
    trajr = order[:ntraj] if traj_steps > 0 else []
    start = {r: (xs[r].copy(), ps[r].copy()) for r in trajr}
    x = torch.from_numpy(np.concatenate(xs)).to(dev)
    p = torch.from_numpy(np.concatenate(ps)).to(dev)
    del xs, ps
    bt = Batch(ns, 0, stream)
    bt.set_potential(boxes[0].pot)
    if skin > 0:
        bt.set_option(5, skin)                    # NCL_OPT_SKIN: neighbour lists
    bt.set_lattices("do", [b.L0 for b in boxes], [b.A for b in boxes], [b.t for b in boxes],
                    [b.automorphisms for b in boxes])
    bt.build_cells(x, "fp32")
    h, mass = 0.002, 1.0
    graph = skin == 0
    perr = []

    def shadow_check(step, W):
        """relative pressure-tensor error of the shadow replicas at `step`"""
        Wg = W.cpu().numpy().reshape(R, 3, 3)
        for r in shadow:
            b = boxes[r]
            sl = slice(off[r], off[r + 1])
            xr, pr = x[sl].cpu().numpy(), p[sl].cpu().numpy()
            Lr, _, _ = oracle.reduce(b.L0, b.A, b.t + step * h, b.automorphisms)
            ref = oracle.forces_cells(xr, Lr, b.pot, want_hash=False)
            V = abs(np.linalg.det(Lr))
            K = pr.T @ pr / mass
            P_or = (K + ref.W) / V
            P_gp = (K + Wg[r]) / V
            perr.append({"step": step, "replica": r, "n": ns[r],
                         "rel_err": float(np.abs(P_gp - P_or).max() / np.abs(P_or).max())})

    F, U, W = bt.compute_forces()
    if shadow:
        shadow_check(0, W)
    hists, wall, done = [], 0.0, 0
    traj_cmp = {}
    while done < nsteps:
        k = min(chunk, nsteps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F, U, W, hist = bt.sllod_run(x, p, h, mass, k, use_graph=graph, history=True)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        hist = hist.cpu().numpy()
        hists.append(hist if not hists else hist[1:])
        done += k
        if shadow:
            shadow_check(done, W)
        if done == traj_steps and traj_steps > 0:
            for r in trajr:
                sl = slice(off[r], off[r + 1])
                traj_cmp[r] = (x[sl].cpu().numpy(), p[sl].cpu().numpy())
    st = bt.stats()
    bt.close()
    hist = np.concatenate(hists)                  # (nsteps + 1, R, 8)
    drift = energy_drift(hist, boxes, h)
    res = {"value": st["pairs"] / 2 * nsteps / wall, "unit": "pairs/s", "steps": nsteps,
           "ms_per_step": 1e3 * wall / nsteps, "ns_per_particle_step": 1e9 * wall / (nsteps * ntot),
           "workload": f"lj2.5_rho0.8_{R}replicas_N{ntot}_sllod_h0.002_{nsteps}steps",
           "replicas": R, "n_total": ntot, "h": h, "graph_replayed": graph,
           "energy_balance_rel_drift": {"max": float(drift.max()), "median": float(np.median(drift))},
           "pairs_note": "pairs/s uses the last step's pair count for every step"}
    if skin > 0:
        res["skin"], res["list_rebuilds"] = skin, st.get("list_rebuilds", 0)
    if perr:
        res["pressure_tensor_shadow"] = {
            "replicas": shadow, "steps": sorted({e["step"] for e in perr}),
            "max_rel_err": max(e["rel_err"] for e in perr),
            "median_rel_err": float(np.median([e["rel_err"] for e in perr])),
            "definition": "max_ab |P_gpu - P_oracle| / max_ab |P_oracle|, P = (sum p p^T / m + W) / V, "
                          "oracle forces on the GPU's FP64 state"}
    trajs = []
    for r in trajr:
        if r not in traj_cmp:
            continue
        b = boxes[r]
        x0, p0 = start[r]
        t1 = time.perf_counter()
        xo, po, ho = oracle.sllod(x0, p0, b.L0, b.A, b.t, b.automorphisms, b.pot, h, mass, traj_steps)
        t_or = time.perf_counter() - t1
        L = oracle.lattice_at(b.L0, b.A, b.t + traj_steps * h)
        d = traj_cmp[r][0] - xo
        d -= np.round(np.linalg.solve(L, d.T)).T @ L.T    # nearest image
        V = abs(np.linalg.det(b.L0))
        hg = hist[:traj_steps + 1, r]
        pdiag_g = (hg[:, 2:5] + hg[:, 5:8]) / V
        pdiag_o = (ho[:, 2:5] + ho[:, 5:8]) / V
        trajs.append({
            "replica": r, "n": ns[r], "steps": traj_steps, "oracle_seconds": t_or,
            "max_abs_dx_sigma": float(np.abs(d).max()),
            "max_rel_dp": float(np.abs(traj_cmp[r][1] - po).max() / np.abs(po).max()),
            "time_avg_pressure_diag_gpu": pdiag_g.mean(axis=0).tolist(),
            "time_avg_pressure_diag_oracle": pdiag_o.mean(axis=0).tolist(),
            "time_avg_pressure_rel_diff": float(np.abs(pdiag_g.mean(0) - pdiag_o.mean(0)).max()
                                                / np.abs(pdiag_o.mean(0)).max()),
            "energy_balance_rel_drift_oracle": float(np.abs(oracle.energy_balance(ho, b.A)).max()
                                                     / abs(0.5 * ho[0, 5:8].sum() + ho[0, 1]))})
    if trajs:
        # the smallest replica in full, then the worst figures over all
        res["oracle_trajectory"] = trajs[0]
        res["oracle_trajectories"] = {
            "replicas": [t["replica"] for t in trajs], "n": [t["n"] for t in trajs], "steps": traj_steps,
            "oracle_seconds": sum(t["oracle_seconds"] for t in trajs),
            "max_abs_dx_sigma": max(t["max_abs_dx_sigma"] for t in trajs),
            "max_rel_dp": max(t["max_rel_dp"] for t in trajs),
            "max_time_avg_pressure_rel_diff": max(t["time_avg_pressure_rel_diff"] for t in trajs)}
    del x, p
    torch.cuda.empty_cache()
    return res, boxes


def run_nemd(a, out):
    r, boxes = nemd_measure(a, nsteps=a.steps, chunk=a.steps, nshadow=0, traj_steps=0, skin=a.skin)
    graph = r["graph_replayed"]
    out.update({
        "metric": ("pair interactions/s (SLLOD step: bin + force + integrate, graph-replayed, FP32 forces)"
                   if graph else
                   f"pair interactions/s (SLLOD step: neighbour lists with skin {a.skin}, rebuilt when the "
                   "skin bound or a remap requires, + force + integrate, FP32 forces)"),
        "value": r["value"], "unit": "pairs/s", "steps": a.steps,
        "ms_per_step": r["ms_per_step"], "ns_per_particle_step": r["ns_per_particle_step"],
        "dtype": "f32 forces, f64 state and lattice",
        "config": {"workload": r["workload"], "replicas": r["replicas"], "n_total": r["n_total"], "h": r["h"]},
        "energy_balance_rel_drift": r["energy_balance_rel_drift"],
        "skin": a.skin, "list_rebuilds": r.get("list_rebuilds", 0), "pairs_note": r["pairs_note"],
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
    # Python's cyclic garbage collector runs only between legs: a full
    # collection in a process holding torch takes tens of milliseconds, and
    # one landing inside a timed loop stalls the host that feeds the GPU (a
    # 35 ms pause in 64 steps of 0.78 ms added 0.5 ms to every step).  Objects
    # without cycles are still freed at once.
    gc.collect()
    gc.disable()
    boxes = None
    if a.workload == "plain":
        boxes = run_plain(a, out)
        if not a.no_16m:
            log("16M precision leg")
            gc.collect()
            out["precision_16m"] = precision_measure(a, max(1, min(a.steps, 10)))
        if not a.no_batch:
            log("batched leg")
            gc.collect()
            r = batch_measure(a, wl.wca_replica_batch(replicas=512), 20)
            out["batched"] = {k: v for k, v in r.items() if k not in ("pairs", "cands", "t_force")}
            out["batched"]["workload"] = f"wca_rho0.8442_{r['replicas']}replicas_N{r['n_total']}_{a.variant}"
            out["batched"]["roofline"] = {
                k: v for k, v in roofline_alu(r["cands"], 2 * r["pairs"], r["t_force"], 1,
                                              f"kb_sweep<{a.variant},fp32>", r["n_total"]).items()
                if k in ("achieved", "frac", "avg_launch_ms", "kernel", "ops_count")}
        if not a.no_nemd:
            log("nemd leg")
            gc.collect()
            r, _ = nemd_measure(a, nsteps=a.nemd_steps, ntraj=a.nemd_traj)
            out["nemd"] = r
    elif a.workload == "batch":
        boxes = run_batch(a, out)
    elif a.workload == "longrun":
        run_longrun(a, out)
    else:
        boxes = run_nemd(a, out)
    if not a.no_copy_probe:
        copy_probe()
    if not a.no_cpu_baseline and a.workload == "plain":
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(boxes, a.cpu_sample)
    print(json.dumps(out), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(boxes, nsample):
    """The FP64 oracle (plain dynamic-size cell list) on a bounded sample of
    the same workload at full N: nsample strain values on all host threads,
    and the first of them again on one thread."""
    import oracle
    ks = [int(round(q * 63 / max(nsample - 1, 1))) for q in range(nsample)]

    def run(k, threads):
        b = boxes[k]
        x = b.positions(oracle.lattice_at(b.L0, b.A, b.t))
        Lr, Mt, _ = oracle.reduce(b.L0, b.A, b.t, b.automorphisms)
        t0 = time.perf_counter()
        r = oracle.forces_cells(x, Lr, b.pot, want_hash=False, threads=threads)
        return r.stats[1] / 2, time.perf_counter() - t0

    tot_pairs, tot_t = 0.0, 0.0
    for k in ks:
        pr, t = run(k, 0)
        tot_pairs += pr
        tot_t += t
    p1, t1 = run(ks[0], 1)
    n = len(boxes[0].frac)
    return {"value": tot_pairs / tot_t, "unit": "pairs/s", "cores": oracle.max_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{len(ks)} strain values (k={ks}) of the same workload at full N, FP64 DS cell list",
            "seconds": tot_t, "ns_per_particle_step": 1e9 * tot_t / (len(ks) * n),
            "one_thread": {"value": p1 / t1, "unit": "pairs/s", "cores": 1, "seconds": t1,
                           "ns_per_particle_step": 1e9 * t1 / n,
                           "sample": f"strain value k={ks[0]} at full N, one thread"}}


if __name__ == "__main__":
    main()
