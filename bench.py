"""Benchmark: cell build + force pass for 1,048,576 LJ particles (r_c = 2.5,
rho = 0.8) under uniaxial elongation (rate 0.5), cycling through 64 strain
values t_k = k T / 64 that cross one lattice remap.  One step = set the
lattice at t_k, bin into cells, sweep neighbourhoods for forces, energy and
virial.  Prints one JSON line.

value = pair interactions / s: interacting pairs (each unordered pair once)
summed over the timed steps, divided by the wall time of those steps.
"""
from __future__ import annotations

import argparse
import json
import math
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


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=64)
    p.add_argument("--warmup", type=int, default=4)
    p.add_argument("--n", type=int, default=1 << 20)
    p.add_argument("--variant", default="do", choices=["do", "ds"])
    p.add_argument("--precision", default="fp32", choices=["fp32", "fp32k", "fp64"])
    p.add_argument("--sweep", default="particle", choices=["tiled", "particle"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=3, help="oracle evaluations in the CPU baseline")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(see DESIGN.md for how the path would shard)"}))
        sys.exit(2)
    import torch
    from paper_1412_3784_amd import Handle

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    boxes = [wl.config2(k=k, n=a.n) for k in range(64)]
    b0 = boxes[0]
    h = Handle(0, stream)
    h.set_potential(b0.pot)
    from paper_1412_3784_amd import nemdcl as ncl
    h.set_option(ncl.NCL_OPT_SWEEP, 0 if a.sweep == "tiled" else 1)
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

    # pair and candidate counts per strain value (untimed)
    pairs, cands = np.zeros(64), np.zeros(64)
    for k in range(64):
        step(k)
        st = h.stats()
        pairs[k], cands[k] = st["pairs"] / 2, st["candidates"]
    for k in range(a.warmup):
        step(k)
    torch.cuda.synchronize()
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
    value = tot_pairs / wall
    ms_per_step = 1e3 * wall / a.steps
    # dominant kernel: the neighbourhood sweep (one launch per step)
    ops = OPS_PER_CANDIDATE * tot_cands + OPS_PER_PAIR * 2 * tot_pairs
    achieved = ops / t_force / 1e9
    out = {
        "metric": "pair interactions/s (bin + force, FP32 offsets, 1e-5 force accuracy)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "ns_per_particle_step": 1e9 * wall / (a.steps * n),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32 (f64 lattice)", "fp32k": "f32+kahan (f64 lattice)", "fp64": "f64"}[a.precision],
        "data": "synthetic",
        "config": {"workload": f"lj2.5_uniaxial_rho0.8_N{n}_64strains_{a.variant}", "n": n,
                   "variant": a.variant, "precision": a.precision, "sweep": a.sweep, "rate": 0.5, "density": 0.8, "rc": 2.5},
        "breakdown_ms": {"build": 1e3 * t_build / a.steps, "force": 1e3 * t_force / a.steps},
        "candidates_per_particle": tot_cands / (a.steps * n),
        "search_efficiency": 2 * tot_pairs / tot_cands,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
                     "frac": achieved / VALU_PEAK_GOPS, "traffic": None,
                     "kernel": f"k_sweep<{a.variant}>", "ops_per_launch": ops / a.steps,
                     "avg_launch_ms": 1e3 * t_force / a.steps},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(boxes, a.cpu_sample)
    h.close()
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
