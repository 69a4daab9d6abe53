"""Benchmark of the DSMC step + DSMC<->LBM mapping hot path on one GPU.

Workload (one "step" of this benchmark = one coupling cycle over the whole
hot path): a 2-D force-driven channel of 512 x 256 cells, 100 hard-sphere
particles per cell (13,107,200 particles, FP64 state), Kn = 0.05 on the
channel height, body force for Ma = 0.1, diffuse walls, Philox seed 2.
Each cycle runs
  10 DSMC steps (move + walls, sort, NTC collisions, sampling every step),
  the DSMC->D2Q37 projection of all 131,072 cells (3rd order),
  one BGK D2Q37 lattice step (edge rows held),
  the LB->DSMC reseed of the 16-cell-wide strip x < 16 (4,096 cells, 3rd order).
The metric is particle-steps per second over whole cycles; cell-maps per
second (projected plus reseeded cells) is reported beside it.

Printed JSON line: metric, value, ..., plus
  roofline: the dominant kernel's algorithmic bytes per launch divided by
            its mean launch time (HIP events on its launch stream), against
            the 8 TB/s HBM peak;
  cpu_baseline: the FP64 oracle timed on this host on one cycle of the same
            workload (single-threaded).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
NX, NY, PPC, KN, MACH, SEED = 512, 256, 100, 0.05, 0.1, 2
STEPS_PER_CYCLE, STRIP = 10, 16

# algorithmic bytes per unit (FP64): a particle is 5 doubles = 40 B
BYTES = {
    # one DSMC step: read the cell-sorted state and write it sorted by the
    # new cells (80 B per particle); per cell the cell_start pair (8 B), the
    # NTC state nbar/sigcmax/rem read + written (48 B) and the 11 moment sums
    # read + written (176 B, sampling every step)
    "step": (80.0, 8 + 48 + 176),
    # classification of a state set from outside: read x, y, vx, vy
    "classify": (32.0, 8 + 9 * 4),
}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed coupling cycles")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=4, help="coupling cycles the CPU oracle is timed on")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three plain 1 GiB device copies (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(strip, cycles):
    """`cycles` coupling cycles of the same workload with the FP64 oracle on the host."""
    import numpy as np

    from oracle import oracle as O

    dt = O.default_dt(KN, NY)
    g = O.body_force_for_mach(KN, NY, MACH)
    sim = O.Sim(NX, NY, PPC, KN, dt=dt, g=g, seed=SEED, capacity=int(NX * NY * PPC * 1.25) + 1024)
    sim.init_maxwell()
    olat = O.lattice(37)
    tau = O.lbm_tau(KN, NY, olat["r"])
    cells = np.asarray(strip, dtype=np.int32)
    t0 = time.perf_counter()
    for _ in range(cycles):
        sim.step(STEPS_PER_CYCLE, sample_every=1)
        f = O.dsmc2lb(sim.averages(), PPC, olat, 3)
        sim.reset_moments()
        f = O.lbm_step(f, olat, NX, NY, tau, g / olat["r"], 1, 1)
        sim.lb2dsmc(olat, 3, f, cells)
    t1 = time.perf_counter()
    n = NX * NY * PPC
    return {"value": n * STEPS_PER_CYCLE * cycles / (t1 - t0), "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d coupling cycles (each 10 DSMC steps with sampling, D2Q37 projection of all cells, one BGK "
                      "step, strip reseed) of the same 512x256x100 channel after its Maxwellian start, "
                      "single-threaded C, %.1f s" % (cycles, t1 - t0)}


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the hot path here is a single-GPU build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1512_08042_amd import ChannelConfig, bgk_tau
    from paper_1512_08042_amd import _lib
    from paper_1512_08042_amd import dsmc as D

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # plain device-to-device copies of known size: 1 GiB read + 1 GiB written each
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = ChannelConfig(nx=NX, ny=NY, ppc=PPC, kn=KN, mach=MACH, seed=SEED).resolved()
    ch = D.Channel(cfg)
    e, w, r = D.lattice(37)
    tau = bgk_tau(KN, NY, r)
    g_lb = cfg.body_force_x / r  # velocity gain per lattice step (lattice time = dx / (r sqrt(kT/m)))
    ncells = NX * NY
    strip = [iy * NX + ix for iy in range(NY) for ix in range(STRIP)]
    cells = torch.tensor(strip, dtype=torch.int32, device="cuda")
    f = torch.empty((37, ncells), dtype=torch.float64, device="cuda")
    ftmp = torch.empty_like(f)
    nparticles = NX * NY * PPC

    def cycle():
        ch.step(STEPS_PER_CYCLE, sample_every=1)
        ch.map_to_lbm(37, 3, out=f)
        ch.reset_moments()
        D.lbm_step(f, NX, NY, 37, tau, g_lb, 1, 1, f_tmp=ftmp)
        ch.map_from_lbm(f, cells, 37, 3)

    for _ in range(args.warmup):
        cycle()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cycle()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = nparticles * STEPS_PER_CYCLE * args.steps / elapsed
    cell_maps = (ncells + len(strip)) * args.steps / elapsed

    # per-kernel times with HIP events on the launch stream, same cycles again
    ch.profile(True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        cycle()
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    ch.profile(False)
    kernels = {}
    for kid, name in enumerate(_lib.KERNEL_NAMES):
        ms, n = ch.profile_read(kid)
        if n:
            kernels[name] = {"ms_total": ms, "launches": n, "us_mean": 1e3 * ms / n}
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
    st = ch.status()
    roof = None
    if dom in BYTES:
        per_p, per_c = BYTES[dom]
        nb = per_p * st["n"] + per_c * ncells
        achieved = nb / (kernels[dom]["us_mean"] * 1e-6) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": dom,
                "bytes_per_launch": nb}
    step_bytes = 80.0 * value  # algorithmic floor of a particle step (read + write the state once)
    out = {
        "metric": "particle-steps/s + cell-maps/s; chosen form vs plain FP64 at equal moment error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2-D force-driven channel 512x256 cells x 100 particles/cell (13,107,200 particles), "
                               "Kn 0.05, Ma 0.1, FP64; cycle = 10 DSMC steps (sampled every step) + DSMC->D2Q37 "
                               "map of all cells + 1 BGK step + LB->DSMC reseed of a 16-cell strip",
                   "particles": nparticles, "cells": ncells, "steps_per_cycle": STEPS_PER_CYCLE},
        "cell_maps_per_s": cell_maps,
        "step_roofline": {"bytes_per_particle_step": 80, "achieved_GBps": round(step_bytes / 1e9, 1),
                          "frac": round(step_bytes / 1e9 / HBM_PEAK_GBPS, 4)},
        "roofline": roof,
        "kernels_us_per_launch": {k: round(v["us_mean"], 2) for k, v in kernels.items()},
        "kernel_ms_per_cycle": {k: round(v["ms_total"] / args.steps, 4) for k, v in kernels.items()},
        "profiled_ms_per_step": 1e3 * (tp1 - tp0) / args.steps,
        "status_bits": st["bits"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(strip, args.cpu_cycles)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
