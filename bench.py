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
            the 8 TB/s HBM peak; traffic = the HBM bytes per launch that
            rocprofv3 counted for the same kernel (FETCH_SIZE and WRITE_SIZE,
            scaled by what the counters read for a plain 1 GiB copy), taken
            from the committed summary under profiles/ while the kernel
            sources are unchanged since it was made, else null;
  cpu_baseline: the FP64 oracle timed on this host on a few cycles of the
            same workload, built with OpenMP on all the cores OpenMP is
            given (value, cores) and single-threaded (the parity build),
            with the core count and CPU model of the host;
  c1:       the quasi-1-D Poiseuille channel (1 x 64 cells, 50 particles per
            cell, Kn 0.1, seed 1) run in full: 2000 DSMC steps sampled every
            step with the D2Q9 projection of the cumulative averages every
            10 steps, on the GPU and, beside it, with the oracle (both
            builds); the final populations of the two are compared;
  adjoint:  the gradient of the coupling-node moment mismatch with respect to
            the body force and the relaxation time (and to the initial
            populations and the DSMC moment averages) on a D2Q37 1024 x 512
            lattice with the 32 rows at each wall coupled to DSMC strips of
            100 particles per cell (Kn 0.1, 200 steps, checkpoints every 20):
            time per gradient, the adjoint and forward lattice kernels against
            the HBM roofline, and the gradient against central differences of
            the library's own forward;
  batched:  256 independent Poiseuille channels of one cell across x, ny
            uniform in 32..512, particles per cell uniform in 20..200, Kn
            log-uniform in [0.01, 1], Ma 0.1, seeds 1000 + r, FP64, 500 steps
            sampled every step: stepped together (tiling chosen by the
            autotuner, steps replayed from a HIP graph) against the plain
            form, one channel context per replica run one after another;
            every replica's moments are compared bit for bit between the two;
  hybrid:   the coupling of Section 4 on a 1024 x 128 channel (Kn 0.05, Ma
            0.1): the DSMC subdomain (512 x 128 cells, 100 particles per
            cell) feeds the buffer-layer column of a D2Q9 lattice subdomain
            with diffuse walls (1 + 512 columns) every 10 lattice steps (40
            DSMC steps), by the equilibrium mapping of Eq. (feq_dsmc) and by
            the full projection: cycles per second, and the velocity profiles
            at x = L0/4 (DSMC), the buffer layer and x = 3 L0/4 (lattice);
  precision: the FP32-state form against plain FP64 on a 2048 x 1024 x 50
            channel (Kn 0.02, Ma 0.1), 500 steps sampled every step in 20
            batches of 25: particle-steps/s of each, and per moment order
            the RMS and mean over cells of z = dm / SE, dm the difference of
            the time-averaged Hermite moments of FP32 (seed 5) and FP64
            (seed 4), SE from batch means (paired, per run combined, and of
            the FP64 run alone), beside the same z of FP64 (seed 5) against
            the same FP64 run -- the sampling noise -- and the values z takes
            without any error; the batch-means SE is also set against the SE
            of independent steps, and against that of batches twice as long.
"""
from __future__ import annotations

import argparse
import csv
import ctypes
import glob
import hashlib
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
    # one DSMC step: read the state once and write it once (80 B per
    # particle); per cell the cell_start pair (8 B), the NTC state
    # nbar/sigcmax/rem read + written (48 B) and the 11 moment sums read +
    # written (176 B, sampling every step).  The library's own per-cell
    # bookkeeping (its gather tables) is not counted: it is how this
    # implementation moves particles, not what the method must move.
    "step": (80.0, 8 + 48 + 176),
    # the move of a settled state, in place: read + write the state, write
    # the group sizes
    "classify": (80.0, 4 + 40),
}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_512x256x100_fp64_traffic.md")
TRACE_SUMMARY = os.path.join(ROOT, "profiles", "dsmc_cycle_512x256x100_fp64_kernel_trace.md")
# the commands whose output the summaries condense (run from the repository root)
TRACE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/trace -o trace -- "
             "python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-precision --no-adjoint --no-batched --no-hybrid --no-c1")
PMC_CMDS = ("rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o fetch -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-precision --no-adjoint --no-batched --no-hybrid --no-c1 --copy-calibration",
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o write -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-precision --no-adjoint --no-batched --no-hybrid --no-c1 --copy-calibration")
# kernel-name prefixes of the library's kernels, by profiling id
KERNEL_PREFIX = {"step": "void dsmc::k_step<", "classify": "void dsmc::k_classify<", "complete": "void dsmc::k_complete<",
                 "project": "void dsmc::k_project<",
                 "reseed_gen": "void dsmc::k_reseed_gen<", "lbm": "void dsmc::k_lbm<"}
# VALU instruction counts of the same cycle (one counter pass): the reseed's
# FP64 work against the FP64 peak
VALU_SUMMARY = os.path.join(ROOT, "profiles", "dsmc_cycle_512x256x100_fp64_valu.md")
VALU_COUNTERS = ("SQ_INSTS_VALU SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_TRANS_F64 "
                 "SQ_WAVES SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64")
VALU_CMD = ("rocprofv3 --pmc " + VALU_COUNTERS + " --output-format csv -d gpurun_out/valu -o valu -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-precision --no-adjoint --no-batched --no-hybrid --no-c1")
FP64_PEAK_TFLOPS = 78.6
# the chip's vector issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles at 2.4 GHz
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
ADJ_TRACE_SUMMARY = os.path.join(ROOT, "profiles", "lbm_adjoint_1024x512_d2q37_kernel_trace.md")
ADJ_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "lbm_adjoint_1024x512_d2q37_traffic.md")
ADJ_TRACE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/adj_trace -o trace -- "
                 "python3 bench.py --adjoint-only")
ADJ_PMC_CMDS = ("rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/adj_fetch -o fetch -- "
                "python3 bench.py --adjoint-only --copy-calibration",
                "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/adj_write -o write -- "
                "python3 bench.py --adjoint-only --copy-calibration")
ADJ_KERNEL_PREFIX = {"lbm_adjoint": "void dsmc::k_lbm_adjoint<", "lbm_step": "void dsmc::k_lbm<"}
# the precision workload's two state widths, a few steps each, and the batched
# workload's steps (profiled apart from the timed runs)
C4_TRACE_SUMMARY = os.path.join(ROOT, "profiles", "k_step_2048x1024x50_fp32_fp64_kernel_trace.md")
C4_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_2048x1024x50_fp32_fp64_traffic.md")
C4_TRACE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/c4_trace -o trace -- "
                "python3 bench.py --profile-c4")
C4_PMC_CMDS = ("rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/c4_fetch -o fetch -- "
               "python3 bench.py --profile-c4 --copy-calibration",
               "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/c4_write -o write -- "
               "python3 bench.py --profile-c4 --copy-calibration")
C4_KERNEL_PREFIX = {"step_fp64": ("void dsmc::k_step<", "double"), "step_fp32": ("void dsmc::k_step<", "float"),
                    "classify_fp64": ("void dsmc::k_classify<", "double"),
                    "classify_fp32": ("void dsmc::k_classify<", "float")}
BAT_TRACE_SUMMARY = os.path.join(ROOT, "profiles", "k_step_batched_256_replicas_kernel_trace.md")
BAT_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_batched_256_replicas_traffic.md")
BAT_TRACE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/bat_trace -o trace -- "
                 "python3 bench.py --profile-batched")
BAT_PMC_CMDS = ("rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/bat_fetch -o fetch -- "
                "python3 bench.py --profile-batched --copy-calibration",
                "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/bat_write -o write -- "
                "python3 bench.py --profile-batched --copy-calibration")


# the precision workload (FP32 state vs FP64): 500 steps sampled every step,
# in 20 batches of 25 steps whose per-cell means give the standard errors
PREC = dict(nx=2048, ny=1024, ppc=50, kn=0.02, mach=0.1)
PREC_SEED_REF, PREC_SEED_ALT = 4, 5
PREC_BATCHES, PREC_BATCH_STEPS = 20, 25
# Hermite components per order: (sum indices, unit-Maxwellian variance), from
# the 11 per-cell sums N, x, y, xx, xy, yy, xxx, xxy, xyy, yyy, zz
HERMITE = {1: [((1,), 1.0), ((2,), 1.0)],
           2: [((3, -1), 2.0), ((4,), 1.0), ((5, -1), 2.0)],
           3: [((6, 1, -3), 6.0), ((7, 2, -1), 2.0), ((8, 1, -1), 2.0), ((9, 2, -3), 6.0)]}
# rows of the per-cell Hermite stack: order of each row and its variance
HROWS = [(0, None)] + [(o, var) for o, comps in HERMITE.items() for _, var in comps]


def _hermite_stack(avg):
    """[10][ncells] per-cell Hermite moments of one batch from its 11 averaged
    sums: the mean count, then per order the velocity Hermite components
    (per-particle means, in units of sqrt(kT/m))."""
    import torch

    n = avg[0]
    inv = 1.0 / torch.where(n > 0, n, torch.ones_like(n))
    rows = [n]
    for comps in HERMITE.values():
        for idx, _ in comps:
            h = avg[idx[0]] * inv
            if len(idx) == 2:  # x_i x_j - delta_ij
                h = h + idx[1]
            elif len(idx) == 3:  # cubic - c * linear
                h = h + idx[2] * avg[idx[1]] * inv
            rows.append(h)
    return torch.stack(rows)


def _precision_run(bits, seed):
    """One run of the precision workload: its per-batch Hermite stacks
    ([batches][rows][cells], on the GPU) and its stepping rate."""
    import torch

    from paper_1512_08042_amd import ChannelConfig
    from paper_1512_08042_amd import dsmc as D

    ch = D.Channel(ChannelConfig(state_bits=bits, seed=seed, **PREC))
    n = ch.status()["n"]
    batches, t_step = [], 0.0
    for _ in range(PREC_BATCHES):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(PREC_BATCH_STEPS, sample_every=1, moved=True)  # only moments are read between calls
        torch.cuda.synchronize()
        t_step += time.perf_counter() - t0
        batches.append(_hermite_stack(ch.sample_moments(reset=True)))
    ch.close()
    del ch
    torch.cuda.empty_cache()
    return torch.stack(batches), n * PREC_BATCHES * PREC_BATCH_STEPS / t_step


def _z_stats(a, b):
    """Per moment order, z of the time-averaged per-cell moments of runs a and
    b (each [batches][rows][cells]) under three standard errors:
      paired:   the batch means of the differences d_k = a_k - b_k,
                z = mean(d) / (sd(d) / sqrt(B)) (Student t, B - 1 dof);
      combined: each run's own batch-means SE, z = dm / sqrt(SE_a^2 + SE_b^2);
      single:   the SE of run b alone, z = dm / SE_b (for two independent
                runs without error, RMS z = sqrt(2) times the t inflation)."""
    import math

    import torch

    B = a.shape[0]
    d = a - b
    dm = d.mean(0)
    se_pair = d.std(0) / math.sqrt(B)
    se_a, se_b = a.std(0) / math.sqrt(B), b.std(0) / math.sqrt(B)
    ok = (a[:, 0] > 0).all(0) & (b[:, 0] > 0).all(0)
    out = {}
    for order in range(4):
        rows = [i for i, (o, _) in enumerate(HROWS) if o == order]
        r = {}
        for name, se in (("paired", se_pair), ("combined", torch.sqrt(se_a ** 2 + se_b ** 2)), ("single", se_b)):
            z = (dm[rows] / se[rows])[:, ok].flatten()
            z2 = z * z
            rms = float(torch.sqrt(z2.mean()))
            # uncertainty of the RMS from the spread of z^2 over cells
            unc = float(z2.std() / math.sqrt(z2.numel())) / (2.0 * rms)
            r[name] = {"rms": round(rms, 4), "rms_unc": round(unc, 4), "mean": round(float(z.mean()), 4)}
        r["n"] = int(ok.sum()) * len(rows)
        out[str(order)] = r
    return out


def _se_calibration(a):
    """For one run: per order, the mean over cells of its batch-means SE over
    the SE of independent steps (variance / (N S), the sampling noise of
    Section 5 with consecutive steps counted as independent), and of the SE
    from batches twice as long over that from the batches used."""
    import math

    import torch

    B = a.shape[0]
    S = B * PREC_BATCH_STEPS
    se = a.std(0) / math.sqrt(B)
    a2 = 0.5 * (a[0::2] + a[1::2])
    se2 = a2.std(0) / math.sqrt(B // 2)
    N = a[:, 0].mean(0)
    ok = (a[:, 0] > 0).all(0)
    out = {}
    for order in range(4):
        rows = [i for i, (o, _) in enumerate(HROWS) if o == order]
        fr = []
        for i in rows:
            var = HROWS[i][1]
            f = torch.sqrt(N / S) if var is None else torch.sqrt(var / (N * S))
            fr.append((se[i] / f)[ok])
        out[str(order)] = {"se_batch_over_independent_steps": round(float(torch.cat(fr).mean()), 3),
                           "se_batch50_over_batch25": round(float((se2[rows] / se[rows])[:, ok].mean()), 3)}
    return out


def profile_c4():
    """8 sampled steps of the precision workload per state width (FP64, then
    FP32): the run the C4 summaries profile.  Returns the step times."""
    import torch

    from paper_1512_08042_amd import ChannelConfig
    from paper_1512_08042_amd import dsmc as D

    out = {}
    for bits in (64, 32):
        ch = D.Channel(ChannelConfig(state_bits=bits, seed=PREC_SEED_REF, **PREC))
        ch.step(2, sample_every=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(6, sample_every=1)
        torch.cuda.synchronize()
        out["fp%d_ms_per_step" % bits] = round(1e3 * (time.perf_counter() - t0) / 6, 4)
        ch.close()
        del ch
        torch.cuda.empty_cache()
    return out


def profile_batched():
    """The batched workload's autotuner steps and 10 steps under its choice:
    the run the batched summaries profile."""
    import torch

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import inputs

    from paper_1512_08042_amd import dsmc as D

    B = BATCH
    reps = inputs.replica_params(B["seed"], B["nrep"])
    for r in reps:
        r["mach"] = B["mach"]
    b = D.Batch(reps)
    tune = b.autotune(B["tune_steps"], 1)
    b.step(0, 1, moved=True)  # as the timed replays run: the state moved between calls
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(10, 1, moved=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = b.status()["n"]
    b.close()
    return {"chosen": tune["chosen"], "ms_per_step": round(1e3 * dt / 10, 4), "particles": n}


def precision_comparison():
    """FP32-state vs FP64 on the precision workload: rates, and the moment
    error of FP32 (seed 5) against FP64 (seed 4) beside that of FP64 (seed 5)
    against the same FP64 run: the sampling noise the FP32 error is stated
    against.  Standard errors from batch means."""
    import math

    ref, v64 = _precision_run(64, PREC_SEED_REF)
    alt64, _ = _precision_run(64, PREC_SEED_ALT)
    z64 = _z_stats(alt64, ref)
    calib = _se_calibration(ref)
    del alt64
    alt32, v32 = _precision_run(32, PREC_SEED_ALT)
    z32 = _z_stats(alt32, ref)
    del alt32, ref
    B = PREC_BATCHES
    t_infl = math.sqrt((B - 1) / (B - 3))
    out = {"workload": "2048x1024 cells x 50 particles/cell (104,857,600 particles), Kn 0.02, Ma 0.1, from the "
                       "Maxwellian start; %d steps sampled every step, in %d batches of %d; FP64 seed %d (reference), "
                       "FP64 seed %d, FP32 state seed %d" % (B * PREC_BATCH_STEPS, B, PREC_BATCH_STEPS,
                                                             PREC_SEED_REF, PREC_SEED_ALT, PREC_SEED_ALT),
           "fp64_particle_steps_per_s": float("%.4g" % v64),
           "fp32_particle_steps_per_s": float("%.4g" % v32),
           "fp32_speedup": round(v32 / v64, 3),
           "moment_z_by_order": {"fp32_seed5_vs_fp64_seed4": z32, "fp64_seed5_vs_fp64_seed4": z64},
           "expected_rms_z_without_error": {"paired": round(t_infl, 4), "combined": round(
               math.sqrt((2 * B - 2) / (2 * B - 4)), 4), "single": round(math.sqrt(2.0) * t_infl, 4)},
           "se_calibration_fp64_seed4": calib}
    return out


# the differentiation workload: D2Q37 lattice 1024 x 512 (edge rows held), Kn
# 0.1 on its 512 rows, Ma 0.1; DSMC strips 32 cells thick at both walls, 100
# particles per cell, stood in for by one 1024 x 64 DSMC channel with the same
# mean free path (rows 0..31 face the lower wall, rows 32..63 the upper one)
ADJ = dict(nx=1024, ny=512, strip=32, ppc=100, kn=0.1, mach=0.1, seed=5, steps=200, every=20,
           dsmc_warm=20, dsmc_sampled=50)


def adjoint_benchmark(reps=3):
    """Times the mismatch gradient of the differentiation workload and
    checks it against central differences of the forward."""
    import numpy as np
    import torch

    from paper_1512_08042_amd import ChannelConfig, bgk_tau, body_force
    from paper_1512_08042_amd import _lib, lbm
    from paper_1512_08042_amd import dsmc as D

    A = ADJ
    nx, ny, q, S = A["nx"], A["ny"], 37, A["strip"]
    nn = nx * ny
    g_acc = body_force(A["kn"], ny, A["mach"])
    lam_cells = A["kn"] * ny
    ch = D.Channel(ChannelConfig(nx=nx, ny=2 * S, ppc=A["ppc"], kn=lam_cells / (2 * S), body_force_x=g_acc,
                                 seed=A["seed"]))
    ch.step(A["dsmc_warm"])
    ch.reset_moments()
    ch.step(A["dsmc_sampled"], sample_every=1)
    avg = ch.sample_moments().contiguous()
    nparticles = ch.status()["n"]
    del ch
    rows = np.r_[0:S, ny - S:ny]
    nodes = torch.tensor((rows[:, None] * nx + np.arange(nx)[None, :]).ravel(), dtype=torch.int32, device="cuda")
    cells = torch.arange(2 * S * nx, dtype=torch.int32, device="cuda")
    e, w, r = D.lattice(q)
    tau = bgk_tau(A["kn"], ny, r)
    g = g_acc / r
    # Poiseuille start: third-order equilibrium of u_x = 4 U y (H - y) / H^2, U = Ma
    yv = (torch.arange(ny, dtype=torch.float64, device="cuda") + 0.5) / ny
    ux = (4.0 * A["mach"] * yv * (1 - yv)).repeat_interleave(nx)
    xi_x = torch.tensor(r * e[:, 0], dtype=torch.float64, device="cuda")[:, None]
    cu = xi_x * ux[None, :]
    wt = torch.tensor(w, dtype=torch.float64, device="cuda")[:, None]
    f0 = (wt * (1 + cu + 0.5 * (cu * cu - ux * ux) + cu * (cu * cu - 3 * ux * ux) / 6)).contiguous()

    def gradient():
        m = avg.clone().requires_grad_(True)
        f = f0.clone().requires_grad_(True)
        g_t = torch.tensor(g, dtype=torch.float64, device="cuda", requires_grad=True)
        t_t = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
        fD = lbm.project_moments(m, A["ppc"], q, 3)
        fN = lbm.rollout(f, g_t, t_t, nx, ny, q, 1, A["steps"], A["every"])
        J = lbm.coupling_mismatch(fN, nodes, fD, cells, q, 3)
        J.backward()
        return float(J.detach()), float(g_t.grad), float(t_t.grad)

    def J_only(gv, tv):
        with torch.no_grad():
            fD = lbm.project_moments(avg, A["ppc"], q, 3)
            fN = lbm.rollout(f0, gv, tv, nx, ny, q, 1, A["steps"], A["every"])
            return float(lbm.coupling_mismatch(fN, nodes, fD, cells, q, 3))

    res = gradient()  # warm-up
    times, ftimes = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = gradient()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        J_only(g, tau)
        torch.cuda.synchronize()
        ftimes.append(time.perf_counter() - t0)
    J, dg, dtau = res
    hg, ht = 1e-4 * g, 1e-4 * tau
    fd_g = (J_only(g + hg, tau) - J_only(g - hg, tau)) / (2 * hg)
    fd_t = (J_only(g, tau + ht) - J_only(g, tau - ht)) / (2 * ht)

    # the two lattice kernels alone, HIP events on the launch stream
    L = _lib.lib()
    cfg = _lib.LbmConfig(nx, ny, q, 1, tau, g)
    s = torch.cuda.current_stream()
    fa, fb = f0.clone(), torch.empty_like(f0)
    lam_a = torch.randn_like(f0)
    # the adjoint kernel alone: a 20-step reverse pass with a checkpoint at
    # every step (nothing recomputed), one finishing reduction per 20 steps
    NADJ = 20
    ckpt = f0.unsqueeze(0).repeat(NADJ, 1, 1).contiguous()
    size = ctypes.c_size_t()
    _lib.check(L.lbm_adjoint_workspace(ctypes.byref(cfg), 1, ctypes.byref(size)), "lbm_adjoint_workspace")
    work = torch.empty(size.value, dtype=torch.uint8, device="cuda")
    grad = torch.zeros(2, dtype=torch.float64, device="cuda")

    def timed(fn, n=50):
        for _ in range(3):
            fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for _ in range(n):
            fn()
        ev1.record(s)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) * 1e3 / n

    # two steps per call: the result lands back in f without a copy
    us_fwd = timed(lambda: L.lbm_step(ctypes.byref(cfg), fa.data_ptr(), fb.data_ptr(), 2, s.cuda_stream)) / 2
    us_adj = timed(lambda: L.lbm_adjoint(ctypes.byref(cfg), ckpt.data_ptr(), NADJ, 1, lam_a.data_ptr(),
                                         grad.data_ptr(), work.data_ptr(), s.cuda_stream), n=10) / NADJ
    us_copy = timed(lambda: fb.copy_(fa))
    us_fwd_kernel = us_fwd
    adj_bytes, fwd_bytes = 24.0 * q * nn, 16.0 * q * nn
    med = sorted(times)[len(times) // 2]
    fmed = sorted(ftimes)[len(ftimes) // 2]
    achieved = adj_bytes / (us_adj * 1e-6) / 1e9
    return {
        "workload": "D2Q37 BGK 1024x512 (3 edge rows held), tau of Eq. (tau) at Kn 0.1 on 512 rows = %.3f, "
                    "g for Ma 0.1; J = 1/2 sum over the 32 rows at each wall (65,536 nodes) of the squared "
                    "mismatch of the ten Hermite coefficients to third order between the lattice after %d steps "
                    "and the D2Q37 projection of DSMC averages (1024x64 DSMC cells, 100 particles/cell, "
                    "%d particles, %d sampled steps); checkpoints every %d steps"
                    % (tau, A["steps"], nparticles, A["dsmc_sampled"], A["every"]),
        "ms_per_gradient": round(1e3 * med, 3),
        "ms_forward_only": round(1e3 * fmed, 3),
        "gradient_node_steps_per_s": nn * A["steps"] / med,
        "J": J, "dJ_dg": dg, "dJ_dtau": dtau,
        "fd_rel_err": {"g": abs(dg - fd_g) / abs(fd_g), "tau": abs(dtau - fd_t) / abs(fd_t)},
        "kernels_us_per_launch": {"lbm_adjoint": round(us_adj, 2), "lbm_step": round(us_fwd_kernel, 2)},
        "roofline": {"bound": "hbm", "kernel": "k_lbm_adjoint", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": stored_traffic("lbm_adjoint", ADJ_TRAFFIC_SUMMARY), "bytes_per_launch": adj_bytes,
                     "forward_kernel_GBps": round(fwd_bytes / (us_fwd_kernel * 1e-6) / 1e9, 1),
                     "copy_GBps": round(2 * 8.0 * q * nn / (us_copy * 1e-6) / 1e9, 1)},
    }


# the batched workload
BATCH = dict(seed=3, nrep=256, mach=0.1, steps=500, graph_steps=10, tune_steps=2)


def batched_comparison():
    """Batched vs plain FP64 on the batched workload: particle-steps/s of
    each over the same 500 sampled steps, and the replicas' moments compared
    bit for bit (equal moment error)."""
    import numpy as np
    import torch

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import inputs

    from paper_1512_08042_amd import ChannelConfig
    from paper_1512_08042_amd import dsmc as D

    B = BATCH
    reps = inputs.replica_params(B["seed"], B["nrep"])
    for r in reps:
        r["mach"] = B["mach"]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    b = D.Batch(reps, stream=stream)
    n = b.status(stream=stream)["n"]
    t0 = time.perf_counter()
    tune = b.autotune(B["tune_steps"], 1, stream=stream)  # real steps: 4 candidates
    stream.synchronize()
    t_tune = time.perf_counter() - t0
    done = B["tune_steps"] * len(tune["particles_per_tile"])
    b.reset_moments(stream=stream)  # average over the steps after tuning
    # replays that leave the state moved for the next one (only moments are
    # read between them); the last steps settle it for the comparison
    b.graph_create(B["graph_steps"], 1, stream=stream, moved=True)
    nrep_launch = (B["steps"] - done - 1) // B["graph_steps"]
    rest = B["steps"] - done - nrep_launch * B["graph_steps"]
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(nrep_launch):
        b.graph_launch(stream=stream)
    b.step(rest, 1, stream=stream)
    stream.synchronize()
    t_batched = time.perf_counter() - t0
    steps_timed = nrep_launch * B["graph_steps"] + rest
    avg_b = b.sample_moments(stream=stream).cpu().numpy()
    st = b.status(stream=stream)
    stream.synchronize()

    # plain: one context per replica (with the tiling the autotuner chose, so
    # that even the moment sums add in the same order), each run for the same
    # 500 steps in turn
    chans = []
    for r in reps:
        c = D.Channel(ChannelConfig(nx=r["nx"], ny=r["ny"], ppc=r["ppc"], kn=r["kn"], mach=r["mach"], seed=r["seed"]))
        c.set_tiling(tune["chosen"])
        chans.append(c)
    for c in chans:  # the autotuner's steps, then the same sampled steps
        c.step(done, sample_every=1)
        c.reset_moments()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in chans:
        c.step(steps_timed, sample_every=1)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = 0
    zsq = {o: [0.0, 0] for o in range(4)}
    for i, c in enumerate(chans):
        c0, c1 = b.replica_cells(i)
        avg_p = c.sample_moments()
        # per-order z of the batched form against the plain one, SE of the
        # time averages with steps counted as independent
        hb = _hermite_stack(torch.from_numpy(avg_b[:, c0:c1]).to(avg_p.device))
        hp = _hermite_stack(avg_p)
        N = hp[0].clamp(min=1.0)
        for row, (order, var) in enumerate(HROWS):
            se = torch.sqrt((N if var is None else var / N) / steps_timed)
            zsq[order][0] += float((((hb[row] - hp[row]) / se) ** 2).sum())
            zsq[order][1] += int(N.numel())
        eq = np.array_equal(avg_p.cpu().numpy(), avg_b[:, c0:c1])
        eq = eq and all(torch.equal(p, q) for p, q in zip(c.particles(), b.replica_particles(i)))
        same += int(eq)
        c.close()
    del chans
    b.close()
    del b
    torch.cuda.empty_cache()
    v_b = n * steps_timed / t_batched
    v_p = n * steps_timed / t_plain
    return {
        "workload": "%d channel replicas (nx 1, ny U{32..512}, ppc U{20..200}, Kn log-U[0.01,1], Ma %.1f, seeds "
                    "1000+r), %d particles, FP64, %d steps sampled every step" % (B["nrep"], B["mach"], n, B["steps"]),
        "batched_particle_steps_per_s": float("%.4g" % v_b),
        "plain_particle_steps_per_s": float("%.4g" % v_p),
        "batched_speedup": round(v_b / v_p, 2),
        "batched_ms_per_step": round(1e3 * t_batched / steps_timed, 4),
        "plain_ms_per_step": round(1e3 * t_plain / steps_timed, 4),
        "batched_timed": "%d graph replays of %d steps (state left moved between them) + %d eager steps, after "
                         "%d autotuner steps" % (nrep_launch, B["graph_steps"], rest, done),
        "autotune": {"particles_per_tile": tune["particles_per_tile"],
                     "ms_per_step": [round(v, 4) for v in tune["ms_per_step"]], "chosen": tune["chosen"],
                     "seconds": round(t_tune, 3)},
        "replicas_bitwise_equal_to_plain": "%d/%d (particles, and moment sums over the %d timed steps)" % (
            same, B["nrep"], steps_timed),
        "moment_z_by_order_vs_plain_fp64": {str(o): round((v[0] / max(v[1], 1)) ** 0.5, 6) for o, v in zsq.items()},
        "step_roofline_frac": round(80.0 * v_b / 1e9 / HBM_PEAK_GBPS, 4),
        "status_bits": st["bits"],
    }


# the hybrid workload (Section 4)
HYB = dict(L0=1024, H=128, ppc=100, kn=0.05, mach=0.1, seed=6, lbm_steps=10, dsmc_per_lbm=4, warm=5, timed=50,
           observe=100)


def hybrid_benchmark():
    """Coupling cycles of the hybrid workload with both mappings: rates and
    the velocity profiles of the two subdomains."""
    import numpy as np
    import torch

    from paper_1512_08042_amd import ChannelConfig, body_force, hard_sphere_viscosity
    from paper_1512_08042_amd import dsmc as D

    Hh = HYB
    H, nx_d = Hh["H"], Hh["L0"] // 2
    nx_l = Hh["L0"] // 2 + 1  # the buffer column, then the lattice subdomain
    e, w, r = D.lattice(9)
    dt = 1.0 / (Hh["dsmc_per_lbm"] * r)  # lattice step = 1/r in units of dx / sqrt(kT/m)
    g = body_force(Hh["kn"], H, Hh["mach"])
    nu = hard_sphere_viscosity(Hh["kn"], H)
    tau = 0.5 + r * nu  # lattice viscosity (tau - 1/2)/r matched to the gas
    ds = Hh["lbm_steps"] * Hh["dsmc_per_lbm"]
    xi_x = torch.tensor(r * e[:, 0], dtype=torch.float64, device="cuda")[:, None]
    out = {"workload": "channel 1024x128, Kn 0.05, Ma 0.1: DSMC subdomain 512x128 cells x 100 particles/cell, D2Q9 "
                       "subdomain (buffer column + 512 columns) x 128 rows with diffuse walls, tau %.3f (viscosity "
                       "matched), %d DSMC steps (dt = lattice step / %d) and %d lattice steps per cycle; %d warm-up, "
                       "%d timed and %d observed cycles from rest" % (tau, ds, Hh["dsmc_per_lbm"], Hh["lbm_steps"],
                                                                      Hh["warm"], Hh["timed"], Hh["observe"])}
    for mapping, name in ((0, "equilibrium"), (1, "full")):
        ch = D.Channel(ChannelConfig(nx=nx_d, ny=H, ppc=Hh["ppc"], kn=Hh["kn"], dt=dt, body_force_x=g,
                                     seed=Hh["seed"]))
        f = torch.tensor(w, dtype=torch.float64, device="cuda")[:, None].repeat(1, nx_l * H).contiguous()
        tmp = torch.empty_like(f)
        avg = torch.empty((11, nx_d * H), dtype=torch.float64, device="cuda")

        def cycle(a=None):
            ch.hybrid_cycle(f, tmp, nx_l, tau, g / r, dsmc_steps=ds, lbm_steps=Hh["lbm_steps"], mapping=mapping,
                            order=2, avg_out=a, moved=True)  # only moments are read between cycles

        for _ in range(Hh["warm"]):
            cycle()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(Hh["timed"]):
            cycle()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        n = ch.status()["n"]
        sums = torch.zeros((4, H), dtype=torch.float64, device="cuda")
        for _ in range(Hh["observe"]):
            cycle(avg)
            m = avg.view(11, H, nx_d)
            sums[0] += m[1, :, nx_d // 4] / m[0, :, nx_d // 4]  # x = L0/4
            sums[1] += m[1, :, nx_d - 1] / m[0, :, nx_d - 1]  # the buffer layer
            fl = f.view(9, H, nx_l)[:, :, nx_l // 2]  # x = 3 L0/4
            rho = fl.sum(0)
            sums[2] += ((fl * xi_x).sum(0) + 0.5 * rho * g / r) / rho
            sums[3] += m[1].sum(1) / m[0].sum(1)  # every DSMC column (the subdomain is periodic along x)
        prof = (sums / Hh["observe"]).cpu().numpy()
        dsmc, buf, lb, dsmc_all = prof
        out[name] = {
            "ms_per_cycle": round(1e3 * t / Hh["timed"], 3),
            "dsmc_particle_steps_per_s": float("%.4g" % (n * ds * Hh["timed"] / t)),
            "lattice_node_steps_per_s": float("%.4g" % (nx_l * H * Hh["lbm_steps"] * Hh["timed"] / t)),
            "centreline_ux": {"dsmc_L0/4": round(float(dsmc[H // 2 - 1: H // 2 + 1].mean()), 5),
                              "buffer_L0/2": round(float(buf[H // 2 - 1: H // 2 + 1].mean()), 5),
                              "lattice_3L0/4": round(float(lb[H // 2 - 1: H // 2 + 1].mean()), 5),
                              "dsmc_all_columns": round(float(dsmc_all[H // 2 - 1: H // 2 + 1].mean()), 5)},
            "profile_rms_lattice_vs_dsmc_L0/4": round(float(np.sqrt(np.mean((lb - dsmc) ** 2)) / abs(dsmc).max()), 4),
            "profile_rms_lattice_vs_dsmc_all_columns": round(
                float(np.sqrt(np.mean((lb - dsmc_all) ** 2)) / abs(dsmc_all).max()), 4),
            "status_bits": ch.status()["bits"],
        }
        ch.close()
        del ch, f, tmp, avg
        torch.cuda.empty_cache()
    return out


def source_hash() -> str:
    """sha256 over the library's kernel sources and its C header."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1512_08042_amd", "csrc", "*.hip")) +
                   glob.glob(os.path.join(ROOT, "paper_1512_08042_amd", "csrc", "*.hpp")))
    files.append(os.path.join(ROOT, "include", "dsmc.h"))
    for p in files:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _stored(summary: str, key: str):
    """{profiling id: value} of the `key` lines of a committed summary, or {}
    when the summary is missing or the sources changed since it was made."""
    try:
        with open(summary) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return {}
    got, src = {}, None
    for ln in lines:
        if ln.startswith("source_sha256:"):
            src = ln.split(":", 1)[1].strip()
        elif ln.startswith(key + " "):
            kid, v = ln[len(key) + 1:].split(":", 1)
            got[kid.strip()] = float(v)
    return got if src == source_hash() else {}


def summarize_valu(valu_dir):
    """VALU instruction counts per launch of the cycle's kernels (one pass of
    VALU_COUNTERS), written to VALU_SUMMARY."""
    rows = _counter_rows(glob.glob(os.path.join(valu_dir, "*counter_collection.csv"))[0])
    per = {}
    for r in rows:
        per.setdefault((r["Kernel_Name"], r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    out = ["# VALU instructions per launch: coupling cycle, 512x256 cells x 100 particles/cell, FP64", "",
           "Command (from the repository root, on one MI355X):", "", "    " + VALU_CMD, "",
           "Counts are wave instructions (64 lanes).  FP64 flop slots = 64 x (ADD + MUL + TRANS) + 128 x FMA: the",
           "FP64 work the kernel issues, every lane counted.", "",
           "| kernel | dispatches | waves | VALU | FP64 add | FP64 mul | FP64 fma | FP64 trans | int32 | int64 |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    by_name = {}
    for (name, _), d in per.items():
        by_name.setdefault(name, []).append(d)
    per_id = {}
    for name in sorted(by_name):
        if "dsmc::" not in name:
            continue
        ds = by_name[name]
        mean = {c: sum(d.get(c, 0.0) for d in ds) / len(ds) for c in ds[0]}
        g = lambda c: mean.get("SQ_INSTS_" + c, 0.0)
        out.append("| `%s` | %d | %.0f | %.0f | %.0f | %.0f | %.0f | %.0f | %.0f | %.0f |" % (
            name, len(ds), mean.get("SQ_WAVES", 0.0), g("VALU"), g("VALU_ADD_F64"), g("VALU_MUL_F64"),
            g("VALU_FMA_F64"), g("VALU_TRANS_F64"), g("VALU_INT32"), g("VALU_INT64")))
        for kid, pre in KERNEL_PREFIX.items():
            if _kernel_of(name, pre):
                fl = 64 * (g("VALU_ADD_F64") + g("VALU_MUL_F64") + g("VALU_TRANS_F64")) + 128 * g("VALU_FMA_F64")
                per_id.setdefault(kid, []).append((len(ds), g("VALU"), fl))
    out += ["", "Per profiling id (all template variants, weighted by dispatches):", ""]
    for kid, v in sorted(per_id.items()):
        n = sum(a for a, _, _ in v)
        out.append("valu_insts_per_launch %s: %.0f" % (kid, sum(a * b for a, b, _ in v) / n))
        out.append("fp64_flop_slots_per_launch %s: %.0f" % (kid, sum(a * c for a, _, c in v) / n))
    out += ["", "source_sha256: " + source_hash()]
    with open(VALU_SUMMARY, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("wrote", VALU_SUMMARY)


def stored_traffic(kernel: str, summary: str = TRAFFIC_SUMMARY):
    """HBM bytes per launch of `kernel` from a committed counter summary, or
    None when the summary is missing or the sources changed since."""
    try:
        with open(summary) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    got, src = None, None
    for ln in lines:
        if ln.startswith("source_sha256:"):
            src = ln.split(":", 1)[1].strip()
        if ln.startswith("traffic_bytes_per_launch %s:" % kernel):
            got = float(ln.split(":", 1)[1].strip())
    return got if (src == source_hash() and got is not None) else None


def _counter_rows(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


# what each summary covers: title, the commands, the kernels reported per
# profiling id (name prefixes), and the files under profiles/
SUMMARIES = {
    "cycle": dict(
        title="coupling cycle, 512x256 cells x 100 particles/cell, FP64",
        trace_cmd=TRACE_CMD, pmc_cmds=PMC_CMDS, prefixes=KERNEL_PREFIX,
        trace_file=TRACE_SUMMARY, traffic_file=TRAFFIC_SUMMARY,
        note=["Each bench cycle: 10 DSMC steps (k_classify once, then cell kernels + k_step per step), the D2Q37",
              "projection, one BGK step and the strip reseed.  Timed and profiled cycles both appear."]),
    "adjoint": dict(
        title="mismatch gradient, D2Q37 1024x512, 200 steps, checkpoints every 20",
        trace_cmd=ADJ_TRACE_CMD, pmc_cmds=ADJ_PMC_CMDS, prefixes=ADJ_KERNEL_PREFIX,
        trace_file=ADJ_TRACE_SUMMARY, traffic_file=ADJ_TRAFFIC_SUMMARY,
        note=["Each gradient: the DSMC2LB projection, 200 forward steps (every 20th keeps a checkpoint), the",
              "Hermite coefficients and their adjoint, then per 20-step segment 19 recomputed forward steps and",
              "20 adjoint steps; the bench also times the two lattice kernels alone and runs central differences."]),
    "c4": dict(
        title="DSMC steps, 2048x1024 cells x 50 particles/cell (104,857,600 particles), FP64 and FP32 state",
        trace_cmd=C4_TRACE_CMD, pmc_cmds=C4_PMC_CMDS, prefixes=C4_KERNEL_PREFIX,
        trace_file=C4_TRACE_SUMMARY, traffic_file=C4_TRAFFIC_SUMMARY,
        note=["Per state width: one channel from its Maxwellian start (Kn 0.02, Ma 0.1, seed 4), 8 DSMC steps",
              "sampled every step (k_classify once, then cell kernels + k_step per step), FP64 first."]),
    "batched": dict(
        title="256 channel replicas stepped together (about 7.55 million particles), FP64",
        trace_cmd=BAT_TRACE_CMD, pmc_cmds=BAT_PMC_CMDS, prefixes=KERNEL_PREFIX,
        trace_file=BAT_TRACE_SUMMARY, traffic_file=BAT_TRAFFIC_SUMMARY,
        note=["The batched workload (nx 1, ny U{32..512}, ppc U{20..200}, Kn log-U[0.01,1], Ma 0.1, seeds",
              "1000+r): the autotuner's 8 steps over four tilings, then 10 steps under the tiling it chose,",
              "sampled every step."]),
}


def _kernel_of(name, spec):
    """Whether kernel `name` belongs to a profiling id: a name prefix, or a
    (prefix, text the name must also hold) pair."""
    if isinstance(spec, tuple):
        return name.startswith(spec[0]) and spec[1] in name
    return name.startswith(spec)


def summarize(which, trace_dir, fetch_dir, write_dir):
    """Writes the two summaries of one workload under profiles/ from rocprofv3 output."""
    W = SUMMARIES[which]
    stats = _counter_rows(glob.glob(os.path.join(trace_dir, "*kernel_stats.csv"))[0])
    out = ["# Kernel trace: " + W["title"], "",
           "Command (from the repository root, on one MI355X):", "", "    " + W["trace_cmd"], ""] + W["note"] + [
           "", "| kernel | calls | mean us | total % |", "|---|---|---|---|"]
    for r in stats:
        name = r["Name"]
        if "dsmc::" not in name and "copyBuffer" not in name:
            continue
        out.append("| `%s` | %s | %.1f | %s |" % (name.replace("|", "/"), r["Calls"], float(r["AverageNs"]) / 1e3,
                                                 r["Percentage"]))
    out.append("")
    out.append("Mean duration per profiling id (all template variants, weighted by calls):")
    out.append("")
    for kid, pre in sorted(W["prefixes"].items()):
        calls = [(float(r["Calls"]), float(r["AverageNs"])) for r in stats if _kernel_of(r["Name"], pre)]
        if calls:
            n = sum(c for c, _ in calls)
            out.append("mean_us %s: %.1f" % (kid, sum(c * a for c, a in calls) / n / 1e3))
    out.append("")
    out.append("source_sha256: " + source_hash())
    with open(W["trace_file"], "w") as fh:
        fh.write("\n".join(out) + "\n")

    # HBM bytes: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), calibrated on
    # the three 1 GiB device copies bench.py --copy-calibration makes
    def per_kernel(rows):
        agg = {}
        for r in rows:
            agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return agg
    fetch = per_kernel(_counter_rows(glob.glob(os.path.join(fetch_dir, "*counter_collection.csv"))[0]))
    write = per_kernel(_counter_rows(glob.glob(os.path.join(write_dir, "*counter_collection.csv"))[0]))
    gib_kib = float(1 << 20)
    cf = [v for v in fetch.get("__amd_rocclr_copyBuffer", []) if v > 0.25 * gib_kib]
    cw = [v for v in write.get("__amd_rocclr_copyBuffer", []) if v > 0.5 * gib_kib]
    f_fetch = gib_kib / (sum(cf) / len(cf))
    f_write = gib_kib / (sum(cw) / len(cw))
    out = ["# HBM traffic per launch: " + W["title"], "",
           "Commands (from the repository root, on one MI355X), one counter per run:", "",
           "    " + W["pmc_cmds"][0], "    " + W["pmc_cmds"][1], "",
           "Calibration: a 1 GiB device-to-device copy reads FETCH_SIZE = %.0f KiB and WRITE_SIZE = %.0f KiB, so"
           % (gib_kib / f_fetch, gib_kib / f_write),
           "bytes = %.3f x FETCH_SIZE + %.3f x WRITE_SIZE (KiB -> bytes x 1024)." % (f_fetch, f_write), "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB per launch |", "|---|---|---|---|---|"]
    per_id = {}
    for name in sorted(fetch):
        if not name.startswith(("void dsmc::", "dsmc::")) or name not in write:
            continue
        mf = sum(fetch[name]) / len(fetch[name])
        mw = sum(write[name]) / len(write[name])
        mb = (mf * f_fetch + mw * f_write) * 1024 / 1e6
        out.append("| `%s` | %d | %.0f | %.0f | %.1f |" % (name, len(fetch[name]), mf, mw, mb))
        for kid, pre in W["prefixes"].items():
            if _kernel_of(name, pre):
                per_id.setdefault(kid, []).extend(
                    [(a * f_fetch + b * f_write) * 1024 for a, b in zip(fetch[name], write[name])])
    out.append("")
    out.append("Per profiling id (all template variants, averaged over dispatches):")
    out.append("")
    for kid, v in sorted(per_id.items()):
        out.append("traffic_bytes_per_launch %s: %.0f" % (kid, sum(v) / len(v)))
    out.append("")
    out.append("source_sha256: " + source_hash())
    with open(W["traffic_file"], "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("wrote", W["trace_file"], W["traffic_file"])


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed coupling cycles")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=8, help="coupling cycles the OpenMP oracle is timed on")
    ap.add_argument("--cpu-cycles-single", type=int, default=2,
                    help="coupling cycles the single-threaded oracle is timed on")
    ap.add_argument("--no-c1", action="store_true", help="skip the quasi-1-D channel run")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32-vs-FP64 comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiation workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-replica workload")
    ap.add_argument("--no-hybrid", action="store_true", help="skip the hybrid-coupling workload")
    ap.add_argument("--hybrid-only", action="store_true",
                    help="run only the hybrid-coupling workload and print its JSON object")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched-replica workload and print its JSON object")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the differentiation workload and print its JSON object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three plain 1 GiB device copies (reference for HBM byte counters)")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write the profiles/ summaries from rocprofv3 output directories and exit")
    ap.add_argument("--summarize-adjoint", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="the same for the differentiation workload")
    ap.add_argument("--summarize-valu", metavar="VALU_DIR",
                    help="write the VALU-count summary of the cycle from a rocprofv3 --pmc directory and exit")
    ap.add_argument("--summarize-c4", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="the same for the precision workload's steps (--profile-c4)")
    ap.add_argument("--summarize-batched", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="the same for the batched workload's steps (--profile-batched)")
    ap.add_argument("--profile-c4", action="store_true",
                    help="run only a few precision-workload steps in FP64 and FP32 state (for rocprofv3)")
    ap.add_argument("--profile-batched", action="store_true",
                    help="run only a few batched-workload steps (for rocprofv3)")
    return ap.parse_args()


def _host():
    """Cores this process may run on and the CPU model, from the OS."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"nproc": nproc, "cpu_count": os.cpu_count(), "cpu_model": model,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def _oracle_cycles(strip, cycles, threads):
    """`cycles` coupling cycles of the C2 workload with the FP64 oracle;
    returns particle-steps/s and seconds (the Maxwellian start untimed)."""
    import numpy as np

    from oracle import oracle as O

    dt = O.default_dt(KN, NY)
    g = O.body_force_for_mach(KN, NY, MACH)
    sim = O.Sim(NX, NY, PPC, KN, dt=dt, g=g, seed=SEED, capacity=int(NX * NY * PPC * 1.25) + 1024,
                threads=threads)
    sim.init_maxwell()
    olat = O.lattice(37)
    tau = O.lbm_tau(KN, NY, olat["r"])
    cells = np.asarray(strip, dtype=np.int32)
    t0 = time.perf_counter()
    for _ in range(cycles):
        sim.step(STEPS_PER_CYCLE, sample_every=1)
        f = O.dsmc2lb(sim.averages(), PPC, olat, 3, threads=threads)
        sim.reset_moments()
        f = O.lbm_step(f, olat, NX, NY, tau, g / olat["r"], 1, 1, threads=threads)
        sim.lb2dsmc(olat, 3, f, cells)
    t1 = time.perf_counter()
    return NX * NY * PPC * STEPS_PER_CYCLE * cycles / (t1 - t0), t1 - t0


def cpu_baseline(strip, cycles, cycles_single):
    """The FP64 oracle on the host: OpenMP build on the cores OpenMP is given
    (the reported value) and the single-threaded parity build."""
    from oracle import oracle as O

    host = _host()
    threads = O.threads_in_use(0)
    v_omp, s_omp = _oracle_cycles(strip, cycles, 0)
    v_one, s_one = _oracle_cycles(strip, cycles_single, None)
    return {"value": v_omp, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": "%d coupling cycles (each 10 DSMC steps with sampling, D2Q37 projection of all cells, one BGK "
                      "step, strip reseed) of the same 512x256x100 channel after its Maxwellian start, C oracle "
                      "built with OpenMP on %d threads, %.1f s; single-threaded build: %d cycles, %.1f s"
                      % (cycles, threads, s_omp, cycles_single, s_one),
            "single_thread": {"value": v_one, "unit": "particle-steps/s", "cores": 1, "cycles": cycles_single,
                              "seconds": round(s_one, 2)},
            "omp": {"threads": threads, "cycles": cycles, "seconds": round(s_omp, 2),
                    "speedup_over_single": round(v_omp / v_one, 2)},
            **host}


C1 = dict(nx=1, ny=64, ppc=50, kn=0.1, mach=0.1, seed=1, steps=2000, map_every=10)


def c1_benchmark():
    """The quasi-1-D channel in full on the GPU and with the oracle."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_1512_08042_amd import ChannelConfig
    from paper_1512_08042_amd import dsmc as D

    c = C1
    n = c["nx"] * c["ny"] * c["ppc"]
    events = c["steps"] // c["map_every"]
    cfg = ChannelConfig(nx=c["nx"], ny=c["ny"], ppc=c["ppc"], kn=c["kn"], mach=c["mach"], seed=c["seed"]).resolved()

    def gpu_run(graph):
        # eager steps, or the 10 steps of an event replayed from a HIP graph
        # (the replays equal eager steps bit for bit)
        ch = D.Channel(cfg)
        stream = torch.cuda.Stream()
        f = torch.empty((9, c["nx"] * c["ny"]), dtype=torch.float64, device="cuda")
        if graph:
            ch.graph_create(c["map_every"], sample_every=1, stream=stream, moved=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(events):
            if graph:
                ch.graph_launch(stream=stream)
            else:
                ch.step(c["map_every"], sample_every=1, stream=stream, moved=True)
            ch.map_to_lbm(9, 2, out=f, stream=stream)
        stream.synchronize()
        dt = time.perf_counter() - t0
        out = f.cpu().numpy()
        st = ch.status()
        ch.close()
        return dt, out, st

    gpu_run(False)  # first launches (code loading) untimed
    t_gpu, f_gpu, st = gpu_run(False)
    t_graph, f_graph, _ = gpu_run(True)
    lat = O.lattice(9)
    res = {}
    for name, threads in (("single_thread", None), ("omp", 0)):
        sim = O.Sim(c["nx"], c["ny"], c["ppc"], c["kn"], dt=cfg.dt, g=cfg.body_force_x, seed=c["seed"],
                    capacity=2 * n + 64, threads=threads)
        sim.init_maxwell()
        t0 = time.perf_counter()
        for _ in range(events):
            sim.step(c["map_every"], sample_every=1)
            f_or = O.dsmc2lb(sim.averages(), c["ppc"], lat, 2, threads=threads)
        dt = time.perf_counter() - t0
        res[name] = {"particle_steps_per_s": n * c["steps"] / dt, "seconds": round(dt, 4),
                     "cores": O.threads_in_use(threads)}
    scale = np.abs(f_or).max()
    return {"workload": "1x64 cells x 50 particles/cell (3,200 particles), Kn 0.1, Ma 0.1, seed 1, FP64; 2000 "
                        "steps sampled every step, D2Q9 projection of the cumulative averages every 10 steps",
            "gpu": {"particle_steps_per_s": n * c["steps"] / t_gpu, "seconds": round(t_gpu, 4),
                    "us_per_step": 1e6 * t_gpu / c["steps"], "cell_maps_per_s": c["nx"] * c["ny"] * events / t_gpu,
                    "status_bits": st["bits"]},
            "gpu_graph": {"particle_steps_per_s": n * c["steps"] / t_graph, "seconds": round(t_graph, 4),
                          "us_per_step": 1e6 * t_graph / c["steps"],
                          "cell_maps_per_s": c["nx"] * c["ny"] * events / t_graph,
                          "equals_eager_bitwise": bool(np.array_equal(f_graph, f_gpu))},
            "oracle": res,
            "final_populations_max_abs_diff_over_max": float(np.abs(f_gpu - f_or).max() / scale)}


def main():
    args = _parse()
    if args.summarize:
        summarize("cycle", *args.summarize)
        return
    if args.summarize_adjoint:
        summarize("adjoint", *args.summarize_adjoint)
        return
    if args.summarize_c4:
        summarize("c4", *args.summarize_c4)
        return
    if args.summarize_valu:
        summarize_valu(args.summarize_valu)
        return
    if args.summarize_batched:
        summarize("batched", *args.summarize_batched)
        return
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
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_benchmark()}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_comparison()}), flush=True)
        return
    if args.hybrid_only:
        print(json.dumps({"hybrid": hybrid_benchmark()}), flush=True)
        return
    if args.profile_c4:
        print(json.dumps({"profile_c4": profile_c4()}), flush=True)
        return
    if args.profile_batched:
        print(json.dumps({"profile_batched": profile_batched()}), flush=True)
        return
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
        # the state stays moved between calls: the strip reseed goes into the
        # moved state, and no call begins with a pass that moves it again
        ch.step(STEPS_PER_CYCLE, sample_every=1, moved=True)
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
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": stored_traffic(dom), "kernel": dom,
                "bytes_per_launch": nb}
    step_bytes = 80.0 * value  # algorithmic floor of a particle step (read + write the state once)
    # the mapping kernels, from the committed trace and counter summaries of
    # this cycle (null when the sources changed since they were made)
    means = _stored(TRACE_SUMMARY, "mean_us")
    valu = _stored(VALU_SUMMARY, "valu_insts_per_launch")
    flops = _stored(VALU_SUMMARY, "fp64_flop_slots_per_launch")
    project_roof = {"bytes_per_launch": 384 * ncells, "event_us": round(kernels["project"]["us_mean"], 2)
                    if "project" in kernels else None, "trace_us": means.get("project")}
    for src in ("event", "trace"):
        t = project_roof[src + "_us"]
        project_roof[src + "_frac"] = round(384 * ncells / (t * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4) if t else None
    if roof is not None and valu.get(dom):
        # share of the chip's vector-instruction issue the kernel uses
        roof["valu_issue_frac"] = round(valu[dom] / (kernels[dom]["us_mean"] * 1e-6) / VALU_ISSUE_PER_S, 4)
    nnew = STRIP * NY * PPC  # about one cell's worth of particles per reseeded cell
    reseed_roof = None
    if means.get("reseed_gen") and flops.get("reseed_gen"):
        t = means["reseed_gen"] * 1e-6
        reseed_roof = {
            "kernel": "k_reseed_gen", "trace_us": means["reseed_gen"],
            "hbm_bytes_per_launch": 296 * len(strip) + 40 * nnew,
            "hbm_frac": round((296 * len(strip) + 40 * nnew) / t / 1e9 / HBM_PEAK_GBPS, 4),
            "fp64_flop_slots_per_launch": flops["reseed_gen"],
            "fp64_flop_slots_per_new_particle": round(flops["reseed_gen"] / nnew, 1),
            "fp64_tflops": round(flops["reseed_gen"] / t / 1e12, 2), "fp64_peak_tflops": FP64_PEAK_TFLOPS,
            "fp64_frac": round(flops["reseed_gen"] / t / 1e12 / FP64_PEAK_TFLOPS, 4),
            "valu_issue_frac": round(valu["reseed_gen"] / t / VALU_ISSUE_PER_S, 4) if valu.get("reseed_gen") else None}
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
        "project_roofline": project_roof,
        "reseed_roofline": reseed_roof,
        "kernels_us_per_launch": {k: round(v["us_mean"], 2) for k, v in kernels.items()},
        "kernel_ms_per_cycle": {k: round(v["ms_total"] / args.steps, 4) for k, v in kernels.items()},
        "profiled_ms_per_step": 1e3 * (tp1 - tp0) / args.steps,
        "status_bits": st["bits"],
    }
    del ch, f, ftmp
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        out["adjoint"] = adjoint_benchmark()
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = batched_comparison()
        torch.cuda.empty_cache()
    if not args.no_hybrid:
        out["hybrid"] = hybrid_benchmark()
        torch.cuda.empty_cache()
    if not args.no_precision:
        out["precision"] = precision_comparison()
    if not args.no_c1:
        out["c1"] = c1_benchmark()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(strip, args.cpu_cycles, args.cpu_cycles_single)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
