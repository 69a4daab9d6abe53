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
  cpu_baseline: the FP64 oracle timed on this host on one cycle of the same
            workload (single-threaded);
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
            channel (Kn 0.02, Ma 0.1): particle-steps/s of each, and per
            moment order the RMS and mean over cells of z = (m32 - m64) / SE,
            m the time-averaged Hermite moments of each run and SE their
            sampling error under the Maxwellian (consecutive steps counted as
            independent, which overstates z), beside the same z between two
            FP64 runs of different seeds: the FP32 form's moment error is
            stated against that sampling noise.
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
    # one DSMC step: read the moved state once and write it once (80 B per
    # particle); per cell the cell_start pair (8 B), the group sizes read and
    # written (40 + 40 B), the NTC state nbar/sigcmax/rem read + written
    # (48 B) and the 11 moment sums read + written (176 B, sampling every step)
    "step": (80.0, 8 + 80 + 48 + 176),
    # the move of a settled state, in place: read + write the state, write
    # the group sizes
    "classify": (80.0, 4 + 40),
}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_512x256x100_fp64_traffic.md")
TRACE_SUMMARY = os.path.join(ROOT, "profiles", "dsmc_cycle_512x256x100_fp64_kernel_trace.md")
# the commands whose output the summaries condense (run from the repository root)
TRACE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/trace -o trace -- "
             "python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-precision --no-adjoint --no-batched --no-hybrid")
PMC_CMDS = ("rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o fetch -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-precision --no-adjoint --no-batched --no-hybrid --copy-calibration",
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o write -- "
            "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-precision --no-adjoint --no-batched --no-hybrid --copy-calibration")
# kernel-name prefixes of the library's kernels, by profiling id
KERNEL_PREFIX = {"step": "void dsmc::k_step<", "classify": "void dsmc::k_classify<"}
ADJ_TRACE_SUMMARY = os.path.join(ROOT, "profiles", "lbm_adjoint_1024x512_d2q37_kernel_trace.md")
ADJ_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "lbm_adjoint_1024x512_d2q37_traffic.md")
ADJ_TRACE_CMD = ("rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/adj_trace -o trace -- "
                 "python3 bench.py --adjoint-only")
ADJ_PMC_CMDS = ("rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/adj_fetch -o fetch -- "
                "python3 bench.py --adjoint-only --copy-calibration",
                "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/adj_write -o write -- "
                "python3 bench.py --adjoint-only --copy-calibration")
ADJ_KERNEL_PREFIX = {"lbm_adjoint": "void dsmc::k_lbm_adjoint<", "lbm_step": "void dsmc::k_lbm<"}


# the precision workload (FP32 state vs FP64)
PREC = dict(nx=2048, ny=1024, ppc=50, kn=0.02, mach=0.1, seed=4)
PREC_WARM, PREC_STEPS = 20, 100
# Hermite components per order: (sum indices, unit-Maxwellian variance), from
# the 11 per-cell sums N, x, y, xx, xy, yy, xxx, xxy, xyy, yyy, zz
HERMITE = {1: [((1,), 1.0), ((2,), 1.0)],
           2: [((3, -1), 2.0), ((4,), 1.0), ((5, -1), 2.0)],
           3: [((6, 1, -3), 6.0), ((7, 2, -1), 2.0), ((8, 1, -1), 2.0), ((9, 2, -3), 6.0)]}


def _moment_z(a, b, steps):
    """Per moment order: z = (m_a - m_b) / SE over cells (and components)."""
    import numpy as np

    N = 0.5 * (a[0] + b[0])
    ok = N > 0
    S = float(steps)
    z = {0: (a[0] - b[0])[ok] / np.sqrt(N[ok] / S)}
    for order, comps in HERMITE.items():
        zs = []
        for idx, var in comps:
            def hermite(m):
                inv = 1.0 / np.where(m[0] > 0, m[0], 1.0)
                h = m[idx[0]] * inv
                if len(idx) == 2:  # x_i x_j - delta_ij
                    h = h + idx[1]
                elif len(idx) == 3:  # cubic - c * linear
                    h = h + idx[2] * m[idx[1]] * inv
                return h
            se = np.sqrt(var / (N * S))
            zs.append(((hermite(a) - hermite(b)) / se)[ok])
        z[order] = np.concatenate(zs)
    return {str(k): {"rms": round(float(np.sqrt(np.mean(v ** 2))), 3), "mean": round(float(np.mean(v)), 3)}
            for k, v in z.items()}


def precision_comparison():
    """FP32-state vs FP64 on the precision workload: rates and moment error,
    beside the seed-to-seed difference of two FP64 runs (the sampling noise)."""
    import torch

    from paper_1512_08042_amd import ChannelConfig
    from paper_1512_08042_amd import dsmc as D

    res, avgs = {}, {}
    n = PREC["nx"] * PREC["ny"] * PREC["ppc"]
    for bits, seed in ((64, PREC["seed"]), (32, PREC["seed"]), (64, PREC["seed"] + 1)):
        cfg = dict(PREC)
        cfg["seed"] = seed
        ch = D.Channel(ChannelConfig(state_bits=bits, **cfg))
        ch.step(PREC_WARM)
        ch.reset_moments()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(PREC_STEPS, sample_every=1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if seed == PREC["seed"]:
            res["fp%d_particle_steps_per_s" % bits] = n * PREC_STEPS / (t1 - t0)
        avgs[(bits, seed)] = ch.sample_moments().cpu().numpy()
        del ch
        torch.cuda.empty_cache()
    out = {"workload": "2048x1024 cells x 50 particles/cell, Kn 0.02, Ma 0.1; %d warm-up steps, %d sampled steps; "
                       "FP32 and FP64 from seed %d, a second FP64 run from seed %d" %
                       (PREC_WARM, PREC_STEPS, PREC["seed"], PREC["seed"] + 1)}
    out.update({k: float("%.4g" % v) for k, v in res.items()})
    out["fp32_speedup"] = round(res["fp32_particle_steps_per_s"] / res["fp64_particle_steps_per_s"], 3)
    s0, s1 = PREC["seed"], PREC["seed"] + 1
    out["moment_z_by_order"] = {"fp32_vs_fp64": _moment_z(avgs[(32, s0)], avgs[(64, s0)], PREC_STEPS),
                                "fp64_seed_to_seed": _moment_z(avgs[(64, s1)], avgs[(64, s0)], PREC_STEPS)}
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
    b.graph_create(B["graph_steps"], 1, stream=stream)
    nrep_launch = (B["steps"] - done) // B["graph_steps"]
    rest = B["steps"] - done - nrep_launch * B["graph_steps"]
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(nrep_launch):
        b.graph_launch(stream=stream)
    if rest:
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
    for i, c in enumerate(chans):
        c0, c1 = b.replica_cells(i)
        eq = np.array_equal(c.sample_moments().cpu().numpy(), avg_b[:, c0:c1])
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
        "batched_timed": "%d graph replays of %d steps%s after %d autotuner steps" % (
            nrep_launch, B["graph_steps"], (" + %d eager" % rest) if rest else "", done),
        "autotune": {"particles_per_tile": tune["particles_per_tile"],
                     "ms_per_step": [round(v, 4) for v in tune["ms_per_step"]], "chosen": tune["chosen"],
                     "seconds": round(t_tune, 3)},
        "replicas_bitwise_equal_to_plain": "%d/%d (particles, and moment sums over the %d timed steps)" % (
            same, B["nrep"], steps_timed),
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
                            order=2, avg_out=a)

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
}


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
        calls = [(float(r["Calls"]), float(r["AverageNs"])) for r in stats if r["Name"].startswith(pre)]
        if calls:
            n = sum(c for c, _ in calls)
            out.append("mean_us %s: %.1f" % (kid, sum(c * a for c, a in calls) / n / 1e3))
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
            if name.startswith(pre):
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
    ap.add_argument("--cpu-cycles", type=int, default=8, help="coupling cycles the CPU oracle is timed on")
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
    if args.summarize:
        summarize("cycle", *args.summarize)
        return
    if args.summarize_adjoint:
        summarize("adjoint", *args.summarize_adjoint)
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
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": stored_traffic(dom), "kernel": dom,
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(strip, args.cpu_cycles)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
