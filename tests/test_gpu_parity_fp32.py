"""GPU parity of the FP32-state form against the FP32-state oracle.

With state_bits = 32 every particle value is stored in FP32 and every write
rounds to the nearest float; the arithmetic is FP64 on both sides.  Integer
outputs (cell_start, counters, new-particle counts) must agree exactly.
Particle values agree exactly except where a 1-ulp FP64 difference of the
device and host transcendentals (log/sin/cos of Box-Muller and of the
scattering angle) straddles an FP32 rounding midpoint, which moves the stored
value by one FP32 ulp (probability about 4e-9 per value): the bar is two FP32
ulps relative.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle import oracle as O

pytestmark = pytest.mark.gpu

F32_TOL = 2.0 * 2.0 ** -23  # two FP32 ulps, relative


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_08042_amd import dsmc as D
    from paper_1512_08042_amd.config import ChannelConfig

    return D, ChannelConfig


def _f32(particles):
    return [np.asarray(a, dtype=np.float32).astype(np.float64) for a in particles]


def _pair32(nx, ny, ppc, kn, g=0.0, dt=None, seed=1, capacity=None, particles=None):
    D, ChannelConfig = _gpu()
    cfg = ChannelConfig(nx=nx, ny=ny, ppc=ppc, kn=kn, dt=dt, body_force_x=g, seed=seed, capacity=capacity,
                        state_bits=32).resolved()
    if particles is not None:
        particles = _f32(particles)
        ch = D.Channel(cfg, particles=[torch.as_tensor(a) for a in particles])
    else:
        ch = D.Channel(cfg)
    assert ch.state.dtype == torch.float32
    ref = O.Sim(nx, ny, ppc, kn, dt=cfg.dt, g=cfg.body_force_x, seed=seed, capacity=cfg.capacity, state32=True)
    if particles is not None:
        ref.load(*particles)
    else:
        ref.init_maxwell()
    return ch, ref, cfg


def _assert_state32(ch, ref, what=""):
    cs = ch.cell_start().cpu().numpy()
    assert np.array_equal(cs, ref.cells()[0]), "cell_start differs " + what
    got = [t.cpu().numpy().astype(np.float64) for t in ch.particles()]
    want = ref.particles()
    for name, g, w in zip("x y vx vy vz".split(), got, want):
        assert g.shape == w.shape, (name, what)
        assert np.array_equal(np.asarray(w, dtype=np.float32).astype(np.float64), w), "oracle value not a float"
        bad = ~np.isclose(g, w, rtol=F32_TOL, atol=F32_TOL)
        assert not bad.any(), "%s differs at %d slots %s (first %s: %r vs %r)" % (
            name, bad.sum(), what, np.where(bad)[0][:3], g[bad][:3], w[bad][:3])


def _assert_counters(ch, ref):
    st = ch.status()
    rc = ref.counters()
    assert st["ncoll"] == rc["ncoll"] and st["ncand"] == rc["ncand"] and st["nwall"] == rc["nwall"], (st, rc)
    assert st["n"] == rc["n"]
    assert st["bits"] == rc["status"], (st, rc)


@pytest.mark.parametrize("shape", [(1, 64, 50), (7, 5, 13)])
def test_fp32_init_matches_oracle(shape):
    nx, ny, ppc = shape
    ch, ref, _ = _pair32(nx, ny, ppc, 0.1, seed=3)
    _assert_state32(ch, ref, what="after init")
    x, y, _, _, _ = ref.particles()
    gx, gy = (t.cpu().numpy().astype(np.float64) for t in ch.particles()[:2])
    assert np.array_equal(gx, x) and np.array_equal(gy, y)  # positions use no transcendental


@pytest.mark.parametrize("nx,ny,n", [(7, 5, 3000), (2, 4, 777)])
def test_fp32_adopt_sorts_like_oracle(nx, ny, n):
    p = inputs.particles(11, nx, ny, n)
    ch, ref, _ = _pair32(nx, ny, 10, 0.1, particles=p, capacity=n * 2)
    _assert_state32(ch, ref, what="after adopt")
    got = [t.cpu().numpy().astype(np.float64) for t in ch.particles()]
    assert all(np.array_equal(g, w) for g, w in zip(got, ref.particles()))


@pytest.mark.parametrize("nx,ny,kn,g", [(6, 8, 0.05, 0.0), (1, 12, 0.02, 0.01), (2, 6, 0.2, 0.05)])
def test_fp32_one_step_from_identical_state(nx, ny, kn, g):
    counts = np.random.default_rng(nx * 100 + ny).integers(0, 60, nx * ny)
    counts[0] = 0
    p = inputs.particles_per_cell(5, nx, ny, counts, vscale=1.0)
    ch, ref, _ = _pair32(nx, ny, 30, kn, g=g, particles=p, capacity=int(counts.sum()) + 64)
    ch.step(1, sample_every=1)
    ref.step(1, sample_every=1)
    _assert_state32(ch, ref, what="after 1 step")
    _assert_counters(ch, ref)
    assert ch.status()["ncoll"] > 0


def test_fp32_channel_c1_steps_and_moments():
    # 64 cells across, 50 particles per cell, Kn 0.1, Ma 0.1 body force, seed 1
    from paper_1512_08042_amd.config import body_force

    g = body_force(0.1, 64, 0.1)
    ch, ref, _ = _pair32(1, 64, 50, 0.1, g=g, seed=1)
    for _ in range(4):
        ch.step(10, sample_every=1)
        ref.step(10, sample_every=1)
    _assert_state32(ch, ref, what="after 40 steps")
    _assert_counters(ch, ref)
    avg = ch.sample_moments().cpu().numpy()
    want = ref.averages()
    scale = np.abs(want).max(axis=1, keepdims=True) + 1.0
    assert np.all(np.abs(avg - want) <= 1e-6 * scale)


def test_fp32_reseed_matches_oracle():
    nx, ny, ppc = 11, 6, 40
    ch, ref, cfg = _pair32(nx, ny, ppc, 0.1, seed=9, capacity=nx * ny * ppc * 2)
    ch.step(3)
    ref.step(3)
    lat = O.lattice(37)
    f = inputs.populations(4, lat["w"], nx * ny, 0.02)
    cells = inputs.strip_cells(nx, ny, 2)
    ch.map_from_lbm(torch.as_tensor(f, device="cuda"), torch.as_tensor(cells, device="cuda"), 37, 3)
    ref.lb2dsmc(lat, 3, f, cells)
    _assert_state32(ch, ref, what="after reseed")
    ch.step(2)
    ref.step(2)
    _assert_state32(ch, ref, what="2 steps after reseed")
    _assert_counters(ch, ref)


def test_fp32_reseed_completed_by_the_next_step():
    nx, ny, ppc = 11, 6, 40
    ch, ref, cfg = _pair32(nx, ny, ppc, 0.1, seed=7, capacity=nx * ny * ppc * 4)
    ch.step(2)
    ref.step(2)
    lat = O.lattice(37)
    f = inputs.populations(5, lat["w"] * 4.0, nx * ny, 0.02)
    cells = inputs.strip_cells(nx, ny, 3)
    ch.map_from_lbm(torch.as_tensor(f, device="cuda"), torch.as_tensor(cells, device="cuda"), 37, 3)
    assert ref.lb2dsmc(lat, 3, f, cells) == 0
    ch.step(2)
    ref.step(2)
    _assert_state32(ch, ref, what="2 steps after reseed, no read in between")
    _assert_counters(ch, ref)


def test_fp32_full_size_one_step():
    # the 512 x 256 x 100 channel: one step from the same caller-written FP32 state
    from paper_1512_08042_amd.config import body_force

    nx, ny, ppc, kn = 512, 256, 100, 0.05
    counts = np.full(nx * ny, ppc)
    p = inputs.particles_per_cell(21, nx, ny, counts, vscale=1.0)
    ch, ref, _ = _pair32(nx, ny, ppc, kn, g=body_force(kn, ny, 0.1), particles=p,
                         capacity=int(counts.sum() * 1.25) + 1024)
    ch.step(1, sample_every=1)
    ref.step(1, sample_every=1)
    _assert_state32(ch, ref, what="512x256x100 after 1 step")
    _assert_counters(ch, ref)


@pytest.mark.parametrize("bits", [64, 32])
def test_precision_workload_full_size(bits):
    # the precision workload at its full size, in the launch configuration
    # the benchmark times: 2048 x 1024 cells x 50 particles (104,857,600),
    # Kn 0.02, Ma 0.1, seed 4, from the Maxwellian start; two steps sampled
    # every step, against the oracle (its OpenMP build, the same bits as the
    # serial one) element by element
    D, ChannelConfig = _gpu()
    cfg = ChannelConfig(nx=2048, ny=1024, ppc=50, kn=0.02, mach=0.1, seed=4, state_bits=bits).resolved()
    ch = D.Channel(cfg)
    ch.step(2, sample_every=1)
    ref = O.Sim(2048, 1024, 50, 0.02, dt=cfg.dt, g=cfg.body_force_x, seed=4, capacity=cfg.capacity,
                state32=bits == 32, threads=0)
    ref.init_maxwell()
    ref.step(2, sample_every=1)
    assert np.array_equal(ch.cell_start().cpu().numpy(), ref.cells()[0]), "cell_start"
    _assert_counters(ch, ref)
    tol = F32_TOL if bits == 32 else 1e-12
    for name, g, w in zip("x y vx vy vz".split(), ch.particles(), ref.particles()):
        g = g.cpu().numpy().astype(np.float64)
        bad = ~np.isclose(g, w, rtol=tol, atol=tol)
        assert not bad.any(), "%s (%d-bit) differs at %d slots (first %s)" % (name, bits, bad.sum(), np.where(bad)[0][:3])
        del g, w, bad
    avg = ch.sample_moments().cpu().numpy()
    want = ref.averages()
    scale = np.abs(want).max(axis=1, keepdims=True) + 1.0
    assert np.all(np.abs(avg - want) <= 1e-12 * scale), "moment averages"
    ch.close()
