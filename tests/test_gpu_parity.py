"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
identical seeded inputs.

Bars: integer outputs (cell_start, sort order, collision/wall counts, new-
particle counts) bit-exact; FP64 state within 1e-12 relative (the only
differences are 1-ulp differences of the device and host transcendentals
log/sin/cos in Box-Muller and the scattering angle); sampled moments within
1e-12 of their scale (different summation order).
"""
import numpy as np
import pytest
import torch

import inputs
from oracle import oracle as O

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_08042_amd import dsmc as D
    from paper_1512_08042_amd.config import ChannelConfig

    return D, ChannelConfig


def _pair(nx, ny, ppc, kn, g=0.0, dt=None, seed=1, capacity=None, particles=None, nbar_mode=0, far_capacity=0,
          kT=1.0):
    D, ChannelConfig = _gpu()
    cfg = ChannelConfig(nx=nx, ny=ny, ppc=ppc, kn=kn, dt=dt, body_force_x=g, seed=seed, capacity=capacity,
                        nbar_mode=nbar_mode, far_capacity=far_capacity, kT_over_m=kT).resolved()
    if particles is not None:
        ch = D.Channel(cfg, particles=[torch.as_tensor(a) for a in particles])
    else:
        ch = D.Channel(cfg)
    ref = O.Sim(nx, ny, ppc, kn, dt=cfg.dt, g=cfg.body_force_x, seed=seed, capacity=cfg.capacity,
                nbar_mode=nbar_mode, kT=kT)
    if particles is not None:
        ref.load(*particles)
    else:
        ref.init_maxwell()
    return ch, ref, cfg


def _assert_state(ch, ref, rtol=RTOL, what=""):
    cs = ch.cell_start().cpu().numpy()
    assert np.array_equal(cs, ref.cells()[0]), "cell_start differs " + what
    got = [t.cpu().numpy() for t in ch.particles()]
    want = ref.particles()
    for name, g, w in zip("x y vx vy vz".split(), got, want):
        assert g.shape == w.shape, (name, what)
        bad = ~np.isclose(g, w, rtol=rtol, atol=rtol)
        assert not bad.any(), "%s differs at %d slots %s (first %s: %r vs %r)" % (
            name, bad.sum(), what, np.where(bad)[0][:3], g[bad][:3], w[bad][:3])


def _assert_cells(ch, ref):
    nbar, sig, rem = (t.cpu().numpy() for t in ch.cell_state())
    _, nbar_r, sig_r, rem_r = ref.cells()
    assert np.allclose(nbar, nbar_r, rtol=RTOL, atol=0)
    assert np.allclose(sig, sig_r, rtol=RTOL, atol=0)
    assert np.allclose(rem, rem_r, rtol=1e-10, atol=1e-12)


def _assert_counters(ch, ref):
    st = ch.status()
    rc = ref.counters()
    assert st["ncoll"] == rc["ncoll"] and st["ncand"] == rc["ncand"] and st["nwall"] == rc["nwall"], (st, rc)
    assert st["n"] == rc["n"]
    assert st["bits"] == rc["status"], (st, rc)


@pytest.mark.parametrize("shape", [(1, 64, 50), (7, 5, 13), (3, 3, 1)])
def test_init_matches_oracle(shape):
    nx, ny, ppc = shape
    ch, ref, _ = _pair(nx, ny, ppc, 0.1, seed=3)
    _assert_state(ch, ref, what="after init")
    x, y, _, _, _ = ref.particles()
    gx, gy = (t.cpu().numpy() for t in ch.particles()[:2])
    assert np.array_equal(gx, x) and np.array_equal(gy, y)  # positions use no transcendental
    _assert_cells(ch, ref)


@pytest.mark.parametrize("nx,ny,n", [(7, 5, 3000), (1, 9, 400), (2, 4, 777), (16, 16, 0)])
def test_adopt_sorts_like_oracle(nx, ny, n):
    p = inputs.particles(11, nx, ny, n)
    ch, ref, _ = _pair(nx, ny, 10, 0.1, particles=p, capacity=max(n, 1) * 2)
    _assert_state(ch, ref, rtol=0.0, what="after adopt")


@pytest.mark.parametrize("nx,ny,kn,g", [(6, 8, 0.05, 0.0), (1, 12, 0.02, 0.01), (2, 6, 0.2, 0.05), (5, 4, 0.01, 0.0)])
def test_one_step_from_identical_state(nx, ny, kn, g):
    counts = np.random.default_rng(nx * 100 + ny).integers(0, 60, nx * ny)
    counts[0] = 0
    counts[-1] = 1
    p = inputs.particles_per_cell(5, nx, ny, counts, vscale=1.0)
    ch, ref, _ = _pair(nx, ny, 30, kn, g=g, particles=p, capacity=int(counts.sum()) + 64)
    ch.step(1, sample_every=1)
    ref.step(1, sample_every=1)
    _assert_state(ch, ref, what="after 1 step")
    _assert_cells(ch, ref)
    _assert_counters(ch, ref)
    assert ch.status()["ncoll"] > 0


@pytest.mark.parametrize("nbar_mode", [0, 1])
def test_channel_c1_steps_and_moments(nbar_mode):
    # 64 cells across, 50 particles per cell, Kn 0.1, Ma 0.1 body force,
    # seed 1: 40 steps with sampling every step, then D2Q9 projection
    from paper_1512_08042_amd.config import body_force

    g = body_force(0.1, 64, 0.1)
    ch, ref, _ = _pair(1, 64, 50, 0.1, g=g, seed=1, nbar_mode=nbar_mode)
    for _ in range(4):
        ch.step(10, sample_every=1)
        ref.step(10, sample_every=1)
    _assert_state(ch, ref, what="after 40 steps")
    _assert_cells(ch, ref)
    _assert_counters(ch, ref)
    avg = ch.sample_moments().cpu().numpy()
    want = ref.averages()
    scale = np.abs(want).max(axis=1, keepdims=True) + 1.0
    assert np.all(np.abs(avg - want) <= 1e-12 * scale)
    f = ch.map_to_lbm(9, 3).cpu().numpy()
    assert np.allclose(f, O.dsmc2lb(want, 50, O.lattice(9), 3), rtol=1e-11, atol=1e-14)


def test_channel_c1_full_run():
    # the quasi-1-D channel in full, as the benchmark runs it: 2000 steps
    # sampled every step, the D2Q9 projection of the cumulative averages
    # every 10 steps (200 events); every event's populations against the
    # oracle's, then the cells and counters (exact) and the state at the end.
    # Over 2000 steps the few-ulp differences of the transcendental functions
    # enter at every collision and wall bounce, and a bounce divides by the
    # normal speed: measured after 2000 steps, positions differ by up to
    # 3.8e-10 cell and velocities by 6e-14 (thermal speed 1), while every
    # integer decision is the oracle's.  The bars are 1e-8 and 1e-11.
    from paper_1512_08042_amd.config import body_force

    g = body_force(0.1, 64, 0.1)
    ch, ref, _ = _pair(1, 64, 50, 0.1, g=g, seed=1)
    lat = O.lattice(9)
    for ev in range(200):
        ch.step(10, sample_every=1)
        ref.step(10, sample_every=1)
        f = ch.map_to_lbm(9, 2).cpu().numpy()
        want = O.dsmc2lb(ref.averages(), 50, lat, 2)
        err = float(np.abs(f - want).max() / np.abs(want).max())
        assert err <= 1e-12, "event %d: populations differ by %.3g of their largest" % (ev, err)
    assert np.array_equal(ch.cell_start().cpu().numpy(), ref.cells()[0]), "cell_start after 2000 steps"
    _assert_cells(ch, ref)
    _assert_counters(ch, ref)
    for name, g, w, tol in zip("x y vx vy vz".split(), ch.particles(), ref.particles(), (1e-8, 1e-8, 1e-11, 1e-11, 1e-11)):
        d = float(np.abs(g.cpu().numpy() - w).max())
        assert d <= tol, "%s differs by %.3g after 2000 steps" % (name, d)


def test_long_jumps_and_small_nx():
    # a time step of several cells makes many particles jump more than one
    # cell: they go through the long-jump list; nx = 1 and 2 alias the x
    # neighbours
    for nx, ny, dt in ((9, 7, 1.3), (1, 8, 2.1), (2, 5, 1.7), (3, 3, 0.9)):
        counts = np.full(nx * ny, 20)
        p = inputs.particles_per_cell(nx + ny, nx, ny, counts, vscale=1.5)
        ch, ref, _ = _pair(nx, ny, 20, 0.5, dt=dt, particles=p, capacity=int(counts.sum()) + 16)
        for it in range(3):
            ch.step(1)
            ref.step(1)
            _assert_state(ch, ref, what="nx=%d step %d" % (nx, it))
        assert ch.status()["nfar"] > 0
        _assert_counters(ch, ref)


@pytest.mark.parametrize("q,order", [(9, 2), (9, 3), (37, 3), (37, 0), (37, 1)])
def test_projection_matches_oracle(q, order):
    D, _ = _gpu()
    m = inputs.moment_sums(q + order, 1000)
    m[0, 17] = 0.0  # an empty cell
    avg = torch.as_tensor(m, device="cuda").contiguous()
    f = D.project_moments(avg, 100, q, order).cpu().numpy()
    want = O.dsmc2lb(m, 100, O.lattice(q), order)
    assert np.allclose(f, want, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("q,order,ncol", [(9, 2, 3), (37, 3, 2), (37, 2, 5)])
def test_reseed_matches_oracle(q, order, ncol):
    nx, ny, ppc = 11, 6, 40
    ch, ref, _ = _pair(nx, ny, ppc, 0.1, seed=9, capacity=nx * ny * ppc * 2)
    ch.step(3)
    ref.step(3)
    lat = O.lattice(q)
    f = inputs.populations(q, lat["w"] * 1.05, nx * ny, 0.04)
    cells = inputs.strip_cells(nx, ny, ncol)[::-1].copy()  # any order
    ch.map_from_lbm(torch.as_tensor(f, device="cuda").contiguous(), torch.as_tensor(cells, device="cuda"), q, order)
    assert ref.lb2dsmc(lat, order, f, cells) == 0
    _assert_state(ch, ref, what="after reseed")
    # and the dynamics continue identically from the reseeded state
    ch.step(2)
    ref.step(2)
    _assert_state(ch, ref, what="after reseed + 2 steps")
    _assert_counters(ch, ref)


def test_reseed_rejections_leave_state():
    nx, ny, ppc = 4, 4, 10
    ch, ref, _ = _pair(nx, ny, ppc, 0.1, seed=2, capacity=nx * ny * ppc + 5)
    lat = O.lattice(9)
    before = [t.cpu().numpy().copy() for t in ch.particles()]
    f = np.repeat(lat["w"][:, None] * 3.0, nx * ny, axis=1)
    ch.map_from_lbm(torch.as_tensor(f, device="cuda"), torch.arange(4, dtype=torch.int32, device="cuda"), 9, 2)
    assert ch.status()["bits"] & 0x4
    for a, b in zip(ch.particles(), before):
        assert np.array_equal(a.cpu().numpy(), b)
    dup = torch.tensor([1, 2, 1], dtype=torch.int32, device="cuda")
    ch.map_from_lbm(torch.as_tensor(f / 3.0, device="cuda"), dup, 9, 2)
    assert ch.status()["bits"] & 0x40
    for a, b in zip(ch.particles(), before):
        assert np.array_equal(a.cpu().numpy(), b)
    assert ch.views().reseed_events == 2


@pytest.mark.parametrize("q,order,ncol,scale", [(9, 2, 3, 1.0), (37, 3, 2, 1.0), (37, 3, 3, 5.0), (37, 2, 0, 1.0)])
def test_reseed_completed_by_the_next_step(q, order, ncol, scale):
    # nothing reads the state between the reseed and the next step, so the
    # step's first pass completes the reseed (kept cells from the old buffer,
    # new particles in place).  scale 5 makes the strip cells dense enough
    # that their tiles exceed the staged size; ncol 0 is an empty cell list.
    nx, ny, ppc = 11, 6, 40
    ch, ref, _ = _pair(nx, ny, ppc, 0.1, seed=4, capacity=nx * ny * ppc * 4)
    ch.step(2)
    ref.step(2)
    lat = O.lattice(q)
    f = inputs.populations(q + ncol, lat["w"] * scale, nx * ny, 0.04)
    cells = inputs.strip_cells(nx, ny, ncol) if ncol else np.zeros(0, np.int32)
    ch.map_from_lbm(torch.as_tensor(f, device="cuda").contiguous(), torch.as_tensor(cells, device="cuda"), q, order)
    assert ref.lb2dsmc(lat, order, f, cells) == 0
    ch.step(3, sample_every=1)
    ref.step(3, sample_every=1)
    _assert_state(ch, ref, what="3 steps after reseed")
    _assert_counters(ch, ref)
    if scale > 1.0:
        assert ch.cell_start().diff().max().item() > 4 * ppc  # the oversized tiles were exercised


@pytest.mark.parametrize("between", ["reseed", "status", "moments"])
def test_reseed_followed_by_other_calls(between):
    # what comes between a reseed and the next step: a second reseed (which
    # completes the first with the copy), a status read (the same), or a read
    # of the moment sums (which leaves it pending for the step)
    nx, ny, ppc = 9, 7, 30
    ch, ref, _ = _pair(nx, ny, ppc, 0.1, seed=12, capacity=nx * ny * ppc * 3)
    ch.step(2, sample_every=1)
    ref.step(2, sample_every=1)
    lat = O.lattice(37)
    f = inputs.populations(3, lat["w"] * 1.2, nx * ny, 0.03)
    cells = inputs.strip_cells(nx, ny, 2)
    ch.map_from_lbm(torch.as_tensor(f, device="cuda"), torch.as_tensor(cells, device="cuda"), 37, 3)
    assert ref.lb2dsmc(lat, 3, f, cells) == 0
    if between == "reseed":
        cells2 = (cells + 4).astype(np.int32)
        f2 = inputs.populations(8, lat["w"] * 0.9, nx * ny, 0.03)
        ch.map_from_lbm(torch.as_tensor(f2, device="cuda"), torch.as_tensor(cells2, device="cuda"), 37, 2)
        assert ref.lb2dsmc(lat, 2, f2, cells2) == 0
    elif between == "status":
        assert ch.status()["n"] == ref.counters()["n"]
    else:
        got = ch.sample_moments().cpu().numpy()
        want = ref.averages()
        scale = np.abs(want).max(axis=1, keepdims=True) + 1.0
        assert np.all(np.abs(got - want) <= 1e-12 * scale)
    ch.step(2, sample_every=1)
    ref.step(2, sample_every=1)
    _assert_state(ch, ref, what="2 steps after the reseed (%s between)" % between)
    _assert_counters(ch, ref)


def test_reseed_then_step_graph():
    # a graph captured right after a reseed starts from the completed state;
    # a replay whose buffer parity would not match is refused before it
    # changes anything, and an eager step then completes the second reseed
    nx, ny, ppc = 8, 6, 30
    ch, ref, _ = _pair(nx, ny, ppc, 0.1, seed=6, capacity=nx * ny * ppc * 3)
    ch.step(2, sample_every=1)
    ref.step(2, sample_every=1)
    lat = O.lattice(9)
    cells = inputs.strip_cells(nx, ny, 2)
    s = torch.cuda.Stream()
    f = torch.as_tensor(inputs.populations(11, lat["w"], nx * ny, 0.03), device="cuda")
    ch.map_from_lbm(f, torch.as_tensor(cells, device="cuda"), 9, 2, stream=s)
    assert ref.lb2dsmc(lat, 2, f.cpu().numpy(), cells) == 0
    ch.graph_create(4, sample_every=1, stream=s)
    for _ in range(2):
        ch.graph_launch(stream=s)
        ref.step(4, sample_every=1)
    s.synchronize()
    _assert_state(ch, ref, what="two replays after a reseed")
    _assert_counters(ch, ref)
    f2 = torch.as_tensor(inputs.populations(12, lat["w"] * 1.1, nx * ny, 0.03), device="cuda")
    ch.map_from_lbm(f2, torch.as_tensor(cells, device="cuda"), 9, 2, stream=s)
    assert ref.lb2dsmc(lat, 2, f2.cpu().numpy(), cells) == 0
    with pytest.raises(RuntimeError):
        ch.graph_launch(stream=s)  # the completed reseed would leave the other buffer current
    ch.step(2, sample_every=1, stream=s)
    ref.step(2, sample_every=1)
    s.synchronize()
    _assert_state(ch, ref, what="an eager step after the refused replay")
    _assert_counters(ch, ref)


def test_rejected_reseed_then_step():
    # a reseed over capacity is rejected on the device: the step that
    # completes it keeps every particle and the cell starts as they were
    nx, ny, ppc = 4, 4, 10
    ch, ref, _ = _pair(nx, ny, ppc, 0.1, seed=2, capacity=nx * ny * ppc + 5)
    lat = O.lattice(9)
    f = np.repeat(lat["w"][:, None] * 3.0, nx * ny, axis=1)
    cells = np.arange(4, dtype=np.int32)
    ch.map_from_lbm(torch.as_tensor(f, device="cuda"), torch.as_tensor(cells, device="cuda"), 9, 2)
    ref.lb2dsmc(lat, 2, f, cells)
    ch.step(2)
    ref.step(2)
    _assert_state(ch, ref, what="2 steps after a rejected reseed")
    _assert_counters(ch, ref)
    assert ch.status()["bits"] & 0x4
    # the next reseed runs normally
    f2 = np.repeat(lat["w"][:, None], nx * ny, axis=1)
    ch.map_from_lbm(torch.as_tensor(f2, device="cuda"), torch.as_tensor(cells, device="cuda"), 9, 2)
    assert ref.lb2dsmc(lat, 2, f2, cells) == 0
    ch.step(1)
    ref.step(1)
    _assert_state(ch, ref, what="a step after the next reseed")


@pytest.mark.parametrize("q,y_mode,g,nsteps", [(9, 0, 0.0, 3), (37, 0, 1e-3, 2), (37, 1, 2e-3, 3), (9, 1, 0.0, 1)])
def test_lbm_step_matches_oracle(q, y_mode, g, nsteps):
    D, _ = _gpu()
    nx, ny = 13, 11
    lat = O.lattice(q)
    f = inputs.populations(q * 7 + y_mode, lat["w"], nx * ny, 0.1)
    got = D.lbm_step(torch.as_tensor(f, device="cuda").contiguous(), nx, ny, q, 0.83, g, y_mode, nsteps)
    want = O.lbm_step(f, lat, nx, ny, 0.83, g, y_mode, nsteps)
    assert np.allclose(got.cpu().numpy(), want, rtol=1e-12, atol=1e-15)


def test_determinism():
    D, ChannelConfig = _gpu()
    cfg = ChannelConfig(nx=8, ny=16, ppc=30, kn=0.05, mach=0.1, seed=5)
    runs = []
    for _ in range(2):
        ch = D.Channel(cfg)
        ch.step(6, sample_every=2)
        runs.append([t.cpu().numpy().copy() for t in ch.particles()] + [ch.sample_moments().cpu().numpy()])
        ch.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_full_size_channel_c2():
    # the benchmark workload at full size: 512 x 256 cells, 100 particles per
    # cell (13,107,200 particles), Kn 0.05, Ma 0.1 body force: two steps with
    # sampling, the DSMC->D2Q37 map of all cells, and the reseed of the
    # 16-cell strip, all compared with the oracle element by element
    from paper_1512_08042_amd.config import body_force

    nx, ny, ppc, kn = 512, 256, 100, 0.05
    g = body_force(kn, ny, 0.1)
    ch, ref, cfg = _pair(nx, ny, ppc, kn, g=g, seed=2)
    ch.step(2, sample_every=1)
    ref.step(2, sample_every=1)
    _assert_state(ch, ref, what="C2 after 2 steps")
    _assert_counters(ch, ref)
    f = ch.map_to_lbm(37, 3)
    want = O.dsmc2lb(ref.averages(), ppc, O.lattice(37), 3)
    assert np.allclose(f.cpu().numpy(), want, rtol=1e-11, atol=1e-14)
    # both sides reseed from the same populations, so that the integer
    # decisions (N_new = floor(rho ppc + R), the accept test C R <= G) see
    # identical inputs
    cells = inputs.strip_cells(nx, ny, 16)
    ch.map_from_lbm(torch.as_tensor(want, device="cuda").contiguous(), torch.as_tensor(cells, device="cuda"), 37, 3)
    assert ref.lb2dsmc(O.lattice(37), 3, want, cells) == 0
    _assert_state(ch, ref, what="C2 after reseed")
