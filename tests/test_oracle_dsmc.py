"""Pins of the oracle's DSMC particle step (CPU only).

Each test checks the oracle against something other than itself: a closed
form, a textbook kinetic-theory result, a conservation law, or brute force
with a library routine.
"""
import math

import numpy as np
import pytest
from scipy import stats

import inputs
from oracle import oracle as O

NO_COLL_KN = 1e9  # mean free path so long that no collision candidate is ever drawn


def _cells_of(x, y, nx, ny):
    ix = np.clip(np.floor(x).astype(np.int64), 0, nx - 1)
    iy = np.clip(np.floor(y).astype(np.int64), 0, ny - 1)
    return iy * nx + ix


def test_init_exact_count_and_maxwellian():
    nx, ny, ppc = 8, 16, 100
    s = O.Sim(nx, ny, ppc, 0.1, seed=11)
    s.init_maxwell()
    x, y, vx, vy, vz = s.particles()
    cs, nbar, sig, rem = s.cells()
    # Section 3.1: a fixed number of molecules is placed in every cell
    assert np.array_equal(cs, np.arange(nx * ny + 1) * ppc)
    c = _cells_of(x, y, nx, ny)
    assert np.array_equal(c, np.repeat(np.arange(nx * ny), ppc))
    n = x.size
    for v in (vx, vy, vz):
        assert abs(v.mean()) < 4.0 / math.sqrt(n)
        assert abs(v.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert stats.kstest(vx, "norm").pvalue > 1e-4
    assert np.all(sig == 6.0) and np.all(nbar == 0.0) and np.all(rem == 0.0)


def test_stable_sort_against_numpy():
    nx, ny = 7, 5
    for seed in range(3):
        p = inputs.particles(seed, nx, ny, 1000)
        s = O.Sim(nx, ny, 10, 0.1, capacity=2000)
        s.load(*p)
        got = s.particles()
        cell = _cells_of(p[0], p[1], nx, ny)
        order = np.argsort(cell, kind="stable")
        for a, b in zip(got, p):
            assert np.array_equal(a, b[order])
        cs = s.cells()[0]
        assert np.array_equal(cs, np.searchsorted(cell[order], np.arange(nx * ny + 1)))


def test_free_flight_matches_parabola():
    # tall channel, particles far from both walls, no collisions: after n
    # steps the state is the exact constant-acceleration trajectory
    nx, ny, n, g, nsteps = 8, 1000, 2000, 0.01, 20
    rng = np.random.default_rng(5)
    x0 = rng.uniform(0, nx, n)
    y0 = rng.uniform(400, 600, n)
    vx0 = rng.normal(0, 1, n)
    vy0 = np.clip(rng.normal(0, 1, n), -3, 3)
    vz0 = np.arange(n) + 0.5  # unique tag, untouched without collisions and walls
    s = O.Sim(nx, ny, 2, NO_COLL_KN, dt=0.177, g=g, capacity=n)
    s.load(x0, y0, vx0, vy0, vz0)
    s.step(nsteps)
    x, y, vx, vy, vz = s.particles()
    idx = np.round(vz - 0.5).astype(np.int64)
    T = nsteps * 0.177
    xe = np.mod(x0[idx] + vx0[idx] * T + 0.5 * g * T * T, nx)
    dx = np.abs(x - xe)
    dx = np.minimum(dx, nx - dx)
    assert dx.max() < 1e-11
    assert np.allclose(vx, vx0[idx] + g * T, atol=1e-13)
    assert np.allclose(y, y0[idx] + vy0[idx] * T, atol=1e-11)
    assert np.array_equal(vy, vy0[idx])
    assert s.counters()["ncoll"] == 0 and s.counters()["nwall"] == 0


@pytest.mark.parametrize("g", [0.0, 0.05])
def test_diffuse_wall_reflection_law(g):
    # every particle starts at y0 heading into the wall y = 0 with the same
    # speed, so all hit at t* = y0 / |vy| and fly the rest of the step with
    # the re-emitted velocity: v_n = y / (dt - t*) must follow the flux-
    # weighted (Rayleigh) law, the tangential components the Gaussian.
    n, dt, y0 = 40000, 0.177, 0.05
    rng = np.random.default_rng(9)
    s = O.Sim(1, 100, 2, NO_COLL_KN, dt=dt, g=g, capacity=n)
    s.load(rng.uniform(0, 1, n), np.full(n, y0), rng.normal(0, 1, n), np.full(n, -1.0), rng.normal(0, 1, n))
    s.step(1)
    x, y, vx, vy, vz = s.particles()
    trem = dt - y0 / 1.0
    vn = y / trem
    assert np.allclose(vy, vn, rtol=1e-12)
    assert s.counters()["nwall"] == n
    assert stats.kstest(vn, "rayleigh").pvalue > 1e-4
    assert abs(vn.mean() - math.sqrt(math.pi / 2)) < 4 * math.sqrt((2 - math.pi / 2) / n)
    assert stats.kstest(vx - g * trem, "norm").pvalue > 1e-4
    assert stats.kstest(vz, "norm").pvalue > 1e-4


def test_diffuse_wall_hit_rate():
    # equilibrium gas between two walls at the gas temperature: the number
    # of wall hits per unit wall length and time is n sqrt(kT/(2 pi m)).
    nx, ny, ppc, nsteps, dt = 16, 8, 100, 100, 0.177
    s = O.Sim(nx, ny, ppc, NO_COLL_KN, dt=dt, seed=3)
    s.init_maxwell()
    s.step(nsteps)
    hits = s.counters()["nwall"]
    expect = 2 * nx * ppc * dt * nsteps / math.sqrt(2 * math.pi)
    assert abs(hits - expect) < 5 * math.sqrt(expect)


def test_collisions_conserve_momentum_and_energy():
    # one cell, no wall contact during the step (vy = 0), many collisions
    n = 1000
    rng = np.random.default_rng(2)
    s = O.Sim(1, 1, n, 0.001, dt=1e-4, capacity=n)
    vx, vz = rng.normal(0, 1, n), rng.normal(0, 1, n)
    s.load(rng.uniform(0, 1, n), rng.uniform(0.2, 0.8, n), vx, np.zeros(n), vz)
    p0 = np.array([vx.sum(), 0.0, vz.sum()])
    e0 = (vx ** 2 + vz ** 2).sum()
    s.step(1)
    _, _, ux, uy, uz = s.particles()
    assert s.counters()["ncoll"] > 50
    assert np.allclose([ux.sum(), uy.sum(), uz.sum()], p0, atol=1e-11)
    assert (ux ** 2 + uy ** 2 + uz ** 2).sum() == pytest.approx(e0, rel=1e-13)


@pytest.mark.parametrize("nbar_mode", [0, 1])
def test_ntc_collision_rate(nbar_mode):
    # Eq. (collisionnumber) with hard spheres: in equilibrium the expected
    # number of accepted collisions per cell and step is
    # 1/2 N Nbar F_N sigma_T <c_r> dt / V_c with <c_r> = 4 sqrt(kT/(pi m)),
    # and F_N sigma_T / V_c follows from Eq. (MFP) with lambda = Kn H.
    nx, ny, ppc, kn = 16, 16, 50, 0.05
    s = O.Sim(nx, ny, ppc, kn, seed=4, nbar_mode=nbar_mode)
    s.init_maxwell()
    lam = kn * ny
    # Eq. (MFP) with number density n = ppc per unit cell (F_N / V_c = 1):
    # sigma_T = pi d^2 = 1 / (sqrt(2) lambda n), and F_N sigma_T / V_c = sigma_T
    n_dens = float(ppc)
    d2 = 1.0 / (math.sqrt(2.0) * math.pi * lam * n_dens)
    K = math.pi * d2
    cr_mean = 4.0 / math.sqrt(math.pi)
    expect = 0.0
    for _ in range(120):
        s.step(1)
        cs, nbar, _, _ = s.cells()
        N = np.diff(cs).astype(np.float64)
        pair = nbar if nbar_mode == 0 else N - 1.0
        expect += float(np.sum(0.5 * N * pair * K * cr_mean * s.dt))
    got = s.counters()["ncoll"]
    assert abs(got - expect) < 5 * math.sqrt(expect), (got, expect)


def _hermite_sums(avg):
    """Per-cell sample means of the orthogonal Hermite components from the averages."""
    N = avg[0]
    m = avg[1:] / N
    return {"x": (m[0], 1.0), "y": (m[1], 1.0), "xx": (m[2] - 1, 2.0), "xy": (m[3], 1.0), "yy": (m[4] - 1, 2.0),
            "xxx": (m[5] - 3 * m[0], 6.0), "xxy": (m[6] - m[1], 2.0), "xyy": (m[7] - m[0], 2.0),
            "yyy": (m[8] - 3 * m[1], 6.0), "zz": (m[9] - 1, 2.0)}


@pytest.mark.parametrize("nsteps,state32", [(0, False), (60, False), (60, True)])
def test_equilibrium_moments_within_standard_errors(nsteps, state32):
    nx, ny, ppc = 16, 16, 100
    s = O.Sim(nx, ny, ppc, 0.1, seed=21, state32=state32)
    s.init_maxwell()
    s.step(nsteps)
    s.reset_moments()
    s.sample_now()
    avg = s.averages()
    N = avg[0]
    assert N.sum() == nx * ny * ppc
    # Var[H_alpha] = alpha! under the unit Maxwellian: per-cell z-scores have
    # unit RMS, and the pooled mean over all cells is within 4.5 SE of 0.
    # (Third-order components are heavy-tailed at 100 particles, so no
    # per-cell maximum is asserted.)
    for name, (mean, var) in _hermite_sums(avg).items():
        z = mean * np.sqrt(N / var)
        assert 0.8 < np.sqrt(np.mean(z ** 2)) < 1.25, name
        pooled = np.sum(mean * N) / math.sqrt(var * N.sum())
        assert abs(pooled) < 4.5, name


def test_sampling_accumulates_cumulative_averages():
    s = O.Sim(2, 3, 20, 0.1, seed=2)
    s.init_maxwell()
    s.step(4, sample_every=2)
    assert s.counters()["nsamples"] == 2
    snap = []
    t = O.Sim(2, 3, 20, 0.1, seed=2)
    t.init_maxwell()
    for _ in range(2):
        t.step(2)
        t.reset_moments()
        t.sample_now()
        snap.append(t.averages())
    assert np.allclose(s.averages(), 0.5 * (snap[0] + snap[1]), rtol=1e-13, atol=1e-12)


def test_low_kn_poiseuille_profile():
    # Force-driven Poiseuille flow at Kn = 0.05 (Section 3.1 set-up, 2-D
    # channel): away from the Knudsen layers the velocity profile is the
    # Navier-Stokes parabola with curvature -g / nu, nu the Chapman-Enskog
    # hard-sphere viscosity (5/16) sqrt(2 pi) 1.016 lambda sqrt(kT/m).
    # Ma 0.2 and two periodic columns keep the statistical error near 2 %;
    # viscous heating at this Mach number changes nu by about 0.2 %.
    nx, ny, ppc, kn, mach = 2, 64, 100, 0.05, 0.2
    g = O.body_force_for_mach(kn, ny, mach)
    s = O.Sim(nx, ny, ppc, kn, g=g, seed=7)
    s.init_maxwell()
    s.step(5000)
    s.reset_moments()
    nb, per = 6, 4000
    curv = []
    yc = np.arange(ny) + 0.5
    lam = kn * ny
    bulk = (yc > 2 * lam) & (yc < ny - 2 * lam)
    for _ in range(nb):
        s.step(per, sample_every=1)
        avg = s.averages()
        s.reset_moments()
        u = (avg[1].reshape(ny, nx).sum(1)) / (avg[0].reshape(ny, nx).sum(1))
        c2 = np.polyfit(yc[bulk] - ny / 2, u[bulk], 2)[0]
        curv.append(2 * c2)
    curv = np.array(curv)
    nu = O.hs_viscosity(kn, ny)
    expect = -g / nu
    se = curv.std(ddof=1) / math.sqrt(nb)
    assert abs(curv.mean() - expect) < max(0.03 * abs(expect), 4 * se), (curv.mean(), expect, se)


def test_fp32_state_rounds_every_stored_value():
    # FP32 state: every stored value is a float, and one step of the FP32
    # form differs from the FP64 form only by the rounding of the stored
    # values (a few FP32 ulps; no collision outcome or wall decision changes
    # on this small box)
    kw = dict(g=0.01, seed=7, capacity=4096)
    a = O.Sim(4, 6, 40, 0.2, state32=True, **kw)
    b = O.Sim(4, 6, 40, 0.2, **kw)
    for s in (a, b):
        s.init_maxwell()
    pa, pb = a.particles(), b.particles()
    for u, v in zip(pa, pb):
        assert np.array_equal(np.asarray(u, dtype=np.float32).astype(np.float64), u)
        assert np.all(np.abs(u - v) <= 2.0 ** -24 * np.abs(v) + 1e-300)  # init: one rounding each
    a.step(1)
    b.step(1)
    assert a.counters()["ncoll"] == b.counters()["ncoll"] and a.counters()["nwall"] == b.counters()["nwall"]
    assert np.array_equal(a.cells()[0], b.cells()[0])
    for u, v in zip(a.particles(), b.particles()):
        assert np.array_equal(np.asarray(u, dtype=np.float32).astype(np.float64), u)
        assert np.all(np.abs(u - v) <= 1e-6 * (np.abs(v) + 1.0))
