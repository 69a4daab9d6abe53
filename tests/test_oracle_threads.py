"""The OpenMP build of the oracle (the CPU baseline of the benchmark) against
the single-threaded build: the same bits for every operation it splits over
threads -- free flight with walls, the stable counting sort, NTC
collisions, sampling, the DSMC2LB projection, the LB2DSMC reconstruction
and the BGK lattice Boltzmann step."""
import numpy as np
import pytest

import inputs
from oracle import oracle as O


def _sim(threads, nx=3, ny=40, ppc=50, kn=0.05, mach=0.1, seed=21, state32=False, dt=None):
    g = O.body_force_for_mach(kn, ny, mach)
    s = O.Sim(nx, ny, ppc, kn, dt=dt, g=g, seed=seed, state32=state32, threads=threads,
              capacity=nx * ny * ppc * 2 + 64)
    s.init_maxwell()
    return s


def _same_state(a, b):
    for u, v in zip(a.particles(), b.particles()):
        assert np.array_equal(u, v)
    for u, v in zip(a.cells(), b.cells()):
        assert np.array_equal(u, v)
    assert a.counters() == b.counters()
    assert np.array_equal(a.averages(), b.averages())


@pytest.mark.parametrize("threads", [0, 3, 8])
@pytest.mark.parametrize("state32", [False, True])
def test_steps_are_bit_identical(threads, state32):
    one, many = _sim(None, state32=state32), _sim(threads, state32=state32)
    assert O.threads_in_use(threads) == (threads or O.threads_in_use(0)) and O.threads_in_use(None) == 1
    for _ in range(3):
        one.step(5, sample_every=1)
        many.step(5, sample_every=1)
        _same_state(one, many)
    c = one.counters()
    assert c["ncoll"] > 0 and c["nwall"] > 0


def test_more_threads_than_particles_and_bounce_limit():
    # empty slot ranges for most threads; a large time step drives particles
    # into the bounce limit, whose status bit must reach the shared flags
    one = _sim(None, nx=1, ny=2, ppc=3, kn=0.5, dt=40.0)
    many = _sim(8, nx=1, ny=2, ppc=3, kn=0.5, dt=40.0)
    one.step(3, sample_every=1)
    many.step(3, sample_every=1)
    _same_state(one, many)
    assert one.counters()["status"] & O.ST_WALL_LIMIT


@pytest.mark.parametrize("q,order", [(9, 2), (37, 3)])
def test_mappings_are_bit_identical(q, order):
    lat = O.lattice(q)
    one, many = _sim(None), _sim(8)
    one.step(6, sample_every=1)
    many.step(6, sample_every=1)
    avg = one.averages()
    f1 = O.dsmc2lb(avg, one.ppc, lat, order)
    f8 = O.dsmc2lb(avg, one.ppc, lat, order, threads=8)
    assert np.array_equal(f1, f8)
    assert np.array_equal(O.dsmc2lb_eq(avg, one.ppc, lat, 2), O.dsmc2lb_eq(avg, one.ppc, lat, 2, threads=8))
    cells = inputs.strip_cells(one.nx, one.ny, 2)
    assert one.lb2dsmc(lat, order, f1, cells) == many.lb2dsmc(lat, order, f8, cells) == 0
    _same_state(one, many)
    one.step(2, sample_every=1)
    many.step(2, sample_every=1)
    _same_state(one, many)


@pytest.mark.parametrize("q,y_mode,x_buffer", [(9, 0, 0), (9, 2, 2), (37, 1, 0), (37, 0, 3)])
def test_lbm_step_is_bit_identical(q, y_mode, x_buffer):
    lat = O.lattice(q)
    nx, ny = 13, 24
    f = inputs.populations(q + 10 * y_mode + x_buffer, lat["w"], nx * ny, 0.05)
    tau = O.lbm_tau(0.1, ny, lat["r"])
    a = O.lbm_step(f, lat, nx, ny, tau, 1e-4, y_mode, 5, x_buffer=x_buffer)
    b = O.lbm_step(f, lat, nx, ny, tau, 1e-4, y_mode, 5, x_buffer=x_buffer, threads=8)
    assert np.array_equal(a, b)
