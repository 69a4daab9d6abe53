"""Pins of the oracle pieces the hybrid loop of Section 4 adds (CPU only):
diffuse walls and held inflow columns in the BGK step, and the equilibrium
mapping of Eq. (feq_dsmc)."""
import numpy as np
import pytest

import inputs
from oracle import oracle as O


def _eq(lat, rho, ux, uy, order=2):
    cu = lat["xi"][:, :1] * ux + lat["xi"][:, 1:] * uy
    uu = ux * ux + uy * uy
    eq = 1 + cu + 0.5 * (cu * cu - uu)
    if order >= 3:
        eq = eq + cu * (cu * cu - 3 * uu) / 6
    return lat["w"][:, None] * rho * eq


def _maxwell_avg(rho, ux, uy, ppc):
    m0 = rho * ppc
    return np.array([m0, m0 * ux, m0 * uy, m0 * (ux * ux + 1), m0 * ux * uy, m0 * (uy * uy + 1),
                     m0 * (ux ** 3 + 3 * ux), m0 * (ux * ux * uy + uy), m0 * (ux * uy * uy + ux),
                     m0 * (uy ** 3 + 3 * uy), m0 * np.ones_like(ux)])


def test_diffuse_walls_conserve_mass():
    lat = O.lattice(9)
    nx, ny = 6, 9
    f = inputs.populations(1, lat["w"], nx * ny, 0.3)
    out = O.lbm_step(f, lat, nx, ny, 0.8, 2e-3, 2, 25)
    assert out.sum() == pytest.approx(f.sum(), rel=1e-13)


def test_gas_at_rest_between_walls_stays_at_rest():
    lat = O.lattice(9)
    nx, ny = 5, 7
    f = _eq(lat, np.full(nx * ny, 1.2), np.zeros(nx * ny), np.zeros(nx * ny))
    out = O.lbm_step(f, lat, nx, ny, 0.9, 0.0, 2, 10)
    assert np.allclose(out, f, rtol=1e-14, atol=1e-16)


def test_walls_are_at_rest_and_give_back_what_they_take():
    # after one step the populations leaving the wall rows carry no momentum
    # along the wall and their mass equals what the node sent into the wall
    lat = O.lattice(9)
    nx, ny = 4, 6
    f = inputs.populations(2, lat["w"], nx * ny, 0.4)
    out = O.lbm_step(f, lat, nx, ny, 1.0, 0.0, 2, 1)  # tau = 1: post-collision = equilibrium
    e = lat["e"]
    up = e[:, 1] > 0
    rows = np.repeat(np.arange(ny), nx)
    for node in np.where(rows == 0)[0]:
        emitted = out[up, node]
        assert (emitted * lat["xi"][up, 0]).sum() == pytest.approx(0.0, abs=1e-15)
        rho = f[:, node].sum()
        ux = (f[:, node] * lat["xi"][:, 0]).sum() / rho
        uy = (f[:, node] * lat["xi"][:, 1]).sum() / rho
        sent = _eq(lat, np.array([rho]), np.array([ux]), np.array([uy]))[e[:, 1] < 0, 0].sum()
        assert emitted.sum() == pytest.approx(sent, rel=1e-13)


def test_force_driven_flow_between_walls_is_a_parabola():
    # steady BGK Poiseuille flow: u(y) = a/(2 nu) y (H - y) + slip, with the
    # lattice viscosity nu = (tau - 1/2)/r^2 and acceleration a = g/r per step
    # (lattice units); the diffuse walls only shift the profile (slip)
    lat = O.lattice(9)
    r = lat["r"]
    nx, ny, tau, g = 1, 24, 0.9, 1e-5
    f = _eq(lat, np.ones(nx * ny), np.zeros(nx * ny), np.zeros(nx * ny))
    out = O.lbm_step(f, lat, nx, ny, tau, g, 2, 6000)
    rho = out.sum(0)
    ux = ((out * lat["xi"][:, :1]).sum(0) + 0.5 * rho * g) / rho / r  # lattice units, half-step shift
    y = np.arange(ny) + 0.5
    C = np.polyfit(y, ux, 2)[0]
    nu = (tau - 0.5) / r ** 2
    assert C == pytest.approx(-(g / r) / (2 * nu), rel=0.01)
    assert np.allclose(ux, ux[::-1], rtol=1e-9)
    assert ux.min() > 0  # slip at the walls


def test_held_inflow_column_drives_the_lattice_it_matches():
    # a held column at the state of the whole lattice keeps everything
    # stationary; the held column itself never changes
    lat = O.lattice(9)
    nx, ny = 8, 5
    f = _eq(lat, np.full(nx * ny, 0.9), np.full(nx * ny, 0.05), np.full(nx * ny, -0.02))
    out = O.lbm_step(f, lat, nx, ny, 0.7, 0.0, 0, 5, x_buffer=1)
    assert np.allclose(out, f, rtol=1e-13)
    g = inputs.populations(3, lat["w"], nx * ny, 0.2)
    out = O.lbm_step(g, lat, nx, ny, 0.7, 1e-3, 2, 3, x_buffer=1)
    cols = np.tile(np.arange(nx), ny)
    assert np.array_equal(out[:, cols == 0], g[:, cols == 0])
    # the column next to it receives the held column's right-moving populations
    e = lat["e"]
    a = int(np.where((e[:, 0] == 1) & (e[:, 1] == 0))[0][0])
    one = O.lbm_step(g, lat, nx, ny, 0.7, 1e-3, 2, 1, x_buffer=1)
    assert np.array_equal(one[a, cols == 1], g[a, cols == 0])


@pytest.mark.parametrize("Q,order", [(9, 2), (37, 2), (37, 3)])
def test_equilibrium_mapping_keeps_only_rho_and_u(Q, order):
    lat = O.lattice(Q)
    avg = inputs.moment_sums(4, 30, scale=5.0)
    f = O.dsmc2lb_eq(avg, 100, lat, order)
    rho = avg[0] / 100
    ux, uy = avg[1] / avg[0], avg[2] / avg[0]
    assert np.allclose(f.sum(0), rho, rtol=1e-13)
    assert np.allclose((f * lat["xi"][:, :1]).sum(0), rho * ux, rtol=1e-12, atol=1e-14)
    assert np.allclose((f * lat["xi"][:, 1:]).sum(0), rho * uy, rtol=1e-12, atol=1e-14)
    # the second-order coefficient is the equilibrium one, rho u u, whatever
    # the sampled pressure tensor was
    hxx = lat["xi"][:, 0] ** 2 - 1
    assert np.allclose((f * hxx[:, None]).sum(0), rho * ux * ux, rtol=1e-11, atol=1e-13)


def test_equilibrium_mapping_equals_the_full_one_for_a_maxwellian():
    lat = O.lattice(9)
    rng = np.random.default_rng(5)
    rho, ux, uy = rng.uniform(0.8, 1.2, 20), rng.uniform(-0.2, 0.2, 20), rng.uniform(-0.2, 0.2, 20)
    avg = _maxwell_avg(rho, ux, uy, 100)
    assert np.allclose(O.dsmc2lb_eq(avg, 100, lat, 2), O.dsmc2lb(avg, 100, lat, 2), rtol=1e-13, atol=1e-16)


def test_equilibrium_mapping_of_an_empty_cell_is_zero():
    lat = O.lattice(9)
    avg = inputs.moment_sums(6, 4)
    avg[:, 2] = 0.0
    f = O.dsmc2lb_eq(avg, 50, lat, 2)
    assert np.all(f[:, 2] == 0.0) and np.all(f[:, [0, 1, 3]] > 0.0)
