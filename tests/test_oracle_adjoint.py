"""Pins of the differentiated lattice oracle (CPU only).

The oracle's gradients come from automatic differentiation of a PyTorch
restatement of the BGK step, the Hermite coefficients and the DSMC2LB
projection.  They are pinned here to things other than themselves:
  * the forward restatement equals the C oracle's BGK step and projection;
  * closed forms on uniform states: the force adds rho g of momentum per step
    whatever tau is, and with g = 0 the non-equilibrium part of a uniform
    state decays by (1 - 1/tau) per step;
  * central differences of the C oracle's forward (an independent code) for
    d/dg, d/dtau, directional derivatives in f0 and in the DSMC moments, and
    the adjoint identity <lam_n, v> = <lam_{n+1}, (d f_{n+1}/d f_n) v> of one
    step;
  * the Hermite coefficients of an equilibrium are rho, rho u, rho u u,
    rho u u u.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle import lbm_adjoint as A
from oracle import oracle as O


def _hermite_np(lat, order):
    x, y = lat["xi"][:, 0], lat["xi"][:, 1]
    rows = [np.ones_like(x)]
    if order >= 1:
        rows += [x, y]
    if order >= 2:
        rows += [x * x - 1, x * y, y * y - 1]
    if order >= 3:
        rows += [x ** 3 - 3 * x, x * x * y - y, x * y * y - x, y ** 3 - 3 * y]
    return np.array(rows)


def _equilibrium(lat, rho, ux, uy):
    cu = lat["xi"][:, :1] * ux + lat["xi"][:, 1:] * uy
    uu = ux * ux + uy * uy
    eq = 1 + cu + 0.5 * (cu * cu - uu)
    if lat["Q"] != 9:
        eq = eq + cu * (cu * cu - 3 * uu) / 6
    return lat["w"][:, None] * rho * eq


def _J_c_oracle(f0, lat, nx, ny, tau, g, y_mode, nsteps, nodes, order, target):
    fN = O.lbm_step(f0, lat, nx, ny, tau, g, y_mode, nsteps)
    a = _hermite_np(lat, order) @ fN[:, nodes]
    return 0.5 * ((a - target) ** 2).sum()


def _grads_torch(f0, lat, nx, ny, tau, g, y_mode, nsteps, nodes, order, target):
    f = torch.tensor(f0, requires_grad=True)
    t = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    gg = torch.tensor(g, dtype=torch.float64, requires_grad=True)
    fN = A.rollout(f, lat, nx, ny, t, gg, y_mode, nsteps)
    a = A.hermite_coefficients(fN, lat, order, nodes)
    J = 0.5 * ((a - torch.as_tensor(target)) ** 2).sum()
    df, dg, dt = torch.autograd.grad(J, (f, gg, t))
    return float(J.detach()), df.numpy(), float(dg), float(dt)


@pytest.mark.parametrize("Q,y_mode,g", [(9, 0, 0.0), (9, 1, 3e-3), (37, 0, 2e-3), (37, 1, 1e-3)])
def test_torch_step_equals_c_oracle(Q, y_mode, g):
    lat = O.lattice(Q)
    nx, ny = 7, 11
    f = inputs.populations(30 + Q, lat["w"], nx * ny, 0.1)
    want = O.lbm_step(f, lat, nx, ny, 0.75, g, y_mode, 4)
    got = A.rollout(torch.tensor(f), lat, nx, ny, 0.75, g, y_mode, 4).numpy()
    assert np.allclose(got, want, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("Q", [9, 37])
def test_uniform_state_momentum_gradient_closed_form(Q):
    # any uniform state on a periodic grid gains rho g of x momentum per node
    # and step: j_x(N) = j_x(0) + N rho g.  For J = 1/2 sum_i (j_x(N) - t_i)^2,
    # dJ/dg = sum_i (j_x(N) - t_i) N rho and dJ/dtau = 0.
    lat = O.lattice(Q)
    nx, ny, N, tau, g = 4, 5, 7, 0.85, 2e-3
    col = inputs.populations(1, lat["w"], 1, 0.2)[:, 0]
    f0 = np.repeat(col[:, None], nx * ny, axis=1)
    nodes = np.array([0, 3, 7, 19])
    target = np.random.default_rng(2).normal(0, 0.1, (3, nodes.size))
    J, _, dg, dt = _grads_torch(f0, lat, nx, ny, tau, g, 0, N, nodes, 1, target)
    rho = col.sum()
    jx_N = (col * lat["xi"][:, 0]).sum() + N * rho * g
    assert dg == pytest.approx(((jx_N - target[1]) * N * rho).sum(), rel=1e-11)
    assert abs(dt) < 1e-12 * (1 + abs(dg))


@pytest.mark.parametrize("Q", [9, 37])
def test_uniform_nonequilibrium_tau_gradient_closed_form(Q):
    # with g = 0, rho and u are conserved, f_eq stays put and a uniform
    # non-equilibrium part decays by (1 - 1/tau) per step, so
    # a_xx(N) = rho ux^2 + (1 - 1/tau)^N d with d = a_xx(0) - rho ux^2.
    lat = O.lattice(Q)
    nx, ny, N, tau, eps = 3, 4, 9, 0.7, 0.05
    rho, ux, uy = 1.1, 0.04, -0.03
    hxx = lat["xi"][:, 0] ** 2 - 1
    col = _equilibrium(lat, np.array([rho]), np.array([ux]), np.array([uy]))[:, 0] + 0.5 * eps * lat["w"] * hxx
    f0 = np.repeat(col[:, None], nx * ny, axis=1)
    nodes = np.array([1, 5, 10])
    target = np.random.default_rng(3).normal(0, 0.1, (6, nodes.size))
    _, _, _, dt = _grads_torch(f0, lat, nx, ny, tau, 0.0, 0, N, nodes, 2, target)
    d = 0.5 * eps * (lat["w"] * hxx * hxx).sum()
    axx_N = rho * ux * ux + (1 - 1 / tau) ** N * d
    want = ((axx_N - target[3]) * N * (1 - 1 / tau) ** (N - 1) / tau ** 2 * d).sum()
    assert dt == pytest.approx(want, rel=1e-9)


@pytest.mark.parametrize("Q,y_mode,nsteps", [(37, 1, 6), (9, 0, 5), (37, 0, 1), (9, 1, 3)])
def test_gradients_match_central_differences_of_c_oracle(Q, y_mode, nsteps):
    lat = O.lattice(Q)
    nx, ny, tau, g = 5, 10, 0.8, 2e-3
    f0 = inputs.populations(40 + Q + y_mode, lat["w"], nx * ny, 0.05)
    nodes = np.array([0, 11, 17, 24, 36, 49])
    target = np.random.default_rng(4).normal(0, 0.05, (10, nodes.size)) + _hermite_np(lat, 3) @ f0[:, nodes]
    args = (lat, nx, ny)
    J, df, dg, dt = _grads_torch(f0, *args, tau, g, y_mode, nsteps, nodes, 3, target)
    assert J == pytest.approx(_J_c_oracle(f0, *args, tau, g, y_mode, nsteps, nodes, 3, target), rel=1e-12)
    h = 1e-5
    fd_g = (_J_c_oracle(f0, *args, tau, g + h, y_mode, nsteps, nodes, 3, target)
            - _J_c_oracle(f0, *args, tau, g - h, y_mode, nsteps, nodes, 3, target)) / (2 * h)
    fd_t = (_J_c_oracle(f0, *args, tau + h, g, y_mode, nsteps, nodes, 3, target)
            - _J_c_oracle(f0, *args, tau - h, g, y_mode, nsteps, nodes, 3, target)) / (2 * h)
    v = np.random.default_rng(5).normal(0, 1, f0.shape) * lat["w"][:, None]
    fd_f = (_J_c_oracle(f0 + h * v, *args, tau, g, y_mode, nsteps, nodes, 3, target)
            - _J_c_oracle(f0 - h * v, *args, tau, g, y_mode, nsteps, nodes, 3, target)) / (2 * h)
    assert dg == pytest.approx(fd_g, rel=1e-6, abs=1e-9)
    assert dt == pytest.approx(fd_t, rel=1e-6, abs=1e-9)
    assert (df * v).sum() == pytest.approx(fd_f, rel=1e-6, abs=1e-9)
    if nsteps > 1:
        assert abs(dt) > 1e-6 and abs(dg) > 1e-6  # the pins are not vacuous


@pytest.mark.parametrize("Q,y_mode", [(37, 1), (9, 0)])
def test_step_vjp_adjoint_identity(Q, y_mode):
    # <lam_n, v> = <lam_{n+1}, D v> with D v from central differences of the
    # C oracle's step (exact for the linear part, O(h^2) otherwise)
    lat = O.lattice(Q)
    nx, ny, tau, g = 6, 9, 0.9, 1e-3
    f = inputs.populations(50 + Q, lat["w"], nx * ny, 0.08)
    rng = np.random.default_rng(6)
    lam_next = rng.normal(0, 1, f.shape)
    lam, dg, dt = A.step_vjp(f, lam_next, lat, nx, ny, tau, g, y_mode)
    h = 1e-6
    for _ in range(3):
        v = rng.normal(0, 1, f.shape) * lat["w"][:, None]
        Dv = (O.lbm_step(f + h * v, lat, nx, ny, tau, g, y_mode, 1)
              - O.lbm_step(f - h * v, lat, nx, ny, tau, g, y_mode, 1)) / (2 * h)
        assert (lam * v).sum() == pytest.approx((lam_next * Dv).sum(), rel=1e-7, abs=1e-9)
    Dg = (O.lbm_step(f, lat, nx, ny, tau, g + h, y_mode, 1) - O.lbm_step(f, lat, nx, ny, tau, g - h, y_mode, 1)) / (2 * h)
    Dt = (O.lbm_step(f, lat, nx, ny, tau + h, g, y_mode, 1) - O.lbm_step(f, lat, nx, ny, tau - h, g, y_mode, 1)) / (2 * h)
    assert dg == pytest.approx((lam_next * Dg).sum(), rel=1e-7, abs=1e-9)
    assert dt == pytest.approx((lam_next * Dt).sum(), rel=1e-7, abs=1e-9)


def test_buffer_rows_pass_cotangents_through():
    # a buffer node's populations are copied forward and streamed unchanged,
    # so its cotangent is the sum of the two paths and carries no tau or g part
    lat = O.lattice(37)
    nx, ny = 4, 8
    f = inputs.populations(60, lat["w"], nx * ny, 0.05)
    lam_next = np.zeros_like(f)
    rows = np.repeat(np.arange(ny), nx)
    lam_next[:, rows < 3] = 1.0  # cotangent only on the lower buffer rows
    lam, dg, dt = A.step_vjp(f, lam_next, lat, nx, ny, 0.8, 1e-3, 1)
    assert np.array_equal(lam[:, rows < 3], lam_next[:, rows < 3])
    assert np.all(lam[:, rows >= 3] == 0.0)
    assert dg == 0.0 and dt == 0.0


@pytest.mark.parametrize("Q,order", [(37, 3), (37, 2), (9, 2), (9, 1)])
def test_projection_matches_c_oracle_and_its_transpose(Q, order):
    lat = O.lattice(Q)
    avg = inputs.moment_sums(7, 40, scale=3.0)
    avg[0, [3, 17]] = 0.0  # empty cells
    want = O.dsmc2lb(avg, 100, lat, order)
    m = torch.tensor(avg, requires_grad=True)
    got = A.project(m, 100, lat, order)
    assert np.allclose(got.detach().numpy(), want, rtol=1e-13, atol=1e-15)
    fbar = np.random.default_rng(8).normal(0, 1, want.shape)
    (mbar,) = torch.autograd.grad(got, m, grad_outputs=torch.tensor(fbar))
    mbar = mbar.numpy()
    assert np.all(mbar[:, [3, 17]] == 0.0) and np.all(mbar[10] == 0.0)
    v = np.random.default_rng(9).normal(0, 1, avg.shape)
    v[0] *= 0.1
    v[:, [3, 17]] = 0.0  # an empty cell stays empty (the projection jumps there)
    h = 1e-3
    Dv = (O.dsmc2lb(avg + h * v, 100, lat, order) - O.dsmc2lb(avg - h * v, 100, lat, order)) / (2 * h)
    assert (mbar * v).sum() == pytest.approx((fbar * Dv).sum(), rel=1e-9)


def test_hermite_coefficients_of_equilibrium():
    # the D2Q37 third-order equilibrium has a(0..3) = rho, rho u, rho u u, rho u u u
    lat = O.lattice(37)
    rng = np.random.default_rng(10)
    rho, ux, uy = rng.uniform(0.8, 1.2, 6), rng.uniform(-0.2, 0.2, 6), rng.uniform(-0.2, 0.2, 6)
    f = _equilibrium(lat, rho, ux, uy)
    a = A.hermite_coefficients(torch.tensor(f), lat, 3, np.arange(6)).numpy()
    want = np.array([rho, rho * ux, rho * uy, rho * ux * ux, rho * ux * uy, rho * uy * uy, rho * ux ** 3,
                     rho * ux * ux * uy, rho * ux * uy * uy, rho * uy ** 3])
    assert np.allclose(a, want, rtol=1e-12, atol=1e-14)


def test_mismatch_gradients_match_central_differences():
    lat = O.lattice(37)
    nx, ny, tau, g, nsteps, ppc = 4, 9, 0.8, 1e-3, 4, 100
    f0 = inputs.populations(70, lat["w"], nx * ny, 0.05)
    nodes = np.array([12, 13, 14, 15, 20, 21])
    cells = np.arange(6)
    avg = inputs.moment_sums(11, 6, scale=2.0)
    res = A.mismatch(f0, lat, nx, ny, tau, g, 1, nsteps, nodes, 3, avg, cells, ppc)
    H = _hermite_np(lat, 3)

    def J(f0_, g_, t_, m_):
        fN = O.lbm_step(f0_, lat, nx, ny, t_, g_, 1, nsteps)
        fD = O.dsmc2lb(m_, ppc, lat, 3)
        return 0.5 * ((H @ fN[:, nodes] - H @ fD[:, cells]) ** 2).sum()

    assert res["J"] == pytest.approx(J(f0, g, tau, avg), rel=1e-12)
    h = 1e-5
    assert res["g_bar"] == pytest.approx((J(f0, g + h, tau, avg) - J(f0, g - h, tau, avg)) / (2 * h), rel=1e-6)
    assert res["tau_bar"] == pytest.approx((J(f0, g, tau + h, avg) - J(f0, g, tau - h, avg)) / (2 * h), rel=1e-6)
    v = np.random.default_rng(12).normal(0, 1, avg.shape)
    assert (res["avg_bar"] * v).sum() == pytest.approx(
        (J(f0, g, tau, avg + h * v) - J(f0, g, tau, avg - h * v)) / (2 * h), rel=1e-6)
