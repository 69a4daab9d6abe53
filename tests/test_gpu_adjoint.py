"""GPU parity of the lattice adjoint against the autograd oracle.

Every entry point is called through the C ABI (or the autograd Functions
that wrap it) on seeded synthetic populations and compared with the oracle's
reverse-mode derivative of the same definition, element by element.

Tolerances: the adjoint sums the same products as the oracle's automatic
differentiation but in another order and with reciprocals (1/tau, 1/rho, 1/6)
where the forward divides; over a few dozen steps each cotangent carries a
relative rounding error of a few hundred FP64 ulps at most, so cotangents are
compared at 1e-11 relative (plus 1e-13 of the largest magnitude), and the
parameter gradients, sums over every node and step, at 1e-10 relative.
"""
import ctypes

import numpy as np
import pytest
import torch

import inputs
from oracle import lbm_adjoint as A
from oracle import oracle as O

pytestmark = pytest.mark.gpu

LAM_RTOL, LAM_ATOL_REL, GRAD_RTOL = 1e-11, 1e-13, 1e-10


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_08042_amd import _lib, lbm

    return _lib, lbm


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _close_lam(got, want, what=""):
    scale = np.abs(want).max() + 1e-300
    bad = ~np.isclose(got, want, rtol=LAM_RTOL, atol=LAM_ATOL_REL * scale)
    assert not bad.any(), "%s: %d entries differ, first %s: %r vs %r" % (
        what, bad.sum(), np.argwhere(bad)[:3].tolist(), got[bad][:3], want[bad][:3])


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _adjoint_step(_lib, nx, ny, q, y_mode, tau, g, f, lam_next):
    L = _lib.lib()
    cfg = _lib.LbmConfig(nx, ny, q, y_mode, tau, g)
    size = ctypes.c_size_t()
    assert L.lbm_adjoint_workspace(ctypes.byref(cfg), 0, ctypes.byref(size)) == 0
    work = torch.empty(size.value, dtype=torch.uint8, device="cuda")
    fd, ld = _dev(f), _dev(lam_next)
    out = torch.full_like(ld, float("nan"))
    grad = torch.zeros(2, dtype=torch.float64, device="cuda")
    assert L.lbm_adjoint_step(ctypes.byref(cfg), fd.data_ptr(), ld.data_ptr(), out.data_ptr(), grad.data_ptr(),
                              work.data_ptr(), _stream()) == 0
    return out.cpu().numpy(), grad.cpu().numpy()


@pytest.mark.parametrize("q,y_mode,nx,ny,g", [
    (9, 0, 13, 11, 0.0),
    (9, 1, 5, 7, 2e-3),
    (37, 1, 37, 29, 1e-3),   # 1073 nodes: five blocks, the last one ragged
    (37, 0, 40, 33, 2e-3),
    (37, 0, 2, 5, 1e-3),     # narrower than the velocities in x
    (37, 1, 1, 9, 1e-3),     # one column, three interior rows
    (9, 0, 1, 1, 1e-3),      # a single node
])
def test_adjoint_step_matches_oracle(q, y_mode, nx, ny, g):
    _lib, _ = _gpu()
    lat = O.lattice(q)
    f = inputs.populations(100 + q + nx, lat["w"], nx * ny, 0.1)
    lam_next = np.random.default_rng(ny).normal(0, 1, f.shape)
    tau = 0.83
    got, grad = _adjoint_step(_lib, nx, ny, q, y_mode, tau, g, f, lam_next)
    want, dg, dt = A.step_vjp(f, lam_next, lat, nx, ny, tau, g, y_mode)
    _close_lam(got, want, "lambda_n")
    assert grad[0] == pytest.approx(dg, rel=GRAD_RTOL, abs=1e-14)
    assert grad[1] == pytest.approx(dt, rel=GRAD_RTOL, abs=1e-14)


def _rollout_gpu(_lib, nx, ny, q, y_mode, tau, g, f0, lam_N, nsteps, every):
    L = _lib.lib()
    cfg = _lib.LbmConfig(nx, ny, q, y_mode, tau, g)
    nn = nx * ny
    f = _dev(f0)
    tmp = torch.empty_like(f)
    nck = max((nsteps + every - 1) // every, 1)
    ckpt = torch.full((nck, q, nn), float("nan"), dtype=torch.float64, device="cuda")
    assert L.lbm_step_checkpointed(ctypes.byref(cfg), f.data_ptr(), tmp.data_ptr(), ckpt.data_ptr(), nsteps, every,
                                   _stream()) == 0
    size = ctypes.c_size_t()
    assert L.lbm_adjoint_workspace(ctypes.byref(cfg), every, ctypes.byref(size)) == 0
    work = torch.empty(size.value, dtype=torch.uint8, device="cuda")
    lam = _dev(lam_N)
    grad = torch.full((2,), 0.25, dtype=torch.float64, device="cuda")  # the entry adds to it
    assert L.lbm_adjoint(ctypes.byref(cfg), ckpt.data_ptr(), nsteps, every, lam.data_ptr(), grad.data_ptr(),
                         work.data_ptr(), _stream()) == 0
    return f.cpu().numpy(), ckpt.cpu().numpy(), lam.cpu().numpy(), grad.cpu().numpy() - 0.25


@pytest.mark.parametrize("nsteps,every", [(45, 20), (45, 1), (45, 45), (45, 64), (20, 20), (1, 20), (0, 20)])
def test_checkpointed_adjoint_matches_oracle(nsteps, every):
    _lib, _ = _gpu()
    q, y_mode, nx, ny, tau, g = 37, 1, 16, 12, 0.8, 1e-3
    lat = O.lattice(q)
    f0 = inputs.populations(7, lat["w"], nx * ny, 0.08)
    lam_N = np.random.default_rng(8).normal(0, 1, f0.shape)
    fN, ckpt, lam0, grad = _rollout_gpu(_lib, nx, ny, q, y_mode, tau, g, f0, lam_N, nsteps, every)
    want_fN, want_lam0, dg, dt = A.rollout_vjp(f0, lam_N, lat, nx, ny, tau, g, y_mode, nsteps)
    assert np.allclose(fN, want_fN, rtol=1e-12, atol=1e-15)
    for k in range((nsteps + every - 1) // every):
        want_k = O.lbm_step(f0, lat, nx, ny, tau, g, y_mode, k * every)
        assert np.allclose(ckpt[k], want_k, rtol=1e-12, atol=1e-15), "checkpoint %d" % k
    _close_lam(lam0, want_lam0, "lambda_0")
    assert grad[0] == pytest.approx(dg, rel=GRAD_RTOL, abs=1e-14)
    assert grad[1] == pytest.approx(dt, rel=GRAD_RTOL, abs=1e-14)


def test_adjoint_is_bitwise_reproducible():
    _lib, _ = _gpu()
    q, nx, ny = 37, 64, 40
    lat = O.lattice(q)
    f0 = inputs.populations(9, lat["w"], nx * ny, 0.05)
    lam_N = np.random.default_rng(10).normal(0, 1, f0.shape)
    r1 = _rollout_gpu(_lib, nx, ny, q, 1, 0.9, 1e-3, f0, lam_N, 30, 7)
    r2 = _rollout_gpu(_lib, nx, ny, q, 1, 0.9, 1e-3, f0, lam_N, 30, 7)
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("q,order", [(37, 3), (9, 2), (37, 1), (9, 0)])
def test_hermite_moments_and_adjoint_match_oracle(q, order):
    _lib, lbm = _gpu()
    lat = O.lattice(q)
    nn = 700
    f = inputs.populations(11, lat["w"], nn, 0.2)
    nodes = np.random.default_rng(12).permutation(nn)[:300].astype(np.int32)
    ft = _dev(f).requires_grad_(True)
    a = lbm.hermite_moments(ft, _dev(nodes, torch.int32), q, order)
    want = A.hermite_coefficients(torch.tensor(f), lat, order, nodes).numpy()
    assert a.shape == want.shape
    assert np.allclose(a.detach().cpu().numpy(), want, rtol=1e-13, atol=1e-15)
    a_bar = np.random.default_rng(13).normal(0, 1, want.shape)
    (f_bar,) = torch.autograd.grad(a, ft, grad_outputs=_dev(a_bar))
    fo = torch.tensor(f, requires_grad=True)
    (want_bar,) = torch.autograd.grad(A.hermite_coefficients(fo, lat, order, nodes), fo, torch.tensor(a_bar))
    assert np.allclose(f_bar.cpu().numpy(), want_bar.numpy(), rtol=1e-13, atol=1e-14)


def test_hermite_moments_flag_ids_outside_the_grid():
    _lib, lbm = _gpu()
    lat = O.lattice(9)
    f = _dev(inputs.populations(14, lat["w"], 10, 0.1))
    a = lbm.hermite_moments(f, _dev(np.array([0, 10, -1, 9], dtype=np.int32), torch.int32), 9, 2).cpu().numpy()
    assert np.isfinite(a[:, [0, 3]]).all() and np.isnan(a[:, [1, 2]]).all()


@pytest.mark.parametrize("q,order", [(37, 3), (37, 2), (9, 3), (9, 2)])
def test_projection_adjoint_matches_oracle(q, order):
    _lib, lbm = _gpu()
    lat = O.lattice(q)
    avg = inputs.moment_sums(15, 1000, scale=3.0)
    avg[0, [5, 700]] = 0.0
    m = _dev(avg).requires_grad_(True)
    f = lbm.project_moments(m, 100, q, order)
    f_bar = np.random.default_rng(16).normal(0, 1, (q, 1000))
    (m_bar,) = torch.autograd.grad(f, m, grad_outputs=_dev(f_bar))
    mo = torch.tensor(avg, requires_grad=True)
    (want,) = torch.autograd.grad(A.project(mo, 100, lat, order), mo, torch.tensor(f_bar))
    got = m_bar.cpu().numpy()
    assert np.all(got[:, [5, 700]] == 0.0) and np.all(got[10] == 0.0)
    assert np.allclose(got, want.numpy(), rtol=1e-12, atol=1e-15 * np.abs(want.numpy()).max())


def test_autograd_mismatch_gradients_match_oracle():
    _lib, lbm = _gpu()
    q, nx, ny, tau, g, nsteps, ppc = 37, 12, 14, 0.85, 2e-3, 25, 100
    lat = O.lattice(q)
    f0 = inputs.populations(17, lat["w"], nx * ny, 0.05)
    nodes = np.arange(3 * nx, 5 * nx, dtype=np.int32)  # two interior rows
    cells = np.arange(nodes.size, dtype=np.int32)
    avg = inputs.moment_sums(18, nodes.size, scale=2.0)
    want = A.mismatch(f0, lat, nx, ny, tau, g, 1, nsteps, nodes, 3, avg, cells, ppc)

    f0_t = _dev(f0).requires_grad_(True)
    g_t = torch.tensor(g, dtype=torch.float64, device="cuda", requires_grad=True)
    tau_t = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
    m_t = _dev(avg).requires_grad_(True)
    fN = lbm.rollout(f0_t, g_t, tau_t, nx, ny, q, y_mode=1, nsteps=nsteps, every=10)
    fD = lbm.project_moments(m_t, ppc, q, 3)
    J = lbm.coupling_mismatch(fN, _dev(nodes, torch.int32), fD, _dev(cells, torch.int32), q, 3)
    J.backward()
    assert float(J.detach()) == pytest.approx(want["J"], rel=1e-12)
    assert float(g_t.grad) == pytest.approx(want["g_bar"], rel=GRAD_RTOL)
    assert float(tau_t.grad) == pytest.approx(want["tau_bar"], rel=GRAD_RTOL)
    _close_lam(f0_t.grad.cpu().numpy(), want["f0_bar"], "dJ/df0")
    _close_lam(m_t.grad.cpu().numpy(), want["avg_bar"], "dJ/davg")


def _c5_problem(lbm, seed=5):
    """D2Q37 1024 x 512 with the max|e_y| = 3 rows at each y edge held, the
    relaxation time of Eq. (tau) at Kn 0.1 on 512 rows, the body force for
    Ma 0.1, Poiseuille initial populations; coupling nodes: the 32 rows at
    each wall, matched with synthetic DSMC averages of 100 particles per cell."""
    from paper_1512_08042_amd.config import bgk_tau, body_force

    q, nx, ny = 37, 1024, 512
    lat = O.lattice(q)
    r = lat["r"]
    tau = bgk_tau(0.1, ny, r)
    g = body_force(0.1, ny, 0.1) / r
    y = (np.arange(ny) + 0.5) / ny
    ux = np.repeat(0.4 * y * (1 - y), nx)
    cu = lat["xi"][:, :1] * ux
    f0 = lat["w"][:, None] * (1 + cu + 0.5 * (cu * cu - ux * ux) + cu * (cu * cu - 3 * ux * ux) / 6)
    rows = np.r_[0:32, ny - 32:ny]
    nodes = (rows[:, None] * nx + np.arange(nx)[None, :]).ravel().astype(np.int32)
    rng = np.random.default_rng(seed)
    uxs = np.repeat(0.4 * y[rows] * (1 - y[rows]), nx) + rng.normal(0, 0.01, nodes.size)
    m0 = 100.0 * (1 + rng.normal(0, 0.02, nodes.size))
    vy = rng.normal(0, 0.01, nodes.size)
    avg = np.array([m0, m0 * uxs, m0 * vy, m0 * (uxs ** 2 + 1), m0 * uxs * vy, m0 * (vy ** 2 + 1),
                    m0 * (uxs ** 3 + 3 * uxs), m0 * (uxs ** 2 * vy + vy), m0 * (uxs * vy ** 2 + uxs),
                    m0 * (vy ** 3 + 3 * vy), m0])
    return dict(q=q, nx=nx, ny=ny, tau=tau, g=g, f0=f0, nodes=nodes, cells=np.arange(nodes.size, dtype=np.int32),
                avg=avg)


def test_full_size_one_adjoint_step_matches_oracle():
    _lib, lbm = _gpu()
    P = _c5_problem(lbm)
    lat = O.lattice(37)
    lam_next = np.random.default_rng(19).normal(0, 1, P["f0"].shape)
    f = O.lbm_step(P["f0"], lat, P["nx"], P["ny"], P["tau"], P["g"], 1, 1)
    got, grad = _adjoint_step(_lib, P["nx"], P["ny"], 37, 1, P["tau"], P["g"], f, lam_next)
    want, dg, dt = A.step_vjp(f, lam_next, lat, P["nx"], P["ny"], P["tau"], P["g"], 1)
    _close_lam(got, want, "lambda_n at 1024 x 512")
    assert grad[0] == pytest.approx(dg, rel=1e-9)
    assert grad[1] == pytest.approx(dt, rel=1e-9)


def test_full_size_gradient_matches_central_differences():
    # 200 steps with checkpoints every 20 at the full size: dJ/dg, dJ/dtau and
    # a directional derivative in f0 against central differences of the
    # library's own forward (a property that holds at any size)
    _lib, lbm = _gpu()
    P = _c5_problem(lbm)
    q, nx, ny, nsteps = 37, P["nx"], P["ny"], 200
    nodes, cells = _dev(P["nodes"], torch.int32), _dev(P["cells"], torch.int32)
    fD = lbm.project_moments(_dev(P["avg"]), 100, q, 3)

    def J(f0, g, tau):
        with torch.no_grad():
            fN = lbm.rollout(f0, g, tau, nx, ny, q, 1, nsteps, 20)
            return float(lbm.coupling_mismatch(fN, nodes, fD, cells, q, 3))

    f0 = _dev(P["f0"]).requires_grad_(True)
    g_t = torch.tensor(P["g"], dtype=torch.float64, device="cuda", requires_grad=True)
    tau_t = torch.tensor(P["tau"], dtype=torch.float64, device="cuda", requires_grad=True)
    Jt = lbm.coupling_mismatch(lbm.rollout(f0, g_t, tau_t, nx, ny, q, 1, nsteps, 20), nodes, fD, cells, q, 3)
    Jt.backward()
    f0d = f0.detach()
    hg, ht = 1e-4 * P["g"], 1e-4 * P["tau"]
    fd_g = (J(f0d, P["g"] + hg, P["tau"]) - J(f0d, P["g"] - hg, P["tau"])) / (2 * hg)
    fd_t = (J(f0d, P["g"], P["tau"] + ht) - J(f0d, P["g"], P["tau"] - ht)) / (2 * ht)
    v = torch.randn(f0d.shape, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    v *= 1e-4 * _dev(O.lattice(37)["w"])[:, None]
    fd_f = (J(f0d + v, P["g"], P["tau"]) - J(f0d - v, P["g"], P["tau"])) / 2
    assert float(g_t.grad) == pytest.approx(fd_g, rel=1e-6)
    assert float(tau_t.grad) == pytest.approx(fd_t, rel=1e-6)
    assert float((f0.grad * v).sum()) == pytest.approx(fd_f, rel=1e-6)
    assert abs(float(g_t.grad)) > 0 and abs(float(tau_t.grad)) > 0
