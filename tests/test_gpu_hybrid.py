"""GPU parity of the hybrid coupling of Section 4: the lattice step with
diffuse walls and held inflow columns, the equilibrium mapping of
Eq. (feq_dsmc), and whole coupling cycles (DSMC subdomain -> buffer-layer
column -> lattice subdomain) against the same cycle composed from the
oracle's pieces.  FP64 values within 1e-12 relative of the oracle (1e-11
after several cycles, where rounding of the sampled averages feeds the
lattice)."""
import ctypes

import numpy as np
import pytest
import torch

import inputs
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_08042_amd import dsmc as D
    from paper_1512_08042_amd.config import ChannelConfig

    return D, ChannelConfig


@pytest.mark.parametrize("q,y_mode,xb,nx,ny,g", [
    (9, 2, 0, 13, 11, 1e-3), (9, 2, 1, 13, 11, 2e-3), (9, 0, 1, 7, 5, 1e-3), (9, 1, 1, 9, 7, 0.0),
    (37, 1, 3, 17, 13, 1e-3), (37, 0, 3, 12, 10, 1e-3), (9, 2, 1, 1, 6, 1e-3), (9, 2, 0, 1, 1, 1e-3),
    (9, 2, 0, 300, 7, 1e-3),
])
def test_lbm_step_with_walls_and_inflow_columns_matches_oracle(q, y_mode, xb, nx, ny, g):
    D, _ = _gpu()
    lat = O.lattice(q)
    f = inputs.populations(q + 10 * y_mode + xb, lat["w"], nx * ny, 0.1)
    got = D.lbm_step(torch.as_tensor(f, device="cuda").contiguous(), nx, ny, q, 0.83, g, y_mode, 4, x_buffer=xb)
    want = O.lbm_step(f, lat, nx, ny, 0.83, g, y_mode, 4, x_buffer=xb)
    assert np.allclose(got.cpu().numpy(), want, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("q,order", [(9, 2), (37, 2), (37, 3)])
def test_equilibrium_mapping_matches_oracle(q, order):
    D, _ = _gpu()
    lat = O.lattice(q)
    avg = inputs.moment_sums(21, 900, scale=4.0)
    avg[0, [3, 500]] = 0.0
    got = D.project_equilibrium(torch.as_tensor(avg, device="cuda"), 100, q, order).cpu().numpy()
    want = O.dsmc2lb_eq(avg, 100, lat, order)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15)


def _oracle_cycle(ref, f_lb, lat, nx_d, nx_l, ny, ppc, tau, g, dsmc_steps, lbm_steps, mapping, order):
    ref.step(dsmc_steps, sample_every=1)
    avg = ref.averages()
    ref.reset_moments()
    cells = np.arange(ny) * nx_d + (nx_d - 1)
    col = (O.dsmc2lb_eq if mapping == 0 else O.dsmc2lb)(avg[:, cells], ppc, lat, order)
    f_lb = f_lb.copy()
    f_lb[:, np.arange(ny) * nx_l] = col
    return O.lbm_step(f_lb, lat, nx_l, ny, tau, g, 2, lbm_steps, x_buffer=1), avg


@pytest.mark.parametrize("mapping,moved", [(0, False), (1, False), (0, True)])
def test_hybrid_cycles_match_the_oracle_composition(mapping, moved):
    # moved: every cycle leaves the DSMC state moved for the next one
    D, ChannelConfig = _gpu()
    nx_d, nx_l, ny, ppc, kn = 8, 10, 12, 30, 0.1
    cfg = ChannelConfig(nx=nx_d, ny=ny, ppc=ppc, kn=kn, mach=0.1, seed=3).resolved()
    ch = D.Channel(cfg)
    ref = O.Sim(nx_d, ny, ppc, kn, dt=cfg.dt, g=cfg.body_force_x, seed=3, capacity=cfg.capacity)
    ref.init_maxwell()
    lat = O.lattice(9)
    tau, g_lb = 0.9, cfg.body_force_x / lat["r"]
    f0 = np.repeat(lat["w"][:, None], nx_l * ny, axis=1)
    f_gpu = torch.as_tensor(f0, device="cuda").contiguous()
    tmp = torch.empty_like(f_gpu)
    f_ref = f0
    avg = torch.empty((11, nx_d * ny), dtype=torch.float64, device="cuda")
    for cyc in range(3):
        ch.hybrid_cycle(f_gpu, tmp, nx_l, tau, g_lb, dsmc_steps=4, lbm_steps=2, mapping=mapping, order=2,
                        avg_out=avg, moved=moved)
        assert ch.status()["moved"] == moved
        f_ref, want_avg = _oracle_cycle(ref, f_ref, lat, nx_d, nx_l, ny, ppc, tau, g_lb, 4, 2, mapping, 2)
        assert np.allclose(f_gpu.cpu().numpy(), f_ref, rtol=1e-11, atol=1e-14), "cycle %d" % cyc
        scale = np.abs(want_avg).max(axis=1, keepdims=True) + 1.0
        assert np.all(np.abs(avg.cpu().numpy() - want_avg) <= 1e-12 * scale), "cycle %d averages" % cyc
    if moved:  # one more step on both sides settles it
        ch.step(1)
        ref.step(1)
    for gp, w in zip(ch.particles(), ref.particles()):
        assert np.allclose(gp.cpu().numpy(), w, rtol=1e-12, atol=1e-12)
    # the buffer column holds the DSMC column's state of the last cycle
    assert not np.allclose(f_ref[:, 0], lat["w"])
    ch.close()


def test_hybrid_cycle_rejects_bad_arguments():
    D, ChannelConfig = _gpu()
    from paper_1512_08042_amd import _lib

    L = _lib.lib()
    stream = torch.cuda.current_stream().cuda_stream
    ch = D.Channel(ChannelConfig(nx=4, ny=6, ppc=10, kn=0.1, seed=1))
    f = torch.ones((9, 5 * 7), dtype=torch.float64, device="cuda")
    tmp = torch.empty_like(f)
    h = _lib.Hybrid(_lib.LbmConfig(5, 7, 9, 2, 0.9, 0.0, 1, 0), 2, 1, 0, 2, 3, 0)  # 7 lattice rows, 6 DSMC rows
    assert L.dsmc_hybrid_cycle(ch._h, ctypes.byref(h), f.data_ptr(), tmp.data_ptr(), None, stream) == _lib.EINVAL
    h = _lib.Hybrid(_lib.LbmConfig(5, 6, 9, 2, 0.9, 0.0, 0, 0), 2, 1, 0, 2, 3, 0)  # no buffer column
    assert L.dsmc_hybrid_cycle(ch._h, ctypes.byref(h), f.data_ptr(), tmp.data_ptr(), None, stream) == _lib.EINVAL
    h = _lib.Hybrid(_lib.LbmConfig(5, 6, 9, 2, 0.9, 0.0, 1, 0), 2, 1, 0, 2, 4, 0)  # DSMC column out of range
    assert L.dsmc_hybrid_cycle(ch._h, ctypes.byref(h), f.data_ptr(), tmp.data_ptr(), None, stream) == _lib.EINVAL
    h = _lib.Hybrid(_lib.LbmConfig(5, 6, 9, 2, 0.9, 0.0, 1, 0), 2, 1, 0, 2, 3, 2)  # unknown flag
    assert L.dsmc_hybrid_cycle(ch._h, ctypes.byref(h), f.data_ptr(), tmp.data_ptr(), None, stream) == _lib.EINVAL
    assert ch.views().step == 0  # nothing ran
    ch.close()
    b = D.Batch([dict(nx=4, ny=6, ppc=10, kn=0.1, seed=1), dict(nx=2, ny=6, ppc=10, kn=0.2, seed=2)])
    h = _lib.Hybrid(_lib.LbmConfig(5, 6, 9, 2, 0.9, 0.0, 1, 0), 2, 1, 0, 2, 3, 0)
    assert L.dsmc_hybrid_cycle(b._h, ctypes.byref(h), f.data_ptr(), tmp.data_ptr(), None, stream) == _lib.ESTATE
    b.close()
