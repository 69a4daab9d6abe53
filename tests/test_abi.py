"""CPU-side checks of the C ABI: the library builds, loads and exports every
symbol include/dsmc.h declares; host-only calls validate their arguments."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1512_08042_amd import _lib, config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dsmc.h")).read()
    return set(re.findall(r"^(?:int|void|const char \*)\s*\*?\s*(\w+)\(", src, re.M))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared()
    assert declared == set(_lib.EXPORTS)
    for name in declared:
        assert getattr(L, name) is not None


def test_query_sizes_validates_config():
    L = _lib.lib()
    c = _lib.Config(4, 8, 10, 0, 1000, 0.1, 0.1, 0.0, 1.0, 6.0, 1, 0, 0)
    s = _lib.Sizes()
    assert L.dsmc_query_sizes(ctypes.byref(c), ctypes.byref(s)) == 0
    assert s.ncells == 32 and s.state_array_bytes == 8000 and s.workspace_bytes > 0
    for field, bad in (("nx", 0), ("kn", 0.0), ("dt", -1.0), ("capacity", 0), ("nbar_mode", 2),
                       ("kT_over_m", float("nan"))):
        d = _lib.Config.from_buffer_copy(c)
        setattr(d, field, bad)
        assert L.dsmc_query_sizes(ctypes.byref(d), ctypes.byref(s)) == _lib.EINVAL, field


def test_null_arguments_rejected_without_gpu():
    L = _lib.lib()
    assert L.dsmc_step(None, 1, 0, None) == _lib.EINVAL
    assert L.dsmc_sample_moments(None, None, 0, None) == _lib.EINVAL
    assert L.map_dsmc_to_lbm(None, 9, 2, None, None) == _lib.EINVAL
    assert L.map_lbm_to_dsmc(None, 9, 2, None, None, 0, None) == _lib.EINVAL
    cfg = _lib.LbmConfig(4, 4, 10, 0, 0.8, 0.0)  # lattice 10 does not exist
    assert L.lbm_step(ctypes.byref(cfg), None, None, 1, None) == _lib.EINVAL
    assert L.dsmc_project_moments(None, 4, 10, 1.0, 9, 2, None, None) == _lib.EINVAL
    assert L.dsmc_strerror(_lib.ECAPACITY) == b"capacity exceeded"
    assert L.dsmc_last_error(None) == b"no context"


@pytest.mark.parametrize("q", [9, 37])
def test_library_lattice_matches_oracle_lattice(q):
    # two independent derivations of the Gauss-Hermite lattice agree
    e = np.zeros((q, 2), dtype=np.int32)
    w = np.zeros(q)
    r = ctypes.c_double()
    assert _lib.lib().dsmc_lattice(q, e.ctypes.data, w.ctypes.data, ctypes.byref(r)) == 0
    lo = O.lattice(q)
    assert np.array_equal(e, lo["e"])
    assert r.value == lo["r"]
    assert np.allclose(w, lo["w"], rtol=4e-16, atol=0)


def test_run_parameters_agree_with_oracle_reading():
    for kn, ny in ((0.1, 64), (0.05, 256), (0.02, 1024), (0.01, 32)):
        assert config.time_step(kn, ny) == O.default_dt(kn, ny)
        assert config.body_force(kn, ny, 0.1) == O.body_force_for_mach(kn, ny, 0.1)
    assert config.bgk_tau(0.1, 64, 3 ** 0.5) == O.lbm_tau(0.1, 64, 3 ** 0.5)


def test_state_precision_sizes():
    # FP32 particle state halves the state arrays; other widths are rejected
    L = _lib.lib()
    s64, s32 = _lib.Sizes(), _lib.Sizes()
    c = _lib.Config(4, 8, 10, 0, 1000, 0.1, 0.1, 0.0, 1.0, 6.0, 1, 0, 0, 64, 0)
    assert L.dsmc_query_sizes(ctypes.byref(c), ctypes.byref(s64)) == 0
    c.state_bits = 32
    assert L.dsmc_query_sizes(ctypes.byref(c), ctypes.byref(s32)) == 0
    assert s64.state_array_bytes == 1000 * 8 and s32.state_array_bytes == 1000 * 4
    assert s32.workspace_bytes == s64.workspace_bytes
    c.state_bits = 16
    assert L.dsmc_query_sizes(ctypes.byref(c), ctypes.byref(s32)) == _lib.EINVAL


def test_adjoint_entries_validate_without_gpu():
    L = _lib.lib()
    cfg = _lib.LbmConfig(100, 30, 37, 1, 0.8, 1e-3)
    size = ctypes.c_size_t()
    assert L.lbm_adjoint_workspace(ctypes.byref(cfg), 20, ctypes.byref(size)) == 0
    al = lambda x: (x + 255) // 256 * 256
    nblk = (3000 + 255) // 256
    state = al(37 * 3000 * 8)
    assert size.value == al(2 * nblk * 8) + state + 19 * state
    assert L.lbm_adjoint_workspace(ctypes.byref(cfg), 0, ctypes.byref(size)) == 0
    assert size.value == al(2 * nblk * 8)
    assert L.lbm_adjoint_workspace(ctypes.byref(cfg), -1, ctypes.byref(size)) == _lib.EINVAL
    bad = _lib.LbmConfig(100, 30, 37, 1, 0.5, 1e-3)  # tau must exceed 1/2
    assert L.lbm_adjoint_workspace(ctypes.byref(bad), 20, ctypes.byref(size)) == _lib.EINVAL
    big = _lib.LbmConfig(1 << 15, 1 << 14, 9, 0, 0.8, 0.0)  # 2^29 nodes: beyond 32-bit plane offsets
    assert L.lbm_adjoint_workspace(ctypes.byref(big), 1, ctypes.byref(size)) == _lib.EINVAL
    p = ctypes.c_void_p(256)  # never dereferenced: these calls return before any GPU work
    assert L.lbm_adjoint(ctypes.byref(cfg), p, 0, 20, p, p, p, None) == 0  # zero steps: nothing to do
    assert L.lbm_adjoint(ctypes.byref(cfg), None, 5, 20, p, p, p, None) == _lib.EINVAL
    assert L.lbm_adjoint(ctypes.byref(cfg), p, 5, 0, p, p, p, None) == _lib.EINVAL
    assert L.lbm_adjoint_step(ctypes.byref(cfg), p, p, p, p, p, None) == _lib.EINVAL  # lam_out aliases lam_next
    assert L.lbm_step_checkpointed(ctypes.byref(cfg), p, p, None, 3, 0, None) == _lib.EINVAL
    assert L.lbm_hermite_moments(37, 3, p, 3000, p, 0, p, None) == 0
    assert L.lbm_hermite_moments(37, 4, p, 3000, p, 5, p, None) == _lib.EINVAL
    assert L.lbm_hermite_moments(10, 2, p, 3000, p, 5, p, None) == _lib.EINVAL
    assert L.lbm_hermite_moments_adjoint(9, 2, None, p, 5, p, 3000, None) == _lib.EINVAL
    assert L.dsmc_project_moments_adjoint(p, p, 0, 100, 1.0, 37, 3, p, None) == 0
    assert L.dsmc_project_moments_adjoint(p, p, 10, 0, 1.0, 37, 3, p, None) == _lib.EINVAL
    assert L.dsmc_project_moments_adjoint(p, p, 10, 100, -1.0, 37, 3, p, None) == _lib.EINVAL


def test_batch_sizes_validate_without_gpu():
    L = _lib.lib()
    common = _lib.Config(1, 1, 1, 0, 100000, 1.0, 1.0, 0.0, 1.0, 6.0, 0, 0, 0)
    reps = (_lib.Replica * 3)(_lib.Replica(1, 40, 50, 0, 0.1, 0.05, 1e-3, 7),
                              _lib.Replica(2, 10, 20, 0, 0.5, 0.1, 0.0, 8),
                              _lib.Replica(1, 64, 30, 0, 0.02, 0.01, 1e-4, 9))
    s = _lib.Sizes()
    assert L.dsmc_batch_query_sizes(ctypes.byref(common), reps, 3, ctypes.byref(s)) == 0
    assert s.ncells == 40 + 20 + 64 and s.workspace_bytes > 0
    one = _lib.Sizes()
    assert L.dsmc_batch_query_sizes(ctypes.byref(common), reps, 1, ctypes.byref(one)) == 0
    assert one.ncells == 40 and one.workspace_bytes < s.workspace_bytes
    assert L.dsmc_batch_query_sizes(ctypes.byref(common), reps, 0, ctypes.byref(s)) == _lib.EINVAL
    bad = (_lib.Replica * 1)(_lib.Replica(1, 40, 50, 0, 0.0, 0.05, 0.0, 7))  # Kn must be positive
    assert L.dsmc_batch_query_sizes(ctypes.byref(common), bad, 1, ctypes.byref(s)) == _lib.EINVAL
    bad[0] = _lib.Replica(1, 0, 50, 0, 0.1, 0.05, 0.0, 7)  # no rows
    assert L.dsmc_batch_query_sizes(ctypes.byref(common), bad, 1, ctypes.byref(s)) == _lib.EINVAL
    assert L.dsmc_set_tiling(None, 100, None) == _lib.EINVAL
    assert L.dsmc_autotune(None, 2, 1, None, None) == _lib.EINVAL
    assert L.dsmc_replica_counters(None, None, None) == _lib.EINVAL


def test_wall_and_inflow_modes_validate_without_gpu():
    L = _lib.lib()
    size = ctypes.c_size_t()
    walls = _lib.LbmConfig(10, 8, 9, 2, 0.8, 1e-3, 1, 0)
    p = ctypes.c_void_p(256)  # never dereferenced
    assert L.lbm_step(ctypes.byref(walls), p, p, 0, None) == 0  # zero steps: valid, nothing to do
    bad = _lib.LbmConfig(10, 8, 37, 2, 0.8, 1e-3, 0, 0)  # walls need |e_y| <= 1
    assert L.lbm_step(ctypes.byref(bad), p, p, 0, None) == _lib.EINVAL
    bad = _lib.LbmConfig(10, 8, 9, 3, 0.8, 1e-3, 0, 0)
    assert L.lbm_step(ctypes.byref(bad), p, p, 0, None) == _lib.EINVAL
    bad = _lib.LbmConfig(10, 8, 9, 0, 0.8, 1e-3, 11, 0)  # more inflow columns than columns
    assert L.lbm_step(ctypes.byref(bad), p, p, 0, None) == _lib.EINVAL
    # the reverse pass covers neither walls nor inflow columns
    assert L.lbm_adjoint_workspace(ctypes.byref(walls), 20, ctypes.byref(size)) == _lib.EINVAL
    inflow = _lib.LbmConfig(10, 8, 9, 0, 0.8, 1e-3, 1, 0)
    assert L.lbm_adjoint_workspace(ctypes.byref(inflow), 20, ctypes.byref(size)) == _lib.EINVAL
    assert L.dsmc_project_equilibrium(p, 10, 100, 1.0, 9, 3, p, None) == _lib.EINVAL  # D2Q9 has no 3rd order
    assert L.dsmc_project_equilibrium(p, 0, 100, 1.0, 9, 2, p, None) == _lib.EINVAL
    h = _lib.Hybrid(walls, 4, 2, 0, 2, 0, 0)
    assert L.dsmc_hybrid_cycle(None, ctypes.byref(h), p, p, None, None) == _lib.EINVAL


def test_size_limits():
    # slots are 32-bit (capacity up to 2^31 - 1) and cells fit 30 bits
    # (nx * ny < 2^30): the largest sizes pass, one more is rejected, and the
    # sizes of the largest grid come out without overflow
    L = _lib.lib()
    s = _lib.Sizes()
    c = _lib.Config(4, 8, 10, 0, 2 ** 31 - 1, 0.1, 0.1, 0.0, 1.0, 6.0, 1, 0, 0)
    assert L.dsmc_query_sizes(ctypes.byref(c), ctypes.byref(s)) == 0
    assert s.state_array_bytes == (2 ** 31 - 1) * 8
    c.capacity = 2 ** 31
    assert L.dsmc_query_sizes(ctypes.byref(c), ctypes.byref(s)) == _lib.EINVAL
    big = _lib.Config(1, 2 ** 30 - 1, 1, 0, 2 ** 31 - 1, 0.1, 0.1, 0.0, 1.0, 6.0, 1, 0, 0)
    assert L.dsmc_query_sizes(ctypes.byref(big), ctypes.byref(s)) == 0
    assert s.ncells == 2 ** 30 - 1 and s.workspace_bytes > 100 * (2 ** 30 - 1)
    for nx, ny in ((2 ** 15, 2 ** 15), (1, 2 ** 30), (70000, 40000)):
        c = _lib.Config(nx, ny, 1, 0, 1000, 0.1, 0.1, 0.0, 1.0, 6.0, 1, 0, 0)
        assert L.dsmc_query_sizes(ctypes.byref(c), ctypes.byref(s)) == _lib.EINVAL, (nx, ny)
