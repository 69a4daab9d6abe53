"""Python binding of libdsmc: device buffers and streams come from PyTorch,
every step of the DSMC particle step and the DSMC<->LBM mappings runs in the
HIP kernels behind the C ABI (include/dsmc.h).  There is no CPU fallback:
without the built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check, lib
from .config import ChannelConfig

NMOM = _lib.NMOM


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def lattice(q: int):
    """(e int[Q,2], w float64[Q], r) of the library's D2Q9 / D2Q37 tables (host copy)."""
    import numpy as np

    n = {9: 9, 37: 37}[q]
    e = np.zeros((n, 2), dtype=np.int32)
    w = np.zeros(n)
    r = ctypes.c_double()
    check(lib().dsmc_lattice(q, e.ctypes.data, w.ctypes.data, ctypes.byref(r)), "dsmc_lattice")
    return e, w, r.value


class Channel:
    """A DSMC channel (periodic x, diffuse walls at y = 0 and y = ny) on one GPU."""

    def __init__(self, cfg: ChannelConfig, particles=None, device: str = "cuda", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1512_08042_amd needs a ROCm GPU; no CPU fallback exists")
        self.cfg = c = cfg.resolved()
        self.device = torch.device(device)
        self._c = _lib.Config(c.nx, c.ny, c.ppc, c.nbar_mode, c.capacity, c.kn, c.dt, c.body_force_x, c.kT_over_m,
                              c.sigcr_max0, c.seed, c.ar_max_tries, c.far_capacity, int(c.state_bits), 0)
        sz = _lib.Sizes()
        check(lib().dsmc_query_sizes(ctypes.byref(self._c), ctypes.byref(sz)), "dsmc_query_sizes")
        self.ncells = int(sz.ncells)
        self.capacity = int(sz.capacity)
        # particle state: FP64, or FP32 storage (the arithmetic is FP64 either way)
        self.state_dtype = torch.float32 if int(c.state_bits) == 32 else torch.float64
        self.state = torch.zeros((2, 5, self.capacity), dtype=self.state_dtype, device=self.device)
        self.workspace = torch.zeros(int(sz.workspace_bytes) + 256, dtype=torch.uint8, device=self.device)
        ws = _ptr(self.workspace)
        self._ws = (ws + 255) & ~255
        b = _lib.Buffers()
        for i in range(2):
            for k in range(5):
                b.state[i][k] = _ptr(self.state[i, k])
        b.workspace = self._ws
        b.workspace_bytes = int(sz.workspace_bytes)
        mode, n = 0, 0
        if particles is not None:
            mode = 1
            n = int(particles[0].numel())
            for k in range(5):
                self.state[0, k, :n].copy_(torch.as_tensor(particles[k], dtype=torch.float64).to(self.state_dtype))
        self._h = ctypes.c_void_p()
        check(lib().dsmc_init(ctypes.byref(self._c), ctypes.byref(b), mode, n, _stream(stream), ctypes.byref(self._h)),
              "dsmc_init")

    # ---- lifecycle -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            torch.cuda.synchronize(self.device)
            lib().dsmc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- the hot path -------------------------------------------------------------
    def step(self, nsteps: int = 1, sample_every: int = 0, stream=None, moved: bool = False):
        """nsteps steps (sampling when (step + 1) % sample_every == 0).  With
        moved=True the state is left moved for the coming step, so the next
        call starts without re-moving it; particles() then refuses until a
        plain step() call (nsteps >= 1) settles it again."""
        if moved:
            check(lib().dsmc_step_moved(self._h, int(nsteps), int(sample_every), _stream(stream)), "dsmc_step_moved",
                  self._h)
        else:
            check(lib().dsmc_step(self._h, int(nsteps), int(sample_every), _stream(stream)), "dsmc_step", self._h)

    def sample_moments(self, reset: bool = False, stream=None) -> torch.Tensor:
        out = torch.empty((NMOM, self.ncells), dtype=torch.float64, device=self.device)
        check(lib().dsmc_sample_moments(self._h, _ptr(out), int(reset), _stream(stream)), "dsmc_sample_moments",
              self._h)
        return out

    def reset_moments(self, stream=None):
        check(lib().dsmc_sample_moments(self._h, None, 1, _stream(stream)), "dsmc_sample_moments", self._h)

    def map_to_lbm(self, lattice_q: int, order: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty((lattice_q, self.ncells), dtype=torch.float64, device=self.device)
        check(lib().map_dsmc_to_lbm(self._h, int(lattice_q), int(order), _ptr(out), _stream(stream)),
              "map_dsmc_to_lbm", self._h)
        return out

    def map_from_lbm(self, f: torch.Tensor, cell_ids: torch.Tensor, lattice_q: int, order: int, stream=None):
        """LB2DSMC reseed of the listed cells from populations f [Q][ncells]
        (Table 1).  Only the new particles are written here; the other
        cells' particles move to their new slots in the next step's first
        pass, or when the state is read first (views(), particles(),
        status()), so cell_ids may be freed once this call's work is done."""
        assert f.dtype == torch.float64 and f.is_contiguous() and f.shape == (lattice_q, self.ncells)
        assert cell_ids.dtype == torch.int32 and cell_ids.is_contiguous()
        check(lib().map_lbm_to_dsmc(self._h, int(lattice_q), int(order), _ptr(f), _ptr(cell_ids),
                                    int(cell_ids.numel()), _stream(stream)), "map_lbm_to_dsmc", self._h)

    # ---- inspection ---------------------------------------------------------------
    def views(self) -> _lib.Views:
        """Current buffer, cell starts and bookkeeping (completes a pending
        reseed first, on the stream of the last call)."""
        v = _lib.Views()
        check(lib().dsmc_get_views(self._h, ctypes.byref(v)), "dsmc_get_views", self._h)
        return v

    def _ws_view(self, addr: int, n: int, dtype) -> torch.Tensor:
        itemsize = torch.tensor([], dtype=dtype).element_size()
        off = addr - _ptr(self.workspace)
        return self.workspace[off:off + n * itemsize].view(dtype)

    def cell_start(self) -> torch.Tensor:
        if self.status()["moved"]:
            raise RuntimeError("the state is moved for the coming step (step(moved=True)); step() settles it")
        return self._ws_view(self.views().cell_start, self.ncells + 1, torch.int32)

    def cell_state(self):
        v = self.views()
        return (self._ws_view(v.nbar, self.ncells, torch.float64), self._ws_view(v.sigcmax, self.ncells, torch.float64),
                self._ws_view(v.rem, self.ncells, torch.float64))

    def status(self, clear: bool = False, stream=None) -> dict:
        s = _lib.Status()
        check(lib().dsmc_read_status(self._h, ctypes.byref(s), int(clear), _stream(stream)), "dsmc_read_status",
              self._h)
        return {"bits": int(s.bits), "n": int(s.n_particles), "ncoll": int(s.ncoll), "ncand": int(s.ncand),
                "nwall": int(s.nwall), "nfar": int(s.nfar), "moved": bool(s.moved)}

    def particles(self):
        """(x, y, vx, vy, vz) device views of the current, cell-sorted state."""
        st = self.status()
        if st["moved"]:
            raise RuntimeError("the state is moved for the coming step (step(moved=True)); step() settles it")
        n = st["n"]
        cur = self.views().current
        return tuple(self.state[cur, k, :n] for k in range(5))

    def set_tiling(self, particles_per_tile: int = 0, stream=None):
        """Tiles of about particles_per_tile particles (0: the default); the
        particles do not depend on it, the moment sums only to rounding."""
        check(lib().dsmc_set_tiling(self._h, int(particles_per_tile), _stream(stream)), "dsmc_set_tiling", self._h)

    def hybrid_cycle(self, f_lb: torch.Tensor, f_tmp: torch.Tensor, lbm_nx: int, tau: float, body_force_x: float,
                     dsmc_steps: int, lbm_steps: int, mapping: int = 0, order: int = 2, dsmc_column: int | None = None,
                     lattice_q: int = 9, x_buffer: int = 1, avg_out: torch.Tensor | None = None, stream=None,
                     moved: bool = False):
        """One cycle of the Section 4 coupling: this channel is the DSMC
        subdomain; f_lb[Q][lbm_nx * ny] the lattice subdomain with diffuse
        walls, its first x_buffer columns the buffer layer fed from DSMC column
        dsmc_column (default: the last) by the equilibrium mapping (mapping 0)
        or the full projection (mapping 1).  avg_out ([11][ncells], optional)
        receives the cycle's DSMC averages.  moved=True leaves the DSMC state
        moved (see step(moved=True))."""
        ny = self.cfg.ny
        assert f_lb.dtype == torch.float64 and f_lb.is_contiguous() and f_lb.shape == (lattice_q, lbm_nx * ny)
        col = self.cfg.nx - 1 if dsmc_column is None else int(dsmc_column)
        h = _lib.Hybrid(_lib.LbmConfig(int(lbm_nx), int(ny), int(lattice_q), 2 if lattice_q == 9 else 1, float(tau),
                                       float(body_force_x), int(x_buffer), 0),
                        int(dsmc_steps), int(lbm_steps), int(mapping), int(order), col, 1 if moved else 0)
        if avg_out is not None:
            assert avg_out.dtype == torch.float64 and avg_out.is_contiguous() and avg_out.shape == (NMOM, self.ncells)
        check(lib().dsmc_hybrid_cycle(self._h, ctypes.byref(h), _ptr(f_lb), _ptr(f_tmp),
                                      _ptr(avg_out) if avg_out is not None else None, _stream(stream)),
              "dsmc_hybrid_cycle", self._h)

    def graph_create(self, nsteps: int, sample_every: int = 0, stream=None, moved: bool = False):
        """Capture one step(nsteps, sample_every, moved=moved) call into a HIP
        graph on `stream` (a torch.cuda.Stream; capture cannot use the null
        stream).  A moved graph replays from a moved state and leaves it moved
        (the first replay on a settled state moves it first)."""
        fn, name = ((lib().dsmc_graph_create_moved, "dsmc_graph_create_moved") if moved else
                    (lib().dsmc_graph_create, "dsmc_graph_create"))
        check(fn(self._h, int(nsteps), int(sample_every), _stream(stream)), name, self._h)

    def graph_launch(self, stream=None):
        """Replay the captured steps from the current step."""
        check(lib().dsmc_graph_launch(self._h, _stream(stream)), "dsmc_graph_launch", self._h)

    def profile(self, enable: bool = True):
        check(lib().dsmc_profile_enable(self._h, int(enable)), "dsmc_profile_enable", self._h)

    def profile_read(self, kernel: int):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(lib().dsmc_profile_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n)), "dsmc_profile_read",
              self._h)
        return ms.value, n.value


class Batch(Channel):
    """Independent channels (replicas) of different size, particles per cell,
    Knudsen number, time step, force and seed, stepped together: every
    replica evolves bit for bit as a Channel with its parameters would.

    replicas: a list of dicts with nx, ny, ppc, kn and optionally dt,
    body_force_x (or mach), seed; common: ChannelConfig-like settings shared
    by all (kT_over_m, sigcr_max0, nbar_mode, state_bits, capacity)."""

    def __init__(self, replicas, kT_over_m: float = 1.0, sigcr_max0: float = 6.0, nbar_mode: int = 0,
                 state_bits: int = 64, capacity: int | None = None, far_capacity: int = 0, device: str = "cuda",
                 stream=None):
        from .config import body_force, time_step

        if not torch.cuda.is_available():
            raise RuntimeError("paper_1512_08042_amd needs a ROCm GPU; no CPU fallback exists")
        self.device = torch.device(device)
        self.nrep = len(replicas)
        reps = (_lib.Replica * self.nrep)()
        self.replicas = []
        npart = 0
        for i, r in enumerate(replicas):
            nx, ny, ppc, kn = int(r.get("nx", 1)), int(r["ny"]), int(r["ppc"]), float(r["kn"])
            dt = float(r["dt"]) if r.get("dt") is not None else time_step(kn, ny, kT_over_m)
            g = r.get("body_force_x")
            if g is None:
                g = body_force(kn, ny, float(r["mach"]), kT_over_m) if r.get("mach") else 0.0
            seed = int(r.get("seed", 1000 + i))
            reps[i] = _lib.Replica(nx, ny, ppc, 0, kn, dt, float(g), seed)
            self.replicas.append(dict(nx=nx, ny=ny, ppc=ppc, kn=kn, dt=dt, body_force_x=float(g), seed=seed))
            npart += nx * ny * ppc
        if capacity is None:
            capacity = int(npart * 1.05) + 1024
        self.cfg = None
        self._reps = reps
        self._c = _lib.Config(1, 1, 1, int(nbar_mode), int(capacity), 1.0, 1.0, 0.0, float(kT_over_m),
                              float(sigcr_max0), 0, 0, int(far_capacity), int(state_bits), 0)
        sz = _lib.Sizes()
        check(lib().dsmc_batch_query_sizes(ctypes.byref(self._c), reps, self.nrep, ctypes.byref(sz)),
              "dsmc_batch_query_sizes")
        self.ncells = int(sz.ncells)
        self.capacity = int(sz.capacity)
        self.state_dtype = torch.float32 if int(state_bits) == 32 else torch.float64
        self.state = torch.zeros((2, 5, self.capacity), dtype=self.state_dtype, device=self.device)
        self.workspace = torch.zeros(int(sz.workspace_bytes) + 256, dtype=torch.uint8, device=self.device)
        self._ws = (_ptr(self.workspace) + 255) & ~255
        b = _lib.Buffers()
        for i in range(2):
            for k in range(5):
                b.state[i][k] = _ptr(self.state[i, k])
        b.workspace = self._ws
        b.workspace_bytes = int(sz.workspace_bytes)
        self._h = ctypes.c_void_p()
        check(lib().dsmc_batch_init(ctypes.byref(self._c), reps, self.nrep, ctypes.byref(b), _stream(stream),
                                    ctypes.byref(self._h)), "dsmc_batch_init")
        # cell ranges of the replicas (their particle ranges follow cell_start)
        self.cell_base = []
        c = 0
        for r in self.replicas:
            self.cell_base.append(c)
            c += r["nx"] * r["ny"]
        self.cell_base.append(c)

    def replica_cells(self, r: int):
        return self.cell_base[r], self.cell_base[r + 1]

    def replica_particles(self, r: int):
        """(x, y, vx, vy, vz) device views of replica r's particles, cell-sorted."""
        c0, c1 = self.replica_cells(r)
        cs = self.cell_start()
        p0, p1 = int(cs[c0]), int(cs[c1])
        cur = self.views().current
        return tuple(self.state[cur, k, p0:p1] for k in range(5))

    def replica_cell_start(self, r: int) -> torch.Tensor:
        """cell_start of replica r relative to its first particle."""
        c0, c1 = self.replica_cells(r)
        cs = self.cell_start()[c0:c1 + 1]
        return cs - cs[0]

    def replica_counters(self, stream=None):
        """[(ncoll, ncand, nwall)] per replica since init."""
        import numpy as np

        out = np.zeros((self.nrep, 3), dtype=np.uint64)
        check(lib().dsmc_replica_counters(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                          _stream(stream)), "dsmc_replica_counters", self._h)
        return out

    def autotune(self, steps_per_trial: int = 2, sample_every: int = 0, stream=None) -> dict:
        t = _lib.Tuning()
        check(lib().dsmc_autotune(self._h, int(steps_per_trial), int(sample_every), ctypes.byref(t),
                                  _stream(stream)), "dsmc_autotune", self._h)
        return {"particles_per_tile": [t.particles_per_tile[i] for i in range(t.ncand)],
                "ms_per_step": [t.ms_per_step[i] for i in range(t.ncand)],
                "chosen": t.particles_per_tile[t.chosen]}


def project_equilibrium(avg: torch.Tensor, ppc: int, lattice_q: int, order: int = 2, kT_over_m: float = 1.0,
                        stream=None) -> torch.Tensor:
    """The equilibrium mapping of Eq. (feq_dsmc) of averages avg[11][ncells] (device FP64)."""
    assert avg.dtype == torch.float64 and avg.is_contiguous() and avg.shape[0] == NMOM
    ncells = avg.shape[1]
    out = torch.empty((lattice_q, ncells), dtype=torch.float64, device=avg.device)
    check(lib().dsmc_project_equilibrium(_ptr(avg), ncells, int(ppc), float(kT_over_m), int(lattice_q), int(order),
                                         _ptr(out), _stream(stream)), "dsmc_project_equilibrium")
    return out


def project_moments(avg: torch.Tensor, ppc: int, lattice_q: int, order: int, kT_over_m: float = 1.0,
                    stream=None) -> torch.Tensor:
    """DSMC2LB projection of given per-cell averages avg[11][ncells] (device FP64)."""
    assert avg.dtype == torch.float64 and avg.is_contiguous() and avg.shape[0] == NMOM
    ncells = avg.shape[1]
    out = torch.empty((lattice_q, ncells), dtype=torch.float64, device=avg.device)
    check(lib().dsmc_project_moments(_ptr(avg), ncells, int(ppc), float(kT_over_m), int(lattice_q), int(order),
                                     _ptr(out), _stream(stream)), "dsmc_project_moments")
    return out


def lbm_step(f: torch.Tensor, nx: int, ny: int, lattice_q: int, tau: float, body_force_x: float = 0.0,
             y_mode: int = 0, nsteps: int = 1, f_tmp: torch.Tensor | None = None, stream=None,
             x_buffer: int = 0) -> torch.Tensor:
    """nsteps BGK steps on f[Q][nx*ny] in place (returns f).  y_mode 0
    periodic, 1 held edge rows, 2 diffuse walls (D2Q9); x_buffer held inflow
    columns."""
    assert f.dtype == torch.float64 and f.is_contiguous() and f.shape == (lattice_q, nx * ny)
    if f_tmp is None:
        f_tmp = torch.empty_like(f)
    cfg = _lib.LbmConfig(int(nx), int(ny), int(lattice_q), int(y_mode), float(tau), float(body_force_x),
                         int(x_buffer), 0)
    check(lib().lbm_step(ctypes.byref(cfg), _ptr(f), _ptr(f_tmp), int(nsteps), _stream(stream)), "lbm_step")
    return f
