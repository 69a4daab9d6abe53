"""Python face of the DSMC-LBM oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads the plain-C FP64 oracle
(``oracle/dsmc_oracle.c``) and adds, in numpy, the pieces the oracle needs
that are not per-particle work:

* the Gauss-Hermite lattices (D2Q9 in closed form, D2Q37 derived here by
  solving the Gauss-Hermite moment conditions, Section 2.1 around
  Eq. (coefficients): the abscissae of the lattice must integrate the
  Hermite weight exactly up to the needed degree);
* the oracle's own reading of the run parameters (time step, body force for
  a target Mach number, LBM relaxation time of Eq. (tau)).

Nothing here is shared with the GPU package; the GPU library derives its
own tables.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dsmc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")

NMOM = 11
MOMENT_NAMES = ("N", "vx", "vy", "vxvx", "vxvy", "vyvy", "vxvxvx", "vxvxvy", "vxvyvy", "vyvyvy", "vzvz")

ST_WALL_LIMIT = 0x1
ST_CAPACITY = 0x4
ST_AR_LIMIT = 0x8
ST_NONFINITE = 0x10
ST_NNEW_LIMIT = 0x20
ST_BAD_CELL = 0x40


def build(force: bool = False, omp: bool = False) -> str:
    """Compile the oracle with contraction off and no fast-math; ``omp`` gives
    the same source built with OpenMP (its loops on all host cores)."""
    path = _OMP_PATH if omp else _LIB_PATH
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-Wno-unknown-pragmas"] + (["-fopenmp"] if omp else []) + ["-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return path


_libs = {}
_omp_default = [1]


def lib(threads=None):
    """The single-threaded oracle, or (``threads`` an int) the OpenMP build set
    to that many threads (0: OpenMP's default, OMP_NUM_THREADS if set, else
    all cores).  Both give the same bits."""
    omp = threads is not None
    L = _libs.get(omp)
    if L is None:
        L = ctypes.CDLL(build(omp=omp))
        P = ctypes.c_void_p
        d, i32, i64, u64, u32 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
        L.or_create.restype = P
        L.or_create.argtypes = [i32, i32, i32, i32, i64, d, d, d, d, d, u64, i32]
        L.or_set_state32.argtypes = [P, i32]
        L.or_destroy.argtypes = [P]
        L.or_init_maxwell.argtypes = [P]
        L.or_load.argtypes = [P, i64, P, P, P, P, P]
        L.or_load.restype = ctypes.c_int
        L.or_step.argtypes = [P, i32, i32]
        L.or_sample_now.argtypes = [P]
        L.or_averages.argtypes = [P, P]
        L.or_reset_moments.argtypes = [P]
        L.or_count.argtypes = [P]
        L.or_count.restype = i64
        L.or_get_particles.argtypes = [P, P, P, P, P, P]
        L.or_get_cells.argtypes = [P, P, P, P, P]
        L.or_set_cells.argtypes = [P, P, P, P]
        L.or_get_counters.argtypes = [P, P]
        L.or_set_step.argtypes = [P, i64]
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_u53.argtypes = [u32, u32]
        L.or_u53.restype = d
        L.or_box_muller.argtypes = [d, d, P]
        L.or_dsmc2lb.argtypes = [P, i32, i32, d, i32, i32, P, P, P]
        L.or_grad_params.argtypes = [P, i64, i32, i32, P, P]
        L.or_grad_G.argtypes = [P, d, d]
        L.or_grad_G.restype = d
        L.or_ar_sample_batch.argtypes = [u64, P, u32, u32, i64, i32, P, P]
        L.or_ar_sample_batch.restype = i64
        L.or_lb2dsmc.argtypes = [P, i32, i32, P, P, P, i32]
        L.or_lb2dsmc.restype = ctypes.c_int
        L.or_lbm_step.argtypes = [i32, i32, i32, P, P, P, P, d, d, i32, i32, P, P, i32]
        L.or_dsmc2lb_eq.argtypes = [P, i32, i32, d, i32, i32, P, P, P]
        L.or_threads.argtypes = [i32]
        L.or_threads.restype = i32
        if omp:
            _omp_default[0] = int(L.or_threads(0))  # OMP_NUM_THREADS, else all cores
        _libs[omp] = L
    if omp:
        L.or_threads(int(threads) if threads else _omp_default[0])
    return L


def threads_in_use(threads=None) -> int:
    """Threads the oracle build selected by ``threads`` runs its loops on."""
    return int(lib(threads).or_threads(0))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def u53(a: int, b: int) -> float:
    return lib().or_u53(a, b)


def box_muller(r1: float, r2: float):
    out = np.zeros(2)
    lib().or_box_muller(r1, r2, _ptr(out))
    return out


# --------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------
# Velocity ordering (the interface order of populations f[a]): shells of
# increasing |e|, counter-clockwise within a shell starting from the first
# octant representative.
_SHELLS_37 = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)]


def _shell(p: int, q: int):
    if p == 0 and q == 0:
        return [(0, 0)]
    if q == 0:
        return [(p, 0), (0, p), (-p, 0), (0, -p)]
    if p == q:
        return [(p, p), (-p, p), (-p, -p), (p, -p)]
    return [(p, q), (q, p), (-q, p), (-p, q), (-p, -q), (-q, -p), (q, -p), (p, -q)]


def _dfact(n: int) -> float:
    """(n-1)!! for even n: the n-th moment of the unit Gaussian."""
    if n % 2:
        return 0.0
    v = 1.0
    for k in range(n - 1, 0, -2):
        v *= k
    return v


def lattice(q: int):
    """Return dict(e=int[Q,2], w=float[Q], r=float, xi=float[Q,2])."""
    if q == 9:
        e = np.array(_shell(0, 0) + _shell(1, 0) + _shell(1, 1), dtype=np.int32)
        w = np.array([4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4)
        r = math.sqrt(3.0)
    elif q == 37:
        e, w, r = _derive_d2q37()
    else:
        raise ValueError("lattice must be 9 or 37")
    xi = np.ascontiguousarray(r * e.astype(np.float64))
    return {"e": np.ascontiguousarray(e, dtype=np.int32), "w": np.ascontiguousarray(w), "r": r, "xi": xi, "Q": q}


_D2Q37 = None
_CONDS_37 = [(0, 0), (2, 0), (4, 0), (2, 2), (6, 0), (4, 2), (8, 0), (6, 2), (4, 4)]


def _system_37(r: float):
    shells = [_shell(p, q) for (p, q) in _SHELLS_37]
    A = np.zeros((len(_CONDS_37), len(shells)))
    b = np.zeros(len(_CONDS_37))
    for i, (p, q) in enumerate(_CONDS_37):
        for s, sh in enumerate(shells):
            A[i, s] = sum((r * ex) ** p * (r * ey) ** q for (ex, ey) in sh)
        b[i] = _dfact(p) * _dfact(q)
    return A, b


def _refine_decimal(W, r, digits=50, iters=6):
    """Newton steps on A(r) W = b in 50-digit decimal arithmetic, so that the
    returned doubles are the correctly rounded solution."""
    import decimal

    ctx = decimal.Context(prec=digits)
    D = ctx.create_decimal
    shells = [_shell(p, q) for (p, q) in _SHELLS_37]
    S = [[D(sum(ex ** p * ey ** q for (ex, ey) in sh)) for sh in shells] for (p, q) in _CONDS_37]
    b = [D(int(_dfact(p) * _dfact(q))) for (p, q) in _CONDS_37]
    deg = [p + q for (p, q) in _CONDS_37]
    x = [D(float(v)) for v in W] + [D(float(r))]
    for _ in range(iters):
        rr = x[8]
        rp = [ctx.power(rr, d) for d in deg]
        F = [ctx.subtract(sum((rp[i] * S[i][s] * x[s] for s in range(8)), D(0)), b[i]) for i in range(9)]
        J = [[rp[i] * S[i][s] for s in range(8)] +
             [sum((D(deg[i]) * rp[i] / rr * S[i][s] * x[s] for s in range(8)), D(0))] for i in range(9)]
        # Gaussian elimination with partial pivoting on J dx = F
        M = [J[i] + [F[i]] for i in range(9)]
        for col in range(9):
            piv = max(range(col, 9), key=lambda i: abs(M[i][col]))
            M[col], M[piv] = M[piv], M[col]
            for i in range(9):
                if i != col:
                    f = M[i][col] / M[col][col]
                    M[i] = [a - f * c for a, c in zip(M[i], M[col])]
        dx = [M[i][9] / M[i][i] for i in range(9)]
        x = [a - d for a, d in zip(x, dx)]
    return np.array([float(v) for v in x[:8]]), float(x[8])


def _derive_d2q37():
    """Gauss-Hermite conditions for the 37-speed 2-D lattice.

    Unknowns: 8 shell weights and the scale r of xi = r e.  Conditions: the
    lattice integrates x^p y^q exactly against the unit Gaussian for the even
    (p, q) listed in _CONDS_37 (odd moments vanish by symmetry, the mirror
    (q, p) follows from the x<->y symmetry of the shells), i.e. every monomial
    of degree <= 9.  For fixed r the conditions are linear in the weights; r
    is the root of det[A(r) | b] near 1.2, found by bisection.
    """
    global _D2Q37
    if _D2Q37 is not None:
        return _D2Q37

    def det(r):
        A, b = _system_37(r)
        return np.linalg.det(np.column_stack([A, b]))

    lo, hi = 1.15, 1.25
    flo, fhi = det(lo), det(hi)
    if flo * fhi > 0:
        raise RuntimeError("D2Q37 scale root not bracketed")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = det(mid)
        if fm == 0.0 or hi - lo < 1e-17:
            break
        if flo * fm < 0:
            hi, fhi = mid, fm
        else:
            lo, flo = mid, fm
    r = 0.5 * (lo + hi)
    A, b = _system_37(r)
    W, *_ = np.linalg.lstsq(A, b, rcond=None)
    # Newton on all nine unknowns (W, r) of A(r) W = b, rows scaled by b,
    # to bring the residual to rounding level.
    deg = np.array([p + q for (p, q) in _CONDS_37], dtype=np.float64)
    for _ in range(8):
        A, b = _system_37(r)
        F = (A @ W - b) / b
        J = np.column_stack([A, (deg / r) * (A @ W)]) / b[:, None]
        step = np.linalg.solve(J, F)
        W = W - step[:8]
        r = r - step[8]
    W, r = _refine_decimal(W, r)
    e, w = [], []
    for (p, q), ws in zip(_SHELLS_37, W):
        for v in _shell(p, q):
            e.append(v)
            w.append(ws)
    _D2Q37 = (np.array(e, dtype=np.int32), np.array(w), float(r))
    return _D2Q37


# --------------------------------------------------------------------------
# run parameters (the oracle's reading)
# --------------------------------------------------------------------------
def mean_free_path(kn: float, ny: int) -> float:
    return kn * float(ny)


def default_dt(kn: float, ny: int, kT: float = 1.0) -> float:
    """dt = min(0.25 dx / sqrt(2kT/m), 0.2 lambda / cbar), cbar = sqrt(8kT/(pi m))."""
    lam = mean_free_path(kn, ny)
    return min(0.25 / math.sqrt(2.0 * kT), 0.2 * lam / math.sqrt(8.0 * kT / math.pi))


def hs_viscosity(kn: float, ny: int, kT: float = 1.0) -> float:
    """Chapman-Enskog hard-sphere kinematic viscosity (5/16) sqrt(2 pi) 1.016 lambda sqrt(kT/m)."""
    return (5.0 / 16.0) * math.sqrt(2.0 * math.pi) * 1.016 * mean_free_path(kn, ny) * math.sqrt(kT)


def body_force_for_mach(kn: float, ny: int, mach: float, kT: float = 1.0) -> float:
    """g giving centreline speed Ma sqrt(kT/m) for a no-slip parabola: u_max = g H^2 / (8 nu)."""
    return 8.0 * hs_viscosity(kn, ny, kT) * mach * math.sqrt(kT) / float(ny) ** 2


def lbm_tau(kn: float, ny: int, r: float) -> float:
    """Eq. (tau): tau = sqrt(pi/8) (c/c_s) Kn H + 1/2, with c/c_s = r."""
    return math.sqrt(math.pi / 8.0) * r * kn * float(ny) + 0.5


# --------------------------------------------------------------------------
# DSMC simulation
# --------------------------------------------------------------------------
class Sim:
    def __init__(self, nx, ny, ppc, kn, dt=None, g=0.0, kT=1.0, sigcr0=6.0, seed=1, capacity=None,
                 nbar_mode=0, ar_max_tries=65536, state32=False, threads=None):
        """state32: particle values are stored in FP32 (every write rounds to the
        nearest float); the arithmetic stays FP64.  threads: None runs the
        single-threaded build, an int the OpenMP build on that many threads
        (0 = OpenMP's default), with the same results bit for bit."""
        self.threads = threads
        self.nx, self.ny, self.ppc = int(nx), int(ny), int(ppc)
        self.ncells = self.nx * self.ny
        self.kn, self.kT, self.g = float(kn), float(kT), float(g)
        self.dt = float(dt) if dt is not None else default_dt(kn, ny, kT)
        self.capacity = int(capacity) if capacity is not None else self.ncells * self.ppc * 2 + 64
        self.seed = int(seed)
        self._h = self._lib().or_create(self.nx, self.ny, self.ppc, int(nbar_mode), self.capacity, self.kn, self.dt,
                                  self.g, self.kT, float(sigcr0), self.seed, int(ar_max_tries))
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        self.state32 = bool(state32)
        self._lib().or_set_state32(self._h, 1 if self.state32 else 0)
        self._destroy = self._lib().or_destroy  # held: at interpreter exit the module may be gone

    def _lib(self):
        return lib(self.threads)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def init_maxwell(self):
        self._lib().or_init_maxwell(self._h)

    def load(self, x, y, vx, vy, vz):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, vx, vy, vz)]
        rc = self._lib().or_load(self._h, len(arrs[0]), *[_ptr(a) for a in arrs])
        if rc != 0:
            raise ValueError("load failed")

    def step(self, nsteps=1, sample_every=0):
        self._lib().or_step(self._h, int(nsteps), int(sample_every))

    def sample_now(self):
        self._lib().or_sample_now(self._h)

    @property
    def n(self):
        return int(self._lib().or_count(self._h))

    def particles(self):
        n = self.n
        out = [np.zeros(n) for _ in range(5)]
        self._lib().or_get_particles(self._h, *[_ptr(a) for a in out])
        return out

    def cells(self):
        cs = np.zeros(self.ncells + 1, dtype=np.int32)
        nbar, sig, rem = (np.zeros(self.ncells) for _ in range(3))
        self._lib().or_get_cells(self._h, _ptr(cs), _ptr(nbar), _ptr(sig), _ptr(rem))
        return cs, nbar, sig, rem

    def set_cells(self, nbar, sigcmax, rem):
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (nbar, sigcmax, rem)]
        self._lib().or_set_cells(self._h, *[_ptr(v) for v in a])

    def counters(self):
        out = np.zeros(8, dtype=np.int64)
        self._lib().or_get_counters(self._h, _ptr(out))
        keys = ("step", "nsamples", "ncoll", "ncand", "nwall", "reseed_events", "status", "n")
        return dict(zip(keys, (int(v) for v in out)))

    def set_step(self, step):
        self._lib().or_set_step(self._h, int(step))

    def averages(self):
        out = np.zeros((NMOM, self.ncells))
        self._lib().or_averages(self._h, _ptr(out))
        return out

    def reset_moments(self):
        self._lib().or_reset_moments(self._h)

    def lb2dsmc(self, lat, order, f, cells):
        f = np.ascontiguousarray(f, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        assert f.shape == (lat["Q"], self.ncells)
        return self._lib().or_lb2dsmc(self._h, lat["Q"], int(order), _ptr(lat["xi"]), _ptr(f), _ptr(cells), len(cells))


def dsmc2lb(avg, ppc, lat, order, kT=1.0, threads=None):
    avg = np.ascontiguousarray(avg, dtype=np.float64)
    ncells = avg.shape[1]
    f = np.zeros((lat["Q"], ncells))
    lib(threads).or_dsmc2lb(_ptr(avg), ncells, int(ppc), float(kT), lat["Q"], int(order), _ptr(lat["w"]),
                     _ptr(lat["xi"]), _ptr(f))
    return f


def grad_params(f_node, lat, order):
    f = np.ascontiguousarray(f_node, dtype=np.float64)
    out = np.zeros(12)
    lib().or_grad_params(_ptr(f), 1, lat["Q"], int(order), _ptr(lat["xi"]), _ptr(out))
    return out


def grad_G(prm, x, y):
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    return lib().or_grad_G(_ptr(prm), float(x), float(y))


def ar_sample(prm, n, seed=1, cell=0, event=0, max_tries=65536):
    prm = np.ascontiguousarray(prm, dtype=np.float64)
    xi = np.zeros((n, 2))
    st = np.zeros(1, dtype=np.uint32)
    tries = lib().or_ar_sample_batch(int(seed), _ptr(prm), int(cell), int(event), int(n), int(max_tries), _ptr(xi),
                                     _ptr(st))
    return xi, int(tries), int(st[0])


def lbm_step(f, lat, nx, ny, tau, gx, y_mode, nsteps, x_buffer=0, threads=None):
    f = np.array(f, dtype=np.float64, copy=True, order="C")
    assert f.shape == (lat["Q"], nx * ny)
    tmp = np.zeros_like(f)
    e = lat["e"]
    ex = np.ascontiguousarray(e[:, 0], dtype=np.int32)
    ey = np.ascontiguousarray(e[:, 1], dtype=np.int32)
    lib(threads).or_lbm_step(int(nx), int(ny), lat["Q"], _ptr(ex), _ptr(ey), _ptr(lat["w"]), _ptr(lat["xi"]), float(tau),
                      float(gx), int(y_mode), int(x_buffer), _ptr(f), _ptr(tmp), int(nsteps))
    return f


def dsmc2lb_eq(avg, ppc, lat, order=2, kT=1.0, threads=None):
    """The equilibrium mapping of Eq. (feq_dsmc) (order 2; order 3 adds the
    third-order equilibrium term)."""
    avg = np.ascontiguousarray(avg, dtype=np.float64)
    ncells = avg.shape[1]
    f = np.zeros((lat["Q"], ncells))
    lib(threads).or_dsmc2lb_eq(_ptr(avg), ncells, int(ppc), float(kT), lat["Q"], int(order), _ptr(lat["w"]),
                        _ptr(lat["xi"]), _ptr(f))
    return f
