// Host side of libdsmc: the C ABI declared in include/dsmc.h.
// Built as one translation unit with the kernel sources (unity build), so
// every kernel is launched from the unit that defines it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/dsmc.h"
#include "dsmc_device.hpp"
#include "step_kernels.hpp"
#include "step_kernels.hip"
#include "map_kernels.hip"
#include "adjoint_kernels.hip"

using namespace dsmc;

namespace {

// ---- lattices -----------------------------------------------------------------
// Ordering (the ABI order of populations): shells of increasing |e|, counter-
// clockwise within a shell from the first-octant representative.
void shell(int p, int q, std::vector<int> &ex, std::vector<int> &ey)
{
    auto add = [&](int a, int b) {
        ex.push_back(a);
        ey.push_back(b);
    };
    if (p == 0 && q == 0) {
        add(0, 0);
    } else if (q == 0) {
        add(p, 0), add(0, p), add(-p, 0), add(0, -p);
    } else if (p == q) {
        add(p, p), add(-p, p), add(-p, -p), add(p, -p);
    } else {
        add(p, q), add(q, p), add(-q, p), add(-p, q), add(-p, -q), add(-q, -p), add(q, -p), add(p, -q);
    }
}

const int SHELLS37[8][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}, {3, 0}, {3, 1}};

long double gauss_moment(int n)  // (n-1)!! for even n
{
    if (n % 2) return 0.0L;
    long double v = 1.0L;
    for (int k = n - 1; k > 0; k -= 2) v *= (long double)k;
    return v;
}

// sum over shell s of e_x^p e_y^q
long double shell_moment(int s, int p, int q)
{
    std::vector<int> ex, ey;
    shell(SHELLS37[s][0], SHELLS37[s][1], ex, ey);
    long double acc = 0.0L;
    for (size_t i = 0; i < ex.size(); ++i) acc += powl((long double)ex[i], p) * powl((long double)ey[i], q);
    return acc;
}

// D2Q37 by the Gauss-Hermite conditions: for a trial scale r the shell
// weights follow from eight moment conditions (a linear solve; this subset
// of the degree <= 8 conditions is the well-conditioned one), and r is the
// root of the residual of the ninth condition, x^8, found by secant
// iteration in extended precision.
bool d2q37_weights(long double r, long double W[8], long double *resid)
{
    static const int cond[8][2] = {{0, 0}, {2, 0}, {4, 0}, {2, 2}, {6, 0}, {4, 2}, {6, 2}, {4, 4}};
    long double A[8][9];
    for (int i = 0; i < 8; ++i) {
        const int p = cond[i][0], q = cond[i][1];
        const long double rp = powl(r, p + q);
        for (int s = 0; s < 8; ++s) A[i][s] = rp * shell_moment(s, p, q);
        A[i][8] = gauss_moment(p) * gauss_moment(q);
    }
    for (int col = 0; col < 8; ++col) {
        int piv = col;
        for (int i = col + 1; i < 8; ++i)
            if (fabsl(A[i][col]) > fabsl(A[piv][col])) piv = i;
        if (A[piv][col] == 0.0L) return false;
        if (piv != col)
            for (int k = 0; k < 9; ++k) {
                const long double t = A[col][k];
                A[col][k] = A[piv][k];
                A[piv][k] = t;
            }
        for (int i = 0; i < 8; ++i) {
            if (i == col) continue;
            const long double m = A[i][col] / A[col][col];
            for (int k = col; k < 9; ++k) A[i][k] -= m * A[col][k];
        }
    }
    for (int s = 0; s < 8; ++s) W[s] = A[s][8] / A[s][s];
    long double m80 = 0.0L;
    for (int s = 0; s < 8; ++s) m80 += W[s] * shell_moment(s, 8, 0);
    *resid = m80 * powl(r, 8) - gauss_moment(8);
    return true;
}

bool make_lattice(int Q, Lattice &L)
{
    std::memset(&L, 0, sizeof(L));
    std::vector<int> ex, ey;
    std::vector<long double> w;
    long double r;
    if (Q == 9) {
        shell(0, 0, ex, ey), shell(1, 0, ex, ey), shell(1, 1, ex, ey);
        w = {4.0L / 9.0L, 1.0L / 9.0L, 1.0L / 9.0L, 1.0L / 9.0L, 1.0L / 9.0L,
             1.0L / 36.0L, 1.0L / 36.0L, 1.0L / 36.0L, 1.0L / 36.0L};
        L.Q = 9;
        L.r = std::sqrt(3.0);
        for (int a = 0; a < 9; ++a) {
            L.w[a] = (double)w[a];
            L.xi[a][0] = L.r * (double)ex[a];
            L.xi[a][1] = L.r * (double)ey[a];
        }
        return true;
    }
    if (Q != 37) return false;
    long double r0 = 1.18L, r1 = 1.21L, W[8], f0, f1;
    if (!d2q37_weights(r0, W, &f0) || !d2q37_weights(r1, W, &f1)) return false;
    for (int it = 0; it < 100; ++it) {
        if (f1 == f0) break;
        const long double r2 = r1 - f1 * (r1 - r0) / (f1 - f0);
        r0 = r1, f0 = f1;
        r1 = r2;
        if (!d2q37_weights(r1, W, &f1)) return false;
        if (fabsl(r1 - r0) < 1e-19L * r1) break;
    }
    r = r1;
    if (!d2q37_weights(r, W, &f1)) return false;
    for (int s = 0; s < 8; ++s) {
        std::vector<int> sx, sy;
        shell(SHELLS37[s][0], SHELLS37[s][1], sx, sy);
        for (size_t i = 0; i < sx.size(); ++i) {
            ex.push_back(sx[i]);
            ey.push_back(sy[i]);
            w.push_back(W[s]);
        }
    }
    L.Q = 37;
    L.r = (double)r;
    for (int a = 0; a < 37; ++a) {
        L.w[a] = (double)w[a];
        L.xi[a][0] = L.r * (double)ex[a];
        L.xi[a][1] = L.r * (double)ey[a];
    }
    return true;
}

template <int Q>
int first_of_shell(int s)
{
    for (int a = 0; a < Q; ++a)
        if (VelSet<Q>::sh[a] == s) return a;
    return 0;
}

struct LatticeTables {
    Lattice q9, q37;
    int e9[9][2], e37[37][2];
    bool ok;
    LatticeTables()
    {
        ok = make_lattice(9, q9) && make_lattice(37, q37);
        for (int a = 0; a < 9; ++a) {
            e9[a][0] = (int)std::lround(q9.xi[a][0] / q9.r);
            e9[a][1] = (int)std::lround(q9.xi[a][1] / q9.r);
        }
        for (int a = 0; a < 37; ++a) {
            e37[a][0] = (int)std::lround(q37.xi[a][0] / q37.r);
            e37[a][1] = (int)std::lround(q37.xi[a][1] / q37.r);
        }
        // the lattice kernels' compile-time velocity sets and shell indices
        // must describe these tables exactly
        for (int a = 0; a < 9; ++a)
            ok = ok && e9[a][0] == VelSet<9>::ex[a] && e9[a][1] == VelSet<9>::ey[a] &&
                 q9.w[a] == q9.w[first_of_shell<9>(VelSet<9>::sh[a])];
        for (int a = 0; a < 37; ++a)
            ok = ok && e37[a][0] == VelSet<37>::ex[a] && e37[a][1] == VelSet<37>::ey[a] &&
                 q37.w[a] == q37.w[first_of_shell<37>(VelSet<37>::sh[a])];
    }
};

const LatticeTables &tables()
{
    static const LatticeTables t;
    return t;
}

// ---- configuration and workspace ---------------------------------------------
size_t al(size_t x) { return (x + 255) & ~size_t(255); }

bool valid_config(const dsmc_config *c)
{
    if (!c) return false;
    if (c->nx < 1 || c->ny < 1 || c->ppc < 1) return false;
    if ((int64_t)c->nx * (int64_t)c->ny > (int64_t)0x3FFFFFFF) return false;
    if (c->capacity < 1 || c->capacity > (int64_t)0x7FFFFFFF) return false;
    if (!(c->kn > 0.0) || !(c->dt > 0.0) || !(c->kT_over_m > 0.0) || !(c->sigcr_max0 > 0.0)) return false;
    if (!std::isfinite(c->kn) || !std::isfinite(c->dt) || !std::isfinite(c->body_force_x)) return false;
    if (!std::isfinite(c->kT_over_m) || !std::isfinite(c->sigcr_max0)) return false;
    if (c->nbar_mode != 0 && c->nbar_mode != 1) return false;
    if (c->state_bits != 0 && c->state_bits != 32 && c->state_bits != 64) return false;
    return true;
}

bool state32(const dsmc_config &c) { return c.state_bits == 32; }

int far_cap_of(const dsmc_config &c)
{
    if (c.far_capacity > 0) return c.far_capacity;
    return (int)(c.capacity < 65536 ? c.capacity : 65536);
}

struct Layout {
    size_t cs0, cs1, grp0, grp1, plan, countnew, farcnt, blocksum, far0, far1, nbar, sigcmax, rem, mom, mark, prm, nnew,
        perm, tstat, kc, ctr, rep, tiles, cell_rep, rstat, comp, complist, appoff, total;
};

// nc: cells of all channels together; nrep: channels
Layout make_layout(const dsmc_config &c, size_t nc, size_t nrep)
{
    const size_t nblk = (nc + 255) / 256;
    const size_t cap = (size_t)c.capacity;
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += al(bytes);
        return at;
    };
    L.cs0 = take((nc + 1) * 4);
    L.cs1 = take((nc + 1) * 4);
    L.grp0 = take(GSTRIDE * nc * 4);
    L.grp1 = take(GSTRIDE * nc * 4);
    L.plan = take(2 * NDIR * nc * 4);
    L.countnew = take(nc * 4);
    L.farcnt = take(2 * nc * 4);
    L.blocksum = take(nblk * 4);
    L.far0 = take((size_t)far_cap_of(c) * 16);
    L.far1 = take((size_t)far_cap_of(c) * 16);
    L.nbar = take(nc * 8);
    L.sigcmax = take(nc * 8);
    L.rem = take(nc * 8);
    L.mom = take(NMOM * nc * 8);
    L.mark = take(nc * 4);
    L.prm = take(nc * 12 * 8);
    L.nnew = take(nc * 4);
    L.perm = take(cap * 12);  // adoption: permutation + cell ids; steps: scratch of oversized tiles
    L.tstat = take(3 * nc * 8);  // per step tile, at its first cell
    L.kc = take(REP_OFFSET + nrep * sizeof(RepConst));  // TileConst, then the channels' constants
    L.ctr = take(sizeof(Counters));
    L.rep = L.kc + REP_OFFSET;
    L.tiles = take(2 * TILE_WORDS * nc * 4);  // at most one tile per cell, in two orders (see set_tiling)
    L.cell_rep = take(nc * 4);
    L.rstat = take(3 * nrep * 8);
    L.comp = take(nc * 4);      // completion of a moved state: reasons per cell,
    L.complist = take(nc * 4);  // the listed cells,
    L.appoff = take(nc * 4);    // a moved reseed's appended particles per list entry
    L.total = o;
    return L;
}

bool valid_replica(const dsmc_replica &r)
{
    if (r.nx < 1 || r.ny < 1 || r.ppc < 1) return false;
    if ((int64_t)r.nx * (int64_t)r.ny > (int64_t)0x3FFFFFFF) return false;
    if (!(r.kn > 0.0) || !(r.dt > 0.0) || !std::isfinite(r.kn) || !std::isfinite(r.dt)) return false;
    return std::isfinite(r.body_force_x);
}

// the channels of a batch: common settings valid, every replica valid, the
// cells and the initial particles within the limits
bool valid_batch(const dsmc_config *c, const dsmc_replica *reps, int32_t nrep, int64_t *ncells, int64_t *npart)
{
    if (!c || !reps || nrep < 1) return false;
    if (c->capacity < 1 || c->capacity > (int64_t)0x7FFFFFFF) return false;
    if (!(c->kT_over_m > 0.0) || !(c->sigcr_max0 > 0.0)) return false;
    if (!std::isfinite(c->kT_over_m) || !std::isfinite(c->sigcr_max0)) return false;
    if (c->nbar_mode != 0 && c->nbar_mode != 1) return false;
    if (c->state_bits != 0 && c->state_bits != 32 && c->state_bits != 64) return false;
    int64_t nc = 0, np = 0;
    for (int32_t r = 0; r < nrep; ++r) {
        if (!valid_replica(reps[r])) return false;
        nc += (int64_t)reps[r].nx * reps[r].ny;
        np += (int64_t)reps[r].nx * reps[r].ny * reps[r].ppc;
        if (nc > (int64_t)0x3FFFFFFF) return false;
    }
    *ncells = nc;
    *npart = np;
    return true;
}

dsmc_replica replica_of(const dsmc_config &c)
{
    dsmc_replica r;
    std::memset(&r, 0, sizeof(r));
    r.nx = c.nx;
    r.ny = c.ny;
    r.ppc = c.ppc;
    r.kn = c.kn;
    r.dt = c.dt;
    r.body_force_x = c.body_force_x;
    r.seed = c.seed;
    return r;
}

struct ProfRec {
    int kid;
    hipEvent_t a, b;
};

// Why the current call failed, set where the failure is found: a static
// string, or null for a HIP runtime error (whose own message is taken).
thread_local const char *t_reason = nullptr;

inline int fail(int code, const char *why)
{
    t_reason = why;
    return code;
}

}  // namespace

struct dsmc_ctx {
    dsmc_config cfg;
    void *st[2][5];  // double, or float when state32
    int32_t *cs[2];
    int32_t *grp[2], *plan, *countnew, *farcnt, *blocksum, *far[2], *mark, *nnew, *perm;
    int32_t *comp, *complist, *appoff;
    double *nbar, *sigcmax, *rem, *mom, *prm;
    Counters *ctr;
    unsigned long long *tstat;
    TileConst *kc;       // device copy of kc_host
    TileConst kc_host;
    int ncells, nblk, far_cap, ntiles;
    double K, s_th;  // K of a single channel (reseed)
    Geometry G;      // geometry of a single channel (reseed, adoption)
    int cur;
    // the channels (one, or the replicas of a batch) and the step tiles:
    // tiles are grouped by shape (TC cells, CH 64-slot chunks of LDS stage),
    // one launch per group
    int nrep;
    std::vector<RepConst> reps;
    RepConst *rep;
    int32_t *tiles, *cell_rep;
    unsigned long long *rstat;
    struct TileGroup {
        int tc, ch, tile0, ntiles;
    };
    std::vector<TileGroup> groups;
    // batches: the tile groups after the first run on side streams forked
    // from the caller's stream and joined back into it (one launch's tail
    // overlaps the next group's work); default priority, created at init
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
    bool forked = false;  // side streams and events exist
    std::vector<int32_t> tiles_host;       // the step's order, then the classify pass's
    int particles_per_tile;
    // a captured step graph: nsteps steps (a dsmc_step call) replayable from
    // any even step aligned with its sampling period
    bool capturing;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    int32_t g_nsteps, g_sample_every, g_cur;
    bool g_moved;  // captured from dsmc_graph_create_moved: replays a moved state and leaves it moved
    int64_t step, nsamples, reseed_events;
    // Inside a dsmc_step call the state between steps is kept already moved
    // for the coming step and partitioned by direction inside every cell
    // (with its group sizes and long-jump list, buffers of parity step & 1);
    // at the end of a dsmc_step call it is settled (moved particles sorted
    // into their cells, collided and sampled), at the end of a
    // dsmc_step_moved call it stays moved.  `classified`: the state is moved.
    bool classified;
    // A reseed leaves the state pending: buffer cur still holds the old
    // particles (cell starts cs[cur]), buffer 1 - cur the marked cells' new
    // particles at their slots after the reseed (cell starts cs[1 - cur]),
    // and the marks and the reseed's error flag are set.  The next step's
    // classify pass completes it (it reads every particle anyway); any other
    // call that reads particles or cell starts settles it first with a copy.
    bool pending;
    // A moved state of one channel may have cells left for the completion
    // pass (k_complete, run before the next step): tiles that ended unmoved
    // (STEP_DEFER) and, after a reseed of the moved state (comp_reseed), the
    // replaced cells, whose new particles sit after the state's last slot.
    bool comp_pending, comp_reseed;
    // the step kernels read the state with non-temporal loads (a state buffer
    // of the nominal particle count below 384 MB, 1.5 x the memory-side cache)
    bool nt_loads;
    hipStream_t last;
    bool prof;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    char err[320];  // what the last failing call reported (dsmc_last_error)
};

namespace {

inline hipStream_t S(void *s) { return (hipStream_t)s; }

// records a failing call's message in the context (dsmc_last_error)
int noted(dsmc_ctx *x, const char *call, int rc)
{
    if (rc != DSMC_OK && x) {
        const char *why = t_reason;
        if (!why) why = rc == DSMC_EHIP ? hipGetErrorString(hipPeekAtLastError()) : "rejected";
        std::snprintf(x->err, sizeof(x->err), "%s: %s (%s)", call, why, dsmc_strerror(rc));
    }
    t_reason = nullptr;
    return rc;
}

template <class F>
int launch(dsmc_ctx *x, int kid, hipStream_t s, F &&f)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = x && x->prof && kid >= 0;
    if (timed) {
        for (hipEvent_t *e : {&e0, &e1}) {
            if (!x->pool.empty()) {
                *e = x->pool.back();
                x->pool.pop_back();
            } else if (hipEventCreate(e) != hipSuccess) {
                return DSMC_EHIP;
            }
        }
        if (hipEventRecord(e0, s) != hipSuccess) return DSMC_EHIP;
    }
    f();
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DSMC_EHIP, hipGetErrorString(e));
    if (timed) {
        if (hipEventRecord(e1, s) != hipSuccess) return DSMC_EHIP;
        x->recs.push_back(ProfRec{kid, e0, e1});
    }
    return DSMC_OK;
}

#define TRY(expr)                  \
    do {                           \
        const int rc_ = (expr);    \
        if (rc_ != DSMC_OK) return rc_; \
    } while (0)

inline unsigned grid_cells_wave(int ncells) { return (unsigned)((ncells + 3) / 4); }
inline unsigned grid_threads(size_t n) { return (unsigned)((n + 255) / 256); }

StepArgs step_args(const dsmc_ctx *x, int32_t cur, int64_t step, bool sample, bool classify)
{
    StepArgs a;
    a.kc = x->kc;
    a.tiles = x->tiles;
    a.r = 0;
    a.dev_step = x->capturing ? 1 : 0;
    a.reseed = 0;
    a.flags = 0;
    a.step = (uint32_t)step;
    a.cur = cur;
    a.sample = sample ? 1 : 0;
    a.classify = classify ? 1 : 0;
    return a;
}

// the fixed part of every step-kernel launch, copied to the workspace
int upload_tile_const(dsmc_ctx *x, hipStream_t s)
{
    TileConst &k = x->kc_host;
    for (int b = 0; b < 2; ++b) {
        for (int j = 0; j < 5; ++j) k.st[b][j] = x->st[b][j];
        k.cs[b] = x->cs[b];
        k.grp[b] = x->grp[b];
        k.far[b] = x->far[b];
        k.farcnt[b] = x->farcnt + (size_t)b * x->ncells;
    }
    k.plan = x->plan;
    k.scr = (double *)x->perm;
    k.scr_i = (int32_t *)((char *)x->perm + (size_t)x->cfg.capacity * 8);
    k.ctr = x->ctr;
    k.tstat = x->tstat;
    k.mom = x->mom;
    k.nbar = x->nbar;
    k.sigcmax = x->sigcmax;
    k.rem = x->rem;
    k.mark = x->mark;
    k.comp = x->comp;
    k.complist = x->complist;
    k.appoff = x->appoff;
    k.nnew = x->nnew;
    k.cap = (int)std::min<int64_t>(x->cfg.capacity, 0x7fffffff);
    k.rep = x->rep;
    k.s_th = x->s_th;
    k.nbar_mode = x->cfg.nbar_mode;
    k.ncells = x->ncells;
    k.far_cap = x->far_cap;
    k.nrep = x->nrep;
    return hipMemcpyAsync(x->kc, &k, sizeof(TileConst), hipMemcpyHostToDevice, s) == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

// the tile shape (TC, CH) a channel of ppc particles per cell gets for a
// target of about `ppt` particles per tile (from the shapes instantiated for
// each state type): as many cells as fit the target, then the LDS stage
// that holds them with a quarter to spare
void tile_shape(bool f32, int ppc, int ppt, int &tc, int &ch)
{
    tc = 4;
    while (tc > 1 && tc * ppc > ppt) tc /= 2;
    const bool small = (double)tc * ppc * 1.25 <= 256.0;
    if (f32) {
        ch = (tc == 4 && small) ? 4 : 8;
    } else {
        while (tc > 1 && (double)tc * ppc * 1.25 > 256.0) tc /= 2;  // FP64 stages of 512 slots are single-cell
        ch = (double)tc * ppc * 1.25 <= 256.0 ? 4 : 8;
    }
}

// releases a captured step graph, after the work enqueued on the context's
// last stream (where a replay runs) has finished
int release_graph(dsmc_ctx *x)
{
    if (!x->gexec && !x->graph) return DSMC_OK;
    if (hipStreamSynchronize(x->last) != hipSuccess) return DSMC_EHIP;
    if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
    if (x->graph) (void)hipGraphDestroy(x->graph);
    x->gexec = nullptr;
    x->graph = nullptr;
    x->g_nsteps = 0;
    return DSMC_OK;
}

// Builds the tile groups for a target of ppt particles per tile (0: the
// default, about 200 for FP64 and 400 for FP32 state) and uploads the tile
// table.  The trajectory does not depend on the tiling (the moment sums only
// to rounding: their summation order follows the tile shape).  A captured
// step graph bakes in the tile shapes, grids and table offsets, so it is
// released: a replay would run the old shapes over the new table.
int set_tiling(dsmc_ctx *x, int ppt, hipStream_t s)
{
    if (release_graph(x) != DSMC_OK) return DSMC_EHIP;
    const bool f32 = state32(x->cfg);
    if (ppt <= 0) ppt = f32 ? 400 : 200;
    static const int SHAPES[2][4][2] = {{{4, 4}, {2, 4}, {1, 4}, {1, 8}}, {{4, 8}, {4, 4}, {2, 8}, {1, 8}}};
    std::vector<int> shape_of(x->nrep);
    for (int r = 0; r < x->nrep; ++r) {
        int tc, ch;
        tile_shape(f32, x->reps[r].ppc, ppt, tc, ch);
        shape_of[r] = -1;
        for (int k = 0; k < 4; ++k)
            if (SHAPES[f32][k][0] == tc && SHAPES[f32][k][1] == ch) shape_of[r] = k;
        if (shape_of[r] < 0) return DSMC_EINVAL;
    }
    x->groups.clear();
    x->tiles_host.clear();
    std::vector<int32_t> rows;  // the same tiles in row-major order
    auto add_tile = [&](std::vector<int32_t> &v, int r, int c) {
        const RepConst &R = x->reps[r];
        const int nx = R.G.nx, ci = c - R.cbase;
        v.insert(v.end(), {c, r, ci / nx, ci % nx});
    };
    for (int k = 0; k < 4; ++k) {
        dsmc_ctx::TileGroup g;
        g.tc = SHAPES[f32][k][0];
        g.ch = SHAPES[f32][k][1];
        g.tile0 = (int)(x->tiles_host.size() / TILE_WORDS);
        for (int r = 0; r < x->nrep; ++r) {
            if (shape_of[r] != k) continue;
            const RepConst &R = x->reps[r];
            const int nx = R.G.nx, ny = R.G.ny, tpr = nx / g.tc;
            if (nx % g.tc == 0 && tpr >= 2 * TILE_BAND) {
                // rows of whole tiles at least two bands wide: band by band,
                // each band row by row
                for (int b0 = 0; b0 < tpr; b0 += TILE_BAND)
                    for (int iy = 0; iy < ny; ++iy)
                        for (int t = b0; t < std::min(b0 + TILE_BAND, tpr); ++t)
                            add_tile(x->tiles_host, r, R.cbase + iy * nx + t * g.tc);
            } else {
                for (int c = R.cbase; c < R.cend; c += g.tc) add_tile(x->tiles_host, r, c);
            }
            for (int c = R.cbase; c < R.cend; c += g.tc) add_tile(rows, r, c);
        }
        g.ntiles = (int)(x->tiles_host.size() / TILE_WORDS) - g.tile0;
        if (g.ntiles > 0) x->groups.push_back(g);
    }
    x->ntiles = (int)(x->tiles_host.size() / TILE_WORDS);
    x->tiles_host.insert(x->tiles_host.end(), rows.begin(), rows.end());
    x->particles_per_tile = ppt;
    if (hipMemcpyAsync(x->tiles, x->tiles_host.data(), x->tiles_host.size() * 4, hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return DSMC_EHIP;
    // the host table must outlive the copy
    return hipStreamSynchronize(s) == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

// the launches of one pass of the tile kernels, one per tile group: kind 0
// = k_classify, 1 = k_step.  The groups touch disjoint cells; with side
// streams the second and later groups run beside the first.
int launch_tiles(const dsmc_ctx *x, int kind, bool move, hipStream_t s, const StepArgs &a0)
{
    const bool defer = (a0.flags & STEP_DEFER) != 0 && move;
    const int ng = (int)x->groups.size();
    const bool fork = x->forked && ng > 1 && ng <= 4;
    if (fork && hipEventRecord(x->ev_fork, s) != hipSuccess) return DSMC_EHIP;
    for (int gi = 0; gi < ng; ++gi) {
        const dsmc_ctx::TileGroup &g = x->groups[(size_t)gi];
        hipStream_t gs = s;
        if (fork && gi > 0) {
            gs = x->side[gi - 1];
            if (hipStreamWaitEvent(gs, x->ev_fork, 0) != hipSuccess) return DSMC_EHIP;
        }
        StepArgs a = a0;
        // the classify pass reads whole cells in place and streams best in
        // row order; the step's gathers read across rows and take the bands
        a.tiles = x->tiles + TILE_WORDS * ((kind == 0 ? (size_t)x->ntiles : 0) + (size_t)g.tile0);
        const unsigned n = (unsigned)g.ntiles;
#define DSMC_LAUNCH(TC, CH, S)                                          \
    do {                                                                \
        if (kind == 0 && defer)                                         \
            k_classify<TC, CH, S, true><<<n, 64, 0, gs>>>(a);           \
        else if (kind == 0)                                             \
            k_classify<TC, CH, S, false><<<n, 64, 0, gs>>>(a);          \
        else if (defer && x->nt_loads)                                  \
            k_step<TC, CH, true, S, true, true><<<n, 64, 0, gs>>>(a);   \
        else if (defer)                                                 \
            k_step<TC, CH, true, S, false, true><<<n, 64, 0, gs>>>(a);  \
        else if (x->nt_loads && move)                                   \
            k_step<TC, CH, true, S, true, false><<<n, 64, 0, gs>>>(a);  \
        else if (x->nt_loads)                                           \
            k_step<TC, CH, false, S, true, false><<<n, 64, 0, gs>>>(a); \
        else if (move)                                                  \
            k_step<TC, CH, true, S, false, false><<<n, 64, 0, gs>>>(a); \
        else                                                            \
            k_step<TC, CH, false, S, false, false><<<n, 64, 0, gs>>>(a); \
    } while (0)
        if (state32(x->cfg)) {
            if (g.tc == 4 && g.ch == 8)
                DSMC_LAUNCH(4, 8, float);
            else if (g.tc == 4)
                DSMC_LAUNCH(4, 4, float);
            else if (g.tc == 2)
                DSMC_LAUNCH(2, 8, float);
            else
                DSMC_LAUNCH(1, 8, float);
        } else {
            if (g.tc == 4)
                DSMC_LAUNCH(4, 4, double);
            else if (g.tc == 2)
                DSMC_LAUNCH(2, 4, double);
            else if (g.ch == 4)
                DSMC_LAUNCH(1, 4, double);
            else
                DSMC_LAUNCH(1, 8, double);
        }
#undef DSMC_LAUNCH
        if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
        if (gs != s) {  // join the side stream back into the caller's
            if (hipEventRecord(x->ev_join[gi - 1], gs) != hipSuccess) return DSMC_EHIP;
            if (hipStreamWaitEvent(s, x->ev_join[gi - 1], 0) != hipSuccess) return DSMC_EHIP;
        }
    }
    return DSMC_OK;
}

// side streams and their events for a batch's tile groups (see dsmc_ctx)
int make_side_streams(dsmc_ctx *x)
{
    for (int k = 0; k < 3; ++k) {
        if (hipStreamCreateWithFlags(&x->side[k], hipStreamNonBlocking) != hipSuccess) return DSMC_EHIP;
        if (hipEventCreateWithFlags(&x->ev_join[k], hipEventDisableTiming) != hipSuccess) return DSMC_EHIP;
    }
    if (hipEventCreateWithFlags(&x->ev_fork, hipEventDisableTiming) != hipSuccess) return DSMC_EHIP;
    x->forked = true;
    return DSMC_OK;
}

// releases what a context owns on the device side and the context itself
void release_ctx(dsmc_ctx *x)
{
    for (int k = 0; k < 3; ++k) {
        if (x->side[k]) (void)hipStreamDestroy(x->side[k]);
        if (x->ev_join[k]) (void)hipEventDestroy(x->ev_join[k]);
    }
    if (x->ev_fork) (void)hipEventDestroy(x->ev_fork);
    delete x;
}

int fill_f64(double *p, size_t n, double v, hipStream_t s)
{
    if (n == 0) return DSMC_OK;
    k_fill_f64<<<grid_threads(n), 256, 0, s>>>(p, n, v);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

int fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t s)
{
    if (n == 0) return DSMC_OK;
    k_fill_i32<<<grid_threads(n), 256, 0, s>>>(p, n, v);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

// exclusive scan of per-cell counts into cs[0..ncells] (cs[ncells] = total)
int scan_counts(dsmc_ctx *x, const int32_t *counts, int32_t *cs, hipStream_t s)
{
    k_block_sums<<<x->nblk, 256, 0, s>>>(counts, x->ncells, x->blocksum);
    k_scan_blocks<<<1, 1024, 0, s>>>(x->blocksum, x->nblk, cs, x->ncells, x->ctr, -1);
    k_block_scan<<<x->nblk, 256, 0, s>>>(counts, x->ncells, x->blocksum, cs);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

const Lattice *lattice_of(int q)
{
    const LatticeTables &t = tables();
    if (!t.ok) return nullptr;
    if (q == 9) return &t.q9;
    if (q == 37) return &t.q37;
    return nullptr;
}

// Checks an lbm_config and fills the step arguments shared by the forward and
// adjoint kernels (lattice, velocities, buffer depth K = max|e_y|).
bool lbm_args(const lbm_config *cfg, LbmArgs &a)
{
    if (!cfg || cfg->nx < 1 || cfg->ny < 1) return false;
    if ((int64_t)cfg->nx * cfg->ny >= ((int64_t)1 << 29)) return false;  // 32-bit byte offsets within a plane
    const Lattice *L = lattice_of(cfg->lattice);
    if (!L || !(cfg->tau > 0.5) || !std::isfinite(cfg->tau) || !std::isfinite(cfg->body_force_x)) return false;
    if (cfg->y_mode < 0 || cfg->y_mode > 2) return false;
    if (cfg->x_buffer < 0 || cfg->x_buffer > cfg->nx) return false;
    const LatticeTables &t = tables();
    std::memset(&a, 0, sizeof(a));
    a.L.Q = L->Q;
    a.L.r = L->r;
    int K = 0;
    for (int q = 0; q < L->Q; ++q) {
        const int ey = cfg->lattice == 9 ? t.e9[q][1] : t.e37[q][1];
        a.L.ws[cfg->lattice == 9 ? VelSet<9>::sh[q] : VelSet<37>::sh[q]] = L->w[q];
        if (std::abs(ey) > K) K = std::abs(ey);
    }
    if (cfg->y_mode == 2 && K != 1) return false;  // walls: lattices with |e_y| <= 1
    a.nx = cfg->nx;
    a.ny = cfg->ny;
    a.y_mode = cfg->y_mode;
    a.K = K;
    a.xb = cfg->x_buffer;
    a.tau = cfg->tau;
    a.gx = cfg->body_force_x;
    return true;
}

// the reverse pass covers periodic y and buffer rows without inflow columns
bool adjoint_supported(const lbm_config *cfg) { return cfg->y_mode != 2 && cfg->x_buffer == 0; }

// launches the lattice step / its adjoint instance that fits the grid
void launch_lbm(const LbmArgs &a, hipStream_t s)
{
    const size_t nn = (size_t)a.nx * a.ny;
    const int R = a.L.Q == 9 ? 1 : 3;
    const bool narrow = a.nx < R || a.ny < R;
#define DSMC_LBM(Q, YM)                                                    \
    do {                                                                   \
        if (narrow)                                                        \
            k_lbm<Q, YM, true><<<grid_threads(nn), 256, 0, s>>>(a);        \
        else                                                               \
            k_lbm<Q, YM, false><<<grid_threads(nn), 256, 0, s>>>(a);       \
    } while (0)
    if (a.L.Q == 9) {
        if (a.y_mode == 2)
            DSMC_LBM(9, 2);
        else if (a.y_mode == 1)
            DSMC_LBM(9, 1);
        else
            DSMC_LBM(9, 0);
    } else {
        if (a.y_mode == 1)
            DSMC_LBM(37, 1);
        else
            DSMC_LBM(37, 0);
    }
#undef DSMC_LBM
}

void launch_lbm_adjoint(const LbmAdjArgs &b, unsigned nblk, hipStream_t s)
{
    const int R = b.L.Q == 9 ? 1 : 3;
    const bool yb = b.y_mode == 1, narrow = b.nx < R || b.ny < R;
#define DSMC_ADJ(Q, YB, NW) k_lbm_adjoint<Q, YB, NW><<<nblk, 256, 0, s>>>(b)
    if (b.L.Q == 9) {
        if (yb) { if (narrow) DSMC_ADJ(9, true, true); else DSMC_ADJ(9, true, false); }
        else { if (narrow) DSMC_ADJ(9, false, true); else DSMC_ADJ(9, false, false); }
    } else {
        if (yb) { if (narrow) DSMC_ADJ(37, true, true); else DSMC_ADJ(37, true, false); }
        else { if (narrow) DSMC_ADJ(37, false, true); else DSMC_ADJ(37, false, false); }
    }
#undef DSMC_ADJ
}

LbmAdjArgs adj_args(const LbmArgs &a, const double *f, const double *lam_in, double *lam_out, double *partial,
                    int accumulate)
{
    LbmAdjArgs b;
    b.f = f;
    b.lam_in = lam_in;
    b.lam_out = lam_out;
    b.partial = partial;
    b.accumulate = accumulate;
    b.L = a.L;
    b.nx = a.nx;
    b.ny = a.ny;
    b.y_mode = a.y_mode;
    b.K = a.K;
    b.tau = a.tau;
    b.gx = a.gx;
    return b;
}

// Adjoint workspace: per-block partial sums, one cotangent buffer and the
// every - 1 states recomputed inside a checkpoint segment.  every = 0: the
// partial sums only (one adjoint step).
struct AdjLayout {
    size_t nblk, partial, lam, states, total;
};

AdjLayout adj_layout(const lbm_config *cfg, int Q, int32_t every)
{
    const size_t nn = (size_t)cfg->nx * cfg->ny, st = nn * (size_t)Q * sizeof(double);
    AdjLayout W;
    W.nblk = (nn + 255) / 256;
    W.partial = 0;
    W.lam = al(2 * W.nblk * sizeof(double));
    if (every == 0) {
        W.states = W.lam;
        W.total = W.lam;
        return W;
    }
    W.states = W.lam + al(st);
    W.total = W.states + (size_t)(every - 1) * al(st);
    return W;
}

HermiteArgs hermite_args(const Lattice &L, int order, const double *f, int64_t nnodes, const int32_t *nodes,
                         int32_t nsel)
{
    HermiteArgs h;
    std::memset(&h, 0, sizeof(h));
    h.f = f;
    h.nodes = nodes;
    h.nnodes = nnodes;
    h.nsel = nsel;
    h.nh = (order + 1) * (order + 2) / 2;  // 1, 3, 6, 10 coefficients up to order 0..3
    h.L = L;
    return h;
}

}  // namespace

extern "C" {

const char *dsmc_strerror(int code)
{
    switch (code) {
        case DSMC_OK: return "ok";
        case DSMC_EINVAL: return "invalid argument";
        case DSMC_ECAPACITY: return "capacity exceeded";
        case DSMC_EHIP: return "HIP runtime error";
        case DSMC_ESTATE: return "invalid call for the current state";
        default: return "unknown error";
    }
}

int dsmc_query_sizes(const dsmc_config *cfg, dsmc_sizes *out)
{
    if (!valid_config(cfg) || !out) return DSMC_EINVAL;
    const Layout L = make_layout(*cfg, (size_t)cfg->nx * cfg->ny, 1);
    out->ncells = (int64_t)cfg->nx * cfg->ny;
    out->capacity = cfg->capacity;
    out->state_array_bytes = (size_t)cfg->capacity * (state32(*cfg) ? 4 : 8);
    out->workspace_bytes = L.total;
    return DSMC_OK;
}

int dsmc_lattice(int32_t lattice, int32_t *e_out, double *w_out, double *r_out)
{
    const Lattice *L = lattice_of(lattice);
    if (!L) return DSMC_EINVAL;
    const LatticeTables &t = tables();
    for (int a = 0; a < L->Q; ++a) {
        if (e_out) {
            e_out[2 * a] = lattice == 9 ? t.e9[a][0] : t.e37[a][0];
            e_out[2 * a + 1] = lattice == 9 ? t.e9[a][1] : t.e37[a][1];
        }
        if (w_out) w_out[a] = L->w[a];
    }
    if (r_out) *r_out = L->r;
    return DSMC_OK;
}

}  // extern "C"

namespace {

// A context over nrep channels (cfg supplies the settings they share; the
// single-channel entry passes its own channel as the only replica).
int init_ctx(const dsmc_config *cfg, const dsmc_replica *reps, int32_t nrep, const dsmc_buffers *buf, int32_t mode,
             int64_t n_load, hipStream_t s, dsmc_ctx **out)
{
    int64_t ncells = 0, npart = 0;
    if (!valid_batch(cfg, reps, nrep, &ncells, &npart)) return DSMC_EINVAL;
    const Layout L = make_layout(*cfg, (size_t)ncells, (size_t)nrep);
    if (buf->workspace_bytes < L.total) return DSMC_EINVAL;
    if (mode != 0 && mode != 1) return DSMC_EINVAL;
    if (mode == 1 && nrep != 1) return DSMC_EINVAL;
    if (mode == 0 && npart > cfg->capacity) return DSMC_ECAPACITY;
    if (mode == 1 && (n_load < 0 || n_load > cfg->capacity)) return n_load < 0 ? DSMC_EINVAL : DSMC_ECAPACITY;
    if (!tables().ok) return DSMC_EINVAL;

    dsmc_ctx *x = new (std::nothrow) dsmc_ctx();
    if (!x) return DSMC_EINVAL;
    x->cfg = *cfg;
    x->err[0] = '\0';
    if (nrep == 1) {  // the channel's own parameters, for the single-channel calls
        x->cfg.nx = reps[0].nx;
        x->cfg.ny = reps[0].ny;
        x->cfg.ppc = reps[0].ppc;
        x->cfg.kn = reps[0].kn;
        x->cfg.dt = reps[0].dt;
        x->cfg.body_force_x = reps[0].body_force_x;
        x->cfg.seed = reps[0].seed;
    }
    char *w = (char *)buf->workspace;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 5; ++k) x->st[b][k] = buf->state[b][k];
    x->cs[0] = (int32_t *)(w + L.cs0);
    x->cs[1] = (int32_t *)(w + L.cs1);
    x->grp[0] = (int32_t *)(w + L.grp0);
    x->grp[1] = (int32_t *)(w + L.grp1);
    x->plan = (int32_t *)(w + L.plan);
    x->countnew = (int32_t *)(w + L.countnew);
    x->farcnt = (int32_t *)(w + L.farcnt);
    x->blocksum = (int32_t *)(w + L.blocksum);
    x->far[0] = (int32_t *)(w + L.far0);
    x->far[1] = (int32_t *)(w + L.far1);
    x->nbar = (double *)(w + L.nbar);
    x->sigcmax = (double *)(w + L.sigcmax);
    x->rem = (double *)(w + L.rem);
    x->mom = (double *)(w + L.mom);
    x->mark = (int32_t *)(w + L.mark);
    x->prm = (double *)(w + L.prm);
    x->nnew = (int32_t *)(w + L.nnew);
    x->perm = (int32_t *)(w + L.perm);
    x->ctr = (Counters *)(w + L.ctr);
    x->tstat = (unsigned long long *)(w + L.tstat);
    x->kc = (TileConst *)(w + L.kc);
    x->rep = (RepConst *)(w + L.rep);
    x->tiles = (int32_t *)(w + L.tiles);
    x->cell_rep = (int32_t *)(w + L.cell_rep);
    x->rstat = (unsigned long long *)(w + L.rstat);
    x->comp = (int32_t *)(w + L.comp);
    x->complist = (int32_t *)(w + L.complist);
    x->appoff = (int32_t *)(w + L.appoff);
    x->ncells = (int)ncells;
    x->nblk = (int)((ncells + 255) / 256);
    x->far_cap = far_cap_of(*cfg);
    x->s_th = std::sqrt(cfg->kT_over_m);
    x->nrep = nrep;
    x->reps.resize(nrep);
    std::vector<int32_t> cell_rep((size_t)ncells);
    int64_t cb = 0, pb = 0;
    for (int32_t r = 0; r < nrep; ++r) {
        const dsmc_replica &q = reps[r];
        RepConst &R = x->reps[r];
        const int64_t nc = (int64_t)q.nx * q.ny;
        R.G.nx = q.nx;
        R.G.ny = q.ny;
        R.G.Lx = (double)q.nx;
        R.G.H = (double)q.ny;
        R.dt = q.dt;
        R.g = q.body_force_x;
        // Eq. (MFP): lambda = 1/(sqrt(2) pi d^2 n), n = ppc F_N / V_c
        R.K = 1.0 / (std::sqrt(2.0) * (q.kn * (double)q.ny) * (double)q.ppc);
        R.k0 = (uint32_t)q.seed;
        R.k1 = (uint32_t)(q.seed >> 32);
        R.cbase = (int32_t)cb;
        R.cend = (int32_t)(cb + nc);
        R.pbase = (int32_t)pb;
        R.ppc = q.ppc;
        for (int64_t c = cb; c < cb + nc; ++c) cell_rep[(size_t)c] = r;
        cb += nc;
        pb += nc * q.ppc;
    }
    x->K = x->reps[0].K;
    x->G = x->reps[0].G;
    x->cur = 0;
    x->step = 0;
    x->nsamples = 0;
    x->reseed_events = 0;
    x->classified = false;
    x->pending = false;
    x->comp_pending = false;
    x->comp_reseed = false;
    {
        const int64_t nominal = mode == 1 ? n_load : npart;
        const int64_t bytes = nominal * 5 * (cfg->state_bits == 32 ? 4 : 8);
        x->nt_loads = bytes <= ((int64_t)384 << 20);
    }
    x->prof = false;
    x->last = s;
    x->capturing = false;
    x->graph = nullptr;
    x->gexec = nullptr;
    x->g_nsteps = 0;

    int rc = DSMC_OK;
    if (hipMemcpyAsync(x->rep, x->reps.data(), sizeof(RepConst) * (size_t)nrep, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(x->cell_rep, cell_rep.data(), 4 * (size_t)ncells, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = DSMC_EHIP;
    if (rc == DSMC_OK) rc = set_tiling(x, 0, s);
    if (rc == DSMC_OK && nrep > 1) rc = make_side_streams(x);
    if (rc == DSMC_OK) {
        k_zero_counters<<<1, 64, 0, s>>>(x->ctr);
        if (hipGetLastError() != hipSuccess) rc = DSMC_EHIP;
    }
    if (rc == DSMC_OK) rc = fill_f64(x->mom, (size_t)NMOM * ncells, 0.0, s);
    if (rc == DSMC_OK) rc = fill_i32(x->farcnt, 2 * (size_t)ncells, 0, s);
    if (rc == DSMC_OK) rc = fill_i32(x->mark, (size_t)ncells, 0, s);
    if (rc == DSMC_OK) rc = fill_i32(x->comp, (size_t)ncells, 0, s);
    if (rc == DSMC_OK) rc = fill_i32((int32_t *)x->tstat, 6 * (size_t)ncells, 0, s);
    if (rc == DSMC_OK) rc = upload_tile_const(x, s);
    if (rc == DSMC_OK && mode == 0) {
        // one launch per channel: its cells, its particles, its seed
        const size_t es = state32(*cfg) ? 4 : 8;
        for (int32_t r = 0; r < nrep && rc == DSMC_OK; ++r) {
            const RepConst &R = x->reps[r];
            InitArgs a;
            for (int k = 0; k < 5; ++k) a.st[k] = (char *)x->st[0][k] + (size_t)R.pbase * es;
            a.cs = x->cs[0] + R.cbase;
            a.nbar = x->nbar + R.cbase;
            a.sigcmax = x->sigcmax + R.cbase;
            a.rem = x->rem + R.cbase;
            a.nx = R.G.nx;
            a.ncells = R.cend - R.cbase;
            a.ppc = R.ppc;
            a.pbase = R.pbase;
            a.s_th = x->s_th;
            a.sigcr0 = cfg->sigcr_max0;
            a.k0 = R.k0;
            a.k1 = R.k1;
            const size_t n = (size_t)a.ncells * R.ppc;
            const size_t nthreads = n > (size_t)a.ncells + 1 ? n : (size_t)a.ncells + 1;
            if (state32(*cfg))
                k_init_maxwell<float><<<grid_threads(nthreads), 256, 0, s>>>(a);
            else
                k_init_maxwell<double><<<grid_threads(nthreads), 256, 0, s>>>(a);
            if (hipGetLastError() != hipSuccess) rc = DSMC_EHIP;
        }
        x->cur = 0;
    } else if (rc == DSMC_OK) {
        // adopt: stable sort of buffer 0 into buffer 1 by cell
        AdoptArgs a;
        for (int k = 0; k < 5; ++k) {
            a.in[k] = x->st[0][k];
            a.out[k] = x->st[1][k];
        }
        a.cellid = x->perm + cfg->capacity;  // second half of the permutation space
        a.counts = x->countnew;
        a.cursor = x->farcnt;
        a.perm = x->perm;
        a.cs = x->cs[1];
        a.G = x->G;
        a.n = n_load;
        {
            rc = fill_i32(x->countnew, (size_t)ncells, 0, s);
            if (rc == DSMC_OK && n_load > 0) {
                if (state32(*cfg))
                    k_adopt_count<float><<<grid_threads((size_t)n_load), 256, 0, s>>>(a);
                else
                    k_adopt_count<double><<<grid_threads((size_t)n_load), 256, 0, s>>>(a);
                if (hipGetLastError() != hipSuccess) rc = DSMC_EHIP;
            }
            if (rc == DSMC_OK) rc = scan_counts(x, x->countnew, x->cs[1], s);
            if (rc == DSMC_OK && n_load > 0) {
                k_adopt_place<<<grid_threads((size_t)n_load), 256, 0, s>>>(a);
                k_adopt_sortcell<<<grid_threads((size_t)ncells), 256, 0, s>>>(a);
                if (state32(*cfg))
                    k_adopt_gather<float><<<grid_threads((size_t)n_load), 256, 0, s>>>(a);
                else
                    k_adopt_gather<double><<<grid_threads((size_t)n_load), 256, 0, s>>>(a);
                if (hipGetLastError() != hipSuccess) rc = DSMC_EHIP;
            }
            if (rc == DSMC_OK) rc = fill_f64(x->nbar, (size_t)ncells, 0.0, s);
            if (rc == DSMC_OK) rc = fill_f64(x->sigcmax, (size_t)ncells, cfg->sigcr_max0, s);
            if (rc == DSMC_OK) rc = fill_f64(x->rem, (size_t)ncells, 0.0, s);
            x->cur = 1;
        }
    }
    if (rc != DSMC_OK) {
        release_ctx(x);
        return rc;
    }
    *out = x;
    return DSMC_OK;
}

}  // namespace

extern "C" {

int dsmc_init(const dsmc_config *cfg, const dsmc_buffers *buf, int32_t mode, int64_t n_load, void *stream,
              dsmc_ctx **out)
{
    if (!out || !valid_config(cfg) || !buf || !buf->workspace) return DSMC_EINVAL;
    *out = nullptr;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 5; ++k)
            if (!buf->state[b][k]) return DSMC_EINVAL;
    if (((uintptr_t)buf->workspace & 255u) != 0) return DSMC_EINVAL;
    const dsmc_replica one = replica_of(*cfg);
    return init_ctx(cfg, &one, 1, buf, mode, n_load, S(stream), out);
}

int dsmc_batch_query_sizes(const dsmc_config *common, const dsmc_replica *reps, int32_t nrep, dsmc_sizes *out)
{
    int64_t nc = 0, np = 0;
    if (!out || !valid_batch(common, reps, nrep, &nc, &np)) return DSMC_EINVAL;
    const Layout L = make_layout(*common, (size_t)nc, (size_t)nrep);
    out->ncells = nc;
    out->capacity = common->capacity;
    out->state_array_bytes = (size_t)common->capacity * (state32(*common) ? 4 : 8);
    out->workspace_bytes = L.total;
    return DSMC_OK;
}

int dsmc_batch_init(const dsmc_config *common, const dsmc_replica *reps, int32_t nrep, const dsmc_buffers *buf,
                    void *stream, dsmc_ctx **out)
{
    if (!out || !buf || !buf->workspace) return DSMC_EINVAL;
    *out = nullptr;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 5; ++k)
            if (!buf->state[b][k]) return DSMC_EINVAL;
    if (((uintptr_t)buf->workspace & 255u) != 0) return DSMC_EINVAL;
    return init_ctx(common, reps, nrep, buf, 0, 0, S(stream), out);
}

static int dsmc_set_tiling_impl(dsmc_ctx *x, int32_t particles_per_tile, void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (particles_per_tile < 0 || particles_per_tile > (1 << 20))
        return fail(DSMC_EINVAL, "particles_per_tile must be in [0, 2^20]");
    hipStream_t s = S(stream);
    x->last = s;
    return set_tiling(x, particles_per_tile, s);
}

static int dsmc_autotune_impl(dsmc_ctx *x, int32_t steps_per_trial, int32_t sample_every, dsmc_tuning *out,
                              void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (steps_per_trial < 1 || sample_every < 0)
        return fail(DSMC_EINVAL, "steps_per_trial must be >= 1 and sample_every >= 0");
    hipStream_t s = S(stream);
    x->last = s;
    const bool f32 = state32(x->cfg);
    const int cand_64[] = {100, 200, 400, 800};
    const int cand_32[] = {200, 400, 800, 1600};
    const int *cand = f32 ? cand_32 : cand_64;
    const int ncand = 4;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return DSMC_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return DSMC_EHIP;
    }
    int rc = DSMC_OK, best = -1;
    double best_ms = 0.0;
    dsmc_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.ncand = ncand;
    for (int k = 0; k < ncand && rc == DSMC_OK; ++k) {
        rc = set_tiling(x, cand[k], s);
        if (rc != DSMC_OK) break;
        // real steps of the run: every tiling gives the same results
        if (hipEventRecord(e0, s) != hipSuccess) rc = DSMC_EHIP;
        if (rc == DSMC_OK) rc = dsmc_step(x, steps_per_trial, sample_every, stream);
        if (rc == DSMC_OK && hipEventRecord(e1, s) != hipSuccess) rc = DSMC_EHIP;
        if (rc == DSMC_OK && hipEventSynchronize(e1) != hipSuccess) rc = DSMC_EHIP;
        float ms = 0.0f;
        if (rc == DSMC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = DSMC_EHIP;
        t.particles_per_tile[k] = cand[k];
        t.ms_per_step[k] = (double)ms / steps_per_trial;
        if (rc == DSMC_OK && (best < 0 || t.ms_per_step[k] < best_ms)) {
            best = k;
            best_ms = t.ms_per_step[k];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DSMC_OK) return rc;
    t.chosen = best;
    rc = set_tiling(x, cand[best], s);
    if (out) *out = t;
    return rc;
}

static int dsmc_replica_counters_impl(dsmc_ctx *x, uint64_t *out, void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (!out) return fail(DSMC_EINVAL, "out is NULL");
    hipStream_t s = S(stream);
    x->last = s;
    k_replica_stats<<<(unsigned)x->nrep, 256, 0, s>>>(x->tstat, x->rep, x->rstat);
    if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    if (hipMemcpyAsync(out, x->rstat, 3 * sizeof(uint64_t) * (size_t)x->nrep, hipMemcpyDeviceToHost, s) !=
        hipSuccess)
        return DSMC_EHIP;
    return hipStreamSynchronize(s) == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

}  // extern "C"

namespace {
// completes a pending reseed by copying the kept cells' particles over
int settle(dsmc_ctx *x, hipStream_t s)
{
    if (!x->pending) return DSMC_OK;
    const int cur = x->cur, nxt = 1 - cur;
    ReseedArgs a;
    std::memset(&a, 0, sizeof(a));
    a.mark = x->mark;
    a.cs_old = x->cs[cur];
    a.cs_new = x->cs[nxt];
    for (int k = 0; k < 5; ++k) {
        a.in[k] = x->st[cur][k];
        a.out[k] = x->st[nxt][k];
    }
    a.ctr = x->ctr;
    a.ncells = x->ncells;
    const unsigned gcopy = (unsigned)((x->ncells + RC_TILE - 1) / RC_TILE);
    TRY(launch(x, DSMC_K_RESEED, s, [&] {
        if (state32(x->cfg))
            k_reseed_copy<float><<<gcopy, 256, 0, s>>>(a);
        else
            k_reseed_copy<double><<<gcopy, 256, 0, s>>>(a);
        k_reseed_done<<<1, 64, 0, s>>>(x->ctr);
    }));
    x->cur = nxt;
    x->pending = false;
    x->classified = false;
    return DSMC_OK;
}
}  // namespace

// ---- the adjoint step without a caller workspace -----------------------------
// lbm_adjoint_step_noalloc keeps the per-block partial sums of dJ/dg and
// dJ/dtau (2 doubles per block of 256 nodes) in this array instead of a
// workspace: every device the library runs on holds one copy of it until the
// process ends.  Each adjoint launch writes every slot it later reads, so the
// array needs no clearing between calls.
constexpr int NOALLOC_MAX_BLOCKS = 16384;  // 4,194,304 nodes
static __device__ __align__(256) double scratch[2 * NOALLOC_MAX_BLOCKS];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
double *noalloc_ptr[NOALLOC_MAX_DEVICES];  // the array's address on each device, once looked up

// The device address of `scratch` on the current device.  The host-side name
// of a __device__ array is not a device address; it is looked up once per
// device (with that device current) and only the looked-up address is used.
int noalloc_scratch(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DSMC_EHIP;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return DSMC_EINVAL;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DSMC_EHIP;
        noalloc_ptr[dev] = (double *)p;
    }
    *out = noalloc_ptr[dev];
    return DSMC_OK;
}

// one adjoint step with the per-block partial sums in `partial` (>= 2 nblk doubles)
int adjoint_step_on(const lbm_config *cfg, const double *f_n, const double *lam_next, double *lam_out,
                    double *grad, double *partial, hipStream_t s)
{
    LbmArgs a;
    if (!lbm_args(cfg, a) || !adjoint_supported(cfg) || !f_n || !lam_next || !lam_out || !grad || !partial)
        return DSMC_EINVAL;
    if (lam_next == lam_out) return DSMC_EINVAL;
    const AdjLayout W = adj_layout(cfg, a.L.Q, 0);
    LbmAdjArgs b = adj_args(a, f_n, lam_next, lam_out, partial + W.partial / sizeof(double), 0);
    launch_lbm_adjoint(b, (unsigned)W.nblk, s);
    k_adjoint_finish<<<1, 256, 0, s>>>(b.partial, (int)W.nblk, grad);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}
}  // namespace

extern "C" {

// The completion pass of a moved state (see STEP_COMPLETE): after a moved
// reseed the replaced cells' recorded long jumps are dropped first, then
// every listed cell is moved as a one-cell classify tile.
static int complete(dsmc_ctx *x, hipStream_t s)
{
    if (!x->comp_pending) return DSMC_OK;
    StepArgs a = step_args(x, x->cur, x->step, false, true);
    a.flags = STEP_COMPLETE | (x->comp_reseed ? STEP_COMP_RESEED : 0);
    const bool f32 = state32(x->cfg);
    int tc = 1, ch = 8;
    tile_shape(f32, x->cfg.ppc, 1, tc, ch);
    const unsigned far_blocks = (unsigned)((std::max<size_t>((size_t)x->far_cap, (size_t)x->ncells) + 255) / 256);
    const unsigned grid = (unsigned)std::min(x->ncells, 4096);
    TRY(launch(x, DSMC_K_CLASSIFY, s, [&] {
        if (x->comp_reseed) {
            for (int pass = 0; pass < 2; ++pass) {
                if (f32)
                    k_comp_far<float><<<far_blocks, 256, 0, s>>>(a, pass);
                else
                    k_comp_far<double><<<far_blocks, 256, 0, s>>>(a, pass);
            }
        }
        if (f32)
            k_complete<8, float><<<grid, 64, 0, s>>>(a);
        else if (ch == 4)
            k_complete<4, double><<<grid, 64, 0, s>>>(a);
        else
            k_complete<8, double><<<grid, 64, 0, s>>>(a);
        if (x->comp_reseed) k_comp_done<<<1, 64, 0, s>>>(x->ctr, 1);
    }));
    if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    x->comp_pending = false;
    x->comp_reseed = false;
    return DSMC_OK;
}

// nsteps steps; the state ends settled, or with moved_end moved for the
// coming step (the call's last step moves and partitions as the others do;
// in a one-channel context it leaves tiles with particles bound for a wall
// unmoved, for a reseed that may come first: see STEP_DEFER)
static int step_run(dsmc_ctx *x, int32_t nsteps, int32_t sample_every, bool moved_end, void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (nsteps < 0 || sample_every < 0) return fail(DSMC_EINVAL, "nsteps and sample_every must be >= 0");
    hipStream_t s = S(stream);
    x->last = s;
    const int nc = x->ncells;
    int rc_tiles = DSMC_OK;
    const bool defer = moved_end && x->nrep == 1;
    if (x->classified && nsteps > 0) TRY(complete(x, s));
    if ((nsteps > 0 || moved_end) && !x->classified) {
        // moves of the coming step for a state set or changed from outside
        const int p = (int)(x->step & 1);
        TRY(fill_i32(x->farcnt, 2 * (size_t)nc, 0, s));
        k_far_reset<<<1, 64, 0, s>>>(x->ctr, p);
        const int fl = (defer && nsteps == 0) ? STEP_DEFER : 0;  // the call's moved state comes from this pass
        if (x->pending) {  // the classify pass completes the reseed into the other buffer
            StepArgs a = step_args(x, 1 - x->cur, x->step, false, true);
            a.reseed = 1;
            a.flags = fl;
            TRY(launch(x, DSMC_K_CLASSIFY, s, [&] {
                rc_tiles = launch_tiles(x, 0, true, s, a);
                k_reseed_done<<<1, 64, 0, s>>>(x->ctr);
            }));
            x->cur = 1 - x->cur;
            x->pending = false;
        } else {
            StepArgs a = step_args(x, x->cur, x->step, false, true);
            a.flags = fl;
            TRY(launch(x, DSMC_K_CLASSIFY, s, [&] { rc_tiles = launch_tiles(x, 0, true, s, a); }));
        }
        TRY(rc_tiles);
        x->classified = true;
        if (fl) x->comp_pending = true;
    }
    for (int32_t it = 0; it < nsteps; ++it) {
        const int cur = x->cur, nxt = 1 - cur;
        const int p = (int)(x->step & 1);
        CellArgs c;
        c.grp = x->grp[p];
        c.plan = x->plan;
        c.farcnt = x->farcnt + (size_t)p * nc;
        c.countnew = x->countnew;
        c.blocksum = x->blocksum;
        c.rep = x->rep;
        c.cell_rep = x->cell_rep;
        c.ncells = nc;
        c.nx1 = x->nrep == 1 ? x->reps[0].G.nx : 0;
        c.ny1 = x->nrep == 1 ? x->reps[0].G.ny : 0;
        c.cs_out = x->cs[nxt];
        c.ctr = x->ctr;
        c.reset_slot = p ^ 1;
        TRY(launch(x, DSMC_K_CELL_COUNT, s, [&] { k_cell_count<<<x->nblk, 256, 0, s>>>(c); }));
        if (x->nblk > 1)  // (one block: the count kernel wrote the starts)
            TRY(launch(x, DSMC_K_CELL_FINAL, s, [&] {
                k_cell_final<<<x->nblk, 256, 0, s>>>(x->countnew, nc, x->blocksum, x->cs[nxt], x->ctr, p ^ 1);
            }));

        const bool sample = sample_every > 0 && ((x->step + 1) % sample_every) == 0;
        const bool move = moved_end || it + 1 < nsteps;  // a dsmc_step call's last step leaves the state settled
        StepArgs a = step_args(x, cur, x->step, sample, false);
        if (defer && it + 1 == nsteps) a.flags = STEP_DEFER;
        TRY(launch(x, DSMC_K_STEP, s, [&] { rc_tiles = launch_tiles(x, 1, move, s, a); }));
        TRY(rc_tiles);
        x->cur = nxt;
        if (sample) x->nsamples += 1;
        x->step += 1;
    }
    if (nsteps > 0) {
        x->classified = moved_end;
        x->comp_pending = defer;
    }
    return DSMC_OK;
}

static int dsmc_step_impl(dsmc_ctx *x, int32_t nsteps, int32_t sample_every, void *stream)
{
    return step_run(x, nsteps, sample_every, false, stream);
}

static int dsmc_step_moved_impl(dsmc_ctx *x, int32_t nsteps, int32_t sample_every, void *stream)
{
    return step_run(x, nsteps, sample_every, true, stream);
}

static int dsmc_sample_moments_impl(dsmc_ctx *x, double *out, int32_t reset, void *stream)
{
    if (!x) return DSMC_EINVAL;
    hipStream_t s = S(stream);
    x->last = s;
    if (out) {
        if (x->nsamples <= 0) return fail(DSMC_ESTATE, "no sample has been taken since the last reset");
        const size_t n = (size_t)NMOM * x->ncells;
        const double Sd = (double)x->nsamples;
        TRY(launch(x, -1, s, [&] { k_average<<<grid_threads(n), 256, 0, s>>>(x->mom, out, n, Sd); }));
    }
    if (reset) {
        TRY(fill_f64(x->mom, (size_t)NMOM * x->ncells, 0.0, s));
        x->nsamples = 0;
    }
    return DSMC_OK;
}

// DSMC2LB of n cells c_off + i c_stride into nodes n_off + i n_stride of
// f_out ([Q][nn_out]); all cells into the same layout by default
static int project(dsmc_ctx *x, const double *mom, double S_, int64_t ncells, int32_t ppc, double kT, int32_t lattice,
                   int32_t order, double *f_out, hipStream_t s, int equilibrium = 0, int n = -1, int c_off = 0,
                   int c_stride = 1, int n_off = 0, int n_stride = 1, int64_t nn_out = -1)
{
    const Lattice *L = lattice_of(lattice);
    if (!L || order < 0 || order > 3 || !f_out || !mom || ncells < 1 || ppc < 1 || !(kT > 0.0))
        return fail(DSMC_EINVAL, "lattice must be 9 or 37, order 0..3, buffers non-NULL, ncells, ppc and kT > 0");
    if (equilibrium && order == 3 && lattice == 9)  // D2Q9 does not carry it
        return fail(DSMC_EINVAL, "the third-order equilibrium needs D2Q37");
    ProjectArgs a;
    a.mom = mom;
    a.f = f_out;
    a.L.Q = L->Q;
    a.L.r = L->r;
    for (int q = 0; q < L->Q; ++q) a.L.ws[L->Q == 9 ? VelSet<9>::sh[q] : VelSet<37>::sh[q]] = L->w[q];
    a.rho_scale = 1.0 / (S_ * (double)ppc);
    a.is1 = 1.0 / std::sqrt(kT);
    a.ncells = (int)ncells;
    a.order = order;
    a.equilibrium = equilibrium;
    a.n = n < 0 ? (int)ncells : n;
    a.c_off = c_off;
    a.c_stride = c_stride;
    a.n_off = n_off;
    a.n_stride = n_stride;
    a.nn_out = nn_out < 0 ? ncells : nn_out;
    if (a.n == 0) return DSMC_OK;
    return launch(x, DSMC_K_PROJECT, s, [&] {
        if (L->Q == 9)
            k_project<9><<<grid_threads((size_t)a.n), 256, 0, s>>>(a);
        else
            k_project<37><<<grid_threads((size_t)a.n), 256, 0, s>>>(a);
    });
}

static int map_dsmc_to_lbm_impl(dsmc_ctx *x, int32_t lattice, int32_t order, double *f_out, void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (x->nrep != 1) return fail(DSMC_ESTATE, "a batch context has no mapping (one channel only)");
    if (!lattice_of(lattice) || order < 0 || order > 3 || !f_out)
        return fail(DSMC_EINVAL, "lattice must be 9 or 37, order 0..3 and f_out non-NULL");
    hipStream_t s = S(stream);
    x->last = s;
    if (x->nsamples <= 0) return fail(DSMC_ESTATE, "no sample has been taken since the last reset");
    return project(x, x->mom, (double)x->nsamples, x->ncells, x->cfg.ppc, x->cfg.kT_over_m, lattice, order, f_out, s);
}

int dsmc_project_moments(const double *avg, int64_t ncells, int32_t ppc, double kT_over_m, int32_t lattice,
                         int32_t order, double *f_out, void *stream)
{
    if (ncells > (int64_t)0x3FFFFFFF) return DSMC_EINVAL;
    return project(nullptr, avg, 1.0, ncells, ppc, kT_over_m, lattice, order, f_out, S(stream));
}

int dsmc_project_equilibrium(const double *avg, int64_t ncells, int32_t ppc, double kT_over_m, int32_t lattice,
                             int32_t order, double *f_out, void *stream)
{
    if (ncells > (int64_t)0x3FFFFFFF || order < 0 || order > 3) return DSMC_EINVAL;
    return project(nullptr, avg, 1.0, ncells, ppc, kT_over_m, lattice, order, f_out, S(stream), 1);
}

static int dsmc_hybrid_cycle_impl(dsmc_ctx *x, const dsmc_hybrid *h, double *f_lb, double *f_tmp, double *avg_out,
                                  void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (!h || !f_lb || !f_tmp) return fail(DSMC_EINVAL, "h, f_lb and f_tmp must be non-NULL");
    if (x->nrep != 1) return fail(DSMC_ESTATE, "a batch context has no hybrid cycle (one channel only)");
    LbmArgs la;
    if (!lbm_args(&h->lbm, la)) return fail(DSMC_EINVAL, "invalid lattice configuration");
    if (h->lbm.ny != x->cfg.ny || h->lbm.x_buffer < 1)
        return fail(DSMC_EINVAL, "the lattice needs the channel's ny and at least one buffer column");
    if (h->dsmc_steps < 1 || h->lbm_steps < 0 || (h->mapping != 0 && h->mapping != 1))
        return fail(DSMC_EINVAL, "dsmc_steps >= 1, lbm_steps >= 0 and mapping 0 or 1 are required");
    if (h->order < 1 || h->order > 3 || (h->mapping == 0 && h->order == 3 && h->lbm.lattice == 9))
        return fail(DSMC_EINVAL, "order must be 1..3 (the third-order equilibrium needs D2Q37)");
    if (h->dsmc_column < 0 || h->dsmc_column >= x->cfg.nx) return fail(DSMC_EINVAL, "dsmc_column outside [0, nx)");
    if (h->flags & ~DSMC_HYBRID_MOVED) return fail(DSMC_EINVAL, "flags must be 0 or DSMC_HYBRID_MOVED");
    hipStream_t s = S(stream);
    x->last = s;
    // the DSMC subdomain, sampled every step over the cycle
    TRY((h->flags & DSMC_HYBRID_MOVED) ? dsmc_step_moved(x, h->dsmc_steps, 1, stream)
                                       : dsmc_step(x, h->dsmc_steps, 1, stream));
    // its buffer-layer column, averaged over the cycle, onto every held
    // inflow column of the lattice
    const int ny = x->cfg.ny;
    for (int32_t col = 0; col < h->lbm.x_buffer; ++col)
        TRY(project(x, x->mom, (double)x->nsamples, x->ncells, x->cfg.ppc, x->cfg.kT_over_m, h->lbm.lattice, h->order,
                    f_lb, s, h->mapping == 0 ? 1 : 0, ny, h->dsmc_column, x->cfg.nx, col, h->lbm.nx,
                    (int64_t)h->lbm.nx * ny));
    TRY(dsmc_sample_moments(x, avg_out, 1, stream));
    // the lattice subdomain
    return lbm_step(&h->lbm, f_lb, f_tmp, h->lbm_steps, stream);
}

static int map_lbm_to_dsmc_impl(dsmc_ctx *x, int32_t lattice, int32_t order, const double *f_in,
                                const int32_t *cell_ids, int32_t nsel, void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (x->nrep != 1) return fail(DSMC_ESTATE, "a batch context has no mapping (one channel only)");
    const Lattice *L = lattice_of(lattice);
    if (!L || (order != 2 && order != 3) || !f_in || nsel < 0 || (nsel > 0 && !cell_ids))
        return fail(DSMC_EINVAL, "lattice must be 9 or 37, order 2 or 3, f_in non-NULL, nsel >= 0 with cell_ids");
    if (nsel > x->ncells) return fail(DSMC_EINVAL, "nsel exceeds the number of cells");
    // a moved state (dsmc_step_moved): the new particles go after its last
    // slot and the replaced cells are completed with the rest before the
    // next step (see STEP_COMPLETE); one reseed per moved state
    const bool moved = x->classified;
    if (moved && x->comp_reseed)
        return fail(DSMC_ESTATE, "the moved state was reseeded already: step before the next reseed");
    hipStream_t s = S(stream);
    x->last = s;
    if (!moved) TRY(settle(x, s));
    const uint32_t event = (uint32_t)x->reseed_events;
    x->reseed_events += 1;
    const int cur = x->cur, nxt = 1 - cur;
    ReseedArgs a;
    a.f = f_in;
    a.cells = cell_ids;
    a.nsel = nsel;
    a.mark = x->mark;
    a.prm = x->prm;
    a.nnew = x->nnew;
    a.cs_old = x->cs[cur];
    a.cs_new = x->cs[nxt];
    a.countnew = x->countnew;
    a.blocksum = x->blocksum;
    for (int k = 0; k < 5; ++k) {
        a.in[k] = x->st[cur][k];
        a.out[k] = x->st[moved ? cur : nxt][k];
    }
    a.moved = moved ? 1 : 0;
    a.appoff = x->appoff;
    a.comp = x->comp;
    a.complist = x->complist;
    a.ctr = x->ctr;
    a.L = *L;
    a.nx = x->cfg.nx;
    a.ncells = x->ncells;
    a.ppc = x->cfg.ppc;
    a.order = order;
    a.ar_max_tries = x->cfg.ar_max_tries > 0 ? x->cfg.ar_max_tries : 65536;
    a.capacity = x->cfg.capacity;
    a.s_th = x->s_th;
    a.k0 = (uint32_t)x->cfg.seed;
    a.k1 = (uint32_t)(x->cfg.seed >> 32);
    a.event = event;
    const unsigned gsel = grid_threads((size_t)(nsel > 0 ? nsel : 1));
    TRY(launch(x, DSMC_K_RESEED, s, [&] {
        if (nsel > 0) k_reseed_prep<<<gsel, 256, 0, s>>>(a);
        k_reseed_count<<<x->nblk, 256, 0, s>>>(a);
        k_reseed_starts<<<x->nblk, 256, 0, s>>>(a);
        if (moved) {
            k_reseed_appoff<<<1, 1024, 0, s>>>(a);
            k_reseed_list<<<gsel, 256, 0, s>>>(a);
        }
        // settled state: the new particles go to buffer nxt; the kept ones
        // follow when the state settles (the next step's classify pass, or
        // settle()).  moved state: they go after its last slot
        if (nsel > 0) {
            if (state32(x->cfg))
                k_reseed_gen<float><<<grid_cells_wave(nsel), 256, 0, s>>>(a);
            else
                k_reseed_gen<double><<<grid_cells_wave(nsel), 256, 0, s>>>(a);
        }
    }));
    if (moved) {
        x->comp_pending = true;
        x->comp_reseed = true;
    } else {
        x->pending = true;
        x->classified = false;
    }
    return DSMC_OK;
}

int lbm_step(const lbm_config *cfg, double *f, double *f_tmp, int32_t nsteps, void *stream)
{
    return lbm_step_checkpointed(cfg, f, f_tmp, nullptr, nsteps, 1, stream);
}

int lbm_step_checkpointed(const lbm_config *cfg, double *f, double *f_tmp, double *ckpt, int32_t nsteps,
                          int32_t every, void *stream)
{
    LbmArgs a;
    if (!lbm_args(cfg, a) || !f || !f_tmp || nsteps < 0 || every < 1) return DSMC_EINVAL;
    hipStream_t s = S(stream);
    const size_t nn = (size_t)cfg->nx * cfg->ny, st = nn * (size_t)a.L.Q;
    double *src = f, *dst = f_tmp;
    for (int32_t it = 0; it < nsteps; ++it) {
        a.f = src;
        a.ft = dst;
        a.keep = (ckpt && it % every == 0) ? ckpt + (size_t)(it / every) * st : nullptr;
        launch_lbm(a, s);
        if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
        double *t2 = src;
        src = dst;
        dst = t2;
    }
    if (src != f) {
        if (hipMemcpyAsync(f, src, st * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return DSMC_EHIP;
    }
    return DSMC_OK;
}

int lbm_adjoint_workspace(const lbm_config *cfg, int32_t every, size_t *bytes)
{
    LbmArgs a;
    if (!lbm_args(cfg, a) || !adjoint_supported(cfg) || every < 0 || !bytes) return DSMC_EINVAL;
    *bytes = adj_layout(cfg, a.L.Q, every).total;
    return DSMC_OK;
}

int lbm_adjoint_step(const lbm_config *cfg, const double *f_n, const double *lam_next, double *lam_out,
                     double *grad, void *work, void *stream)
{
    if (!work) return DSMC_EINVAL;
    return adjoint_step_on(cfg, f_n, lam_next, lam_out, grad, (double *)work, S(stream));
}

int lbm_adjoint_step_noalloc(const lbm_config *cfg, const double *f_n, const double *lam_next, double *lam_out,
                             double *grad, void *stream)
{
    LbmArgs a;
    if (!lbm_args(cfg, a)) return DSMC_EINVAL;
    if (adj_layout(cfg, a.L.Q, 0).nblk > (size_t)NOALLOC_MAX_BLOCKS) return DSMC_ECAPACITY;
    double *partial = nullptr;
    TRY(noalloc_scratch(&partial));
    return adjoint_step_on(cfg, f_n, lam_next, lam_out, grad, partial, S(stream));
}

int lbm_adjoint(const lbm_config *cfg, const double *ckpt, int32_t nsteps, int32_t every, double *lam,
                double *grad, void *work, void *stream)
{
    LbmArgs a;
    if (!lbm_args(cfg, a) || !adjoint_supported(cfg) || !ckpt || !lam || !grad || !work || nsteps < 0 || every < 1)
        return DSMC_EINVAL;
    if (nsteps == 0) return DSMC_OK;
    const AdjLayout W = adj_layout(cfg, a.L.Q, every);
    hipStream_t s = S(stream);
    const size_t nn = (size_t)cfg->nx * cfg->ny, st = nn * (size_t)a.L.Q;
    double *partial = (double *)((char *)work + W.partial);
    double *lam_tmp = (double *)((char *)work + W.lam);
    double *states = (double *)((char *)work + W.states);
    double *cur = lam, *other = lam_tmp;
    bool first = true;
    const int32_t nseg = (nsteps + every - 1) / every;
    for (int32_t k = nseg - 1; k >= 0; --k) {
        const int32_t s0 = k * every;
        const int32_t len = std::min(every, nsteps - s0);
        const double *base = ckpt + (size_t)k * st;
        // recompute the segment's states f_{s0+1} .. f_{s0+len-1}
        a.keep = nullptr;
        for (int32_t i = 1; i < len; ++i) {
            a.f = i == 1 ? base : states + (size_t)(i - 2) * st;
            a.ft = states + (size_t)(i - 1) * st;
            launch_lbm(a, s);
        }
        for (int32_t i = len - 1; i >= 0; --i) {
            const double *fn = i == 0 ? base : states + (size_t)(i - 1) * st;
            LbmAdjArgs b = adj_args(a, fn, cur, other, partial, first ? 0 : 1);
            launch_lbm_adjoint(b, (unsigned)W.nblk, s);
            first = false;
            double *t2 = cur;
            cur = other;
            other = t2;
        }
        if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    }
    k_adjoint_finish<<<1, 256, 0, s>>>(partial, (int)W.nblk, grad);
    if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    if (cur != lam) {
        if (hipMemcpyAsync(lam, cur, st * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return DSMC_EHIP;
    }
    return DSMC_OK;
}

int lbm_hermite_moments(int32_t lattice, int32_t order, const double *f, int64_t nnodes, const int32_t *nodes,
                        int32_t nsel, double *a_out, void *stream)
{
    const Lattice *L = lattice_of(lattice);
    if (!L || order < 0 || order > 3 || nnodes < 1 || nsel < 0) return DSMC_EINVAL;
    if (nsel == 0) return DSMC_OK;
    if (!f || !nodes || !a_out) return DSMC_EINVAL;
    HermiteArgs h = hermite_args(*L, order, f, nnodes, nodes, nsel);
    h.a = a_out;
    k_hermite_moments<<<grid_threads((size_t)nsel), 256, 0, S(stream)>>>(h);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

int lbm_hermite_moments_adjoint(int32_t lattice, int32_t order, const double *a_bar, const int32_t *nodes,
                                int32_t nsel, double *f_bar, int64_t nnodes, void *stream)
{
    const Lattice *L = lattice_of(lattice);
    if (!L || order < 0 || order > 3 || nnodes < 1 || nsel < 0) return DSMC_EINVAL;
    if (nsel == 0) return DSMC_OK;
    if (!a_bar || !nodes || !f_bar) return DSMC_EINVAL;
    HermiteArgs h = hermite_args(*L, order, nullptr, nnodes, nodes, nsel);
    h.a_bar = a_bar;
    h.f_bar = f_bar;
    k_hermite_moments_adjoint<<<grid_threads((size_t)nsel), 256, 0, S(stream)>>>(h);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

int dsmc_project_moments_adjoint(const double *f_bar, const double *avg, int64_t ncells, int32_t ppc,
                                 double kT_over_m, int32_t lattice, int32_t order, double *avg_bar, void *stream)
{
    const Lattice *L = lattice_of(lattice);
    if (!L || order < 0 || order > 3 || ncells < 0 || ncells > (int64_t)0x3FFFFFFF || ppc < 1) return DSMC_EINVAL;
    if (!(kT_over_m > 0.0) || !std::isfinite(kT_over_m)) return DSMC_EINVAL;
    if (ncells == 0) return DSMC_OK;
    if (!f_bar || !avg || !avg_bar) return DSMC_EINVAL;
    ProjectAdjArgs p;
    p.f_bar = f_bar;
    p.avg = avg;
    p.avg_bar = avg_bar;
    p.L = *L;
    p.ncells = (int)ncells;
    p.ppc = ppc;
    p.order = order;
    p.s1 = std::sqrt(kT_over_m);
    k_project_adjoint<<<grid_threads((size_t)ncells), 256, 0, S(stream)>>>(p);
    return hipGetLastError() == hipSuccess ? DSMC_OK : DSMC_EHIP;
}

static int dsmc_read_status_impl(dsmc_ctx *x, dsmc_status *out, int32_t clear, void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (!out) return fail(DSMC_EINVAL, "out is NULL");
    hipStream_t s = S(stream);
    TRY(settle(x, s));
    Counters h;
    int32_t n = 0, n_re = 0;
    k_tile_stats<<<1, 1024, 0, s>>>(x->tstat, x->ncells, x->ctr);
    if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    if (hipMemcpyAsync(&h, x->ctr, sizeof(Counters), hipMemcpyDeviceToHost, s) != hipSuccess) return DSMC_EHIP;
    if (hipMemcpyAsync(&n, x->cs[x->cur] + x->ncells, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return DSMC_EHIP;
    if (x->comp_reseed &&  // a moved reseed not yet completed: its count, if it goes ahead
        hipMemcpyAsync(&n_re, x->cs[1 - x->cur] + x->ncells, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return DSMC_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return DSMC_EHIP;
    if (x->comp_reseed && h.reseed_err == 0u) n = n_re;
    out->bits = h.status;
    out->moved = x->classified ? 1u : 0u;
    out->n_particles = n;
    out->ncoll = h.ncoll;
    out->ncand = h.ncand;
    out->nwall = h.nwall;
    out->nfar = h.nfar_total + h.nfar[0] + h.nfar[1];
    if (clear) {
        k_clear_status<<<1, 64, 0, s>>>(x->ctr);
        if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    }
    return DSMC_OK;
}

static int dsmc_get_views_impl(dsmc_ctx *x, dsmc_views *out)
{
    if (!x) return DSMC_EINVAL;
    if (!out) return fail(DSMC_EINVAL, "out is NULL");
    TRY(settle(x, x->last));  // a pending reseed, on the stream of the last call
    out->current = x->cur;
    out->cell_start = x->cs[x->cur];
    out->nbar = x->nbar;
    out->sigcmax = x->sigcmax;
    out->rem = x->rem;
    out->mom_sums = x->mom;
    out->nsamples = x->nsamples;
    out->step = x->step;
    out->reseed_events = x->reseed_events;
    return DSMC_OK;
}

static int dsmc_profile_enable_impl(dsmc_ctx *x, int32_t enable)
{
    if (!x) return DSMC_EINVAL;
    x->prof = enable != 0;
    return DSMC_OK;
}

static int dsmc_profile_read_impl(dsmc_ctx *x, int32_t kernel, double *ms_total, int64_t *launches)
{
    if (!x) return DSMC_EINVAL;
    if (kernel < 0 || kernel >= DSMC_K_COUNT) return fail(DSMC_EINVAL, "unknown kernel id");
    double tot = 0.0;
    int64_t cnt = 0;
    std::vector<ProfRec> keep;
    for (const ProfRec &r : x->recs) {
        if (r.kid != kernel) {
            keep.push_back(r);
            continue;
        }
        if (hipEventSynchronize(r.b) != hipSuccess) return DSMC_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return DSMC_EHIP;
        tot += ms;
        cnt += 1;
        x->pool.push_back(r.a);
        x->pool.push_back(r.b);
    }
    x->recs.swap(keep);
    if (ms_total) *ms_total = tot;
    if (launches) *launches = cnt;
    return DSMC_OK;
}

static int graph_create(dsmc_ctx *x, int32_t nsteps, int32_t sample_every, bool moved, void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (nsteps < 2 || (nsteps & 1) || sample_every < 0)
        return fail(DSMC_EINVAL, "nsteps must be even and >= 2, sample_every >= 0");
    if (sample_every > 0 && nsteps % sample_every != 0)
        return fail(DSMC_EINVAL, "nsteps must be a multiple of sample_every");
    hipStream_t s = S(stream);
    if (s == nullptr) return fail(DSMC_EINVAL, "capture needs a created stream, not the null stream");
    TRY(settle(x, s));  // a pending reseed is completed first
    TRY(release_graph(x));
    // capture one dsmc_step call with steps counted from 0; the host-side
    // bookkeeping of the capture is undone afterwards (nothing ran)
    // (a graph of dsmc_step calls begins with the moving pass of a settled
    // state; one of dsmc_step_moved calls starts from, and ends in, a moved one)
    const int64_t step = x->step, nsamples = x->nsamples;
    const int cur = x->cur;
    const bool prof = x->prof, classified = x->classified, comp_pending = x->comp_pending;
    x->step = 0;
    x->prof = false;
    x->capturing = true;
    x->classified = moved;
    x->comp_pending = false;  // (a pending completion runs eagerly before a replay)
    int rc = DSMC_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = DSMC_EHIP;
    const int rc_step = rc == DSMC_OK ? step_run(x, nsteps, sample_every, moved, stream) : DSMC_OK;
    hipGraph_t g = nullptr;
    if (rc == DSMC_OK && hipStreamEndCapture(s, &g) != hipSuccess) rc = DSMC_EHIP;
    if (rc == DSMC_OK) rc = rc_step;
    if (rc == DSMC_OK && hipGraphInstantiate(&x->gexec, g, nullptr, nullptr, 0) != hipSuccess) rc = DSMC_EHIP;
    x->capturing = false;
    x->step = step;
    x->nsamples = nsamples;
    x->cur = cur;
    x->prof = prof;
    x->classified = classified;
    x->comp_pending = comp_pending;
    if (rc != DSMC_OK) {
        if (g) (void)hipGraphDestroy(g);
        x->gexec = nullptr;
        return rc;
    }
    x->graph = g;
    x->g_nsteps = nsteps;
    x->g_sample_every = sample_every;
    x->g_cur = cur;
    x->g_moved = moved;
    return DSMC_OK;
}

static int dsmc_graph_launch_impl(dsmc_ctx *x, void *stream)
{
    if (!x) return DSMC_EINVAL;
    if (!x->gexec) return fail(DSMC_ESTATE, "no step graph (none created, or released by a re-tiling)");
    // the captured parities and sampling pattern must hold from this step (a
    // pending reseed, completed first, moves the state to the other buffer);
    // checked before anything is enqueued
    const int cur = x->pending ? 1 - x->cur : x->cur;
    if ((x->step & 1) || cur != x->g_cur)
        return fail(DSMC_ESTATE, "the current step must be even, on the state buffer the graph was captured with");
    if (x->g_sample_every > 0 && x->step % x->g_sample_every != 0)
        return fail(DSMC_ESTATE, "the current step is not aligned with the graph's sampling period");
    if (x->step + x->g_nsteps > (int64_t)0xFFFFFFFF) return fail(DSMC_ESTATE, "step counter beyond 2^32");
    if (!x->g_moved && x->classified)
        return fail(DSMC_ESTATE, "the state is moved (dsmc_step_moved) and the graph starts from a settled one");
    hipStream_t s = S(stream);
    if (x->g_moved && !x->classified) {
        TRY(step_run(x, 0, 0, true, stream));  // the moving pass first (completes a pending reseed)
        if (x->cur != x->g_cur)
            return fail(DSMC_ESTATE, "the moved state is on the other buffer than the graph was captured with");
    }
    if (x->g_moved) TRY(complete(x, s));  // cells left unmoved, or a moved reseed
    TRY(settle(x, s));
    x->last = s;
    k_set_step_base<<<1, 64, 0, s>>>(x->ctr, (uint32_t)x->step);
    if (hipGetLastError() != hipSuccess) return DSMC_EHIP;
    if (hipGraphLaunch(x->gexec, s) != hipSuccess) return DSMC_EHIP;
    if (x->g_moved) x->comp_pending = x->nrep == 1;  // its last step left wall tiles unmoved
    x->step += x->g_nsteps;
    if (x->g_sample_every > 0) x->nsamples += x->g_nsteps / x->g_sample_every;
    return DSMC_OK;
}

int dsmc_set_tiling(dsmc_ctx *x, int32_t particles_per_tile, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_set_tiling", dsmc_set_tiling_impl(x, particles_per_tile, stream));
}

int dsmc_autotune(dsmc_ctx *x, int32_t steps_per_trial, int32_t sample_every, dsmc_tuning *out, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_autotune", dsmc_autotune_impl(x, steps_per_trial, sample_every, out, stream));
}

int dsmc_replica_counters(dsmc_ctx *x, uint64_t *out, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_replica_counters", dsmc_replica_counters_impl(x, out, stream));
}

int dsmc_step(dsmc_ctx *x, int32_t nsteps, int32_t sample_every, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_step", dsmc_step_impl(x, nsteps, sample_every, stream));
}

int dsmc_step_moved(dsmc_ctx *x, int32_t nsteps, int32_t sample_every, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_step_moved", dsmc_step_moved_impl(x, nsteps, sample_every, stream));
}

int dsmc_sample_moments(dsmc_ctx *x, double *out, int32_t reset, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_sample_moments", dsmc_sample_moments_impl(x, out, reset, stream));
}

int map_dsmc_to_lbm(dsmc_ctx *x, int32_t lattice, int32_t order, double *f_out, void *stream)
{
    t_reason = nullptr;
    return noted(x, "map_dsmc_to_lbm", map_dsmc_to_lbm_impl(x, lattice, order, f_out, stream));
}

int dsmc_hybrid_cycle(dsmc_ctx *x, const dsmc_hybrid *h, double *f_lb, double *f_tmp, double *avg_out, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_hybrid_cycle", dsmc_hybrid_cycle_impl(x, h, f_lb, f_tmp, avg_out, stream));
}

int map_lbm_to_dsmc(dsmc_ctx *x, int32_t lattice, int32_t order, const double *f_in, const int32_t *cell_ids,
                    int32_t nsel, void *stream)
{
    t_reason = nullptr;
    return noted(x, "map_lbm_to_dsmc", map_lbm_to_dsmc_impl(x, lattice, order, f_in, cell_ids, nsel, stream));
}

int dsmc_read_status(dsmc_ctx *x, dsmc_status *out, int32_t clear, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_read_status", dsmc_read_status_impl(x, out, clear, stream));
}

int dsmc_get_views(dsmc_ctx *x, dsmc_views *out)
{
    t_reason = nullptr;
    return noted(x, "dsmc_get_views", dsmc_get_views_impl(x, out));
}

int dsmc_profile_enable(dsmc_ctx *x, int32_t enable)
{
    t_reason = nullptr;
    return noted(x, "dsmc_profile_enable", dsmc_profile_enable_impl(x, enable));
}

int dsmc_profile_read(dsmc_ctx *x, int32_t kernel, double *ms_total, int64_t *launches)
{
    t_reason = nullptr;
    return noted(x, "dsmc_profile_read", dsmc_profile_read_impl(x, kernel, ms_total, launches));
}

int dsmc_graph_create(dsmc_ctx *x, int32_t nsteps, int32_t sample_every, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_graph_create", graph_create(x, nsteps, sample_every, false, stream));
}

int dsmc_graph_create_moved(dsmc_ctx *x, int32_t nsteps, int32_t sample_every, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_graph_create_moved", graph_create(x, nsteps, sample_every, true, stream));
}

int dsmc_graph_launch(dsmc_ctx *x, void *stream)
{
    t_reason = nullptr;
    return noted(x, "dsmc_graph_launch", dsmc_graph_launch_impl(x, stream));
}

const char *dsmc_last_error(const dsmc_ctx *x)
{
    if (!x) return "no context";
    return x->err;
}

void dsmc_destroy(dsmc_ctx *x)
{
    if (!x) return;
    if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
    if (x->graph) (void)hipGraphDestroy(x->graph);
    for (const ProfRec &r : x->recs) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : x->pool) (void)hipEventDestroy(e);
    release_ctx(x);
}

}  // extern "C"
