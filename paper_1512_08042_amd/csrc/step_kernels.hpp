// Kernel argument blocks and declarations shared by the kernel sources and
// the host side of libdsmc (passed by value; all pointers are device memory).
#pragma once

#include <utility>

#include "dsmc_device.hpp"

namespace dsmc {

// NTC constants of one step's collisions
struct NtcParams {
    double K, dt;       // F_N sigma_T / V_c and the time step
    uint32_t k0, k1;    // Philox key
    uint32_t step;      // index of the step whose collisions these are
    int nbar_mode;
    int cbase;          // first cell of the channel (draws are keyed by the cell's index inside it)
};

// One channel of a context.  A context holds one channel, or a batch of
// independent channels (replicas) stored one after the other in the cell
// and particle arrays; every replica keeps its own geometry, time step,
// force, collision constant and Philox key, and its random draws are keyed
// by cell and slot indices inside the replica, so each replica evolves
// exactly as the same channel alone would.
struct RepConst {
    Geometry G;
    double dt, g, K;       // time step, acceleration, F_N sigma_T / V_c
    uint32_t k0, k1;       // Philox key (the replica's seed)
    int32_t cbase, cend;   // its cells [cbase, cend) in the context's cell arrays
    int32_t pbase;         // its first particle slot (fixed: no particle leaves its channel)
    int32_t ppc;
};

// Per-cell partition of a moved state: inside every old cell's slot range
// the particles are grouped by direction code 0..9 (the 9 near moves, then
// long jumps), each group in slot order; grp[c][d] holds the first slot of
// group d and grp[c][NGRP] the end of the cell's range.
constexpr int NGRP = NDIR + 1;
constexpr int GSTRIDE = NGRP + 1;  // per cell: first slot of each group, then the cell end

// Everything the step kernels need that stays fixed for a context; kept in
// device memory (inside the workspace) so that a launch passes a pointer
// and a few words instead of a large argument block.
struct TileConst {
    void *st[2][5];          // the two state buffers (x, y, vx, vy, vz; double or float)
    int32_t *cs[2];          // their cell_start
    int32_t *grp[2];         // [ncells][GSTRIDE] first slot of every group and the cell end, by step parity
    int32_t *far[2];         // long-jump lists, by step parity
    int32_t *farcnt[2];      // [ncells] long jumps arriving per cell, by step parity
    const int32_t *plan;     // [ncells][2 * NDIR] arriving near groups of the step (see k_cell_count)
    double *scr;             // [capacity] scratch of oversized tiles
    int32_t *scr_i;          // [capacity] scratch of oversized tiles
    Counters *ctr;
    unsigned long long *tstat;  // [tiles][3] running collisions, candidates and wall hits of every tile
    double *mom;             // [11][ncells] sums
    double *nbar, *sigcmax, *rem;
    int32_t *mark;           // [ncells] cells of a pending reseed (list index + 1, else 0)
    // a moved state's completion pass (k_complete): per cell its reason to
    // be completed (1: its tile ended unmoved, 2: a reseed replaced it), the
    // listed cells, and a moved reseed's new particles (first slot after
    // the appended base, count) per reseed list entry
    int32_t *comp, *complist, *appoff;
    const int32_t *nnew;
    const RepConst *rep;     // [nrep] the channels (stored right after this block, at REP_OFFSET)
    double s_th;             // sqrt(kT/m)
    int nbar_mode, ncells, far_cap, nrep;
    int cap;                 // slots of a state buffer (bound of every source slot)
};

// the channels' constants follow the TileConst block in device memory, so a
// tile reaches its channel's fields with one scalar load from the argument
constexpr size_t REP_OFFSET = (sizeof(TileConst) + 63) & ~size_t(63);

// The tile table: per tile its first cell, its channel, and that cell's row
// and column in the channel.  A channel whose rows hold a whole number of
// tiles, at least two bands wide, lists its tiles in bands of TILE_BAND tiles
// across x, each band row by row: the tiles of the rows above and below a
// cell, which read its source groups, then run a few tiles apart instead of
// a whole row apart and share the cache lines those groups split.
constexpr int TILE_WORDS = 4;
constexpr int TILE_BAND = 8;

// One launch of a step kernel.  k_step: the DSMC step `step` (collisions
// of that step, then the move of step + 1), reading buffer cur and writing
// 1 - cur.  k_classify (classify = 1): the move of step `step` for the
// settled state in buffer cur, in place; with `reseed`, the state of a
// pending reseed instead: the kept cells' particles are read from buffer
// 1 - cur (at its cell starts) and the marked cells' new particles from
// buffer cur, all moved into buffer cur.  Buffers of parity step & 1 hold
// the partition read by the step's sort.
//
// A moved state (a call that ends moved, see dsmc_step_moved) may be
// reseeded before the next step, and a reseed changes the cell starts that
// key the wall draws of the coming move.  So the last step of such a call
// (flags STEP_DEFER) leaves every tile with a particle bound for a wall
// unmoved: it writes the tile settled, in place, and lists its cells.
// k_complete (flags STEP_COMPLETE) later moves the listed cells one by one
// as k_classify would, keyed by the cell starts after the reseed, if any,
// and moves a reseeded cell's new particles, which the reseed appended
// after the state's last slot.
constexpr int STEP_DEFER = 1;
constexpr int STEP_COMPLETE = 2;
constexpr int STEP_COMP_RESEED = 4;  // with STEP_COMPLETE: a moved reseed precedes it

struct StepArgs {
    const TileConst *kc;
    const int32_t *tiles;  // [tiles][TILE_WORDS]: first cell, replica, and the first cell's row and column
    uint32_t step;
    int cur, sample, classify;
    int r;                 // replica of the tile (the launch's, or set by the tile kernel from the table)
    int dev_step;          // step graphs: add the device step base to `step`
    int reseed;            // k_classify: complete a pending reseed (see above)
    int flags;             // STEP_DEFER (k_step), STEP_COMPLETE (k_complete)

    // the blocks are read through the constant address space: they do not
    // change while a kernel runs, so their fields come in by scalar loads
    __device__ const __attribute__((address_space(4))) TileConst &K() const
    {
        return *(const __attribute__((address_space(4))) TileConst *)kc;
    }
    __device__ const __attribute__((address_space(4))) RepConst &R() const
    {
        return ((const __attribute__((address_space(4))) RepConst *)((const __attribute__((address_space(4))) char *)kc +
                                                                     REP_OFFSET))[r];
    }

    __device__ Geometry geo() const
    {
        Geometry g;
        g.nx = R().G.nx;
        g.ny = R().G.ny;
        g.Lx = R().G.Lx;
        g.H = R().G.H;
        return g;
    }
    __device__ int po() const { return classify ? (int)(step & 1u) : (int)((step + 1u) & 1u); }
    template <class S>
    __device__ const S *in(int k) const { return (const S *)K().st[cur][k]; }
    template <class S>
    __device__ S *out(int k) const { return (S *)K().st[classify ? cur : 1 - cur][k]; }
    template <class S>
    __device__ const S *old_in(int k) const { return (const S *)K().st[1 - cur][k]; }  // reseed: kept cells
    __device__ const int32_t *cs_old() const { return K().cs[cur]; }
    __device__ const int32_t *cs_new() const { return K().cs[classify ? cur : 1 - cur]; }
    __device__ const int32_t *grp_in() const { return K().grp[step & 1u]; }
    __device__ int32_t *grp_out() const { return K().grp[po()]; }
    __device__ const int32_t *far_in() const { return K().far[step & 1u]; }
    __device__ int32_t *farcnt_in() const { return K().farcnt[step & 1u]; }
    __device__ int far_in_slot() const { return (int)(step & 1u); }
    __device__ int32_t *far_out() const { return K().far[po()]; }
    __device__ int32_t *farcnt_out() const { return K().farcnt[po()]; }
    __device__ int far_out_slot() const { return po(); }
    __device__ MoveParams M1() const
    {
        MoveParams M;
        M.dt = R().dt;
        M.g = R().g;
        M.s_th = K().s_th;
        M.k0 = R().k0;
        M.k1 = R().k1;
        M.step = classify ? step : step + 1u;
        return M;
    }
    __device__ NtcParams N() const
    {
        NtcParams P;
        P.K = R().K;
        P.dt = R().dt;
        P.k0 = R().k0;
        P.k1 = R().k1;
        P.step = step;
        P.nbar_mode = K().nbar_mode;
        P.cbase = R().cbase;
        return P;
    }
};

struct CellArgs {
    const int32_t *grp;      // [ncells][GSTRIDE] group starts and cell end of the moved state
    int32_t *plan;           // [ncells][2 * NDIR] out: each cell's arriving near groups, in sorted order
    const int32_t *farcnt;   // [ncells] long jumps arriving per cell
    int32_t *countnew;
    int32_t *blocksum;
    const RepConst *rep;     // the channels
    const int32_t *cell_rep; // [ncells] channel of every cell
    int ncells;
    int nx1, ny1;            // > 0: one channel of nx1 x ny1 cells (rep and cell_rep are not read)
    // one block (ncells <= 256): the cell starts are written here too, and
    // the step's counters retired, as k_cell_final does for larger grids
    int32_t *cs_out;
    Counters *ctr;
    int reset_slot;
};

// the initial Maxwellian of one channel: its cells start at cs, nbar, ...
// (already offset to its first cell), its particles at st (offset to its
// first slot); cell starts are written as pbase + c * ppc
struct InitArgs {
    void *st[5];  // double or float
    int32_t *cs;
    double *nbar, *sigcmax, *rem;
    int nx, ncells, ppc, pbase;
    double s_th, sigcr0;
    uint32_t k0, k1;
};

struct AdoptArgs {
    const void *in[5];  // double or float
    void *out[5];
    int32_t *cellid, *counts, *cursor, *perm;
    const int32_t *cs;
    Geometry G;
    int64_t n;
};

struct ReseedArgs {
    const double *f;     // [Q][ncells]
    const int32_t *cells;
    int nsel;
    int32_t *mark;       // [ncells], 0 = not listed, else list index + 1
    double *prm;         // [nsel][12]
    int32_t *nnew;       // [nsel]
    const int32_t *cs_old;
    int32_t *cs_new;
    int32_t *countnew;
    int32_t *blocksum;
    const void *in[5];  // double or float
    void *out[5];
    Counters *ctr;
    Lattice L;
    int nx, ncells, ppc, order, ar_max_tries;
    int64_t capacity;
    double s_th;
    uint32_t k0, k1, event;
    // a reseed of a moved state (moved != 0): the new particles of list
    // entry i go to the moved buffer (out) from slot cs_old[ncells] +
    // appoff[i]; the replaced cells are listed for the completion pass
    int moved;
    int32_t *appoff, *comp, *complist;
};

// Velocity sets in the ABI order (shells of increasing |e|, counter-clockwise
// within a shell from the first-octant representative) as compile-time
// tables, so the lattice kernels keep only the scale r and one weight per
// shell in registers; the host checks them against its lattice tables.
template <int Q>
struct VelSet;
template <>
struct VelSet<9> {
    static constexpr int R = 1;  // largest |e| component
    static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int sh[9] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
};
template <>
struct VelSet<37> {
    static constexpr int R = 3;
    static constexpr int ex[37] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, 1, -1, -2, -2, -1, 1, 2,
                                   2, -2, -2, 2, 3, 0, -3, 0, 3, 1, -1, -3, -3, -1, 1, 3};
    static constexpr int ey[37] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 1, 2, 2, 1, -1, -2, -2, -1,
                                   2, 2, -2, -2, 0, 3, 0, -3, 1, 3, 3, 1, -1, -3, -3, -1};
    static constexpr int sh[37] = {0, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4,
                                   5, 5, 5, 5, 6, 6, 6, 6, 7, 7, 7, 7, 7, 7, 7, 7};
};

// Element i of plane q of a [Q][nn] array, addressed as a uniform plane base
// plus a 32-bit byte offset (the host keeps nn * 8 below 2^32), so the loads
// and stores take one 32-bit register per lane instead of a 64-bit address.
__device__ __forceinline__ const double *plane_ptr(const double *base, size_t nn, int q, uint32_t i)
{
    return (const double *)((const char *)(base + (size_t)q * nn) + (size_t)(uint32_t)(i * 8u));
}
__device__ __forceinline__ double *plane_ptr(double *base, size_t nn, int q, uint32_t i)
{
    return (double *)((char *)(base + (size_t)q * nn) + (size_t)(uint32_t)(i * 8u));
}

// acc += C v for a compile-time integer C (nothing for 0, an add for +-1)
template <int C>
__device__ __forceinline__ void cmad(double &acc, double v)
{
    if constexpr (C == 1)
        acc += v;
    else if constexpr (C == -1)
        acc -= v;
    else if constexpr (C != 0)
        acc += (double)C * v;
}

// f(std::integral_constant<int, q>) for q = 0 .. N-1, unrolled at compile time
template <class F, int... qs>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, qs...>)
{
    (f(std::integral_constant<int, qs>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

struct LatShells {
    int Q;         // 9 or 37
    double r;      // xi_q = r e_q
    double ws[8];  // weight of each shell
};

// DSMC2LB of n cells c_off + i c_stride into nodes n_off + i n_stride of f
struct ProjectArgs {
    const double *mom;  // sums [11][ncells]
    double *f;          // [Q][nn_out]
    LatShells L;        // r and the shell weights
    double rho_scale;   // 1 / (samples the sums hold * particles per cell)
    double is1;         // 1 / sqrt(kT/m)
    int ncells, order;
    int equilibrium;    // 1: only rho and u enter (Eq. (feq_dsmc)); 0: the full projection
    int n, c_off, c_stride, n_off, n_stride;
    int64_t nn_out;
};

struct LbmArgs {
    const double *f;
    double *ft;
    double *keep;  // when not null, also receives f (a checkpoint of the step's input)
    LatShells L;
    int nx, ny, y_mode, K;
    int xb;        // held inflow columns 0 .. xb-1
    double tau, gx;
};

struct LbmAdjArgs {
    const double *f;       // populations entering the step [Q][nx*ny]
    const double *lam_in;  // cotangent of the step's output
    double *lam_out;       // cotangent of its input
    double *partial;       // [gridDim.x][2]: per-block (dJ/dg, dJ/dtau)
    int accumulate;        // add to partial (else overwrite)
    LatShells L;
    int nx, ny, y_mode, K;
    double tau, gx;
};

struct HermiteArgs {
    const double *f;      // [Q][nnodes]
    const int32_t *nodes; // [nsel]
    double *a;            // [nh][nsel]
    const double *a_bar;  // [nh][nsel]
    double *f_bar;        // [Q][nnodes]
    int64_t nnodes;
    int nsel, nh;
    Lattice L;
};

struct ProjectAdjArgs {
    const double *f_bar;  // [Q][ncells]
    const double *avg;    // [11][ncells]
    double *avg_bar;      // [11][ncells]
    Lattice L;
    int ncells, ppc, order;
    double s1;            // sqrt(kT/m)
};

// TC cells per tile (one wave); tiles of up to 64*CH particles are staged in
// LDS; S is the stored particle type (double, or float with FP64 arithmetic)
template <int TC, int CH, class S, bool DEFER>
__global__ void k_classify(StepArgs a);
template <int TC, int CH, bool MOVE, class S, bool NT, bool DEFER>
__global__ void k_step(StepArgs a);
__global__ void k_cell_count(CellArgs a);
__global__ void k_scan_blocks(int32_t *blocksum, int nblk, int32_t *cs_out, int ncells, Counters *ctr,
                              int reset_slot);
__global__ void k_average(const double *mom, double *out, size_t n, double S);
template <class S>
__global__ void k_init_maxwell(InitArgs a);
template <class S>
__global__ void k_adopt_count(AdoptArgs a);
__global__ void k_block_sums(const int32_t *counts, int ncells, int32_t *blocksum);
__global__ void k_cell_final(const int32_t *counts, int ncells, const int32_t *blocksum, int32_t *cs, Counters *ctr,
                             int reset_slot);
__global__ void k_block_scan(const int32_t *counts, int ncells, const int32_t *blockoff, int32_t *cs);
__global__ void k_adopt_place(AdoptArgs a);
__global__ void k_adopt_sortcell(AdoptArgs a);
template <class S>
__global__ void k_adopt_gather(AdoptArgs a);
__global__ void k_fill_f64(double *p, size_t n, double v);
__global__ void k_fill_i32(int32_t *p, size_t n, int32_t v);
__global__ void k_zero_counters(Counters *c);
template <int CH, class S>
__global__ void k_complete(StepArgs a);
template <class S>
__global__ void k_comp_far(StepArgs a, int pass);
__global__ void k_comp_done(Counters *ctr, int reseed);
__global__ void k_reseed_appoff(ReseedArgs a);
__global__ void k_reseed_list(ReseedArgs a);
__global__ void k_clear_status(Counters *c);
__global__ void k_tile_stats(const unsigned long long *tstat, int ntiles, Counters *c);
__global__ void k_set_step_base(Counters *c, uint32_t step);
__global__ void k_replica_stats(const unsigned long long *tstat, const RepConst *rep, unsigned long long *out);
__global__ void k_far_reset(Counters *c, int slot);

template <int Q>
__global__ void k_project(ProjectArgs a);
__global__ void k_reseed_prep(ReseedArgs a);
__global__ void k_reseed_count(ReseedArgs a);
__global__ void k_reseed_starts(ReseedArgs a);
template <class S>
__global__ void k_reseed_copy(ReseedArgs a);
template <class S>
__global__ void k_reseed_gen(ReseedArgs a);
__global__ void k_reseed_done(Counters *ctr);
// lattice step (YM: y_mode 0 periodic, 1 buffer rows, 2 diffuse walls) and
// its adjoint (YB: y_mode 1) for Q velocities;
// NARROW: the grid is narrower than the largest velocity component
template <int Q, int YM, bool NARROW>
__global__ void k_lbm(LbmArgs a);
template <int Q, bool YB, bool NARROW>
__global__ void k_lbm_adjoint(LbmAdjArgs a);
__global__ void k_adjoint_finish(const double *partial, int nblk, double *grad);
__global__ void k_hermite_moments(HermiteArgs a);
__global__ void k_hermite_moments_adjoint(HermiteArgs a);
__global__ void k_project_adjoint(ProjectAdjArgs a);

}  // namespace dsmc
