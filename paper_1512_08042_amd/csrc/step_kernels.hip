// DSMC particle step on gfx950: move + wall + cell index, deterministic
// stable counting sort, NTC hard-sphere collisions, moment sampling.
//
// Design.  Particles move at most one cell per step in all but rare cases,
// so the stable sort by new cell is fixed by the (old cell, direction)
// groups, direction d one of the 9 moves inside the 3x3 neighbourhood (or a
// long jump): inside new cell c the order is "arriving groups by old cell,
// each group in old-slot order".  Between two steps of a call the state is
// kept moved for the coming step and partitioned by direction inside every
// old cell, with the group sizes beside it, so that each group is one
// contiguous run.  One step is then
//   cell kernels  (one thread per new cell) sum the groups arriving in c and
//                 scan the counts into the new cell_start;
//   k_step        (one wave per tile of TC cells) gathers the tile's groups,
//                 runs the NTC collisions and the moment sample on the
//                 staged tile, moves it for the next step and writes it out
//                 partitioned by the next step's directions.
// The state is read once and written once per step; nothing depends on the
// order of atomic operations.
#include <climits>

#include "dsmc_device.hpp"
#include "step_kernels.hpp"

namespace dsmc {

__device__ __forceinline__ void add_moments(double *acc, double vx, double vy, double vz)
{
    acc[0] += 1.0;
    acc[1] += vx;
    acc[2] += vy;
    acc[3] += vx * vx;
    acc[4] += vx * vy;
    acc[5] += vy * vy;
    acc[6] += vx * vx * vx;
    acc[7] += vx * vx * vy;
    acc[8] += vx * vy * vy;
    acc[9] += vy * vy * vy;
    acc[10] += vz * vz;
}

// ---- block-level integer scan helpers (256 threads) -------------------------
__device__ __forceinline__ int block_reduce_256(int v, int *lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    const int t = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return t;
}

// exclusive prefix of v over the 256 threads of the block
__device__ __forceinline__ int block_exscan_256(int v, int *lds)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        if (lane >= off) inc += u;
    }
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; ++k) woff += lds[k];
    __syncthreads();
    return woff + inc - v;
}

// append a long jump of the particle written to slot q (old cell o, new cell nc)
__device__ __forceinline__ void record_far(int32_t *far, int32_t *farcnt, Counters *ctr, int slot, int far_cap, int q,
                                           int o, int nc)
{
    atomicAdd(&farcnt[nc], 1);
    const uint32_t idx = atomicAdd(&ctr->nfar[slot], 1u);
    if (idx < (uint32_t)far_cap) {
        far[4 * (size_t)idx + 0] = q;
        far[4 * (size_t)idx + 1] = o;
        far[4 * (size_t)idx + 2] = nc;
        far[4 * (size_t)idx + 3] = -1;
    } else {
        atomicOr(&ctr->status, ST_FAR_OVERFLOW);
    }
}

// ---- tiles of cells, one wave each ------------------------------------------------
constexpr int NTC_ROUND = 32;  // NTC candidates drawn per round (all cells of a tile)

// Tiles of four cells keep their cells' NTC state and running moment sums
// in LDS from the set-up to their use: held in registers across the gather,
// these spilled to scratch (about 3 KB of scratch traffic per tile).  The
// smaller tiles keep them in registers and their LDS at 8 KB.
template <int TC, bool STASH = (TC == 4)>
struct CellStash {
};
template <int TC>
struct CellStash<TC, true> {
    double ntcs[3][TC];            // nbar, sigcmax, rem of each cell
    double mprev[NMOM][TC];        // the moment sums before this step
};

template <int TC, int CH, class S>
struct TileLds : CellStash<TC> {
    static constexpr int CAP = 64 * CH;
    S v[3][CAP];                   // vx, vy, vz of the tile's particles (stored precision), in new-slot order;
                                   // positions stay in registers of the lane that owns the slot
    // arrays of different phases share their space (each phase ends at a
    // barrier): the NTC draws (collisions) and the long jumps' source slots
    // (gather), then the group keys (move to write)
    union {
        int32_t kr[CAP];           // next-step group (low 6 bits) and rank inside it, per slot
        struct {
            double dr[5][NTC_ROUND];   // one round of NTC draws: R, cos(theta), sin(theta), cos(phi), sin(phi)
            int32_t di[2][NTC_ROUND];  // ... and the candidate pairs (i, j)
        };
    };
    long long mc[TC];              // NTC candidates of each cell this step
    int32_t csn[TC + 1];           // cell starts of the tile after the sort
    int32_t tix[TC], tiy[TC];      // cell coordinates
    int32_t anyfar;                // long jumps arrive in some cell of the tile
    int32_t kdelta;                // wall-draw keys: slot + kdelta (a completed cell's starts after a reseed)
    // the 9 near groups arriving in each cell, in the order of the sort (by
    // source cell; groups without a source last, empty); the keys and sizes
    // only where long jumps arrive
    int32_t gsrc[TC][NDIR];        // their first source slots
    int32_t gstart[TC][NDIR];      // their first slots inside the cell
    int32_t gkey[TC][NDIR];        // their source cells (INT_MAX: none)
    int32_t gn[TC][NDIR];          // their sizes
    int32_t nfin[TC];              // long jumps arriving in each cell
    int32_t rsrc[TC];              // classify after a reseed: first old slot of a kept cell, -1 for a new one
    int32_t run[TC * NGRP];        // sizes of the next step's groups of the tile's cells ...
    int32_t excl[TC * NGRP];       // ... and their offsets inside each cell
};

// cell (0 .. ntc-1) of tile slot i (0 <= i < nt)
template <int TC, int CH, class S>
__device__ __forceinline__ int tile_cell(const TileLds<TC, CH, S> &L, int ntc, int D0, int i)
{
    int t = 0;
#pragma unroll
    for (int u = 1; u < TC; ++u) t += (i >= L.csn[u] - D0) ? 1 : 0;  // csn[u] = tile end for u > ntc
    return t;
}

// source slot of the particle that the sort puts at offset r of tile cell t
// when a near group holds that offset; -1 otherwise (a long jump's slot).
// The group is the last one starting at or before r (empty groups start where
// the next one does).  Without long jumps in the tile (`gaps` false) the near
// groups fill the cell from offset 0 and every offset is in its group; with
// them, offsets before the first group or after a group's end are long
// jumps' slots.
template <int TC, int CH, class S>
__device__ __forceinline__ int tile_source(const TileLds<TC, CH, S> &L, int t, int r, bool gaps)
{
    int k = 0;
#pragma unroll
    for (int u = 1; u < NDIR; ++u) k += (r >= L.gstart[t][u]) ? 1 : 0;
    const int off = r - L.gstart[t][k];
    if (gaps && (off < 0 || off >= L.gn[t][k])) return -1;
    return L.gsrc[t][k] + off;
}

// ---- long jumps (moves of more than one cell; rare) ---------------------------
// The pass that moved the particles recorded each long jump (slot, old cell,
// new cell) in a list of far_cap entries and counted all of them.  When more
// were counted than the list holds, the list is incomplete and the long jumps
// are found in the partitioned state itself instead: they are the DIR_FAR
// group of every cell of the channel, and each one's new cell follows from
// its stored position exactly as the recording pass found it.
__device__ __forceinline__ bool far_listed(const StepArgs &a)
{
    return a.K().ctr->nfar[a.far_in_slot()] <= (uint32_t)a.K().far_cap;
}

// new cell (index in the context) of the long jump in input slot q
template <class S>
__device__ __forceinline__ int far_new_cell(const StepArgs &a, int q)
{
    int nix, niy;
    cell_xy(a.geo(), (double)a.template in<S>(0)[q], (double)a.template in<S>(1)[q], nix, niy);
    return a.R().cbase + niy * a.geo().nx + nix;
}

// Long jumps arriving in tile cell t, from the list (one lane per cell):
// every near group is preceded in the sort by the long jumps from smaller
// source cells; counts them and shifts the group starts.
template <int TC, int CH, class S>
__device__ void tile_far_shift(const StepArgs &a, TileLds<TC, CH, S> &L, int t, int c, int nfin)
{
    const uint32_t nf = a.K().ctr->nfar[a.far_in_slot()];
    int shift[NDIR];
#pragma unroll
    for (int k = 0; k < NDIR; ++k) shift[k] = 0;
    int found = 0;
    for (uint32_t e = 0; e < nf; ++e) {
        if (a.far_in()[4 * (size_t)e + 2] != c) continue;
        ++found;
        const int o = a.far_in()[4 * (size_t)e + 1];
#pragma unroll
        for (int k = 0; k < NDIR; ++k)
            if (o < L.gkey[t][k]) shift[k] += 1;
    }
#pragma unroll
    for (int k = 0; k < NDIR; ++k) L.gstart[t][k] += shift[k];
    if (found != nfin) atomicOr(&a.K().ctr->status, ST_INTERNAL);
    a.farcnt_in()[c] = 0;
}

// The same after an overflow, by the whole wave: lane l scans the DIR_FAR
// groups of the channel's cells l, l + 64, ...; the per-lane shifts and
// counts are summed over the wave (integers: exact in any order).  c0 is the
// tile's first cell; lane t < ntc holds nfin of tile cell t.
template <int TC, int CH, class S>
__device__ void tile_far_shift_scan(const StepArgs &a, TileLds<TC, CH, S> &L, int c0, int ntc, int nfin)
{
    const int lane = threadIdx.x;
    const int cb = a.R().cbase, ce = a.R().cend;
    int shift[TC][NDIR], found[TC];
#pragma unroll
    for (int t = 0; t < TC; ++t) {
        found[t] = 0;
#pragma unroll
        for (int k = 0; k < NDIR; ++k) shift[t][k] = 0;
    }
    for (int o = cb + lane; o < ce; o += 64) {
        const int32_t *g = a.grp_in() + (size_t)o * GSTRIDE + DIR_FAR;
        for (int q = g[0]; q < g[1]; ++q) {
            const int t = far_new_cell<S>(a, q) - c0;
#pragma unroll
            for (int u = 0; u < TC; ++u) {
                if (u != t || u >= ntc) continue;
                found[u] += 1;
#pragma unroll
                for (int k = 0; k < NDIR; ++k)
                    if (o < L.gkey[u][k]) shift[u][k] += 1;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < TC; ++t) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) found[t] += __shfl_xor(found[t], off, 64);
#pragma unroll
        for (int k = 0; k < NDIR; ++k) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) shift[t][k] += __shfl_xor(shift[t][k], off, 64);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TC; ++t) {
        if (t != lane || t >= ntc) continue;
#pragma unroll
        for (int k = 0; k < NDIR; ++k) L.gstart[t][k] += shift[t][k];
        if (found[t] != nfin) atomicOr(&a.K().ctr->status, ST_INTERNAL);
        if (nfin > 0) a.farcnt_in()[c0 + t] = 0;
    }
}

// total size of tile cell t's near groups from source cells before o
template <int TC, int CH, class S>
__device__ __forceinline__ int near_before(const TileLds<TC, CH, S> &L, int t, int o)
{
    int r = 0;
    for (int k = 0; k < NDIR; ++k)
        if (L.gkey[t][k] < o) r += L.gn[t][k];
    return r;
}

// stages the long jump from input slot q at offset r of tile cell t (see
// tile_far_gather)
template <int TC, int CH, class S>
__device__ __forceinline__ void far_put(const StepArgs &a, const TileLds<TC, CH, S> &L, S *const *s, int n_old,
                                        int32_t *pick, int t, int q, int r)
{
    const int D0 = L.csn[0];
    const int slot = L.csn[t] - D0 + r;
    if (q < 0 || q >= n_old || slot >= L.csn[t + 1] - D0) {
        atomicOr(&a.K().ctr->status, ST_INTERNAL);
        return;
    }
#pragma unroll
    for (int k = 2; k < 5; ++k) s[k][slot] = a.template in<S>(k)[q];
    if (pick) {
        pick[slot] = q;
    } else {
        s[0][slot] = a.template in<S>(0)[q];
        s[1][slot] = a.template in<S>(1)[q];
    }
}

// Stages the long jumps arriving in the tile at their sorted slots: after
// the near groups of smaller source cells and the long jumps of smaller
// (source cell, source slot).  s[2..4] address the tile's velocity stage;
// positions go to s[0], s[1] too, or, when `pick` is given (positions kept in
// the owner lanes' registers), the source slot goes to pick[slot] for the
// owner lane to fetch.  From the list, lanes take entries in turn.  After an
// overflow, lane l scans the DIR_FAR groups of a contiguous block of the
// channel's cells twice: it counts the tile's arrivals in its block, adds the
// counts of the lanes before it (the earlier source cells), then stages its
// arrivals in (source cell, slot) order.
template <int TC, int CH, class S>
__device__ void tile_far_gather(const StepArgs &a, const TileLds<TC, CH, S> &L, S *const *s, int c0, int ntc,
                                int n_old, int32_t *pick)
{
    const int lane = threadIdx.x;
    if (far_listed(a)) {
        const uint32_t nf = a.K().ctr->nfar[a.far_in_slot()];
        for (uint32_t e = lane; e < nf; e += 64) {
            const int nc = a.far_in()[4 * (size_t)e + 2];
            if (nc < c0 || nc >= c0 + ntc) continue;
            const int t = nc - c0;
            const int q = a.far_in()[4 * (size_t)e], o = a.far_in()[4 * (size_t)e + 1];
            int r = near_before<TC, CH, S>(L, t, o);
            for (uint32_t f = 0; f < nf; ++f) {
                if (a.far_in()[4 * (size_t)f + 2] != nc) continue;
                const int o2 = a.far_in()[4 * (size_t)f + 1], q2 = a.far_in()[4 * (size_t)f];
                if (o2 < o || (o2 == o && q2 < q)) ++r;
            }
            far_put<TC, CH, S>(a, L, s, n_old, pick, t, q, r);
        }
        return;
    }
    const int cb = a.R().cbase, ce = a.R().cend;
    const int blk = (ce - cb + 63) / 64;
    const int o0 = min(cb + lane * blk, ce), o1 = min(o0 + blk, ce);
    int cnt[TC];
#pragma unroll
    for (int t = 0; t < TC; ++t) cnt[t] = 0;
    for (int o = o0; o < o1; ++o) {
        const int32_t *g = a.grp_in() + (size_t)o * GSTRIDE + DIR_FAR;
        for (int q = g[0]; q < g[1]; ++q) {
            const int t = far_new_cell<S>(a, q) - c0;
#pragma unroll
            for (int u = 0; u < TC; ++u)
                if (u == t && u < ntc) cnt[u] += 1;
        }
    }
    // exclusive prefix over the lanes: the arrivals from the earlier blocks
#pragma unroll
    for (int t = 0; t < TC; ++t) {
        int inc = cnt[t];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(inc, off, 64);
            if (lane >= off) inc += v;
        }
        cnt[t] = inc - cnt[t];
    }
    for (int o = o0; o < o1; ++o) {
        const int32_t *g = a.grp_in() + (size_t)o * GSTRIDE + DIR_FAR;
        for (int q = g[0]; q < g[1]; ++q) {
            const int t = far_new_cell<S>(a, q) - c0;
#pragma unroll
            for (int u = 0; u < TC; ++u) {
                if (u != t || u >= ntc) continue;
                far_put<TC, CH, S>(a, L, s, n_old, pick, u, q, near_before<TC, CH, S>(L, u, o) + cnt[u]);
                cnt[u] += 1;
            }
        }
    }
}

// The groups arriving in every cell of the tile, in the order of the stable
// sort: by source cell, each group in source-slot order.  The state read
// here keeps every old cell's particles partitioned by move direction, so a
// near group (source cell s, direction d) is the contiguous run that starts
// after the groups 0 .. d-1 of s; the cell pass before the step wrote each
// cell's plan: the first source slot and the offset inside the cell of its 9
// near groups in sorted order (plan[c][0..8] and plan[c][9..17]), loaded with
// the tile's other per-cell data.  Where long jumps arrive (rare), the
// groups' source cells and sizes are rebuilt and every group preceded by long
// jumps from smaller source cells is shifted.
template <int TC, int CH, class S>
__device__ void tile_groups(const StepArgs &a, TileLds<TC, CH, S> &L, int ntc, int nfin)
{
    const int lane = threadIdx.x, nx = a.geo().nx;
    if (lane < TC) L.nfin[lane] = nfin;
    if (lane == 0) L.anyfar = 0;
    __syncthreads();
    if (ballot64(lane < ntc && nfin > 0) == 0) return;  // no long jumps arrive in the tile
    if (lane < TC * NDIR) {
        const int t = lane / NDIR, k = lane - t * NDIR;
        int key[NDIR], dir[NDIR];
        arrival_order(nx, a.geo().ny, L.tix[t], L.tiy[t], a.R().cbase, key, dir);
        int kk = 0;
#pragma unroll
        for (int u = 0; u < NDIR; ++u) kk = u == k ? key[u] : kk;
        L.gkey[t][k] = kk;
        const int end = k + 1 < NDIR ? L.gstart[t][k + 1] : L.csn[t + 1] - L.csn[t] - L.nfin[t];
        L.gn[t][k] = t < ntc ? end - L.gstart[t][k] : 0;
    }
    __syncthreads();
    if (far_listed(a)) {
        if (lane < ntc && nfin > 0)
            tile_far_shift<TC, CH, S>(a, L, lane, a.R().cbase + L.tiy[lane] * nx + L.tix[lane], nfin);
    } else {
        tile_far_shift_scan<TC, CH, S>(a, L, a.R().cbase + L.tiy[0] * nx + L.tix[0], ntc, nfin);
    }
    if (lane == 0) L.anyfar = 1;
    __syncthreads();
}

// ---- NTC collisions of the tile (Eq. (collisionnumber)) ---------------------------
// Per cell: update the running mean of N, form the candidate count
// 1/2 N Nbar K sigcmax dt + rem (K = F_N sigma_T / V_c), draw candidate pairs
// uniformly (i != j), accept with probability c_r / sigcmax (hard spheres)
// and scatter isotropically in the centre-of-mass frame.  Candidate k of
// cell c at step s draws from counters (2k, c, s, COLL) and (2k+1, c, s,
// COLL).  The draws do not depend on the velocities, so a round of up to
// NTC_ROUND/TC candidates per cell is drawn by the lanes of the wave at
// once; one lane per cell then runs its candidates in order.
template <int TC, int CH, class S>
__device__ __forceinline__ void ntc_draws(TileLds<TC, CH, S> &L, const NtcParams &P, int c0, int ntc, long long k0)
{
    constexpr int KC = NTC_ROUND / TC;
    const int lane = threadIdx.x;
    const int t = lane / KC;
    const long long k = k0 + (lane - t * KC);
    if (lane < NTC_ROUND && t < ntc && k < L.mc[t]) {
        const uint32_t N = (uint32_t)(L.csn[t + 1] - L.csn[t]);
        const uint32_t c = (uint32_t)(c0 + t - P.cbase);  // the cell's index inside its channel
        const U4 u = draw(P.k0, P.k1, (uint32_t)(2 * k), c, P.step, TAG_COLL, 0u);
        const uint32_t i = (uint32_t)(((uint64_t)u.x * (uint64_t)N) >> 32);
        uint32_t j = (uint32_t)(((uint64_t)u.y * (uint64_t)(N - 1)) >> 32);
        if (j >= i) j += 1;
        const U4 w = draw(P.k0, P.k1, (uint32_t)(2 * k + 1), c, P.step, TAG_COLL, 0u);
        const double cth = 2.0 * u53(w.x, w.y) - 1.0;
        double sphi, cphi;
        sincos_turn(u53(w.z, w.w), sphi, cphi);  // phi = 2 pi R
        L.di[0][lane] = (int32_t)i;
        L.di[1][lane] = (int32_t)j;
        L.dr[0][lane] = u53(u.z, u.w);
        L.dr[1][lane] = cth;
        L.dr[2][lane] = sqrt(1.0 - cth * cth);
        L.dr[3][lane] = cphi;
        L.dr[4][lane] = sphi;
    }
}

template <int TC, int CH, class S>
__device__ __forceinline__ void ntc_chain(S *vx, S *vy, S *vz, const TileLds<TC, CH, S> &L, int e0,
                                          int n, double &sig, unsigned long long &ncoll)
{
    for (int e = e0; e < e0 + n; ++e) {
        const int i = L.di[0][e], j = L.di[1][e];
        const double vxi = vx[i], vyi = vy[i], vzi = vz[i];
        const double vxj = vx[j], vyj = vy[j], vzj = vz[j];
        const double dx = vxi - vxj, dy = vyi - vyj, dz = vzi - vzj;
        const double cr = sqrt(dx * dx + dy * dy + dz * dz);
        if (cr > sig) sig = cr;
        if (cr / sig > L.dr[0][e]) {
            const double cth = L.dr[1][e], sth = L.dr[2][e], cphi = L.dr[3][e], sphi = L.dr[4][e];
            const double rx = cr * cth;
            const double ry = cr * sth * cphi;
            const double rz = cr * sth * sphi;
            const double mx = 0.5 * (vxi + vxj);
            const double my = 0.5 * (vyi + vyj);
            const double mz = 0.5 * (vzi + vzj);
            vx[i] = (S)(mx + 0.5 * rx), vy[i] = (S)(my + 0.5 * ry), vz[i] = (S)(mz + 0.5 * rz);
            vx[j] = (S)(mx - 0.5 * rx), vy[j] = (S)(my - 0.5 * ry), vz[j] = (S)(mz - 0.5 * rz);
            ncoll += 1;
        }
    }
}

// v* address the tile's velocities (LDS or global), slot 0 = first of the tile
template <int TC, int CH, class S>
__device__ __forceinline__ void tile_ntc(S *vx, S *vy, S *vz, TileLds<TC, CH, S> &L,
                                         const NtcParams &P, int c0, int ntc, bool own, double &nbar,
                                         double &sig, double &rem, unsigned long long &ncoll,
                                         unsigned long long &ncand)
{
    constexpr int KC = NTC_ROUND / TC;
    const int lane = threadIdx.x;
    const int D0 = L.csn[0];
    long long M = 0;
    int s0 = 0;
    if (lane < TC) L.mc[lane] = 0;
    if (own) {
        const int N = L.csn[lane + 1] - L.csn[lane];
        s0 = L.csn[lane] - D0;
        const double Nd = (double)N;
        nbar = nbar + (Nd - nbar) / (double)(P.step + 1);
        const double pairf = (P.nbar_mode == 1) ? (Nd - 1.0) : nbar;
        double X = 0.5 * Nd * pairf * P.K * sig * P.dt + rem;
        if (!(X > 0.0)) X = 0.0;
        const double Mf = floor(X);
        rem = X - Mf;
        M = N < 2 ? 0 : (long long)Mf;
        L.mc[lane] = M;
    }
    __syncthreads();
    for (long long k0 = 0; ballot64(lane < ntc && M > k0) != 0; k0 += KC) {
        ntc_draws<TC, CH, S>(L, P, c0, ntc, k0);
        __syncthreads();
        if (lane < ntc && M > k0) {
            const int n = (int)min(M - k0, (long long)KC);
            ntc_chain<TC, CH, S>(vx + s0, vy + s0, vz + s0, L, lane * KC, n, sig, ncoll);
            ncand += (unsigned long long)n;
        }
        __syncthreads();
    }
}

// moment sample: a team of 64/TC lanes per cell; the lane that owns sum m of
// cell t (see tile_kernel) adds the team total to the running sum
template <int TC, int CH, class S>
__device__ __forceinline__ void tile_sample(const S *vx, const S *vy, const S *vz,
                                            const TileLds<TC, CH, S> &L, int ntc, bool mown, double mprev,
                                            double *mdst)
{
    constexpr int T = 64 / TC;
    const int lane = threadIdx.x, team = lane / T, lt = lane - team * T;
    const int D0 = L.csn[0];
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    if (team < ntc) {
        const int s0 = L.csn[team] - D0, e0 = L.csn[team + 1] - D0;
        for (int i = s0 + lt; i < e0; i += T) add_moments(acc, vx[i], vy[i], vz[i]);
    }
    const double tot = team_reduce_scatter16<T>(acc, lt);
    if (mown) *mdst = mprev + tot;
}

// ---- the move and the grouping of the moved particles ---------------------------
constexpr int KEY_WALL = 63;  // marks a particle whose move crosses a wall (done in a second pass)

// direction code of a particle of tile cell t now at (x, y)
template <int TC, int CH, class S>
__device__ __forceinline__ int tile_dir(const StepArgs &a, const TileLds<TC, CH, S> &L, int t, double x, double y)
{
    int nix, niy;
    cell_xy(a.geo(), x, y, nix, niy);
    return direction(a.geo().nx, L.tix[t], L.tiy[t], nix, niy);
}

// Free flight over the coming step of the particles of one 64-slot chunk
// (slots b0 .. b0+63 of the tile) that do not reach a wall, in place; their
// direction codes go to kr.  A particle that would cross a wall is left as
// it is and marked KEY_WALL.  Returns whether the chunk has such particles.
template <int TC, int CH, class S>
__device__ __forceinline__ bool move_chunk_free(const StepArgs &a, const TileLds<TC, CH, S> &L, S &px, S &py,
                                                S *const *s, int32_t *kr, int ntc, int nt, int b0)
{
    const int i = b0 + (int)threadIdx.x;
    bool wall = false;
    if (i < nt) {
        const int t = tile_cell<TC, CH, S>(L, ntc, L.csn[0], i);
        const double dt = a.R().dt, g = a.R().g, H = a.R().G.H, Lx = a.R().G.Lx;
        double x = px, vx = s[2][i];
        const double y = py, vy = s[3][i];
        // the no-wall branch of move_particle, written out
        const double yn = y + vy * dt;
        if (yn < 0.0 || yn > H) {
            wall = true;
            kr[i] = KEY_WALL;
        } else {
            x = x + vx * dt + 0.5 * g * dt * dt;
            vx = vx + g * dt;
            // periodic wrap; inside (0, Lx) floor(x / Lx) is 0 and x stays as it is
            if (!(x > 0.0 && x < Lx)) {
                double xw = x - Lx * floor(x / Lx);
                if (xw < 0.0) xw = xw + Lx;
                if (xw >= Lx) xw = 0.0;
                x = xw;
            }
            // the stored (for FP32 state: rounded) position decides the cell
            const S xs = (S)x, ys = (S)yn;
            px = xs;
            py = ys;
            s[2][i] = (S)vx;
            kr[i] = t * NGRP + tile_dir<TC, CH, S>(a, L, t, (double)xs, (double)ys);
        }
    }
    return ballot64(wall) != 0;
}

// the particles of one chunk marked KEY_WALL: the full move with walls
template <int TC, int CH, class S>
__device__ void move_chunk_walls(const StepArgs &a, const TileLds<TC, CH, S> &L, S &px, S &py, S *const *s,
                                 int32_t *kr, int ntc, int nt, int b0, int &walls, bool &limit)
{
    const int i = b0 + (int)threadIdx.x;
    if (i < nt && kr[i] == KEY_WALL) {
        const int t = tile_cell<TC, CH, S>(L, ntc, L.csn[0], i);
        double x = px, y = py, vx = s[2][i], vy = s[3][i], vz = s[4][i];
        // wall draws are keyed by the slot inside the channel (of the settled
        // state the move starts from: see STEP_COMPLETE for L.kdelta)
        walls += move_particle(a.geo(), a.M1(), (uint32_t)(L.csn[0] + L.kdelta + i - a.R().pbase), x, y, vx, vy, vz,
                               limit);
        const S xs = (S)x, ys = (S)y;
        px = xs;
        py = ys;
        s[2][i] = (S)vx;
        s[3][i] = (S)vy;
        s[4][i] = (S)vz;
        kr[i] = t * NGRP + tile_dir<TC, CH, S>(a, L, t, (double)xs, (double)ys);
    }
}

// Stable rank of every particle of one chunk inside its next-step group
// (key t * NGRP + d, in kr), continuing from earlier chunks: L.run[key]
// holds the size of each group so far (zero before the first chunk).  One
// ballot per bit of the key gives every lane the chunk's lanes that share
// its key; its rank is the count of those below it, and the highest of them
// adds the chunk's share to the group size.
template <int TC, int CH, class S>
__device__ __forceinline__ void rank_chunk(TileLds<TC, CH, S> &L, int32_t *kr, int nt, int b0)
{
    constexpr int KB = TC * NGRP > 32 ? 6 : (TC * NGRP > 16 ? 5 : 4);  // bits of a key
    const int lane = threadIdx.x;
    const int i = b0 + lane;
    const bool act = i < nt;
    const int key = act ? kr[i] : 0;
    uint64_t same = ballot64(act);
#pragma unroll
    for (int b = 0; b < KB; ++b) {
        const bool bit = ((key >> b) & 1) != 0;
        const uint64_t m = ballot64(act && bit);
        same &= bit ? m : ~m;
    }
    if (act) {
        const int below = rank_below(same);
        const int before = L.run[key];
        kr[i] = ((before + below) << 6) | key;
        if ((same >> lane) == 1ull) L.run[key] = before + below + 1;  // the last of its key in the chunk
    }
}

// offsets of the tile cells' next-step groups inside each cell (sizes in
// L.run), published as absolute first slots with the cell end: lane
// t * NGRP + d scans the sizes of cell t's groups below d across its lanes
template <int TC, int CH, class S>
__device__ __forceinline__ void tile_group_offsets(const StepArgs &a, TileLds<TC, CH, S> &L, int c0, int ntc)
{
    const int lane = threadIdx.x;
    __syncthreads();
    const int t = lane / NGRP, d = lane - t * NGRP;
    const bool act = lane < ntc * NGRP;
    const int own = act ? L.run[lane] : 0;
    int inc = own;
#pragma unroll
    for (int off = 1; off < NGRP; off <<= 1) {
        const int v = __shfl_up(inc, off, 64);
        if (d >= off) inc += v;
    }
    if (act) {
        L.excl[lane] = inc - own;
        a.grp_out()[(size_t)(c0 + t) * GSTRIDE + d] = L.csn[t] + inc - own;
    }
    if (lane < ntc) a.grp_out()[(size_t)(c0 + lane) * GSTRIDE + NGRP] = L.csn[lane + 1];
    __syncthreads();
}

// ---- the step kernel ------------------------------------------------------------------
// One wave per tile of TC consecutive cells.
//   GATHER (a DSMC step): the particles that the step's sort puts in the
//     tile's cells are gathered group by group from the moved, partitioned
//     state, collided (NTC) and sampled; with MOVE they are then moved for
//     the next step, partitioned by direction inside their cells and
//     written out with the next step's group sizes; without MOVE (the last
//     step of a call) they are written out in sorted order.
//   no GATHER (k_classify): a settled state is moved for the coming step
//     and partitioned in place.
// STAGED tiles (at most 64*CH particles) are staged in LDS; larger ones run
// the same steps on the tile's destination range in global memory.
template <int TC, int CH, class S, bool GATHER, bool MOVE, bool STAGED, bool NT, bool DEFER>
__device__ void tile_body(const StepArgs &a, TileLds<TC, CH, S> &L, int c0, int ntc, int nt, int n_old, bool own_ntc,
                          double &nbar, double &sig, double &rem, bool mown, double mprev, double *mdst,
                          unsigned long long &ncoll, unsigned long long &ncand, int &walls, bool &limit)
{
    const int lane = threadIdx.x;
    const int D0 = L.csn[0];
    S *s[5];
    int32_t *kr;
    // STAGED: the positions of slot 64 b + lane stay in xr[b], yr[b] of this
    // lane from the gather to the write (every phase maps slots to lanes so)
    S xr[CH], yr[CH];
    if (STAGED) {
        s[0] = s[1] = nullptr;
#pragma unroll
        for (int k = 2; k < 5; ++k) s[k] = L.v[k - 2];
        kr = L.kr;
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) s[k] = a.template out<S>(k) + D0;  // k_classify: out == in (in place)
        kr = a.K().scr_i + D0;
    }

    // 1. gather
    if (STAGED) {
        // every load of the tile in flight at once
        S g[CH][5];
        bool g_ok[CH];
        // the state arrays' addresses are read here, where the gather uses
        // them (the empty asm hides the buffer index from the compiler, which
        // otherwise loads every address at the kernel's start and keeps them
        // live in SGPRs, spilling others: measured 355 -> 220 us for the
        // classify pass on a 512 x 256 x 100 channel)
        int ib = __builtin_amdgcn_readfirstlane(a.cur);
        asm volatile("" : "+s"(ib));
        const S *ip[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) ip[k] = (const S *)a.K().st[ib][k];
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            const int i = 64 * b + lane;
            int src = -1;
            if (i < nt) {
                if (GATHER) {
                    const int t = tile_cell<TC, CH, S>(L, ntc, D0, i);
                    src = tile_source<TC, CH, S>(L, t, i - (L.csn[t] - D0), L.anyfar != 0);
                    if (src >= n_old) {
                        src = -1;
                        atomicOr(&a.K().ctr->status, ST_INTERNAL);
                    }
                } else {
                    src = D0 + i;
                }
            }
            bool old = false;  // classify after a reseed: a kept cell's particle, from the old buffer
            if (!GATHER && a.reseed && i < nt) {
                const int t = tile_cell<TC, CH, S>(L, ntc, D0, i);
                if (L.rsrc[t] >= 0) {
                    src = L.rsrc[t] + (i - (L.csn[t] - D0));
                    old = true;
                }
            }
            g_ok[b] = src >= 0;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const S *p = &(old ? a.template old_in<S>(k) : ip[k])[src];
                if constexpr (NT)
                    g[b][k] = src >= 0 ? __builtin_nontemporal_load(p) : (S)0;
                else
                    g[b][k] = src >= 0 ? *p : (S)0;
            }
        }
        __builtin_amdgcn_s_setprio(0);  // the gather is issued
        // every slot of the tile is staged: a slot that no near group fills
        // holds zeros until the long jump that the sort puts there fills it,
        // and its long-jump source slot is marked absent until then
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            const int i = 64 * b + lane;
            xr[b] = g[b][0];
            yr[b] = g[b][1];
            if (i < nt) {
#pragma unroll
                for (int k = 2; k < 5; ++k) L.v[k - 2][i] = g[b][k];
                if (GATHER && !g_ok[b]) L.kr[i] = -1;
            }
        }
        if (GATHER && L.anyfar) {
            __syncthreads();
            tile_far_gather<TC, CH, S>(a, L, s, c0, ntc, n_old, L.kr);
            __syncthreads();
            // long jumps: the owner lane fetches the positions
#pragma unroll
            for (int b = 0; b < CH; ++b) {
                const int i = 64 * b + lane;
                if (i < nt && !g_ok[b]) {
                    const int q = L.kr[i];  // in [0, n_old) when written (tile_far_gather checks)
                    if (q >= 0) {
                        xr[b] = a.template in<S>(0)[q];
                        yr[b] = a.template in<S>(1)[q];
                    }
                }
            }
        }
        __syncthreads();
    } else if (GATHER) {
        for (int i = lane; i < nt; i += 64) {
            const int t = tile_cell<TC, CH, S>(L, ntc, D0, i);
            const int src = tile_source<TC, CH, S>(L, t, i - (L.csn[t] - D0), L.anyfar != 0);
            if (src >= n_old) atomicOr(&a.K().ctr->status, ST_INTERNAL);
            if (src < 0 || src >= n_old) continue;
#pragma unroll
            for (int k = 0; k < 5; ++k) s[k][i] = a.template in<S>(k)[src];
        }
        if (L.anyfar) tile_far_gather<TC, CH, S>(a, L, s, c0, ntc, n_old, nullptr);
        __threadfence();
        __syncthreads();
    } else if (a.reseed) {  // classify after a reseed: the kept cells' particles into place first
        for (int i = lane; i < nt; i += 64) {
            const int t = tile_cell<TC, CH, S>(L, ntc, D0, i);
            if (L.rsrc[t] < 0) continue;
            const int q = L.rsrc[t] + (i - (L.csn[t] - D0));
#pragma unroll
            for (int k = 0; k < 5; ++k) s[k][i] = a.template old_in<S>(k)[q];
        }
        __threadfence();
        __syncthreads();
    }

    // 2. collisions and 3. sample
    if (GATHER) {
        if constexpr (TC == 4) {
            if (own_ntc) {
                nbar = L.ntcs[0][lane];
                sig = L.ntcs[1][lane];
                rem = L.ntcs[2][lane];
            }
        }
        tile_ntc<TC, CH, S>(s[2], s[3], s[4], L, a.N(), c0, ntc, own_ntc, nbar, sig, rem, ncoll, ncand);
        if (own_ntc) {  // the cells' NTC state is final here (stored now: nothing stays live to the end)
            a.K().nbar[c0 + lane] = nbar;
            a.K().sigcmax[c0 + lane] = sig;
            a.K().rem[c0 + lane] = rem;
        }
        if (!STAGED) __threadfence();
        __syncthreads();
        if constexpr (TC == 4) {  // the moment sums' address is formed again here rather than held
            constexpr int T = 64 / TC, SPAN = T / 16;
            const int team = lane / T, lt = lane - team * T;
            if (mown) {
                mprev = L.mprev[lt / SPAN][team];
                mdst = a.K().mom + (size_t)(lt / SPAN) * a.K().ncells + c0 + team;
            }
        }
        if (a.sample) tile_sample<TC, CH, S>(s[2], s[3], s[4], L, ntc, mown, mprev, mdst);
    }

    if (!MOVE) {
        if (STAGED) {
#pragma unroll
            for (int b = 0; b < CH; ++b) {
                const int i = 64 * b + lane;
                if (i < nt) {
                    a.template out<S>(0)[D0 + i] = xr[b];
                    a.template out<S>(1)[D0 + i] = yr[b];
#pragma unroll
                    for (int k = 2; k < 5; ++k) a.template out<S>(k)[D0 + i] = L.v[k - 2][i];
                }
            }
        }
        return;  // unstaged: already in place, in sorted order
    }

    // STEP_DEFER: a tile with a particle that may reach a wall in the coming
    // move ends settled, in place, and its cells are listed for k_complete
    // (the test is the move's own wall test with a margin: deferring a tile
    // that needs no wall draw changes nothing)
    if constexpr (DEFER) {
        const double dt = a.R().dt, H = a.R().G.H, tol = 1e-9 * H;
        bool w = false;
        if (STAGED) {
#pragma unroll
            for (int b = 0; b < CH; ++b) {
                const int i = 64 * b + lane;
                if (i < nt) {
                    const double yn = (double)yr[b] + (double)L.v[1][i] * dt;
                    w |= !(yn > tol && yn < H - tol);
                }
            }
        } else {
            for (int i = lane; i < nt; i += 64) {
                const double yn = (double)s[1][i] + (double)s[3][i] * dt;
                w |= !(yn > tol && yn < H - tol);
            }
        }
        if (ballot64(w) != 0) {
            if (STAGED) {
#pragma unroll
                for (int b = 0; b < CH; ++b) {
                    const int i = 64 * b + lane;
                    if (i < nt) {
                        a.template out<S>(0)[D0 + i] = xr[b];
                        a.template out<S>(1)[D0 + i] = yr[b];
#pragma unroll
                        for (int k = 2; k < 5; ++k) a.template out<S>(k)[D0 + i] = L.v[k - 2][i];
                    }
                }
            }  // unstaged: already in place, in sorted order
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&a.K().ctr->ncomp, (uint32_t)ntc);
            base = __shfl(base, 0, 64);
            if (lane < ntc) {
                a.K().complist[base + lane] = c0 + lane;
                a.K().comp[c0 + lane] = 1;
            }
            return;
        }
    }

    // 4. move for the next step (walls in a second pass), grouped by (cell,
    // direction) in slot order
    bool anywall = false;
    S dx = (S)0, dy = (S)0;  // stand-ins for the positions of slots beyond the tile
    if (STAGED) {
#pragma unroll
        for (int b = 0; b < CH; ++b)
            if (64 * b < nt) anywall |= move_chunk_free<TC, CH, S>(a, L, xr[b], yr[b], s, kr, ntc, nt, 64 * b);
    } else {
        for (int b0 = 0; b0 < nt; b0 += 64) {
            const int i = b0 + lane;
            anywall |= move_chunk_free<TC, CH, S>(a, L, i < nt ? s[0][i] : dx, i < nt ? s[1][i] : dy, s, kr, ntc, nt,
                                                  b0);
        }
    }
    if (!STAGED) __threadfence();
    __syncthreads();
    if (anywall) {
        if (STAGED) {
#pragma unroll
            for (int b = 0; b < CH; ++b)
                if (64 * b < nt)
                    move_chunk_walls<TC, CH, S>(a, L, xr[b], yr[b], s, kr, ntc, nt, 64 * b, walls, limit);
        } else {
            for (int b0 = 0; b0 < nt; b0 += 64) {
                const int i = b0 + lane;
                move_chunk_walls<TC, CH, S>(a, L, i < nt ? s[0][i] : dx, i < nt ? s[1][i] : dy, s, kr, ntc, nt, b0,
                                            walls, limit);
            }
        }
        if (!STAGED) __threadfence();
        __syncthreads();
    }
    for (int b0 = 0; b0 < nt; b0 += 64) rank_chunk<TC, CH, S>(L, kr, nt, b0);
    tile_group_offsets<TC, CH, S>(a, L, c0, ntc);

    // 5. write out, partitioned by group inside each cell
    if (STAGED) {
        int ob = a.classify ? a.cur : 1 - a.cur;  // the output arrays, read here likewise
        ob = __builtin_amdgcn_readfirstlane(ob);
        asm volatile("" : "+s"(ob));
        S *op[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) op[k] = (S *)a.K().st[ob][k];
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            const int i = 64 * b + lane;
            if (i < nt) {
                const int k6 = kr[i], key = k6 & 63, t = key / NGRP;
                const int q = L.csn[t] + L.excl[key] + (k6 >> 6);
                op[0][q] = xr[b];
                op[1][q] = yr[b];
#pragma unroll
                for (int k = 2; k < 5; ++k) op[k][q] = L.v[k - 2][i];
            }
        }
    } else {
        __threadfence();
        __syncthreads();
        for (int k = 0; k < 5; ++k) {
            for (int i = lane; i < nt; i += 64) a.K().scr[D0 + i] = s[k][i];
            __threadfence();
            __syncthreads();
            for (int i = lane; i < nt; i += 64) {
                const int k6 = kr[i], key = k6 & 63, t = key / NGRP;
                a.template out<S>(k)[L.csn[t] + L.excl[key] + (k6 >> 6)] = a.K().scr[D0 + i];
            }
            __threadfence();
            __syncthreads();
        }
    }
    // long jumps of the next step go to the far list
#pragma unroll
    for (int b = 0; b < (STAGED ? CH : 1); ++b) {
        for (int i = STAGED ? 64 * b + lane : lane; i < nt; i += 64) {
            const int k6 = kr[i], key = k6 & 63, t = key / NGRP;
            if (key - t * NGRP == DIR_FAR) {
                const int q = L.csn[t] + L.excl[key] + (k6 >> 6);
                int nix, niy;
                cell_xy(a.geo(), STAGED ? (double)xr[b] : (double)a.template out<S>(0)[q],
                        STAGED ? (double)yr[b] : (double)a.template out<S>(1)[q], nix, niy);
                record_far(a.far_out(), a.farcnt_out(), a.K().ctr, a.far_out_slot(), a.K().far_cap, q, c0 + t,
                           a.R().cbase + niy * a.geo().nx + nix);
            }
            if (STAGED) break;
        }
    }
}

// Workgroups are dealt to the chip's 8 XCDs round-robin, each XCD with its
// own L2.  Tile t of the launch is given to block b so that every XCD runs
// one contiguous range of tiles: neighbouring tiles read each other's source
// groups (and the cache lines their runs share) from the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int x = b & 7, i = b >> 3;  // the block's XCD and its rank there
    const int q = n >> 3, r = n & 7;  // XCD x runs q + (x < r) tiles
    return x * q + min(x, r) + i;
}

// NT: the gather reads the state with non-temporal loads (see k_step)
// cc: the cell of a STEP_COMPLETE pass (TC 1), else -1 (tiles from the table)
template <int TC, int CH, class S, bool GATHER, bool MOVE, bool NT, bool DEFER = false>
__device__ __forceinline__ void tile_kernel(const StepArgs &a0, int cc = -1)
{
    static_assert(TC == 1 || TC == 2 || TC == 4, "tile sizes with teams of >= 16 lanes");
    static_assert(TC * NGRP <= 64 && NTC_ROUND <= 64, "");
    static_assert(GATHER || MOVE, "");
    __shared__ TileLds<TC, CH, S> L;
    constexpr int T = 64 / TC, SPAN = T / 16;
    const int lane = threadIdx.x;
    // the tile: up to TC consecutive cells of one channel, its entry in the
    // tile table (first cell, channel, that cell's row and column)
    // Odd steps run the tiles in the opposite order.  The state is larger than
    // the memory-side cache, and each step reads what the one before wrote; run
    // backwards, a step starts on the lines written last, which are the ones
    // still in that cache.  (Graph replays start at even steps: the parity of
    // the launch's step is the parity of the step.)
    StepArgs a = a0;
    int c0, iy0, ix0;
    if (cc >= 0) {  // one channel: its first replica entry
        c0 = cc;
        a.r = 0;
        iy0 = cc / a.R().G.nx;
        ix0 = cc - iy0 * a.R().G.nx;
    } else {
        const int tx = xcd_tile((int)blockIdx.x, (int)gridDim.x);
        const int tile = (a0.step & 1u) ? (int)gridDim.x - 1 - tx : tx;
        const __attribute__((address_space(4))) int32_t *td =
            (const __attribute__((address_space(4))) int32_t *)a0.tiles + TILE_WORDS * (size_t)tile;
        c0 = td[0];
        a.r = td[1];
        iy0 = td[2];
        ix0 = td[3];
    }
    // a step graph is captured with steps counted from 0 and replayed from
    // the step the host sets (an even one, so every parity is unchanged)
    if (a0.dev_step) a.step += ((const __attribute__((address_space(4))) Counters *)a.K().ctr)->step_base;
    const int nc = a.K().ncells, nx = a.geo().nx, cb = a.R().cbase, ce = a.R().cend;
    const int ntc = min(TC, ce - c0);

    // classify after a reseed (one channel): a rejected reseed (error flag)
    // keeps every cell's particles at its old slots and restores the old
    // cell starts; otherwise a marked cell's new particles are in place and
    // every other cell's particles move over from the old buffer
    const bool rs = !GATHER && a.reseed;
    const bool rerr = rs && ((const __attribute__((address_space(4))) Counters *)a.K().ctr)->reseed_err != 0u;
    const int32_t *const cs_old = a.K().cs[1 - a.cur];

    // The waves of a SIMD take turns by priority: a tile up to the issue of
    // its gather runs at a raised one, so that the two load rounds the tile
    // waits on leave as early as possible.
    __builtin_amdgcn_s_setprio(2);
    // set-up: every per-cell quantity of the tile is loaded in one round
    if (cc >= 0) {
        // the listed cell's settled particles: its slots in the moved state,
        // or, when a moved reseed that went ahead replaced it, its new
        // particles after the state's last slot; wall draws keyed by its
        // start after that reseed
        if (lane == 0) {
            const bool acc = (a0.flags & STEP_COMP_RESEED) &&
                             ((const __attribute__((address_space(4))) Counters *)a.K().ctr)->reseed_err == 0u;
            const int32_t *cs = a.K().cs[a.cur];
            const int mk = acc ? a.K().mark[cc] : 0;
            int src = cs[cc], n = cs[cc + 1] - cs[cc];
            if (mk > 0) {
                src = cs[nc] + a.K().appoff[mk - 1];
                n = a.K().nnew[mk - 1];
            }
            L.csn[0] = src;
            L.csn[1] = src + n;
            L.kdelta = (acc ? a.K().cs[1 - a.cur][cc] : cs[cc]) - src;
            a.K().mark[cc] = 0;
            a.K().comp[cc] = 0;
        }
    } else {
        if (lane <= TC) L.csn[lane] = (rerr ? cs_old : a.cs_new())[min(c0 + lane, ce)];
        if (lane == 0) L.kdelta = 0;
    }
    if (lane < TC * NGRP) L.run[lane] = 0;  // the next step's group sizes, counted by the rank
    if (rs && lane < TC) {
        const int c = min(c0 + lane, ce - 1);
        const bool fresh = !rerr && lane < ntc && a.K().mark[c] != 0;
        L.rsrc[lane] = fresh ? -1 : cs_old[c];
        if (lane < ntc) {  // the tile owns its cells' marks and starts
            a.K().mark[c] = 0;
            if (rerr) a.K().cs[a.cur][c] = cs_old[c];
        }
        if (rerr && lane == 0 && c0 + ntc == ce) a.K().cs[a.cur][ce] = cs_old[ce];
    }
    if (lane < TC) {  // the cells' rows and columns (a tile may run over row ends in narrow channels)
        int ix = ix0 + min(lane, ce - 1 - c0), iy = iy0;
#pragma unroll
        for (int u = 1; u < TC; ++u)
            if (ix >= nx) {
                ix -= nx;
                iy += 1;
            }
        L.tix[lane] = ix;
        L.tiy[lane] = iy;
    }
    double nbar = 0.0, sig = 0.0, rem = 0.0;
    int nfin = 0;
    if (GATHER && lane < ntc) nfin = a.farcnt_in()[c0 + lane];
    const bool own_ntc = GATHER && lane < ntc;  // this lane runs the collisions of tile cell `lane`
    if (own_ntc) {
        if constexpr (TC == 4) {
            L.ntcs[0][lane] = a.K().nbar[c0 + lane];
            L.ntcs[1][lane] = a.K().sigcmax[c0 + lane];
            L.ntcs[2][lane] = a.K().rem[c0 + lane];
        } else {
            nbar = a.K().nbar[c0 + lane];
            sig = a.K().sigcmax[c0 + lane];
            rem = a.K().rem[c0 + lane];
        }
    }
    const int team = lane / T, lt = lane - team * T, mslot = lt / SPAN;
    const bool mown = GATHER && a.sample && team < ntc && (lt % SPAN) == 0 && mslot < NMOM;
    double *const mdst = a.K().mom + (size_t)(mown ? mslot : 0) * nc + c0 + (mown ? team : 0);
    double mprev = 0.0;
    if (mown) {
        if constexpr (TC == 4)
            L.mprev[mslot][team] = *mdst;
        else
            mprev = *mdst;
    }
    double *const mdst_held = TC == 4 ? nullptr : mdst;
    const int n_old = GATHER ? a.K().cap : 0;  // source slots are checked against the buffer
    if (GATHER) {  // the tile's cells' plans (see tile_groups), in the same round of loads
#pragma unroll
        for (int e = lane; e < TC * 2 * NDIR; e += 64) {
            const int t = e / (2 * NDIR), f = e - t * (2 * NDIR);
            const int v = t < ntc ? a.K().plan[(size_t)(c0 + t) * (2 * NDIR) + f] : 0;
            if (f < NDIR)
                L.gsrc[t][f] = v;
            else
                L.gstart[t][f - NDIR] = v;
        }
    }
    __syncthreads();
    if (GATHER) tile_groups<TC, CH, S>(a, L, ntc, nfin);
    const int D0 = L.csn[0];
    const int nt = L.csn[ntc] - D0;

    unsigned long long ncoll = 0, ncand = 0;
    int walls = 0;
    bool limit = false;
    if (nt <= TileLds<TC, CH, S>::CAP)
        tile_body<TC, CH, S, GATHER, MOVE, true, NT, DEFER>(a, L, c0, ntc, nt, n_old, own_ntc, nbar, sig, rem, mown,
                                                            mprev, mdst_held, ncoll, ncand, walls, limit);
    else
        tile_body<TC, CH, S, GATHER, MOVE, false, NT, DEFER>(a, L, c0, ntc, nt, n_old, own_ntc, nbar, sig, rem, mown,
                                                             mprev, mdst_held, ncoll, ncand, walls, limit);

    // the tile's running counters.  Collisions and candidates were counted by
    // the lanes that ran the cells' collisions (lanes below TC); wall hits on
    // any lane, and in most tiles on none.  Every tile owns its entry; the
    // add is an atomic without return only so that the wave need not wait for
    // a read, which would queue behind all of the tile's stores.
    unsigned long long tcoll = 0, tcand = 0, twall = 0;
#pragma unroll
    for (int u = 0; u < TC; ++u) {
        tcoll += lane_u64(ncoll, u);
        tcand += lane_u64(ncand, u);
    }
    if (ballot64(walls != 0) != 0) twall = wave_sum_u64((unsigned long long)walls);
    const unsigned long long tadd = lane == 0 ? tcoll : (lane == 1 ? tcand : twall);
    // running counters of the tile, kept at its first cell (valid for any tiling)
    if (lane < 3 && tadd != 0) atomicAdd(a.K().tstat + 3 * (size_t)c0 + lane, tadd);
    if (MOVE && ballot64(limit) != 0 && lane == 0) atomicOr(&a.K().ctr->status, ST_WALL_LIMIT);
}

// FP32 tiles of four chunks at five waves per SIMD: without the collisions
// and the sampling they fit 96 VGPRs with a few spills in the cold wall
// path.  FP64 tiles stay at four: at five their positions spill around the
// rank and the write-out (measured 367 against 425 us on a 512 x 256 x 100
// channel).
// DEFER: the moving pass that leaves a call's state moved (see STEP_DEFER)
template <int TC, int CH, class S, bool DEFER>
__global__ __launch_bounds__(64, (CH == 4 && sizeof(S) == 4) ? 5 : 4) void k_classify(StepArgs a)
{
    tile_kernel<TC, CH, S, false, true, true, DEFER>(a);  // whole cells, read once: non-temporal
}

// four waves per SIMD: the tile fits 128 VGPRs (a few spills in the cold
// wall path) and about 9.4 KB of LDS (FP64, 2 cells x 4 chunks), so 16 tiles
// share a CU; measured 8 % faster than three waves with no spills
//
// NT (chosen on the host): the state read by the gather is dead once read,
// and the state written is what the next step reads.  When a buffer is not
// much larger than the 256 MB memory-side cache, non-temporal loads leave
// the written state there for the next step (measured: +4 % at 0.3 GB); at
// twice its size and more, the L2 reuse of the lines that neighbouring tiles
// share matters more and plain loads win (-1.5 % with NT at 0.5 GB).
// DEFER (with MOVE): the last step of a call that leaves the state moved
template <int TC, int CH, bool MOVE, class S, bool NT, bool DEFER>
__global__ __launch_bounds__(64, 4) void k_step(StepArgs a)
{
    tile_kernel<TC, CH, S, true, MOVE, NT, DEFER>(a);
}

// The completion pass of a moved state (see STEP_COMPLETE): the listed
// cells one by one, each a one-cell classify tile; a block takes list
// entries b, b + grid, ...  Launched with flags STEP_COMPLETE and, after a
// moved reseed, STEP_COMP_RESEED.
template <int CH, class S>
__global__ __launch_bounds__(64, 4) void k_complete(StepArgs a)
{
    const uint32_t n = ((const volatile Counters *)a.K().ctr)->ncomp;
    for (uint32_t e = blockIdx.x; e < n; e += gridDim.x) {
        tile_kernel<1, CH, S, false, true, true>(a, a.K().complist[e]);
        __syncthreads();
    }
}
template __global__ void k_complete<4, double>(StepArgs);
template __global__ void k_complete<8, double>(StepArgs);
template __global__ void k_complete<8, float>(StepArgs);

// Before the completion pass after a moved reseed that went ahead: the long
// jumps the step recorded for the replaced cells' old particles are void.
// From a complete list (pass 0, one thread per entry) they are dropped (new
// cell -1) and taken off the arrival counts.  After an overflow of the list
// the counts are rebuilt instead: pass 0 clears them, pass 1 (one thread
// per cell) counts the long jumps of every cell that keeps its moved state
// (neither replaced nor listed for completion) from its partitioned groups;
// the completion adds those of the listed cells.  The long-jump total drops
// by the void ones in either case.
template <class S>
__global__ __launch_bounds__(256) void k_comp_far(StepArgs a, int pass)
{
    const Counters *ct = a.K().ctr;
    if (ct->reseed_err != 0u) return;
    const int slot = (int)(a.step & 1u);
    const uint32_t nf = ct->nfar[slot];
    const bool listed = nf <= (uint32_t)a.K().far_cap;
    const int nc = a.K().ncells;
    int32_t *cnt = a.K().farcnt[slot];
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long dropped = 0;
    if (listed && pass == 0) {
        if (i < nf) {
            int32_t *e = a.K().far[slot] + 4 * i;
            const int o = e[1], d = e[2];
            if (d >= 0 && o >= 0 && o < nc && a.K().mark[o] != 0) {
                e[2] = -1;
                atomicSub(&cnt[d], 1);
                dropped = 1;
            }
        }
    } else if (!listed && pass == 0) {
        if (i < (size_t)nc) cnt[i] = 0;
    } else if (!listed && pass == 1 && i < (size_t)nc) {
        // (a cell that ended unmoved recorded no long jumps and has no groups yet)
        const int o = (int)i;
        const int32_t *g = a.K().grp[slot] + (size_t)o * GSTRIDE + DIR_FAR;
        if ((a.K().comp[o] & 1) == 0) {
            if (a.K().mark[o] != 0) {
                dropped = (unsigned long long)(g[1] - g[0]);
            } else {
                for (int q = g[0]; q < g[1]; ++q) atomicAdd(&cnt[far_new_cell<S>(a, q)], 1);
            }
        }
    }
    dropped = wave_sum_u64(dropped);
    if ((threadIdx.x & 63) == 0 && dropped)
        atomicAdd(&a.K().ctr->nfar_total, ~dropped + 1ull);  // minus: the sum with nfar[] stays exact mod 2^64
}

template __global__ void k_comp_far<double>(StepArgs, int);
template __global__ void k_comp_far<float>(StepArgs, int);

// after the completion pass of a moved reseed: the reseed is over and the
// list is empty (without a reseed the next step's cell pass empties it)
__global__ void k_comp_done(Counters *ctr, int reseed)
{
    if (threadIdx.x == 0) {
        ctr->ncomp = 0u;
        if (reseed) {
            ctr->reseed_err = 0u;
            ctr->reseed_new = 0ull;
            ctr->reseed_removed = 0ull;
        }
    }
}

#define DSMC_TILE_INSTANCES(TC, CH, S)                                    \
    template __global__ void k_classify<TC, CH, S, false>(StepArgs);      \
    template __global__ void k_classify<TC, CH, S, true>(StepArgs);       \
    template __global__ void k_step<TC, CH, true, S, false, false>(StepArgs);  \
    template __global__ void k_step<TC, CH, false, S, false, false>(StepArgs); \
    template __global__ void k_step<TC, CH, true, S, true, false>(StepArgs);   \
    template __global__ void k_step<TC, CH, false, S, true, false>(StepArgs);  \
    template __global__ void k_step<TC, CH, true, S, false, true>(StepArgs);   \
    template __global__ void k_step<TC, CH, true, S, true, true>(StepArgs);
DSMC_TILE_INSTANCES(4, 4, double)
DSMC_TILE_INSTANCES(2, 4, double)
DSMC_TILE_INSTANCES(1, 4, double)
DSMC_TILE_INSTANCES(1, 8, double)
DSMC_TILE_INSTANCES(4, 8, float)
DSMC_TILE_INSTANCES(4, 4, float)
DSMC_TILE_INSTANCES(2, 8, float)
DSMC_TILE_INSTANCES(1, 8, float)
#undef DSMC_TILE_INSTANCES

// Particles arriving in every cell with the step's sort, their block sums,
// and the cell's plan for the step kernel: its 9 near groups in the order of
// the stable sort (by source cell, sources beyond a wall or aliased last and
// empty), plan[c][k] the first source slot and plan[c][9 + k] the offset
// inside the cell of the k-th (long jumps not counted: the step shifts them)
__global__ __launch_bounds__(256) void k_cell_count(CellArgs a)
{
    __shared__ int lds[4];
    __shared__ int32_t stage[256 * 2 * NDIR];  // the block's plans, stored out in one contiguous sweep
    const int c0 = blockIdx.x * 256, c = c0 + threadIdx.x;
    int total = 0;
    if (c < a.ncells) {
        int nx = a.nx1, ny = a.ny1, cb = 0;
        if (nx <= 0) {  // a batch: the cell's channel
            const RepConst &R = a.rep[a.cell_rep[c]];
            nx = R.G.nx;
            ny = R.G.ny;
            cb = R.cbase;
        }
        const int cix = (c - cb) % nx, ciy = (c - cb) / nx;
        int key[NDIR], dir[NDIR];
        arrival_order(nx, ny, cix, ciy, cb, key, dir);
        int32_t *const pl = stage + threadIdx.x * (2 * NDIR);
#pragma unroll
        for (int k = 0; k < NDIR; ++k) {
            int first = 0, n = 0;
            if (key[k] != 0x7fffffff) {
                const int32_t *g = a.grp + (size_t)key[k] * GSTRIDE + dir[k];
                first = g[0];
                n = g[1] - g[0];
            }
            pl[k] = first;
            pl[NDIR + k] = total;
            total += n;
        }
        total += a.farcnt[c];
        a.countnew[c] = total;
    }
    __syncthreads();
    // 16-byte stores of consecutive plan words (a block's plans start on a
    // 16-byte boundary: 256 * 72 bytes apart)
    const int nwords = min(256, a.ncells - c0) * (2 * NDIR);
    int4 *const dst = (int4 *)(a.plan + (size_t)c0 * (2 * NDIR));
    const int4 *const src = (const int4 *)stage;
    for (int i = threadIdx.x; i < nwords / 4; i += 256) dst[i] = src[i];
    for (int i = (nwords / 4) * 4 + threadIdx.x; i < nwords; i += 256) a.plan[(size_t)c0 * (2 * NDIR) + i] = stage[i];
    const int bsum = block_reduce_256(total, lds);
    if (threadIdx.x == 0) a.blocksum[blockIdx.x] = bsum;
    if (gridDim.x == 1) {  // the whole grid: its cell starts too (no k_cell_final launch)
        const int ex = block_exscan_256(total, lds);
        if (c < a.ncells) a.cs_out[c] = ex;
        if (threadIdx.x == 255) a.cs_out[a.ncells] = ex + total;
        if (threadIdx.x == 0 && a.reset_slot >= 0) {
            a.ctr->nfar_total += a.ctr->nfar[a.reset_slot];
            a.ctr->nfar[a.reset_slot] = 0u;
            a.ctr->ncomp = 0u;
        }
    }
}

// exclusive scan of the block sums (one workgroup of 1024); writes the grand
// total to cs_out[ncells]
__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t *blocksum, int nblk, int32_t *cs_out, int ncells,
                                                     Counters *ctr, int reset_slot)
{
    if (reset_slot >= 0 && threadIdx.x == 0) {
        // the long-jump list of parity reset_slot belonged to the previous
        // step, whose sort is complete; the coming k_step refills it
        ctr->nfar_total += ctr->nfar[reset_slot];
        ctr->nfar[reset_slot] = 0u;
    }
    __shared__ int lds[16];
    __shared__ int carry_s;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < nblk; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int v = i < nblk ? blocksum[i] : 0;
        int inc = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int u = __shfl_up(inc, off, 64);
            if (lane >= off) inc += u;
        }
        if (lane == 63) lds[w] = inc;
        __syncthreads();
        int woff = 0;
        for (int k = 0; k < w; ++k) woff += lds[k];
        const int carry = carry_s;
        if (i < nblk) blocksum[i] = carry + woff + inc - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry_s = carry + woff + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) cs_out[ncells] = carry_s;
}

// averages = sums / S
__global__ __launch_bounds__(256) void k_average(const double *mom, double *out, size_t n, double S)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = mom[i] / S;
}

// ---- initial state: ppc Maxwellian particles per cell ----------------------
template <class S>
__global__ __launch_bounds__(256) void k_init_maxwell(InitArgs a)
{
    const size_t g = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (g <= (size_t)a.ncells) a.cs[g] = (int32_t)((size_t)a.pbase + g * (size_t)a.ppc);
    if (g < (size_t)a.ncells) {
        a.nbar[g] = 0.0;
        a.sigcmax[g] = a.sigcr0;
        a.rem[g] = 0.0;
    }
    if (g >= (size_t)a.ncells * (size_t)a.ppc) return;
    const int c = (int)(g / (size_t)a.ppc);
    const int ix = c % a.nx, iy = c / a.nx;
    const U4 p = draw(a.k0, a.k1, 0u, (uint32_t)g, 0u, TAG_INIT, 0u);
    const U4 b = draw(a.k0, a.k1, 1u, (uint32_t)g, 0u, TAG_INIT, 0u);
    const U4 e = draw(a.k0, a.k1, 2u, (uint32_t)g, 0u, TAG_INIT, 0u);
    double z0, z1, zz0, zz1;
    box_muller(u53(b.x, b.y), u53(b.z, b.w), z0, z1);
    box_muller(u53(e.x, e.y), u53(e.z, e.w), zz0, zz1);
    ((S *)a.st[0])[g] = (S)inside_cell(ix, u53(p.x, p.y));
    ((S *)a.st[1])[g] = (S)inside_cell(iy, u53(p.z, p.w));
    ((S *)a.st[2])[g] = (S)(a.s_th * z0);
    ((S *)a.st[3])[g] = (S)(a.s_th * z1);
    ((S *)a.st[4])[g] = (S)(a.s_th * zz0);
}
template __global__ void k_init_maxwell<double>(InitArgs);
template __global__ void k_init_maxwell<float>(InitArgs);

// ---- adoption of a caller-written, unsorted particle set -------------------
template <class S>
__global__ __launch_bounds__(256) void k_adopt_count(AdoptArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n) return;
    int ix, iy;
    cell_xy(a.G, (double)((const S *)a.in[0])[p], (double)((const S *)a.in[1])[p], ix, iy);
    const int c = iy * a.G.nx + ix;
    a.cellid[p] = c;
    atomicAdd(&a.counts[c], 1);
}
template __global__ void k_adopt_count<double>(AdoptArgs);
template __global__ void k_adopt_count<float>(AdoptArgs);

// generic block sums of per-cell counts
__global__ __launch_bounds__(256) void k_block_sums(const int32_t *counts, int ncells, int32_t *blocksum)
{
    __shared__ int lds[4];
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int v = c < ncells ? counts[c] : 0;
    const int s = block_reduce_256(v, lds);
    if (threadIdx.x == 0) blocksum[blockIdx.x] = s;
}

// generic exclusive scan of per-cell counts given scanned block sums
// Cell starts of the coming sort in one pass: block b adds up the block sums
// of blocks 0 .. b-1 itself (at most a few hundred integers, exact in any
// order), then scans its own 256 counts; the last block writes the total.
// Block 0 also retires the long-jump list of parity reset_slot (the previous
// step's, already sorted), which the coming step refills, and empties the
// completion list of a moved state (its pass, if any, ran before).
__global__ __launch_bounds__(256) void k_cell_final(const int32_t *counts, int ncells, const int32_t *blocksum,
                                                    int32_t *cs, Counters *ctr, int reset_slot)
{
    __shared__ int lds[4];
    const int b = blockIdx.x;
    if (b == 0 && threadIdx.x == 0 && reset_slot >= 0) {
        ctr->nfar_total += ctr->nfar[reset_slot];
        ctr->nfar[reset_slot] = 0u;
        ctr->ncomp = 0u;
    }
    int part = 0;
    for (int i = threadIdx.x; i < b; i += 256) part += blocksum[i];
    const int off = block_reduce_256(part, lds);
    const int c = b * 256 + threadIdx.x;
    const int v = c < ncells ? counts[c] : 0;
    const int ex = block_exscan_256(v, lds);
    if (c < ncells) cs[c] = off + ex;
    if (b == (int)gridDim.x - 1 && threadIdx.x == 255) cs[ncells] = off + ex + v;
}

__global__ __launch_bounds__(256) void k_block_scan(const int32_t *counts, int ncells, const int32_t *blockoff,
                                                    int32_t *cs)
{
    __shared__ int lds[4];
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int v = c < ncells ? counts[c] : 0;
    const int ex = block_exscan_256(v, lds);
    if (c < ncells) cs[c] = blockoff[blockIdx.x] + ex;
}

__global__ __launch_bounds__(256) void k_adopt_place(AdoptArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n) return;
    const int c = a.cellid[p];
    const int pos = a.cs[c] + atomicAdd(&a.cursor[c], 1);
    a.perm[pos] = (int32_t)p;
}

// slot order inside each cell (the placement above is in atomic order)
__global__ __launch_bounds__(256) void k_adopt_sortcell(AdoptArgs a)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= a.G.nx * a.G.ny) return;
    const int s = a.cs[c], e = a.cs[c + 1];
    for (int i = s + 1; i < e; ++i) {
        const int v = a.perm[i];
        int j = i - 1;
        while (j >= s && a.perm[j] > v) {
            a.perm[j + 1] = a.perm[j];
            --j;
        }
        a.perm[j + 1] = v;
    }
    a.cursor[c] = 0;
}

template <class S>
__global__ __launch_bounds__(256) void k_adopt_gather(AdoptArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= a.n) return;
    const int p = a.perm[q];
#pragma unroll
    for (int k = 0; k < 5; ++k) ((S *)a.out[k])[q] = ((const S *)a.in[k])[p];
}
template __global__ void k_adopt_gather<double>(AdoptArgs);
template __global__ void k_adopt_gather<float>(AdoptArgs);

__global__ __launch_bounds__(256) void k_fill_f64(double *p, size_t n, double v)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, size_t n, int32_t v)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_counters(Counters *c)
{
    if (threadIdx.x == 0) {
        c->status = 0u;
        c->reseed_err = 0u;
        c->nfar[0] = 0u;
        c->nfar[1] = 0u;
        c->ncoll = 0ull;
        c->ncand = 0ull;
        c->nwall = 0ull;
        c->nfar_total = 0ull;
        c->reseed_new = 0ull;
        c->reseed_removed = 0ull;
        c->step_base = 0u;
        c->ncomp = 0u;
    }
}

// the first step of the step graph about to be replayed
__global__ void k_set_step_base(Counters *c, uint32_t step)
{
    if (threadIdx.x == 0) c->step_base = step;
}

// discard the long-jump list of one parity (its classification is void)
__global__ void k_far_reset(Counters *c, int slot)
{
    if (threadIdx.x == 0) c->nfar[slot] = 0u;
}

__global__ void k_clear_status(Counters *c)
{
    if (threadIdx.x == 0) c->status = 0u;
}

// totals of the per-tile counters (one workgroup of 1024)
// totals of the tile counters (kept at the tiles' first cells: n entries)
__global__ __launch_bounds__(1024) void k_tile_stats(const unsigned long long *tstat, int n, Counters *c)
{
    __shared__ unsigned long long part[3][16];
    unsigned long long v[3] = {0ull, 0ull, 0ull};
    for (int t = threadIdx.x; t < n; t += 1024) {
        v[0] += tstat[3 * (size_t)t];
        v[1] += tstat[3 * (size_t)t + 1];
        v[2] += tstat[3 * (size_t)t + 2];
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = wave_sum_u64(v[k]);
        if (lane == 0) part[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot[3] = {0ull, 0ull, 0ull};
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 16; ++i) tot[k] += part[k][i];
        c->ncoll = tot[0];
        c->ncand = tot[1];
        c->nwall = tot[2];
    }
}

// per channel: the sums of its cells' tile counters -> out[r][3]
__global__ __launch_bounds__(256) void k_replica_stats(const unsigned long long *tstat, const RepConst *rep,
                                                       unsigned long long *out)
{
    __shared__ unsigned long long part[3][4];
    const RepConst &R = rep[blockIdx.x];
    unsigned long long v[3] = {0ull, 0ull, 0ull};
    for (int c = R.cbase + (int)threadIdx.x; c < R.cend; c += 256) {
        v[0] += tstat[3 * (size_t)c];
        v[1] += tstat[3 * (size_t)c + 1];
        v[2] += tstat[3 * (size_t)c + 2];
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = wave_sum_u64(v[k]);
        if (lane == 0) part[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        out[3 * (size_t)blockIdx.x + k] = part[k][0] + part[k][1] + part[k][2] + part[k][3];
    }
}

}  // namespace dsmc
