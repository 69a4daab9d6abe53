// DSMC particle step on gfx950: move + wall + cell index, deterministic
// stable counting sort, NTC hard-sphere collisions, moment sampling.
//
// Design.  The particles are sorted by cell at the start of a step and move
// at most one cell per step in all but rare cases, so the destination of a
// particle is fixed by its (old cell o, direction d) group, d one of the 9
// moves inside the 3x3 neighbourhood: a stable order inside a new cell c is
// "groups in increasing old-cell order, and slot order inside a group".
// Every particle's direction code for the coming step is known before the
// step starts (k_step writes it for the state it produces; k_classify
// computes it for a state set from outside).  One step is then
//   cell kernels  (one thread per new cell) sum the groups that arrive in c,
//                 scan, and give every group its first destination slot;
//   k_step        (one workgroup per tile of new cells) gather the tile's
//                 particles from its neighbour cells, redo their move (the
//                 random numbers are counter-based, so it is bit-identical),
//                 run the NTC collisions and the moment sample on the staged
//                 tile, write it out contiguously, and classify the next
//                 step's moves.
// The state is read once and written once per step, plus one code byte per
// particle; nothing depends on the order of atomic operations.
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

// ---- NTC collisions of one cell (Eq. (collisionnumber)) -----------------------
// Update the running mean of N, form the candidate count
// 1/2 N Nbar K sigcmax dt + rem (K = F_N sigma_T / V_c), draw candidate
// pairs uniformly (i != j), accept with probability c_r / sigcmax (hard
// spheres), scatter isotropically in the centre-of-mass frame.  Candidate k
// of cell c at step s draws from counters (2k, c, s, COLL) and, when
// accepted, (2k+1, c, s, COLL).  v* address the cell's velocities (LDS or
// global).
__device__ __forceinline__ void ntc_cell(double *vx, double *vy, double *vz, int N, uint32_t c, const NtcParams &P,
                                         double &nbar, double &sig, double &rem, unsigned long long &ncoll,
                                         unsigned long long &ncand)
{
    const double Nd = (double)N;
    nbar = nbar + (Nd - nbar) / (double)(P.step + 1);
    const double pairf = (P.nbar_mode == 1) ? (Nd - 1.0) : nbar;
    double X = 0.5 * Nd * pairf * P.K * sig * P.dt + rem;
    if (!(X > 0.0)) X = 0.0;
    const double Mf = floor(X);
    rem = X - Mf;
    if (N < 2) return;
    const long long M = (long long)Mf;
    for (long long k = 0; k < M; ++k) {
        const U4 u = draw(P.k0, P.k1, (uint32_t)(2 * k), c, P.step, TAG_COLL, 0u);
        const uint32_t i = (uint32_t)(((uint64_t)u.x * (uint64_t)(uint32_t)N) >> 32);
        uint32_t j = (uint32_t)(((uint64_t)u.y * (uint64_t)(uint32_t)(N - 1)) >> 32);
        if (j >= i) j += 1;
        const double vxi = vx[i], vyi = vy[i], vzi = vz[i];
        const double vxj = vx[j], vyj = vy[j], vzj = vz[j];
        const double dx = vxi - vxj, dy = vyi - vyj, dz = vzi - vzj;
        const double cr = sqrt(dx * dx + dy * dy + dz * dz);
        if (cr > sig) sig = cr;
        const double R = u53(u.z, u.w);
        ncand += 1;
        if (cr / sig > R) {
            const U4 w = draw(P.k0, P.k1, (uint32_t)(2 * k + 1), c, P.step, TAG_COLL, 0u);
            const double cth = 2.0 * u53(w.x, w.y) - 1.0;
            const double sth = sqrt(1.0 - cth * cth);
            double sphi, cphi;
            sincos_turn(u53(w.z, w.w), sphi, cphi);  // phi = 2 pi R
            const double rx = cr * cth;
            const double ry = cr * sth * cphi;
            const double rz = cr * sth * sphi;
            const double mx = 0.5 * (vxi + vxj);
            const double my = 0.5 * (vyi + vyj);
            const double mz = 0.5 * (vzi + vzj);
            const double ax = mx + 0.5 * rx, ay = my + 0.5 * ry, az = mz + 0.5 * rz;
            const double bx = mx - 0.5 * rx, by = my - 0.5 * ry, bz = mz - 0.5 * rz;
            vx[i] = ax, vy[i] = ay, vz[i] = az;
            vx[j] = bx, vy[j] = by, vz[j] = bz;
            ncoll += 1;
        }
    }
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

// append a long jump of the particle in slot q (old cell o, new cell nc)
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

// ---- the move of a settled state (one wave per cell) --------------------------
// Free flight (with walls) of every particle of the current, cell-sorted
// state over the coming step, written back in place, with its direction
// code, the per-cell counts of the 9 (cell, direction) groups and the
// long-jump list.  Runs for the first step of every dsmc_step call;
// inside a call k_step moves the state it writes.
__global__ __launch_bounds__(256) void k_classify(ClassifyArgs a)
{
    const int lane = threadIdx.x & 63;
    const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (o >= a.ncells) return;  // wave-uniform
    const int start = a.cs[o], end = a.cs[o + 1];
    const int nx = a.G.nx;
    const int oix = o % nx, oiy = o / nx;
    int run[NDIR];
#pragma unroll
    for (int d = 0; d < NDIR; ++d) run[d] = 0;
    bool limit = false;
    int walls = 0;
    for (int p0 = start; p0 < end; p0 += 64) {
        const int p = p0 + lane;
        int d = DIR_NONE, nc = 0;
        if (p < end) {
            double x = a.st[0][p], y = a.st[1][p], vx = a.st[2][p], vy = a.st[3][p], vz = a.st[4][p];
            walls += move_particle(a.G, a.M, (uint32_t)p, x, y, vx, vy, vz, limit);
            a.st[0][p] = x;
            a.st[1][p] = y;
            a.st[2][p] = vx;
            a.st[3][p] = vy;
            a.st[4][p] = vz;
            int nix, niy;
            cell_xy(a.G, x, y, nix, niy);
            d = direction(nx, oix, oiy, nix, niy);
            nc = niy * nx + nix;
        }
#pragma unroll
        for (int dd = 0; dd < NDIR; ++dd) run[dd] += __popcll(ballot64(d == dd));
        if (p < end) {
            a.code[p] = (uint8_t)d;
            if (d == DIR_FAR) record_far(a.far, a.farcnt, a.ctr, a.far_slot, a.far_cap, p, o, nc);
        }
    }
    if (lane < NDIR) {
        int v = 0;
#pragma unroll
        for (int dd = 0; dd < NDIR; ++dd)
            if (lane == dd) v = run[dd];
        a.cnt[(size_t)lane * a.ncells + o] = v;
    }
    const unsigned long long wsum = wave_sum_u64((unsigned long long)walls);
    if (lane == 0 && wsum) atomicAdd(&a.ctr->nwall, wsum);
    if (ballot64(limit) != 0 && lane == 0) atomicOr(&a.ctr->status, ST_WALL_LIMIT);
}

// ---- inverse of the new sort: source slot of every new slot -----------------
// One wave per old cell, in slot order: a particle of group (o, d) goes to
// new slot base[d][o] + (number of earlier particles of o with the same d),
// counted with one ballot per direction.  (Long jumps get theirs in
// k_cell_final.)
__global__ __launch_bounds__(256) void k_invert(InvertArgs a)
{
    const int lane = threadIdx.x & 63;
    const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (o >= a.ncells) return;
    const int start = a.cs[o], end = a.cs[o + 1];
    const int n = a.cs[a.ncells];
    int b[NDIR];
#pragma unroll
    for (int d = 0; d < NDIR; ++d) b[d] = a.base[(size_t)d * a.ncells + o];
    for (int p0 = start; p0 < end; p0 += 64) {
        const int p = p0 + lane;
        const int d = p < end ? (int)a.code[p] : DIR_NONE;
        int q = -1;
#pragma unroll
        for (int dd = 0; dd < NDIR; ++dd) {
            const uint64_t m = ballot64(d == dd);
            if (d == dd) q = b[dd] + rank_below(m);
            b[dd] += __popcll(m);
        }
        if (d < NDIR) {
            if (q >= 0 && q < n) a.from[q] = p;
            else atomicOr(&a.ctr->status, ST_INTERNAL);
        }
    }
}

// ---- the DSMC step, organised by destination tile --------------------------------
// The state it reads has already been moved (by k_classify or by the
// previous k_step) and carries each particle's direction code and rank.
// One workgroup per tile of TC consecutive new cells (their particles are
// the contiguous new slots [D0, D0 + nt)):
//   1. gather: copy every new slot's particle from its source slot (from
//      k_invert), positions to the new buffer, velocities to the stage;
//   2. NTC collisions of the step, one lane per new cell, on the stage;
//   3. a team of 256/TC lanes per cell: moment sample (when due), then
//      either the settled state out (last step of a call) or the next
//      step's move of every particle, written out with its direction code;
//      the (cell, direction) counts are summed in LDS.
constexpr int ST_PMAX = 896;  // tile particles that fit the LDS stage
constexpr int ST_PER_THREAD = (ST_PMAX + 255) / 256;

template <int TC>
struct StepLds {
    double v[5][ST_PMAX];  // x, y, vx, vy, vz of the tile's particles
    int32_t csn[TC + 1];
    int32_t cnt[TC * NDIR];
};

template <int TC, bool STAGE>
__device__ __forceinline__ void step_tile(const StepArgs &a, StepLds<TC> &L, int c0, int ntc, int D0, int nt)
{
    constexpr int T = 256 / TC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nx = a.G.nx, nc = a.ncells;
    double *const ovx = a.out[2] + D0, *const ovy = a.out[3] + D0, *const ovz = a.out[4] + D0;
    double *const ox = a.out[0] + D0, *const oy = a.out[1] + D0;
    double *const sx = STAGE ? L.v[0] : ox;
    double *const sy = STAGE ? L.v[1] : oy;
    double *const svx = STAGE ? L.v[2] : ovx;
    double *const svy = STAGE ? L.v[3] : ovy;
    double *const svz = STAGE ? L.v[4] : ovz;
    const int n_old = a.cs_old[nc];

    // 1. gather
    for (int r0 = 0; r0 < nt; r0 += 256 * ST_PER_THREAD) {
        double x[ST_PER_THREAD], y[ST_PER_THREAD], vx[ST_PER_THREAD], vy[ST_PER_THREAD], vz[ST_PER_THREAD];
        int pp[ST_PER_THREAD];
#pragma unroll
        for (int r = 0; r < ST_PER_THREAD; ++r) {
            const int slot = r0 + tid + 256 * r;
            pp[r] = slot < nt ? a.from[D0 + slot] : -1;
            if (pp[r] >= n_old) pp[r] = -1;
        }
#pragma unroll
        for (int r = 0; r < ST_PER_THREAD; ++r) {
            if (pp[r] >= 0) {
                x[r] = a.in[0][pp[r]];
                y[r] = a.in[1][pp[r]];
                vx[r] = a.in[2][pp[r]];
                vy[r] = a.in[3][pp[r]];
                vz[r] = a.in[4][pp[r]];
            }
        }
#pragma unroll
        for (int r = 0; r < ST_PER_THREAD; ++r) {
            const int slot = r0 + tid + 256 * r;
            if (slot >= nt) continue;
            if (pp[r] < 0) {
                atomicOr(&a.ctr->status, ST_INTERNAL);
                continue;
            }
            sx[slot] = x[r];
            sy[slot] = y[r];
            svx[slot] = vx[r];
            svy[slot] = vy[r];
            svz[slot] = vz[r];
        }
    }
    __threadfence_block();
    __syncthreads();

    // 2. NTC collisions of this step, one lane per new cell
    {
        unsigned long long ncoll = 0, ncand = 0;
        if (tid < ntc) {
            const int c = c0 + tid;
            const int s0 = L.csn[tid] - D0, N = L.csn[tid + 1] - L.csn[tid];
            double nbar = a.nbar[c], sig = a.sigcmax[c], rem = a.rem[c];
            ntc_cell(svx + s0, svy + s0, svz + s0, N, (uint32_t)c, a.N, nbar, sig, rem, ncoll, ncand);
            a.nbar[c] = nbar;
            a.sigcmax[c] = sig;
            a.rem[c] = rem;
        }
        if (wave == 0) {
            ncoll = wave_sum_u64(ncoll);
            ncand = wave_sum_u64(ncand);
            if (lane == 0 && ncoll) atomicAdd(&a.ctr->ncoll, ncoll);
            if (lane == 0 && ncand) atomicAdd(&a.ctr->ncand, ncand);
        }
    }
    if (!STAGE) __threadfence_block();
    __syncthreads();

    // 3. one team per cell: sample, then move (or settle) and write out
    int walls = 0;
    bool limit = false;
    {
        const int team = tid / T, lt = tid % T;
        double acc[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0;
        const bool live = team < ntc;
        const int o = c0 + (live ? team : 0);
        const int oix = o % nx, oiy = o / nx;
        const int s0 = live ? L.csn[team] - D0 : 0, e0 = live ? L.csn[team + 1] - D0 : 0;
        if (a.sample) {
            for (int i = s0 + lt; i < e0; i += T) add_moments(acc, svx[i], svy[i], svz[i]);
            const double tot = team_reduce_scatter16<T>(acc, lt);
            constexpr int SPAN = T / 16;
            const int slot = (lt / SPAN) & 15;
            if (live && (lt % SPAN) == 0 && slot < NMOM) a.mom[(size_t)slot * nc + o] += tot;
        }
        for (int i = s0 + lt; i < e0; i += T) {
            double x = sx[i], y = sy[i], vx = svx[i], vy = svy[i], vz = svz[i];
            if (a.classify) {
                walls += move_particle(a.G, a.M1, (uint32_t)(D0 + i), x, y, vx, vy, vz, limit);
                int nix, niy;
                cell_xy(a.G, x, y, nix, niy);
                const int d = direction(nx, oix, oiy, nix, niy);
                a.code_out[D0 + i] = (uint8_t)d;
                if (d == DIR_FAR)
                    record_far(a.far_out, a.farcnt, a.ctr, a.far_slot ^ 1, a.far_cap, D0 + i, o, niy * nx + nix);
                else
                    atomicAdd(&L.cnt[team * NDIR + d], 1);
            }
            if (STAGE || a.classify) {
                ox[i] = x;
                oy[i] = y;
                ovx[i] = vx;
                ovy[i] = vy;
                ovz[i] = vz;
            }
        }
    }
    __syncthreads();
    if (a.classify) {
        for (int k = tid; k < ntc * NDIR; k += 256) {
            const int cl = k / NDIR, d = k - cl * NDIR;
            a.cnt[(size_t)d * nc + c0 + cl] = L.cnt[k];
        }
    }
    const unsigned long long wsum = wave_sum_u64((unsigned long long)walls);
    if (lane == 0 && wsum) atomicAdd(&a.ctr->nwall, wsum);
    if (ballot64(limit) != 0 && lane == 0) atomicOr(&a.ctr->status, ST_WALL_LIMIT);
}

template <int TC>
__global__ __launch_bounds__(256) void k_step(StepArgs a)
{
    __shared__ StepLds<TC> L;
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * TC;
    const int ntc = min(TC, a.ncells - c0);
    if (tid <= TC) L.csn[tid] = a.cs_new[min(c0 + tid, a.ncells)];
    if (tid < TC * NDIR) L.cnt[tid] = 0;
    __syncthreads();
    const int D0 = L.csn[0];
    const int nt = L.csn[ntc] - D0;
    if (nt <= ST_PMAX)
        step_tile<TC, true>(a, L, c0, ntc, D0, nt);
    else
        step_tile<TC, false>(a, L, c0, ntc, D0, nt);
}

template __global__ void k_step<4>(StepArgs);
template __global__ void k_step<8>(StepArgs);
template __global__ void k_step<16>(StepArgs);

// counts arriving in every cell of the new sort, and their block sums
__global__ __launch_bounds__(256) void k_cell_count(CellArgs a)
{
    __shared__ int lds[4];
    const int c = blockIdx.x * 256 + threadIdx.x;
    int total = 0;
    if (c < a.ncells) {
        const int cix = c % a.nx, ciy = c / a.nx;
#pragma unroll
        for (int d = 0; d < NDIR; ++d) {
            const int src = source_cell(a.nx, a.ny, cix, ciy, d);
            if (src >= 0) total += a.cnt[(size_t)d * a.ncells + src];
        }
        total += a.farcnt[c];
        a.countnew[c] = total;
    }
    const int bsum = block_reduce_256(total, lds);
    if (threadIdx.x == 0) a.blocksum[blockIdx.x] = bsum;
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

// new cell_start, first destination slot of every arriving group, and the
// destinations of long jumps into the cell
__global__ __launch_bounds__(256) void k_cell_final(CellArgs a)
{
    __shared__ int lds[4];
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int v = c < a.ncells ? a.countnew[c] : 0;
    const int ex = block_exscan_256(v, lds);
    if (c >= a.ncells) return;
    const int cs = a.blocksum[blockIdx.x] + ex;
    a.cs_new[c] = cs;

    const int cix = c % a.nx, ciy = c / a.nx;
    int srcs[NDIR], dirs[NDIR], cnts[NDIR];
    int ns = 0;
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
        const int src = source_cell(a.nx, a.ny, cix, ciy, d);
        if (src >= 0) {
            srcs[ns] = src;
            dirs[ns] = d;
            cnts[ns] = a.cnt[(size_t)d * a.ncells + src];
            ++ns;
        }
    }
    // order the arriving groups by old cell (insertion sort of <= 9)
    for (int i = 1; i < ns; ++i) {
        const int s = srcs[i], d = dirs[i], n = cnts[i];
        int j = i - 1;
        while (j >= 0 && srcs[j] > s) {
            srcs[j + 1] = srcs[j];
            dirs[j + 1] = dirs[j];
            cnts[j + 1] = cnts[j];
            --j;
        }
        srcs[j + 1] = s;
        dirs[j + 1] = d;
        cnts[j + 1] = n;
    }
    const int nfar_in = a.farcnt[c];
    const uint32_t nf = min(a.ctr->nfar[a.far_slot], (uint32_t)a.far_cap);
    int acc = 0;
    for (int i = 0; i < ns; ++i) {
        int before_far = 0;
        if (nfar_in > 0) {
            for (uint32_t e = 0; e < nf; ++e)
                if (a.far[4 * (size_t)e + 2] == c && a.far[4 * (size_t)e + 1] < srcs[i]) ++before_far;
        }
        a.base[(size_t)dirs[i] * a.ncells + srcs[i]] = cs + acc + before_far;
        acc += cnts[i];
    }
    if (nfar_in > 0) {
        for (uint32_t e = 0; e < nf; ++e) {
            if (a.far[4 * (size_t)e + 2] != c) continue;
            const int po = a.far[4 * (size_t)e + 1], pp = a.far[4 * (size_t)e];
            int rank = 0;
            for (int i = 0; i < ns; ++i)
                if (srcs[i] < po) rank += cnts[i];
            for (uint32_t f = 0; f < nf; ++f)
                if (a.far[4 * (size_t)f + 2] == c && a.far[4 * (size_t)f] < pp) ++rank;
            a.far[4 * (size_t)e + 3] = cs + rank;
            a.from[cs + rank] = pp;
        }
        a.farcnt[c] = 0;
    }
}

// averages = sums / S
__global__ __launch_bounds__(256) void k_average(const double *mom, double *out, size_t n, double S)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = mom[i] / S;
}

// ---- initial state: ppc Maxwellian particles per cell ----------------------
__global__ __launch_bounds__(256) void k_init_maxwell(InitArgs a)
{
    const size_t g = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (g <= (size_t)a.ncells) a.cs[g] = (int32_t)(g * (size_t)a.ppc);
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
    a.st[0][g] = inside_cell(ix, u53(p.x, p.y));
    a.st[1][g] = inside_cell(iy, u53(p.z, p.w));
    a.st[2][g] = a.s_th * z0;
    a.st[3][g] = a.s_th * z1;
    a.st[4][g] = a.s_th * zz0;
}

// ---- adoption of a caller-written, unsorted particle set -------------------
__global__ __launch_bounds__(256) void k_adopt_count(AdoptArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n) return;
    int ix, iy;
    cell_xy(a.G, a.in[0][p], a.in[1][p], ix, iy);
    const int c = iy * a.G.nx + ix;
    a.cellid[p] = c;
    atomicAdd(&a.counts[c], 1);
}

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

__global__ __launch_bounds__(256) void k_adopt_gather(AdoptArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= a.n) return;
    const int p = a.perm[q];
#pragma unroll
    for (int k = 0; k < 5; ++k) a.out[k][q] = a.in[k][p];
}

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
    }
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

}  // namespace dsmc
