// DSMC particle step on gfx950: move + wall + cell index, deterministic
// stable counting sort, NTC hard-sphere collisions, moment sampling.
//
// Sort design.  The particles are sorted by cell at the start of a step and
// move at most one cell per step in all but rare cases, so the destination
// of a particle is fixed by its (old cell o, direction d) group, d one of the
// 9 moves inside the 3x3 neighbourhood: a stable order inside a new cell c
// is "groups in increasing old-cell order, and slot order inside a group".
//   pass 1  (one wave per old cell)  move every particle, count the 9 groups
//           with wave ballots, record long jumps ("far") in a short list;
//   cell    (one thread per new cell) sum the groups that arrive in c, scan,
//           and give every group its first destination slot;
//   pass 2  (one wave per old cell)  repeat the identical move (the random
//           numbers are counter-based, so it is bit-identical) and write
//           each particle to base[d] + rank inside its group.
// The state is read twice and written once per step; nothing depends on the
// order of atomic operations.
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

// wave-reduce the 11 per-lane partial sums and add them to cell o's sums
__device__ __forceinline__ void flush_moments(double *acc, double *mom, int o, int ncells, int lane)
{
#pragma unroll
    for (int k = 0; k < NMOM; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NMOM; ++k) mom[(size_t)k * ncells + o] += acc[k];
    }
}

template <bool SCATTER>
__global__ __launch_bounds__(256) void k_pass(PassArgs a)
{
    const int lane = threadIdx.x & 63;
    const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (o >= a.ncells) return;  // wave-uniform
    const int start = a.cs[o], end = a.cs[o + 1];
    const int nx = a.G.nx;
    const int oix = o % nx, oiy = o / nx;

    int run[NDIR];
    int gbase[NDIR];
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
        run[d] = 0;
        gbase[d] = SCATTER ? a.base[(size_t)d * a.ncells + o] : 0;
    }
    double acc[NMOM];
#pragma unroll
    for (int k = 0; k < NMOM; ++k) acc[k] = 0.0;
    int walls = 0;
    bool limit = false;
    uint32_t nfar = 0;
    if (SCATTER) nfar = min(a.ctr->nfar, (uint32_t)a.far_cap);

    for (int p0 = start; p0 < end; p0 += 64) {
        const int p = p0 + lane;
        const bool act = p < end;
        int d = DIR_NONE, nc = 0;
        double x = 0.0, y = 0.0, vx = 0.0, vy = 0.0, vz = 0.0;
        if (act) {
            x = a.in[0][p];
            y = a.in[1][p];
            vx = a.in[2][p];
            vy = a.in[3][p];
            vz = a.in[4][p];
            if (!SCATTER && a.sample) add_moments(acc, vx, vy, vz);
            walls += move_particle(a.G, a.M, (uint32_t)p, x, y, vx, vy, vz, limit);
            int nix, niy;
            cell_xy(a.G, x, y, nix, niy);
            nc = niy * nx + nix;
            d = direction(nx, oix, oiy, nix, niy);
        }
        if (!SCATTER && d == DIR_FAR) {
            atomicAdd(&a.farcnt[nc], 1);
            const uint32_t idx = atomicAdd(&a.ctr->nfar, 1u);
            if (idx < (uint32_t)a.far_cap) {
                a.far[4 * (size_t)idx + 0] = p;
                a.far[4 * (size_t)idx + 1] = o;
                a.far[4 * (size_t)idx + 2] = nc;
                a.far[4 * (size_t)idx + 3] = -1;
            } else {
                atomicOr(&a.ctr->status, ST_FAR_OVERFLOW);
            }
        }
        uint64_t m[NDIR];
#pragma unroll
        for (int dd = 0; dd < NDIR; ++dd) m[dd] = ballot64(d == dd);
        if (SCATTER && act) {
            int dest = -1;
            if (d < NDIR) {
                int r = 0, b = 0;
                uint64_t mm = 0;
#pragma unroll
                for (int dd = 0; dd < NDIR; ++dd) {
                    if (d == dd) {
                        r = run[dd];
                        b = gbase[dd];
                        mm = m[dd];
                    }
                }
                dest = b + r + rank_below(mm);
            } else {
                for (uint32_t e = 0; e < nfar; ++e) {
                    if (a.far[4 * (size_t)e] == p) {
                        dest = a.far[4 * (size_t)e + 3];
                        break;
                    }
                }
            }
            if (dest >= 0) {
                a.out[0][dest] = x;
                a.out[1][dest] = y;
                a.out[2][dest] = vx;
                a.out[3][dest] = vy;
                a.out[4][dest] = vz;
            }
        }
#pragma unroll
        for (int dd = 0; dd < NDIR; ++dd) run[dd] += __popcll(m[dd]);
    }

    if (!SCATTER) {
        if (lane < NDIR) {
            int v = 0;
#pragma unroll
            for (int dd = 0; dd < NDIR; ++dd)
                if (lane == dd) v = run[dd];
            a.cnt[(size_t)lane * a.ncells + o] = v;
        }
        if (a.sample) flush_moments(acc, a.mom, o, a.ncells, lane);
        const unsigned long long wsum = wave_sum_u64((unsigned long long)walls);
        if (lane == 0 && wsum) atomicAdd(&a.ctr->nwall, wsum);
        if (ballot64(limit) != 0 && lane == 0) atomicOr(&a.ctr->status, ST_WALL_LIMIT);
    }
}

template __global__ void k_pass<false>(PassArgs);
template __global__ void k_pass<true>(PassArgs);

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
__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t *blocksum, int nblk, int32_t *cs_out, int ncells)
{
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
    const uint32_t nf = min(a.ctr->nfar, (uint32_t)a.far_cap);
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
        }
        a.farcnt[c] = 0;
    }
}

// ---- NTC collisions (Eq. (collisionnumber)), one lane per cell ---------------
// Per cell: update the running mean of N, form the candidate count
// 1/2 N Nbar K sigcmax dt + rem (K = F_N sigma_T / V_c), draw candidate
// pairs uniformly (i != j), accept with probability c_r / sigcmax, scatter
// isotropically in the centre-of-mass frame.  Candidate k draws from
// counters (2k, c, step, COLL) and, when accepted, (2k+1, c, step, COLL).
__global__ __launch_bounds__(256) void k_collide(CollideArgs a)
{
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the long-jump list of the step that just finished is no longer needed
        a.ctr->nfar_total += a.ctr->nfar;
        a.ctr->nfar = 0u;
    }
    const int c = blockIdx.x * 256 + threadIdx.x;
    unsigned long long ncoll = 0, ncand = 0;
    if (c < a.ncells) {
        const int start = a.cs[c];
        const int N = a.cs[c + 1] - start;
        const double Nd = (double)N;
        double nbar = a.nbar[c];
        nbar = nbar + (Nd - nbar) / (double)(a.step + 1);
        a.nbar[c] = nbar;
        double sig = a.sigcmax[c];
        const double pairf = (a.nbar_mode == 1) ? (Nd - 1.0) : nbar;
        double X = 0.5 * Nd * pairf * a.K * sig * a.dt + a.rem[c];
        if (!(X > 0.0)) X = 0.0;
        const double Mf = floor(X);
        a.rem[c] = X - Mf;
        if (N >= 2) {
            const long long M = (long long)Mf;
            double *vxp = a.v[0] + start;
            double *vyp = a.v[1] + start;
            double *vzp = a.v[2] + start;
            for (long long k = 0; k < M; ++k) {
                const U4 u = draw(a.k0, a.k1, (uint32_t)(2 * k), (uint32_t)c, a.step, TAG_COLL, 0u);
                const uint32_t i = (uint32_t)(((uint64_t)u.x * (uint64_t)(uint32_t)N) >> 32);
                uint32_t j = (uint32_t)(((uint64_t)u.y * (uint64_t)(uint32_t)(N - 1)) >> 32);
                if (j >= i) j += 1;
                const double vxi = vxp[i], vyi = vyp[i], vzi = vzp[i];
                const double vxj = vxp[j], vyj = vyp[j], vzj = vzp[j];
                const double dx = vxi - vxj, dy = vyi - vyj, dz = vzi - vzj;
                const double cr = sqrt(dx * dx + dy * dy + dz * dz);
                if (cr > sig) sig = cr;
                const double R = u53(u.z, u.w);
                ncand += 1;
                if (cr / sig > R) {
                    const U4 w = draw(a.k0, a.k1, (uint32_t)(2 * k + 1), (uint32_t)c, a.step, TAG_COLL, 0u);
                    const double cth = 2.0 * u53(w.x, w.y) - 1.0;
                    const double sth = sqrt(1.0 - cth * cth);
                    const double phi = TWO_PI * u53(w.z, w.w);
                    const double rx = cr * cth;
                    const double ry = cr * sth * cos(phi);
                    const double rz = cr * sth * sin(phi);
                    const double mx = 0.5 * (vxi + vxj);
                    const double my = 0.5 * (vyi + vyj);
                    const double mz = 0.5 * (vzi + vzj);
                    vxp[i] = mx + 0.5 * rx;
                    vyp[i] = my + 0.5 * ry;
                    vzp[i] = mz + 0.5 * rz;
                    vxp[j] = mx - 0.5 * rx;
                    vyp[j] = my - 0.5 * ry;
                    vzp[j] = mz - 0.5 * rz;
                    ncoll += 1;
                }
            }
        }
        a.sigcmax[c] = sig;
    }
    ncoll = wave_sum_u64(ncoll);
    ncand = wave_sum_u64(ncand);
    if (lane == 0) {
        if (ncoll) atomicAdd(&a.ctr->ncoll, ncoll);
        if (ncand) atomicAdd(&a.ctr->ncand, ncand);
    }
}

// ---- sampling of the current state (one wave per cell) ----------------------
__global__ __launch_bounds__(256) void k_sample(SampleArgs a)
{
    const int lane = threadIdx.x & 63;
    const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (o >= a.ncells) return;
    const int start = a.cs[o], end = a.cs[o + 1];
    double acc[NMOM];
#pragma unroll
    for (int k = 0; k < NMOM; ++k) acc[k] = 0.0;
    for (int p = start + lane; p < end; p += 64) add_moments(acc, a.v[0][p], a.v[1][p], a.v[2][p]);
    flush_moments(acc, a.mom, o, a.ncells, lane);
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
        c->nfar = 0u;
        c->reseed_err = 0u;
        c->pad = 0u;
        c->ncoll = 0ull;
        c->ncand = 0ull;
        c->nwall = 0ull;
        c->nfar_total = 0ull;
    }
}

__global__ void k_clear_status(Counters *c)
{
    if (threadIdx.x == 0) c->status = 0u;
}

}  // namespace dsmc
