// DSMC<->LBM mapping kernels and the BGK lattice step on gfx950.
// Method: Di Staso, Clercx, Succi & Toschi, arXiv:1512.08042, Section 2.
#include "dsmc_device.hpp"
#include "step_kernels.hpp"

namespace dsmc {

// ---- DSMC2LB (Eq. (discretefunctions)) -------------------------------------
// From the cumulative averages of the sampled sums: rho = <N>/ppc (the mass
// scale of the appendix), the absolute-frame Hermite coefficients a(1..3)
// of Eq. (nordercoefficients) from the raw velocity moments (in units of
// sqrt(kT/m)), and f_a = w_a sum_{n<=order} a(n):H(n)(xi_a)/n!.  D2Q9
// cannot carry H_xxx and H_yyy (they vanish on its nodes): those terms are
// left out there.  With `equilibrium` only rho and u enter, a(n) being
// those of the local equilibrium (rho u, rho u u, rho u u u): Eq.
// (feq_dsmc).
// With xi_a = r e_a (e_a integer), the sum over n is a cubic polynomial in
// e_a whose ten coefficients are formed once per cell; each population is
// then a few multiply-adds with e_a's components folded in at compile time,
// all Q stores of a thread issued back to back.  (Splitting a cell's
// populations over two to eight threads, for more waves in flight, was no
// faster: 10.4 to 12.0 us against 10.4 us for 131,072 cells on D2Q37.)
template <int Q>
__global__ __launch_bounds__(256) void k_project(ProjectArgs a)
{
#pragma clang fp contract(fast)
    using V = VelSet<Q>;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int c = a.c_off + i * a.c_stride;
    const size_t node = (size_t)a.n_off + (size_t)i * a.n_stride;
    const int nc = a.ncells;
    double m[NMOM];
#pragma unroll
    for (int k = 0; k < NMOM; ++k) m[k] = a.mom[(size_t)k * nc + c];
    // coefficients of e^0, e_x, e_y, e_x^2, e_x e_y, e_y^2, e_x^3, e_x^2 e_y, e_x e_y^2, e_y^3
    double p0 = 0.0, px = 0.0, py = 0.0, pxx = 0.0, pxy = 0.0, pyy = 0.0;
    double pxxx = 0.0, pxxy = 0.0, pxyy = 0.0, pyyy = 0.0;
    if (m[0] > 0.0) {
        const int order = a.order;
        const double r = a.L.r, r2 = r * r, r3 = r2 * r;
        const double rho = m[0] * a.rho_scale;
        const double im = a.is1 / m[0];
        const double ex = m[1] * im, ey = m[2] * im;
        double a1x = 0.0, a1y = 0.0, a2xx = 0.0, a2xy = 0.0, a2yy = 0.0;
        double a3xxx = 0.0, a3xxy = 0.0, a3xyy = 0.0, a3yyy = 0.0;
        if (order >= 1) {
            a1x = rho * ex;
            a1y = rho * ey;
        }
        if (a.equilibrium) {
            if (order >= 2) {
                a2xx = a1x * ex;
                a2xy = a1x * ey;
                a2yy = a1y * ey;
            }
            if (order >= 3) {
                a3xxx = a2xx * ex;
                a3xxy = a2xx * ey;
                a3xyy = a2xy * ey;
                a3yyy = a2yy * ey;
            }
        } else {
            const double im2 = im * a.is1, im3 = im2 * a.is1;
            if (order >= 2) {
                a2xx = rho * (m[3] * im2 - 1.0);
                a2xy = rho * (m[4] * im2);
                a2yy = rho * (m[5] * im2 - 1.0);
            }
            if (order >= 3) {
                a3xxx = rho * (m[6] * im3 - 3.0 * ex);
                a3xxy = rho * (m[7] * im3 - ey);
                a3xyy = rho * (m[8] * im3 - ex);
                a3yyy = rho * (m[9] * im3 - 3.0 * ey);
            }
        }
        if (Q == 9) a3xxx = a3yyy = 0.0;
        // a(2):H(2)/2 and a(3):H(3)/6 written out in powers of e = xi / r
        p0 = rho - 0.5 * (a2xx + a2yy);
        px = r * (a1x - 0.5 * (a3xxx + a3xyy));
        py = r * (a1y - 0.5 * (a3yyy + a3xxy));
        pxx = 0.5 * r2 * a2xx;
        pxy = r2 * a2xy;
        pyy = 0.5 * r2 * a2yy;
        pxxx = r3 * a3xxx * (1.0 / 6.0);
        pxxy = 0.5 * r3 * a3xxy;
        pxyy = 0.5 * r3 * a3xyy;
        pyyy = r3 * a3yyy * (1.0 / 6.0);
    }
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int X = V::ex[q], Y = V::ey[q];
        double v = p0;
        cmad<X>(v, px);
        cmad<Y>(v, py);
        cmad<X * X>(v, pxx);
        cmad<X * Y>(v, pxy);
        cmad<Y * Y>(v, pyy);
        cmad<X * X * X>(v, pxxx);
        cmad<X * X * Y>(v, pxxy);
        cmad<X * Y * Y>(v, pxyy);
        cmad<Y * Y * Y>(v, pyyy);
        a.f[(size_t)q * a.nn_out + node] = a.L.ws[V::sh[q]] * v;
    });
}
template __global__ void k_project<9>(ProjectArgs);
template __global__ void k_project<37>(ProjectArgs);

// ---- LB2DSMC (Section 2.2, Table 1) ------------------------------------------
// Table 1 steps 1-3 on node populations f[q * stride]: rho, u, comoving and
// density-normalised a(2), a(3) about u, M = max |component|, C = 1 + 30 M.
// prm: rho, ux, uy, a2xx, a2xy, a2yy, a3xxx, a3xxy, a3xyy, a3yyy, M, C.
// Q is fixed at compile time so that the node's Q loads are all issued at
// once; the sums run over q in order.
template <int Q>
__device__ void grad_params(const double *f, size_t stride, const Lattice &L, int order, double *prm)
{
    double fq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) fq[q] = f[(size_t)q * stride];
    double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double fa = fq[q];
        rho += fa;
        jx += fa * L.xi[q][0];
        jy += fa * L.xi[q][1];
    }
    for (int k = 0; k < 12; ++k) prm[k] = 0.0;
    prm[0] = rho;
    if (!(rho > 0.0)) return;
    const double ux = jx / rho, uy = jy / rho;
    double sxx = 0, sxy = 0, syy = 0, sxxx = 0, sxxy = 0, sxyy = 0, syyy = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double fa = fq[q];
        const double cx = L.xi[q][0] - ux, cy = L.xi[q][1] - uy;
        sxx += fa * (cx * cx - 1.0);
        sxy += fa * (cx * cy);
        syy += fa * (cy * cy - 1.0);
        sxxx += fa * (cx * cx * cx - 3.0 * cx);
        sxxy += fa * (cx * cx * cy - cy);
        sxyy += fa * (cx * cy * cy - cx);
        syyy += fa * (cy * cy * cy - 3.0 * cy);
    }
    double a2xx = sxx / rho, a2xy = sxy / rho, a2yy = syy / rho;
    double a3xxx = sxxx / rho, a3xxy = sxxy / rho, a3xyy = sxyy / rho, a3yyy = syyy / rho;
    if (order < 3) {
        a3xxx = 0.0;
        a3xxy = 0.0;
        a3xyy = 0.0;
        a3yyy = 0.0;
    }
    if (Q == 9) {
        a3xxx = 0.0;
        a3yyy = 0.0;
    }
    if (order < 2) {
        a2xx = 0.0;
        a2xy = 0.0;
        a2yy = 0.0;
    }
    const double comp[7] = {a2xx, a2xy, a2yy, a3xxx, a3xxy, a3xyy, a3yyy};
    double M = 0.0;
    for (int k = 0; k < 7; ++k) {
        const double v = fabs(comp[k]);
        if (v > M) M = v;
    }
    prm[1] = ux;
    prm[2] = uy;
    prm[3] = a2xx;
    prm[4] = a2xy;
    prm[5] = a2yy;
    prm[6] = a3xxx;
    prm[7] = a3xxy;
    prm[8] = a3xyy;
    prm[9] = a3yyy;
    prm[10] = M;
    prm[11] = 1.0 + 30.0 * M;
}

// G of Eq. (distr_outeq) at xi: 1 + a(2):H(2)/2! + a(3):H(3)/3!
__device__ __forceinline__ double grad_G(const double *p, double x, double y)
{
    const double hxx = x * x - 1.0, hxy = x * y, hyy = y * y - 1.0;
    const double hxxx = x * x * x - 3.0 * x, hxxy = x * x * y - y;
    const double hxyy = x * y * y - x, hyyy = y * y * y - 3.0 * y;
    const double t2 = p[3] * hxx + 2.0 * p[4] * hxy + p[5] * hyy;
    const double t3 = p[6] * hxxx + 3.0 * p[7] * hxxy + 3.0 * p[8] * hxyy + p[9] * hyyy;
    return 1.0 + t2 / 2.0 + t3 / 6.0;
}

// one thread per listed cell: mark the cell, Table 1 steps 1-3, and the
// number of new particles floor(rho ppc + R) (mass conservation at the
// coupling site), R from counters (0, c, e, RESEED_N)
__global__ __launch_bounds__(256) void k_reseed_prep(ReseedArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    unsigned long long add_new = 0, add_removed = 0;
    if (i < a.nsel) {
        const int c = a.cells[i];
        a.nnew[i] = 0;
        bool ok = true;
        if (c < 0 || c >= a.ncells) {
            atomicOr(&a.ctr->reseed_err, ST_BAD_CELL);
            ok = false;
        } else if (atomicCAS(&a.mark[c], 0, i + 1) != 0) {
            atomicOr(&a.ctr->reseed_err, ST_BAD_CELL);
            ok = false;
        }
        if (ok) {
            double *pr = a.prm + (size_t)i * 12;
            if (a.L.Q == 9)
                grad_params<9>(a.f + c, (size_t)a.ncells, a.L, a.order, pr);
            else
                grad_params<37>(a.f + c, (size_t)a.ncells, a.L, a.order, pr);
            const U4 r = draw(a.k0, a.k1, 0u, (uint32_t)c, a.event, TAG_RESEED_N, 0u);
            const double target = pr[0] * (double)a.ppc + u53(r.x, r.y);
            bool finite = true;
            for (int k = 0; k < 12; ++k)
                if (!isfinite(pr[k])) finite = false;
            int nn = 0;
            if (!finite) {
                atomicOr(&a.ctr->status, ST_NONFINITE);
                nn = 0;
            } else if (target >= 16777215.0) {
                atomicOr(&a.ctr->status, ST_NNEW_LIMIT);
                nn = 16777215;
            } else if (target >= 1.0) {
                nn = (int)floor(target);
            }
            if (!(pr[0] > 0.0)) nn = 0;
            a.nnew[i] = nn;
            add_new = (unsigned long long)nn;
            add_removed = (unsigned long long)(a.cs_old[c + 1] - a.cs_old[c]);
        }
    }
    // the reseed's totals: one add per wave (adds to one address serialise)
    add_new = wave_sum_u64(add_new);
    add_removed = wave_sum_u64(add_removed);
    if ((threadIdx.x & 63) == 0) {
        if (add_new) atomicAdd(&a.ctr->reseed_new, add_new);
        if (add_removed) atomicAdd(&a.ctr->reseed_removed, add_removed);
    }
}

// per-cell particle counts after the reseed, and their block sums
__global__ __launch_bounds__(256) void k_reseed_count(ReseedArgs a)
{
    __shared__ int lds[4];
    const int c = blockIdx.x * 256 + threadIdx.x;
    int v = 0;
    if (c < a.ncells) {
        const int mk = a.mark[c];
        v = mk ? a.nnew[mk - 1] : (a.cs_old[c + 1] - a.cs_old[c]);
        a.countnew[c] = v;
    }
    // block sum (same reduction as the step's cell count)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) a.blocksum[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

// The reseed's new cell starts in one pass: block b adds up the block sums
// of blocks 0 .. b-1 itself (at most a few hundred integers, exact in any
// order) and scans its own 256 counts.  The last thread also decides whether
// the reseed goes ahead, from the 64-bit totals of the listed cells (the
// 32-bit starts are meaningless when that total is above capacity).
__global__ __launch_bounds__(256) void k_reseed_starts(ReseedArgs a)
{
    __shared__ int lds[4];
    const int b = blockIdx.x;
    int part = 0;
    for (int i = threadIdx.x; i < b; i += 256) part += a.blocksum[i];
    const int off = block_reduce_256(part, lds);
    const int c = b * 256 + threadIdx.x;
    const int v = c < a.ncells ? a.countnew[c] : 0;
    const int ex = block_exscan_256(v, lds);
    if (c < a.ncells) a.cs_new[c] = off + ex;
    if (b == (int)gridDim.x - 1 && threadIdx.x == 255) {
        a.cs_new[a.ncells] = off + ex + v;
        Counters *ct = a.ctr;
        if (ct->reseed_err & ST_BAD_CELL) ct->status |= ST_BAD_CELL;
        const long long total =
            (long long)a.cs_old[a.ncells] + (long long)ct->reseed_new - (long long)ct->reseed_removed;
        if (total > a.capacity) {
            ct->reseed_err |= ST_CAPACITY;
            ct->status |= ST_CAPACITY;
        }
    }
}

// Kept cells of a pending reseed (when no step completes it): one
// workgroup per tile of RC_TILE cells streams the tile's old particles and
// copies those of unmarked cells to their new slots (the identity when the
// reseed was rejected, in which case cell_start is restored as well), and
// clears the tile's marks.
constexpr int RC_TILE = 64;

template <class S>
__global__ __launch_bounds__(256) void k_reseed_copy(ReseedArgs a)
{
    __shared__ int s_old[RC_TILE + 1], s_new[RC_TILE + 1], s_keep[RC_TILE];
    const int tid = threadIdx.x;
    const int c0 = blockIdx.x * RC_TILE;
    const int nt = min(RC_TILE, a.ncells - c0);
    const bool err = a.ctr->reseed_err != 0u;
    if (tid <= RC_TILE) {
        const int c = min(c0 + tid, a.ncells);
        s_old[tid] = a.cs_old[c];
        s_new[tid] = err ? a.cs_old[c] : a.cs_new[c];
    }
    if (tid < RC_TILE) {
        s_keep[tid] = (tid < nt) && (err || a.mark[c0 + tid] == 0);
        if (tid < nt) a.mark[c0 + tid] = 0;
    }
    __syncthreads();
    if (err) {
        if (tid < nt) a.cs_new[c0 + tid] = s_old[tid];
        if (c0 + nt == a.ncells && tid == 0) a.cs_new[a.ncells] = s_old[nt];
    }
    const int P0 = s_old[0], P1 = s_old[nt];
    for (int p = P0 + tid; p < P1; p += 256) {
        int lo = 0, hi = nt;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_old[mid] <= p) lo = mid;
            else hi = mid;
        }
        if (!s_keep[lo]) continue;
        const int q = s_new[lo] + (p - s_old[lo]);
#pragma unroll
        for (int k = 0; k < 5; ++k) ((S *)a.out[k])[q] = ((const S *)a.in[k])[p];
    }
}
template __global__ void k_reseed_copy<double>(ReseedArgs);
template __global__ void k_reseed_copy<float>(ReseedArgs);

// Listed cells: one wave per listed cell generates its new particles
// (Table 1 steps 4-6) into the cell's new slots.  Four waves per SIMD: the
// cell's Grad parameters are read from LDS (the same address on every lane)
// rather than held in registers, so that a strip of up to 4 cells per SIMD
// runs in one round.
template <class S>
__global__ __launch_bounds__(256, 4) void k_reseed_gen(ReseedArgs a)
{
    __shared__ double s_prm[4][12];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 4 + w;
    if (i >= a.nsel) return;  // (whole waves: no barrier follows)
    if (a.ctr->reseed_err != 0u) return;
    const int c = a.cells[i];
    const int nn = a.nnew[i];
    const int d0 = a.moved ? a.cs_old[a.ncells] + a.appoff[i] : a.cs_new[c];
    if (lane < 12) s_prm[w][lane] = a.prm[(size_t)i * 12 + lane];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double *prm = s_prm[w];
    const double C = prm[11];
    const int ix = c % a.nx, iy = c / a.nx;
    bool limit = false;
    // Table 1 steps 4-5 for new particle k of the cell: Box-Muller tries
    // from counters (2t, c, e, RESEED|k), accepted when C R <= G(xi) with R
    // from counters (2t+1, c, e, RESEED|k); after ar_max_tries rejections the
    // last try is kept and the AR-limit status bit is raised.  Every lane
    // samples one particle at a time, one try per pass; a lane whose
    // particle is done takes the next unassigned ordinal, so the wave's
    // passes follow the mean number of tries (about C) rather than the
    // slowest lane's.  The draws are keyed by the ordinal, so the result does
    // not depend on which lane samples which particle.
    int k = lane;       // ordinal of this lane's particle
    long long t = 0;    // its tries so far
    int next = 64;      // first ordinal not yet assigned
    while (ballot64(k < nn) != 0) {
        bool fin = false;
        if (k < nn) {
            const U4 A = draw(a.k0, a.k1, (uint32_t)(2 * t), (uint32_t)c, a.event, TAG_RESEED, (uint32_t)k);
            const U4 B = draw(a.k0, a.k1, (uint32_t)(2 * t + 1), (uint32_t)c, a.event, TAG_RESEED, (uint32_t)k);
            double z0, z1;
            box_muller(u53(A.x, A.y), u53(A.z, A.w), z0, z1);
            const double R = u53(B.x, B.y);
            const double G = grad_G(prm, z0, z1);
            t += 1;
            if (C * R <= G) {
                fin = true;
            } else if (t >= a.ar_max_tries) {
                limit = true;
                fin = true;
            }
            if (fin) {  // the in-plane velocity (Table 1 step 6) is final here
                const int q = d0 + k;
                ((S *)a.out[2])[q] = (S)(a.s_th * (z0 + prm[1]));
                ((S *)a.out[3])[q] = (S)(a.s_th * (z1 + prm[2]));
            }
        }
        const uint64_t m = ballot64(fin);
        if (fin) {
            k = next + rank_below(m);
            t = 0;
        }
        next += __popcll(m);
    }
    // position (uniform in the cell) and out-of-plane velocity (Maxwellian)
    // of every new particle, one ordinal per lane: no rejection step here
    for (int kk = lane; kk < nn; kk += 64) {
        double zz0, zz1;
        const U4 Pp = draw(a.k0, a.k1, 0u, (uint32_t)c, a.event, TAG_RESEED_POS, (uint32_t)kk);
        const U4 V = draw(a.k0, a.k1, 1u, (uint32_t)c, a.event, TAG_RESEED_POS, (uint32_t)kk);
        box_muller(u53(V.x, V.y), u53(V.z, V.w), zz0, zz1);
        const int q = d0 + kk;
        ((S *)a.out[0])[q] = (S)inside_cell(ix, u53(Pp.x, Pp.y));
        ((S *)a.out[1])[q] = (S)inside_cell(iy, u53(Pp.z, Pp.w));
        ((S *)a.out[4])[q] = (S)(a.s_th * zz0);
    }
    if (__ballot(limit) != 0 && lane == 0) atomicOr(&a.ctr->status, ST_AR_LIMIT);
}

template __global__ void k_reseed_gen<double>(ReseedArgs);
template __global__ void k_reseed_gen<float>(ReseedArgs);

// A reseed of a moved state: the first slot of every list entry's new
// particles after the state's last slot (an exclusive scan of the counts in
// list order, one workgroup: each thread sums a run of entries, the runs'
// sums are scanned across the waves), and whether they fit the buffer
// there: the replaced particles keep their slots until the next step, so
// this needs room for both (a reseed that does not fit is skipped, as one
// above capacity is).
__global__ __launch_bounds__(1024) void k_reseed_appoff(ReseedArgs a)
{
    __shared__ long long wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int per = (a.nsel + 1023) / 1024;
    const int i0 = min(t * per, a.nsel), i1 = min(i0 + per, a.nsel);
    long long part = 0;
    for (int i = i0; i < i1; ++i) part += a.nnew[i];
    long long inc = part;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long v = __shfl_up(inc, off, 64);
        if (lane >= off) inc += v;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    long long before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    long long run = before + inc - part;
    for (int i = i0; i < i1; ++i) {
        a.appoff[i] = (int)min(run, (long long)0x7fffffff);
        run += a.nnew[i];
    }
    if (t == 1023 && (long long)a.cs_old[a.ncells] + before + inc > a.capacity) {
        a.ctr->reseed_err |= ST_CAPACITY;
        a.ctr->status |= ST_CAPACITY;
    }
}

// ... and the listing: a reseed that goes ahead lists every replaced cell
// not listed already (one add per wave on the list length); one that is
// skipped clears the marks, since no completion will read them
__global__ __launch_bounds__(256) void k_reseed_list(ReseedArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool ok = a.ctr->reseed_err == 0u;
    bool add = false;
    int c = -1;
    if (i < a.nsel) {
        c = a.cells[i];
        if (c >= 0 && c < a.ncells) {
            if (ok)
                add = (atomicOr(&a.comp[c], 2) == 0);
            else
                a.mark[c] = 0;
        }
    }
    const uint64_t m = ballot64(add);
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (m != 0 && lane == 0) base = atomicAdd(&a.ctr->ncomp, (uint32_t)__popcll(m));
    base = __shfl(base, 0, 64);
    if (add) a.complist[base + rank_below(m)] = c;
}

// the end of a reseed (its cells' marks were cleared as the state settled)
__global__ void k_reseed_done(Counters *ctr)
{
    if (threadIdx.x == 0) {
        ctr->reseed_err = 0u;
        ctr->reseed_new = 0ull;
        ctr->reseed_removed = 0ull;
    }
}

// ---- BGK lattice step (Section 3.1), one thread per node, push streaming ----
// periodic index in [0, n) for any shift (grids narrower than the velocities too)
__device__ __forceinline__ int wrap_index(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// The node's neighbour columns and rows for offsets -R..R: wrapped column
// index, start of the row (row * nx) and whether the row keeps what streams
// into it.  YM 1 (buffer rows): only interior rows keep anything; YM 2
// (walls): rows beyond the grid are walls; YM 0: y is periodic.  Rows beyond
// the grid are clamped to it so that an address formed from them stays in
// bounds.  NARROW: the grid is narrower than R in x or y (full modulo).
template <int R>
struct Nbr {
    int col[2 * R + 1];
    int row[2 * R + 1];
    bool in[2 * R + 1];
};

template <int R, int YM, bool NARROW>
__device__ __forceinline__ void neighbours(int ix, int iy, int nx, int ny, int K, Nbr<R> &n)
{
#pragma unroll
    for (int d = -R; d <= R; ++d) {
        int c = ix + d;
        if (NARROW) {
            c = wrap_index(c, nx);
        } else {
            c += c < 0 ? nx : 0;
            c -= c >= nx ? nx : 0;
        }
        n.col[d + R] = c;
        int y = iy + d;
        if (YM != 0) {
            n.in[d + R] = YM == 1 ? (y >= K && y < ny - K) : (y >= 0 && y < ny);
            y = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
        } else {
            n.in[d + R] = true;
            if (NARROW) {
                y = wrap_index(y, ny);
            } else {
                y += y < 0 ? ny : 0;
                y -= y >= ny ? ny : 0;
            }
        }
        n.row[d + R] = y * nx;
    }
}

template <int Q, int YM, bool NARROW>
__device__ __forceinline__ void lbm_node(const LbmArgs &a, int node)
{
#pragma clang fp contract(fast)
    using V = VelSet<Q>;
    constexpr int R = V::R;
    const int nx = a.nx, ny = a.ny;
    const size_t nn = (size_t)nx * ny;
    const int ix = node % nx, iy = node / nx;
    // held nodes (buffer rows, inflow columns) are neither collided nor overwritten
    const bool held = (YM == 1 && (iy < a.K || iy >= ny - a.K)) || ix < a.xb;
    const double r = a.L.r;
    double fe[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) fe[q] = *plane_ptr(a.f, nn, q, (uint32_t)node);
    if (a.keep) {
#pragma unroll
        for (int q = 0; q < Q; ++q) *plane_ptr(a.keep, nn, q, (uint32_t)node) = fe[q];
    }
    if (!held) {
        // rho and the momentum from the integer velocity components
        double rho = 0.0, ex = 0.0, ey = 0.0;
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            rho += fe[q];
            cmad<V::ex[q]>(ex, fe[q]);
            cmad<V::ey[q]>(ey, fe[q]);
        });
        const double g = a.gx, itau = 1.0 / a.tau;
        const double cf = 1.0 - 0.5 * itau, k1 = 1.0 - itau;
        const double irho = 1.0 / rho;
        const double ux = (r * ex + 0.5 * rho * g) * irho;
        const double uy = r * ey * irho;
        const double uu = ux * ux + uy * uy;
        const double rux = r * ux, ruy = r * uy, rg = r * g, gux = g * ux;
        double wr[8], fr[8];  // per shell: w rho / tau and (1 - 1/(2 tau)) w rho
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            wr[s] = a.L.ws[s] * rho * itau;
            fr[s] = cf * a.L.ws[s] * rho;
        }
        // post-collision f - (f - f_eq)/tau + force, with f_eq = w rho E(xi.u)
        // and force (1 - 1/(2 tau)) w rho [xi_x g (1 + xi.u) - g u_x]
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int s = V::sh[q];
            double cu = 0.0, cg = 0.0;
            cmad<V::ex[q]>(cu, rux);
            cmad<V::ey[q]>(cu, ruy);
            cmad<V::ex[q]>(cg, rg);
            double eq = 1.0 + cu + 0.5 * (cu * cu - uu);
            if (Q != 9) eq += cu * (cu * cu - 3.0 * uu) * (1.0 / 6.0);
            fe[q] = k1 * fe[q] + wr[s] * eq + fr[s] * (cg + cg * cu - gux);
        });
    }
    // push along e_q; held nodes also keep their own populations.  What
    // streams into a held node is dropped; with walls (YM 2, |e_y| <= 1) what
    // streams through a wall is taken up by it and given back to the same
    // node as the rest equilibrium of the mass it took
    Nbr<R> nb;
    neighbours<R, YM, NARROW>(ix, iy, nx, ny, a.K, nb);
    double wall_lo = 0.0, wall_hi = 0.0;
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if (held) *plane_ptr(a.ft, nn, q, (uint32_t)node) = fe[q];
        const int jx2 = nb.col[V::ex[q] + R];
        const bool in = YM == 0 || nb.in[V::ey[q] + R];
        if (YM == 2 && !in) {
            if constexpr (V::ey[q] < 0)
                wall_lo += fe[q];
            else
                wall_hi += fe[q];
        }
        if (in && jx2 >= a.xb)
            *plane_ptr(a.ft, nn, q, (uint32_t)(nb.row[V::ey[q] + R] + jx2)) = fe[q];
    });
    if (YM == 2 && !held && (iy == 0 || iy == ny - 1)) {
        double wup = 0.0, wdn = 0.0;  // weight of the directions pointing up / down
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (V::ey[q] > 0) wup += a.L.ws[V::sh[q]];
            if constexpr (V::ey[q] < 0) wdn += a.L.ws[V::sh[q]];
        });
        const double rlo = wall_lo / wup, rhi = wall_hi / wdn;
        static_for<Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (V::ey[q] > 0)
                if (iy == 0) *plane_ptr(a.ft, nn, q, (uint32_t)node) = a.L.ws[V::sh[q]] * rlo;
            if constexpr (V::ey[q] < 0)
                if (iy == ny - 1) *plane_ptr(a.ft, nn, q, (uint32_t)node) = a.L.ws[V::sh[q]] * rhi;
        });
    }
}

template <int Q, int YM, bool NARROW>
__global__ __launch_bounds__(256, 4) void k_lbm(LbmArgs a)
{
    const int node = blockIdx.x * 256 + threadIdx.x;
    if (node >= a.nx * a.ny) return;
    lbm_node<Q, YM, NARROW>(a, node);
}

#define DSMC_LBM_INSTANCES(Q, YM)                                 \
    template __global__ void k_lbm<Q, YM, false>(LbmArgs);        \
    template __global__ void k_lbm<Q, YM, true>(LbmArgs);
DSMC_LBM_INSTANCES(9, 0)
DSMC_LBM_INSTANCES(9, 1)
DSMC_LBM_INSTANCES(9, 2)
DSMC_LBM_INSTANCES(37, 0)
DSMC_LBM_INSTANCES(37, 1)
#undef DSMC_LBM_INSTANCES

}  // namespace dsmc
