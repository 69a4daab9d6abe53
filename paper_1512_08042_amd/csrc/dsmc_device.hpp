// Device-side building blocks of the DSMC step and the DSMC<->LBM mappings
// (gfx950, wave64).  Method: Di Staso, Clercx, Succi & Toschi,
// arXiv:1512.08042.  Every floating-point expression here is written in the
// same operation order as the step it implements and the library is built
// with -ffp-contract=off, so the integer decisions (cell indices, pair
// choices, accept/reject) follow from IEEE-rounded arithmetic only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsmc {

// Philox counter word 3 carries (tag << 24) | aux.
constexpr uint32_t TAG_INIT = 1u;
constexpr uint32_t TAG_WALL = 2u;
constexpr uint32_t TAG_COLL = 3u;
constexpr uint32_t TAG_RESEED_N = 4u;
constexpr uint32_t TAG_RESEED = 5u;
constexpr uint32_t TAG_RESEED_POS = 6u;

constexpr int MAX_BOUNCES = 16;
constexpr int NMOM = 11;
constexpr int NDIR = 9;     // 3x3 neighbourhood of the old cell
constexpr int DIR_FAR = 9;  // moved more than one cell in x or y
constexpr int DIR_NONE = 10;

constexpr uint32_t ST_WALL_LIMIT = 0x1u;
constexpr uint32_t ST_FAR_OVERFLOW = 0x2u;
constexpr uint32_t ST_CAPACITY = 0x4u;
constexpr uint32_t ST_AR_LIMIT = 0x8u;
constexpr uint32_t ST_NONFINITE = 0x10u;
constexpr uint32_t ST_NNEW_LIMIT = 0x20u;
constexpr uint32_t ST_BAD_CELL = 0x40u;
constexpr uint32_t ST_INTERNAL = 0x80u;

constexpr double TWO_PI = 6.283185307179586;

// Counters shared by all kernels of a context (device memory).
struct Counters {
    uint32_t status;
    uint32_t reseed_err;  // per-reseed error flags (cleared at each reseed)
    uint32_t nfar[2];     // long jumps of the step, double-buffered by step parity
    unsigned long long ncoll, ncand, nwall, nfar_total;
    unsigned long long reseed_new, reseed_removed;  // particle totals of the reseed in progress
    uint32_t step_base;   // first step of a replayed step graph (added to the steps it was captured with)
    uint32_t ncomp;       // cells listed for the completion pass of a moved state (see k_complete)
};

struct U4 {
    uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon et al., SC'11): ten rounds, each two 32x32->64
// products of counter words 0 and 2 with the round multipliers, mixed with
// the other two words and the round key; the key is bumped by the Weyl
// increments between rounds.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64 product each (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(uint32_t k0, uint32_t k1, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t tag,
                                   uint32_t aux)
{
    return philox(w0, w1, w2, (tag << 24) | (aux & 0xFFFFFFu), k0, k1);
}

// uniform in [0,1) with 53 random bits: a supplies the top 32, b the next 21
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    const uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)m * (1.0 / 9007199254740992.0);
}

// ---- elementary functions on the ranges this library needs -------------------
// The general-purpose FP64 sin/cos/log handle every argument and cost
// thousands of instructions; here the arguments are restricted, so short
// exact reductions and Taylor series suffice (a few ulp).

// cos(2 pi r) and sin(2 pi r) for r in [0, 1).  8r = k + f splits the turn
// into octants exactly (scaling by 8 and subtracting the integer part are
// exact); on each octant the angle is reduced to theta = g pi/4 with g in
// [0, 1] (g = f on even octants, 1 - f on odd ones, both exact), where the
// Taylor series of sin and cos to degree 19 / 20 are exact to rounding
// (remainder below 1e-21).
__device__ __forceinline__ void sincos_turn(double r, double &s, double &c)
{
    const double t = r * 8.0;
    const int k = (int)t;
    const double f = t - (double)k;
    const double g = (k & 1) ? 1.0 - f : f;
    const double th = g * 0.78539816339744830962;  // pi/4
    const double q = th * th;
    // sin(th) = th (1 - q/3! + q^2/5! - ... - q^9/19!)
    double ps = -1.0 / 121645100408832000.0;  // -1/19!
    ps = fma(ps, q, 1.0 / 355687428096000.0);
    ps = fma(ps, q, -1.0 / 1307674368000.0);
    ps = fma(ps, q, 1.0 / 6227020800.0);
    ps = fma(ps, q, -1.0 / 39916800.0);
    ps = fma(ps, q, 1.0 / 362880.0);
    ps = fma(ps, q, -1.0 / 5040.0);
    ps = fma(ps, q, 1.0 / 120.0);
    ps = fma(ps, q, -1.0 / 6.0);
    const double sn = fma(th * q, ps, th);
    // cos(th) = 1 - q/2! + q^2/4! - ... + q^10/20!
    double pc = 1.0 / 2432902008176640000.0;  // 1/20!
    pc = fma(pc, q, -1.0 / 6402373705728000.0);
    pc = fma(pc, q, 1.0 / 20922789888000.0);
    pc = fma(pc, q, -1.0 / 87178291200.0);
    pc = fma(pc, q, 1.0 / 479001600.0);
    pc = fma(pc, q, -1.0 / 3628800.0);
    pc = fma(pc, q, 1.0 / 40320.0);
    pc = fma(pc, q, -1.0 / 720.0);
    pc = fma(pc, q, 1.0 / 24.0);
    pc = fma(pc, q, -0.5);
    const double cs = fma(q, pc, 1.0);
    // angle = (k + f) pi/4 -> quadrant identities
    switch (k & 7) {
        case 0: c = cs; s = sn; break;    // theta
        case 1: c = sn; s = cs; break;    // pi/2 - theta
        case 2: c = -sn; s = cs; break;   // pi/2 + theta
        case 3: c = -cs; s = sn; break;   // pi - theta
        case 4: c = -cs; s = -sn; break;  // pi + theta
        case 5: c = -sn; s = -cs; break;  // 3pi/2 - theta
        case 6: c = sn; s = -cs; break;   // 3pi/2 + theta
        default: c = cs; s = -sn; break;  // 2pi - theta
    }
}

// natural log of x in (0, 1] (a normal double): x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), log m = 2 atanh(s), s = (m-1)/(m+1), |s| < 0.1716,
// atanh by its odd series to s^27 (remainder below 1e-22); e ln 2 with ln 2
// split in a short high part and a correction (the Cody-Waite split used by
// fdlibm's e_log.c, whose high part has trailing zero bits so that e times it
// is exact).
__device__ __forceinline__ double log_unit(double x)
{
    const long long bits = __double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    double m = __longlong_as_double((bits & 0x000fffffffffffffLL) | 0x3ff0000000000000LL);  // [1, 2)
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e += 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double q = s * s;
    double p = 1.0 / 27.0;
    p = fma(p, q, 1.0 / 25.0);
    p = fma(p, q, 1.0 / 23.0);
    p = fma(p, q, 1.0 / 21.0);
    p = fma(p, q, 1.0 / 19.0);
    p = fma(p, q, 1.0 / 17.0);
    p = fma(p, q, 1.0 / 15.0);
    p = fma(p, q, 1.0 / 13.0);
    p = fma(p, q, 1.0 / 11.0);
    p = fma(p, q, 1.0 / 9.0);
    p = fma(p, q, 1.0 / 7.0);
    p = fma(p, q, 1.0 / 5.0);
    p = fma(p, q, 1.0 / 3.0);
    const double lm = 2.0 * fma(s * q, p, s);
    const double ln2_hi = 6.93147180369123816490e-01, ln2_lo = 1.90821492927058770002e-10;
    return fma((double)e, ln2_hi, fma((double)e, ln2_lo, lm));
}

// Box-Muller pair from two uniforms; 1 - r1 is in (0, 1]
__device__ __forceinline__ void box_muller(double r1, double r2, double &z0, double &z1)
{
    const double rad = sqrt(-2.0 * log_unit(1.0 - r1));
    double s, c;
    sincos_turn(r2, s, c);
    z0 = rad * c;
    z1 = rad * s;
}

// uniform coordinate inside cell i: a sum that rounds up to the far edge is
// pulled back to the largest double below it
__device__ __forceinline__ double inside_cell(int i, double r)
{
    double v = (double)i + r;
    const double hi = (double)(i + 1);
    if (v >= hi) v = nextafter(hi, 0.0);
    return v;
}

struct Geometry {
    int nx, ny;
    double Lx, H;
};

__device__ __forceinline__ void cell_xy(const Geometry &G, double x, double y, int &ix, int &iy)
{
    ix = (int)floor(x);
    iy = (int)floor(y);
    ix = ix < 0 ? 0 : (ix > G.nx - 1 ? G.nx - 1 : ix);
    iy = iy < 0 ? 0 : (iy > G.ny - 1 ? G.ny - 1 : iy);
}

struct MoveParams {
    double dt, g, s_th;  // time step, acceleration along x, sqrt(kT/m)
    uint32_t k0, k1;     // Philox key
    uint32_t step;       // global step index
};

// Free flight of one particle over dt under the constant acceleration g
// along x, between diffuse walls at y = 0 and y = H: on a wall hit the
// particle is re-emitted from the wall with a flux-weighted normal speed and
// Gaussian tangential components at the wall temperature, and finishes the
// remaining time.  Bounce b of the particle in slot p draws from counters
// (2b, p, step, WALL) and (2b+1, p, step, WALL).  Returns the wall hits.
__device__ __forceinline__ int move_particle(const Geometry &G, const MoveParams &M, uint32_t p, double &x, double &y,
                                             double &vx, double &vy, double &vz, bool &limit)
{
    const double g = M.g, H = G.H;
    double t = M.dt;
    int b = 0;
    for (;;) {
        const double yn = y + vy * t;
        const bool cross = (yn < 0.0 || yn > H);
        if (cross && b < MAX_BOUNCES) {
            const double wall = (yn < 0.0) ? 0.0 : H;
            const double th = (wall - y) / vy;
            x = x + vx * th + 0.5 * g * th * th;
            y = wall;
            const U4 a = draw(M.k0, M.k1, (uint32_t)(2 * b), p, M.step, TAG_WALL, 0u);
            const U4 c = draw(M.k0, M.k1, (uint32_t)(2 * b + 1), p, M.step, TAG_WALL, 0u);
            const double vn = M.s_th * sqrt(-2.0 * log_unit(1.0 - u53(a.x, a.y)));
            double z0, z1;
            box_muller(u53(a.z, a.w), u53(c.x, c.y), z0, z1);
            vx = M.s_th * z0;
            vz = M.s_th * z1;
            vy = (wall == 0.0) ? vn : -vn;
            t = t - th;
            b += 1;
            continue;
        }
        if (cross) {
            limit = true;
            const double wall = (yn < 0.0) ? 0.0 : H;
            const double th = (wall - y) / vy;
            x = x + vx * th + 0.5 * g * th * th;
            vx = vx + g * th;
            y = wall;
            break;
        }
        x = x + vx * t + 0.5 * g * t * t;
        vx = vx + g * t;
        y = yn;
        break;
    }
    double xw = x - G.Lx * floor(x / G.Lx);
    if (xw < 0.0) xw = xw + G.Lx;
    if (xw >= G.Lx) xw = 0.0;
    x = xw;
    return b;
}

// Direction code of a move from cell (oix, oiy) to (nix, niy): 3*(dy+1) +
// (dx+1) for moves inside the 3x3 neighbourhood (dx taken modulo nx, +1
// preferred over -1 when both name the same cell), DIR_FAR otherwise.
__device__ __forceinline__ int direction(int nx, int oix, int oiy, int nix, int niy)
{
    const int dy = niy - oiy;
    if (dy < -1 || dy > 1) return DIR_FAR;
    int dl = nix - oix;
    if (dl < 0) dl += nx;
    int dx;
    if (dl == 0)
        dx = 0;
    else if (dl == 1)
        dx = 1;
    else if (dl == nx - 1)
        dx = -1;
    else
        return DIR_FAR;
    return (dy + 1) * 3 + (dx + 1);
}

// Source cell from which direction d reaches target (cix, ciy), or -1 when
// no source exists (outside the channel, or an alias of another direction
// when nx <= 2).
__device__ __forceinline__ int source_cell(int nx, int ny, int cix, int ciy, int d)
{
    const int dy = d / 3 - 1, dx = d % 3 - 1;
    const int siy = ciy - dy;
    if (siy < 0 || siy >= ny) return -1;
    int six = cix - dx;
    if (six < 0) six += nx;
    if (six >= nx) six -= nx;
    if (six < 0 || six >= nx) return -1;
    if (direction(nx, six, siy, cix, ciy) != d) return -1;
    return siy * nx + six;
}

// The near groups arriving in cell (cix, ciy) of a channel whose first cell
// is cb, in the order of the stable sort by new cell: by source cell.  For
// each rank k, dir[k] is the direction of the k-th group and key[k] its
// source cell (cb + index inside the channel), INT_MAX for a direction
// without a source (beyond a wall, or an alias when nx <= 2); those come last.
// Source cells of different directions differ, so the order is strict.
__device__ __forceinline__ void arrival_order(int nx, int ny, int cix, int ciy, int cb, int *key, int *dir)
{
    int kd[NDIR];
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
        const int sc = source_cell(nx, ny, cix, ciy, d);
        kd[d] = sc >= 0 ? cb + sc : 0x7fffffff;
    }
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
        int rank = 0;
#pragma unroll
        for (int e = 0; e < NDIR; ++e) rank += (kd[e] < kd[d] || (kd[e] == kd[d] && e < d)) ? 1 : 0;
#pragma unroll
        for (int k = 0; k < NDIR; ++k) {
            if (k == rank) {
                key[k] = kd[d];
                dir[k] = d;
            }
        }
    }
}

// ---- wave64 helpers --------------------------------------------------------
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// number of set bits of m in lanes below this lane
__device__ __forceinline__ int rank_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// the value of v on lane u (u wave-uniform), read into scalar registers
__device__ __forceinline__ unsigned long long lane_u64(unsigned long long v, int u)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), u);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of 16 per-lane values over a team of T lanes (T = 16, 32 or 64, teams
// aligned inside the wave), returned "scattered": afterwards lane lt of the
// team holds the team total of value (lt / (T/16)) & 15.  Four exchange
// steps halve the values each lane carries (17 shuffles for 16 values
// instead of 16 * log2(T)); the remaining steps are plain butterflies.
// Additions happen in a fixed order, so results are deterministic.
template <int T>
__device__ __forceinline__ double team_reduce_scatter16(double *v, int lt)
{
    double a[8], b[4], c[2], d;
    {
        constexpr int off = T / 2;
        const bool hi = (lt & off) != 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double keep = hi ? v[8 + i] : v[i];
            const double send = hi ? v[i] : v[8 + i];
            a[i] = keep + __shfl_xor(send, off, 64);
        }
    }
    {
        constexpr int off = T / 4;
        const bool hi = (lt & off) != 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double keep = hi ? a[4 + i] : a[i];
            const double send = hi ? a[i] : a[4 + i];
            b[i] = keep + __shfl_xor(send, off, 64);
        }
    }
    {
        constexpr int off = T / 8;
        const bool hi = (lt & off) != 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const double keep = hi ? b[2 + i] : b[i];
            const double send = hi ? b[i] : b[2 + i];
            c[i] = keep + __shfl_xor(send, off, 64);
        }
    }
    {
        constexpr int off = T / 16;
        const bool hi = (lt & off) != 0;
        const double keep = hi ? c[1] : c[0];
        const double send = hi ? c[0] : c[1];
        d = keep + __shfl_xor(send, off, 64);
    }
#pragma unroll
    for (int off = T / 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
    return d;
}

// ---- lattices ----------------------------------------------------------------
struct Lattice {
    int Q;
    double r;
    double w[37];
    double xi[37][2];
};

}  // namespace dsmc
