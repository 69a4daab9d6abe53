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

constexpr double TWO_PI = 6.283185307179586;

// Counters shared by all kernels of a context (device memory).
struct Counters {
    uint32_t status;
    uint32_t nfar;        // long jumps recorded in the current step
    uint32_t reseed_err;  // per-reseed error flags (cleared at each reseed)
    uint32_t pad;
    unsigned long long ncoll, ncand, nwall, nfar_total;
    unsigned long long reseed_new, reseed_removed;  // particle totals of the reseed in progress
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
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
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

// Box-Muller pair from two uniforms; 1 - r1 is in (0, 1]
__device__ __forceinline__ void box_muller(double r1, double r2, double &z0, double &z1)
{
    const double rad = sqrt(-2.0 * log(1.0 - r1));
    const double ang = TWO_PI * r2;
    z0 = rad * cos(ang);
    z1 = rad * sin(ang);
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
            const double vn = M.s_th * sqrt(-2.0 * log(1.0 - u53(a.x, a.y)));
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

// ---- wave64 helpers --------------------------------------------------------
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// number of set bits of m in lanes below this lane
__device__ __forceinline__ int rank_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
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

// ---- lattices ----------------------------------------------------------------
struct Lattice {
    int Q;
    double r;
    double w[37];
    double xi[37][2];
};

}  // namespace dsmc
