/*
 * DSMC-LBM oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 implementation of what the GPU library
 * computes, written from Di Staso, Clercx, Succi & Toschi, "DSMC-LBM mapping
 * scheme for rarefied and non-rarefied gas flows" (arXiv:1512.08042).  Only the
 * test suite, the package smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or constant generator with the
 * GPU library; the quadrature tables it uses are derived by oracle/oracle.py.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (oracle/oracle.py).
 * Contraction is off so that every floating-point operation is rounded exactly
 * as written, which is what lets the GPU side reproduce the integer decisions.
 * The same source built with -fopenmp runs its per-particle and per-cell loops
 * on all host cores (the CPU baseline of the benchmark).  Every loop so split
 * is over independent particles or cells (draws are keyed by slot or cell,
 * sums per cell keep their order), counters are integer reductions, and the
 * counting sort gives each thread's slot range its own offsets inside each
 * cell, so the threaded build's results are bit-identical to the single-
 * threaded one (checked by the tests).
 *
 * Conventions (the paper works in SI units; the unit system below is the
 * nondimensionalisation of its appendix "Scaling factors"):
 *   cell size 1 in x and y, channel height H = ny, periodic length Lx = nx;
 *   speeds in units where kT/m is the configured kT_over_m (1 by default);
 *   mean free path lambda = Kn * H (Kn on the channel height, Section 3.1);
 *   hard spheres with F_N sigma_T / V_c = 1/(sqrt(2) lambda ppc), which is the
 *   hard-sphere mean-free-path relation of Eq. (MFP) with n = ppc F_N / V_c.
 *
 * Parity-unpinned parts: none of the functions below lacks a pin; see the
 * tests under tests/ (test_oracle_*.py) for what pins each one.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_NMOM 11
#define OR_MAX_BOUNCES 16

/* counter tags: Philox counter word 3 is (tag << 24) | aux */
#define OR_TAG_INIT 1u
#define OR_TAG_WALL 2u
#define OR_TAG_COLL 3u
#define OR_TAG_RESEED_N 4u
#define OR_TAG_RESEED 5u
#define OR_TAG_RESEED_POS 6u

/* status bits */
#define OR_ST_WALL_LIMIT 0x1u
#define OR_ST_CAPACITY 0x4u
#define OR_ST_AR_LIMIT 0x8u
#define OR_ST_NONFINITE 0x10u
#define OR_ST_NNEW_LIMIT 0x20u
#define OR_ST_BAD_CELL 0x40u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the */
/* round key bumped by the Weyl constants between rounds.                    */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t tag, uint32_t aux,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {w0, w1, w2, (tag << 24) | (aux & 0xFFFFFFu)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in [0,1) from two 32-bit words: top 32 bits from a, low 21
 * bits from the high bits of b; the integer converts to double exactly. */
double or_u53(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)m * (1.0 / 9007199254740992.0);
}

/* Box-Muller: two independent standard normals from two uniforms (Table 1,
 * step 4 names the transformation).  1 - r1 lies in (0, 1]. */
void or_box_muller(double r1, double r2, double out[2])
{
    double rad = sqrt(-2.0 * log(1.0 - r1));
    double ang = 6.283185307179586 * r2;
    out[0] = rad * cos(ang);
    out[1] = rad * sin(ang);
}

/* ------------------------------------------------------------------------ */
/* threads of the OpenMP build (1 in the plain build)                       */
/* ------------------------------------------------------------------------ */
int32_t or_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

static int nthreads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* simulation state                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny, ppc, nbar_mode, ar_max_tries, ncells;
    int64_t capacity;
    double kn, dt, g, kT, sigcr0;
    uint64_t seed;
    double lambda, K, Lx, H, s_th;
    int64_t n;
    double *x, *y, *vx, *vy, *vz;
    double *tx, *ty, *tvx, *tvy, *tvz; /* scratch of the same capacity */
    int32_t *cell_start;                /* ncells + 1 */
    int32_t *cellid;                    /* per particle scratch */
    double *nbar, *sigcmax, *rem;       /* per cell */
    double *mom;                        /* [11][ncells] sums */
    int64_t nsamples, step, reseed_events;
    int64_t ncoll, ncand, nwall;
    uint32_t status;
    int32_t state32;                    /* 1: particle state stored in FP32 */
} or_sim;

/* Stored particle values: with FP32 state every value written to the
 * particle arrays is rounded to the nearest float; the arithmetic itself is
 * FP64 on the stored values. */
static double stv(const or_sim *s, double v) { return s->state32 ? (double)(float)v : v; }

static void *xalloc(size_t n) { void *p = calloc(n ? n : 1, 1); return p; }

or_sim *or_create(int32_t nx, int32_t ny, int32_t ppc, int32_t nbar_mode, int64_t capacity, double kn,
                  double dt, double g, double kT, double sigcr0, uint64_t seed, int32_t ar_max_tries)
{
    if (nx < 1 || ny < 1 || ppc < 1 || capacity < 1 || !(kn > 0) || !(dt > 0) || !(kT > 0)) return NULL;
    or_sim *s = (or_sim *)xalloc(sizeof(or_sim));
    s->nx = nx; s->ny = ny; s->ppc = ppc; s->nbar_mode = nbar_mode; s->capacity = capacity;
    s->kn = kn; s->dt = dt; s->g = g; s->kT = kT; s->sigcr0 = sigcr0; s->seed = seed;
    s->ar_max_tries = ar_max_tries > 0 ? ar_max_tries : 65536;
    s->ncells = nx * ny;
    s->Lx = (double)nx;
    s->H = (double)ny;
    s->lambda = kn * s->H;
    /* Eq. (MFP): lambda = 1/(sqrt(2) pi d^2 n) with n = ppc F_N / V_c, so
     * F_N sigma_T / V_c = 1 / (sqrt(2) lambda ppc). */
    s->K = 1.0 / (sqrt(2.0) * s->lambda * (double)ppc);
    s->s_th = sqrt(kT);
    size_t cap = (size_t)capacity, nc = (size_t)s->ncells;
    s->x = xalloc(cap * 8); s->y = xalloc(cap * 8); s->vx = xalloc(cap * 8);
    s->vy = xalloc(cap * 8); s->vz = xalloc(cap * 8);
    s->tx = xalloc(cap * 8); s->ty = xalloc(cap * 8); s->tvx = xalloc(cap * 8);
    s->tvy = xalloc(cap * 8); s->tvz = xalloc(cap * 8);
    s->cellid = xalloc(cap * 4);
    s->cell_start = xalloc((nc + 1) * 4);
    s->nbar = xalloc(nc * 8); s->sigcmax = xalloc(nc * 8); s->rem = xalloc(nc * 8);
    s->mom = xalloc(nc * OR_NMOM * 8);
    for (size_t c = 0; c < nc; ++c) s->sigcmax[c] = sigcr0;
    return s;
}

void or_destroy(or_sim *s)
{
    if (!s) return;
    free(s->x); free(s->y); free(s->vx); free(s->vy); free(s->vz);
    free(s->tx); free(s->ty); free(s->tvx); free(s->tvy); free(s->tvz);
    free(s->cellid); free(s->cell_start); free(s->nbar); free(s->sigcmax); free(s->rem);
    free(s->mom); free(s);
}

/* cell index: ix = floor(x), iy = floor(y) clamped to the top row (a
 * particle exactly on y = H belongs to the last row). */
static int32_t cell_of(const or_sim *s, double x, double y)
{
    int32_t ix = (int32_t)floor(x);
    int32_t iy = (int32_t)floor(y);
    if (ix < 0) ix = 0;
    if (ix > s->nx - 1) ix = s->nx - 1;
    if (iy < 0) iy = 0;
    if (iy > s->ny - 1) iy = s->ny - 1;
    return iy * s->nx + ix;
}

/* uniform position inside cell (ix, iy); a sum that rounds up to the next
 * cell edge is pulled back to the largest double below it. */
static double inside(int32_t i, double r)
{
    double v = (double)i + r;
    double hi = (double)(i + 1);
    if (v >= hi) v = nextafter(hi, 0.0);
    return v;
}

/* stable counting sort of the particle set by cell index (ties keep slot
 * order), rebuilding cell_start.  With T threads, thread t owns the slot
 * range [t n / T, (t+1) n / T); inside every cell the ranges follow each
 * other in thread order, each in slot order, which is the serial order. */
static void sort_by_cell(or_sim *s)
{
    int32_t nc = s->ncells;
    int T = nthreads();
    int32_t *cnt = (int32_t *)xalloc((size_t)T * (nc + 1) * 4);
#pragma omp parallel num_threads(T)
    {
#ifdef _OPENMP
        const int t = omp_get_thread_num(), Tn = omp_get_num_threads(); /* Tn <= T */
#else
        const int t = 0, Tn = 1;
#endif
        int64_t lo = s->n * t / Tn, hi = s->n * (t + 1) / Tn;
        int32_t *mine = cnt + (size_t)t * (nc + 1);
        for (int64_t p = lo; p < hi; ++p) {
            s->cellid[p] = cell_of(s, s->x[p], s->y[p]);
            mine[s->cellid[p]] += 1;
        }
#pragma omp barrier
#pragma omp single
        {
            int32_t acc = 0;
            for (int32_t c = 0; c < nc; ++c) {
                s->cell_start[c] = acc;
                for (int u = 0; u < Tn; ++u) {
                    int32_t k = cnt[(size_t)u * (nc + 1) + c];
                    cnt[(size_t)u * (nc + 1) + c] = acc;
                    acc += k;
                }
            }
            s->cell_start[nc] = acc;
        }
        for (int64_t p = lo; p < hi; ++p) {
            int32_t c = s->cellid[p];
            int64_t d = mine[c]++;
            s->tx[d] = s->x[p]; s->ty[d] = s->y[p];
            s->tvx[d] = s->vx[p]; s->tvy[d] = s->vy[p]; s->tvz[d] = s->vz[p];
        }
    }
    double *tp;
    tp = s->x; s->x = s->tx; s->tx = tp;
    tp = s->y; s->y = s->ty; s->ty = tp;
    tp = s->vx; s->vx = s->tvx; s->tvx = tp;
    tp = s->vy; s->vy = s->tvy; s->tvy = tp;
    tp = s->vz; s->vz = s->tvz; s->tvz = tp;
    free(cnt);
}

/* Initial state: exactly ppc particles in every cell (Section 3.1 places a
 * fixed number of computational molecules in each cell), uniform in the cell,
 * velocities from the Maxwellian at the reference temperature drawn by
 * Box-Muller. Particle g = c*ppc + k of cell c uses counters (d, g, 0, INIT). */
/* FP32 particle state (1) or FP64 (0); set before the state is first written */
void or_set_state32(or_sim *s, int32_t on) { s->state32 = on ? 1 : 0; }

void or_init_maxwell(or_sim *s)
{
    int64_t n = (int64_t)s->ncells * s->ppc;
    if (n > s->capacity) { s->status |= OR_ST_CAPACITY; n = 0; }
    s->n = n;
#pragma omp parallel for schedule(static)
    for (int32_t c = 0; c < s->ncells; ++c) {
        int32_t ix = c % s->nx, iy = c / s->nx;
        for (int32_t k = 0; k < s->ppc; ++k) {
            int64_t gi = (int64_t)c * s->ppc + k;
            if (gi >= n) break;
            uint32_t a[4], b[4], e[4];
            double z[2], zz[2];
            draw(s->seed, 0u, (uint32_t)gi, 0u, OR_TAG_INIT, 0u, a);
            draw(s->seed, 1u, (uint32_t)gi, 0u, OR_TAG_INIT, 0u, b);
            draw(s->seed, 2u, (uint32_t)gi, 0u, OR_TAG_INIT, 0u, e);
            or_box_muller(or_u53(b[0], b[1]), or_u53(b[2], b[3]), z);
            or_box_muller(or_u53(e[0], e[1]), or_u53(e[2], e[3]), zz);
            s->x[gi] = stv(s, inside(ix, or_u53(a[0], a[1])));
            s->y[gi] = stv(s, inside(iy, or_u53(a[2], a[3])));
            s->vx[gi] = stv(s, s->s_th * z[0]);
            s->vy[gi] = stv(s, s->s_th * z[1]);
            s->vz[gi] = stv(s, s->s_th * zz[0]);
        }
    }
    for (int32_t c = 0; c <= s->ncells; ++c) {
        int64_t v = (int64_t)c * s->ppc;
        s->cell_start[c] = (int32_t)(v < n ? v : n);
    }
}

/* Adopt an arbitrary particle set (positions must lie in [0,Lx) x [0,H]). */
int or_load(or_sim *s, int64_t n, const double *x, const double *y, const double *vx, const double *vy,
            const double *vz)
{
    if (n < 0 || n > s->capacity) return -1;
    s->n = n;
    memcpy(s->x, x, (size_t)n * 8); memcpy(s->y, y, (size_t)n * 8);
    memcpy(s->vx, vx, (size_t)n * 8); memcpy(s->vy, vy, (size_t)n * 8);
    memcpy(s->vz, vz, (size_t)n * 8);
    for (int64_t p = 0; p < n; ++p) {
        s->x[p] = stv(s, s->x[p]); s->y[p] = stv(s, s->y[p]);
        s->vx[p] = stv(s, s->vx[p]); s->vy[p] = stv(s, s->vy[p]); s->vz[p] = stv(s, s->vz[p]);
    }
    sort_by_cell(s);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* free flight under the body force, with fully diffuse isothermal walls     */
/* ------------------------------------------------------------------------ */
/* The channel is driven by a constant acceleration g along x (the force-
 * driven plane Poiseuille flow of Section 3.1) and bounded by walls at y = 0
 * and y = H with full diffuse reflection at the reference temperature
 * (caption of the velocity-profile figure).  The x motion is the exact
 * constant-acceleration update; a wall hit resets all three components:
 * normal speed from the flux-weighted (Rayleigh) law, tangential components
 * Gaussian.  Bounce b of the particle in slot p at step s draws from counters
 * (2b, p, s, WALL) and (2b+1, p, s, WALL). */
static int move_one(const or_sim *s, int64_t p, double *px, double *py, double *pvx, double *pvy, double *pvz,
                    int *limit)
{
    double x = *px, y = *py, vx = *pvx, vy = *pvy, vz = *pvz;
    double g = s->g, H = s->H;
    double t = s->dt;
    int b = 0;
    for (;;) {
        double yn = y + vy * t;
        if ((yn < 0.0 || yn > H) && b < OR_MAX_BOUNCES) {
            double wall = (yn < 0.0) ? 0.0 : H;
            double th = (wall - y) / vy;
            x = x + vx * th + 0.5 * g * th * th;
            y = wall;
            uint32_t a[4], c[4];
            draw(s->seed, (uint32_t)(2 * b), (uint32_t)p, (uint32_t)s->step, OR_TAG_WALL, 0u, a);
            draw(s->seed, (uint32_t)(2 * b + 1), (uint32_t)p, (uint32_t)s->step, OR_TAG_WALL, 0u, c);
            double vn = s->s_th * sqrt(-2.0 * log(1.0 - or_u53(a[0], a[1])));
            double z[2];
            or_box_muller(or_u53(a[2], a[3]), or_u53(c[0], c[1]), z);
            vx = s->s_th * z[0];
            vz = s->s_th * z[1];
            vy = (wall == 0.0) ? vn : -vn;
            t = t - th;
            b += 1;
            continue;
        }
        if (yn < 0.0 || yn > H) {
            /* bounce limit reached: stop the particle on the wall it hits */
            *limit = 1;
            double wall = (yn < 0.0) ? 0.0 : H;
            double th = (wall - y) / vy;
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
    /* periodic x */
    double Lx = s->Lx;
    double xw = x - Lx * floor(x / Lx);
    if (xw < 0.0) xw = xw + Lx;
    if (xw >= Lx) xw = 0.0;
    *px = stv(s, xw); *py = stv(s, y); *pvx = stv(s, vx); *pvy = stv(s, vy); *pvz = stv(s, vz);
    return b;
}

/* ------------------------------------------------------------------------ */
/* No-Time-Counter collisions, hard spheres (Eq. (collisionnumber))          */
/* ------------------------------------------------------------------------ */
/* Per cell: N_cand = 1/2 N Nbar F_N (sigma_T c_r)_max dt / V_c plus the
 * carried fraction; candidate pairs are drawn uniformly (with replacement
 * across candidates, i != j within one); a pair collides with probability
 * c_r / c_r,max (hard-sphere cross section), and the post-collision relative
 * velocity is isotropic (hard-sphere scattering).  sigcmax stores
 * (sigma_T c_r)_max / sigma_T, a speed, and grows when exceeded.
 * Candidate k of cell c at step s draws from counters (2k, c, s, COLL) and,
 * when accepted, (2k+1, c, s, COLL). */
static void collide_cell(or_sim *s, int32_t c, int64_t *pcand, int64_t *pcoll)
{
    int32_t start = s->cell_start[c];
    int32_t N = s->cell_start[c + 1] - start;
    double Nd = (double)N;
    s->nbar[c] = s->nbar[c] + (Nd - s->nbar[c]) / (double)(s->step + 1);
    double pairf = (s->nbar_mode == 1) ? (Nd - 1.0) : s->nbar[c];
    double X = 0.5 * Nd * pairf * s->K * s->sigcmax[c] * s->dt + s->rem[c];
    if (!(X > 0.0)) X = 0.0;
    double M = floor(X);
    s->rem[c] = X - M;
    if (N < 2) return;
    int64_t ncand = (int64_t)M;
    for (int64_t k = 0; k < ncand; ++k) {
        uint32_t u[4];
        draw(s->seed, (uint32_t)(2 * k), (uint32_t)c, (uint32_t)s->step, OR_TAG_COLL, 0u, u);
        uint32_t i = (uint32_t)(((uint64_t)u[0] * (uint64_t)(uint32_t)N) >> 32);
        uint32_t j = (uint32_t)(((uint64_t)u[1] * (uint64_t)(uint32_t)(N - 1)) >> 32);
        if (j >= i) j += 1;
        int64_t pi = start + (int64_t)i, pj = start + (int64_t)j;
        double dx = s->vx[pi] - s->vx[pj];
        double dy = s->vy[pi] - s->vy[pj];
        double dz = s->vz[pi] - s->vz[pj];
        double cr = sqrt(dx * dx + dy * dy + dz * dz);
        if (cr > s->sigcmax[c]) s->sigcmax[c] = cr;
        double R = or_u53(u[2], u[3]);
        *pcand += 1;
        if (cr / s->sigcmax[c] > R) {
            uint32_t w[4];
            draw(s->seed, (uint32_t)(2 * k + 1), (uint32_t)c, (uint32_t)s->step, OR_TAG_COLL, 0u, w);
            double cth = 2.0 * or_u53(w[0], w[1]) - 1.0;
            double sth = sqrt(1.0 - cth * cth);
            double phi = 6.283185307179586 * or_u53(w[2], w[3]);
            double rx = cr * cth;
            double ry = cr * sth * cos(phi);
            double rz = cr * sth * sin(phi);
            double mx = 0.5 * (s->vx[pi] + s->vx[pj]);
            double my = 0.5 * (s->vy[pi] + s->vy[pj]);
            double mz = 0.5 * (s->vz[pi] + s->vz[pj]);
            s->vx[pi] = stv(s, mx + 0.5 * rx); s->vy[pi] = stv(s, my + 0.5 * ry); s->vz[pi] = stv(s, mz + 0.5 * rz);
            s->vx[pj] = stv(s, mx - 0.5 * rx); s->vy[pj] = stv(s, my - 0.5 * ry); s->vz[pj] = stv(s, mz - 0.5 * rz);
            *pcoll += 1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* cumulative sampling of the velocity moments up to third order            */
/* ------------------------------------------------------------------------ */
/* Per cell, add N and the sums of vx, vy, vx^2, vx vy, vy^2, vx^3, vx^2 vy,
 * vx vy^2, vy^3 and vz^2 (raw velocities) to the running sums (the
 * cumulative averages that feed DSMC2LB, Section 2.1). */
static void sample_all(or_sim *s)
{
    int32_t nc = s->ncells;
#pragma omp parallel for schedule(static)
    for (int32_t c = 0; c < nc; ++c) {
        double acc[OR_NMOM];
        for (int k = 0; k < OR_NMOM; ++k) acc[k] = 0.0;
        for (int32_t p = s->cell_start[c]; p < s->cell_start[c + 1]; ++p) {
            double a = s->vx[p], b = s->vy[p], z = s->vz[p];
            acc[0] += 1.0;
            acc[1] += a;
            acc[2] += b;
            acc[3] += a * a;
            acc[4] += a * b;
            acc[5] += b * b;
            acc[6] += a * a * a;
            acc[7] += a * a * b;
            acc[8] += a * b * b;
            acc[9] += b * b * b;
            acc[10] += z * z;
        }
        for (int k = 0; k < OR_NMOM; ++k) s->mom[(size_t)k * nc + c] += acc[k];
    }
    s->nsamples += 1;
}

/* One DSMC step: move (with walls), index and sort, collide, sample. */
void or_step(or_sim *s, int32_t nsteps, int32_t sample_every)
{
    for (int32_t it = 0; it < nsteps; ++it) {
        int64_t nw = 0, ncand = 0, ncoll = 0;
        int lim = 0;
#pragma omp parallel for schedule(static) reduction(+ : nw) reduction(| : lim)
        for (int64_t p = 0; p < s->n; ++p)
            nw += move_one(s, p, &s->x[p], &s->y[p], &s->vx[p], &s->vy[p], &s->vz[p], &lim);
        s->nwall += nw;
        if (lim) s->status |= OR_ST_WALL_LIMIT;
        sort_by_cell(s);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : ncand, ncoll)
        for (int32_t c = 0; c < s->ncells; ++c) collide_cell(s, c, &ncand, &ncoll);
        s->ncand += ncand;
        s->ncoll += ncoll;
        if (sample_every > 0 && ((s->step + 1) % sample_every) == 0) sample_all(s);
        s->step += 1;
    }
}

/* explicit sampling of the current state (used to check sampling alone) */
void or_sample_now(or_sim *s) { sample_all(s); }

void or_averages(const or_sim *s, double *out)
{
    size_t tot = (size_t)s->ncells * OR_NMOM;
    for (size_t i = 0; i < tot; ++i) out[i] = s->nsamples > 0 ? s->mom[i] / (double)s->nsamples : 0.0;
}

void or_reset_moments(or_sim *s)
{
    memset(s->mom, 0, (size_t)s->ncells * OR_NMOM * 8);
    s->nsamples = 0;
}

int64_t or_count(const or_sim *s) { return s->n; }

void or_get_particles(const or_sim *s, double *x, double *y, double *vx, double *vy, double *vz)
{
    memcpy(x, s->x, (size_t)s->n * 8); memcpy(y, s->y, (size_t)s->n * 8);
    memcpy(vx, s->vx, (size_t)s->n * 8); memcpy(vy, s->vy, (size_t)s->n * 8);
    memcpy(vz, s->vz, (size_t)s->n * 8);
}

void or_get_cells(const or_sim *s, int32_t *cell_start, double *nbar, double *sigcmax, double *rem)
{
    memcpy(cell_start, s->cell_start, (size_t)(s->ncells + 1) * 4);
    memcpy(nbar, s->nbar, (size_t)s->ncells * 8);
    memcpy(sigcmax, s->sigcmax, (size_t)s->ncells * 8);
    memcpy(rem, s->rem, (size_t)s->ncells * 8);
}

void or_set_cells(or_sim *s, const double *nbar, const double *sigcmax, const double *rem)
{
    memcpy(s->nbar, nbar, (size_t)s->ncells * 8);
    memcpy(s->sigcmax, sigcmax, (size_t)s->ncells * 8);
    memcpy(s->rem, rem, (size_t)s->ncells * 8);
}

/* counters: step, nsamples, ncoll, ncand, nwall, reseed_events, status */
void or_get_counters(const or_sim *s, int64_t out[8])
{
    out[0] = s->step; out[1] = s->nsamples; out[2] = s->ncoll; out[3] = s->ncand;
    out[4] = s->nwall; out[5] = s->reseed_events; out[6] = (int64_t)s->status; out[7] = s->n;
}

void or_set_step(or_sim *s, int64_t step) { s->step = step; }

/* ------------------------------------------------------------------------ */
/* Hermite machinery (Eqs. (series)-(seriestrunc)), 2-D velocity space       */
/* ------------------------------------------------------------------------ */
/* Probabilists' Hermite tensors: H_i = x_i, H_ij = x_i x_j - d_ij,
 * H_ijk = x_i x_j x_k - (x_i d_jk + x_j d_ik + x_k d_ij). Coefficient order
 * used throughout: a2 = (xx, xy, yy), a3 = (xxx, xxy, xyy, yyy). */

/* DSMC2LB projection (Eq. (discretefunctions)): from the cumulative averages
 * of one cell build a(0..3) (Eq. (nordercoefficients), absolute frame,
 * density scaled so that ppc particles are rho = 1 as in the appendix's mass
 * scale) and evaluate f_a = w_a sum_n a(n) : H(n)(xi_a) / n!.
 * avg: [11][ncells] time averages of the sampled sums; f: [Q][ncells].
 * On a lattice that cannot carry H_xxx, H_yyy (D2Q9, Q = 9) those two terms
 * are left out. */
void or_dsmc2lb(const double *avg, int32_t ncells, int32_t ppc, double kT, int32_t Q, int32_t order,
                const double *w, const double *xi, double *f)
{
    double s1 = sqrt(kT);
#pragma omp parallel for schedule(static)
    for (int32_t c = 0; c < ncells; ++c) {
        double m[OR_NMOM];
        for (int k = 0; k < OR_NMOM; ++k) m[k] = avg[(size_t)k * ncells + c];
        if (!(m[0] > 0.0)) {
            for (int32_t a = 0; a < Q; ++a) f[(size_t)a * ncells + c] = 0.0;
            continue;
        }
        double rho = m[0] / (double)ppc;
        double ex = (m[1] / m[0]) / s1, ey = (m[2] / m[0]) / s1;
        double s2 = s1 * s1, s3 = s2 * s1;
        double exx = (m[3] / m[0]) / s2, exy = (m[4] / m[0]) / s2, eyy = (m[5] / m[0]) / s2;
        double exxx = (m[6] / m[0]) / s3, exxy = (m[7] / m[0]) / s3;
        double exyy = (m[8] / m[0]) / s3, eyyy = (m[9] / m[0]) / s3;
        double a1x = rho * ex, a1y = rho * ey;
        double a2xx = rho * (exx - 1.0), a2xy = rho * exy, a2yy = rho * (eyy - 1.0);
        double a3xxx = rho * (exxx - 3.0 * ex), a3xxy = rho * (exxy - ey);
        double a3xyy = rho * (exyy - ex), a3yyy = rho * (eyyy - 3.0 * ey);
        for (int32_t a = 0; a < Q; ++a) {
            double x = xi[2 * a], y = xi[2 * a + 1];
            double v = rho;
            if (order >= 1) v += a1x * x + a1y * y;
            if (order >= 2) {
                double hxx = x * x - 1.0, hxy = x * y, hyy = y * y - 1.0;
                v += 0.5 * (a2xx * hxx + 2.0 * a2xy * hxy + a2yy * hyy);
            }
            if (order >= 3) {
                double hxxy = x * x * y - y, hxyy = x * y * y - x;
                double t3 = 3.0 * a3xxy * hxxy + 3.0 * a3xyy * hxyy;
                if (Q != 9) {
                    double hxxx = x * x * x - 3.0 * x, hyyy = y * y * y - 3.0 * y;
                    t3 += a3xxx * hxxx + a3yyy * hyyy;
                }
                v += t3 / 6.0;
            }
            f[(size_t)a * ncells + c] = w[a] * v;
        }
    }
}

/* LB2DSMC, Table 1 steps 1-3 for one node: from populations f[a] (stride
 * `stride`) compute rho, u = sum f xi / rho, and the comoving, density-
 * normalised coefficients a2 (3) and a3 (4) about u; then M (largest
 * magnitude of the retained components) and C = 1 + 30 M.
 * out: rho, ux, uy, a2xx, a2xy, a2yy, a3xxx, a3xxy, a3xyy, a3yyy, M, C. */
void or_grad_params(const double *f, int64_t stride, int32_t Q, int32_t order, const double *xi, double out[12])
{
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int32_t a = 0; a < Q; ++a) {
        double fa = f[(size_t)a * stride];
        rho += fa;
        jx += fa * xi[2 * a];
        jy += fa * xi[2 * a + 1];
    }
    for (int k = 0; k < 12; ++k) out[k] = 0.0;
    out[0] = rho;
    if (!(rho > 0.0)) return;
    double ux = jx / rho, uy = jy / rho;
    double sxx = 0, sxy = 0, syy = 0, sxxx = 0, sxxy = 0, sxyy = 0, syyy = 0;
    for (int32_t a = 0; a < Q; ++a) {
        double fa = f[(size_t)a * stride];
        double cx = xi[2 * a] - ux, cy = xi[2 * a + 1] - uy;
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
    if (order < 3) { a3xxx = 0; a3xxy = 0; a3xyy = 0; a3yyy = 0; }
    if (Q == 9) { a3xxx = 0; a3yyy = 0; }
    if (order < 2) { a2xx = 0; a2xy = 0; a2yy = 0; }
    double M = 0.0;
    double comp[7] = {a2xx, a2xy, a2yy, a3xxx, a3xxy, a3xyy, a3yyy};
    for (int k = 0; k < 7; ++k) {
        double v = fabs(comp[k]);
        if (v > M) M = v;
    }
    out[1] = ux; out[2] = uy;
    out[3] = a2xx; out[4] = a2xy; out[5] = a2yy;
    out[6] = a3xxx; out[7] = a3xxy; out[8] = a3xyy; out[9] = a3yyy;
    out[10] = M;
    out[11] = 1.0 + 30.0 * M;
}

/* G of Eq. (distr_outeq) at xi (comoving, density-normalised, so a0 = 1 and
 * a1 = 0): 1 + a2:H2/2! + a3:H3/3!. prm as produced by or_grad_params. */
double or_grad_G(const double prm[12], double x, double y)
{
    double hxx = x * x - 1.0, hxy = x * y, hyy = y * y - 1.0;
    double hxxx = x * x * x - 3.0 * x, hxxy = x * x * y - y;
    double hxyy = x * y * y - x, hyyy = y * y * y - 3.0 * y;
    double t2 = prm[3] * hxx + 2.0 * prm[4] * hxy + prm[5] * hyy;
    double t3 = prm[6] * hxxx + 3.0 * prm[7] * hxxy + 3.0 * prm[8] * hxyy + prm[9] * hyyy;
    return 1.0 + t2 / 2.0 + t3 / 6.0;
}

/* Table 1 steps 4-5 for new particle k of cell c in reseed event e: try
 * xi from Box-Muller on counters (2t, c, e, RESEED|k), accept when
 * C R <= G(xi) with R from counters (2t+1, c, e, RESEED|k).  After
 * max_tries rejections the last try is kept and the status bit is set.
 * Returns the number of tries. */
static int64_t ar_sample(uint64_t seed, const double prm[12], uint32_t c, uint32_t e, uint32_t k, int32_t max_tries,
                         double xi_out[2], uint32_t *status)
{
    double C = prm[11];
    int64_t t = 0;
    for (;;) {
        uint32_t a[4], b[4];
        draw(seed, (uint32_t)(2 * t), c, e, OR_TAG_RESEED, k, a);
        draw(seed, (uint32_t)(2 * t + 1), c, e, OR_TAG_RESEED, k, b);
        double z[2];
        or_box_muller(or_u53(a[0], a[1]), or_u53(a[2], a[3]), z);
        double R = or_u53(b[0], b[1]);
        double G = or_grad_G(prm, z[0], z[1]);
        t += 1;
        xi_out[0] = z[0];
        xi_out[1] = z[1];
        if (C * R <= G) break;
        if (t >= max_tries) { *status |= OR_ST_AR_LIMIT; break; }
    }
    return t;
}

/* batch AR sampling for statistics: n particles k = 0..n-1 of cell `c`,
 * event `e`; xi_out is [n][2]; returns the total number of tries. */
int64_t or_ar_sample_batch(uint64_t seed, const double prm[12], uint32_t c, uint32_t e, int64_t n, int32_t max_tries,
                           double *xi_out, uint32_t *status)
{
    int64_t tries = 0;
    for (int64_t k = 0; k < n; ++k) tries += ar_sample(seed, prm, c, e, (uint32_t)k, max_tries, &xi_out[2 * k], status);
    return tries;
}

/* LB2DSMC reconstruction (Section 2.2, Table 1) on the listed cells.
 * f: [Q][ncells] populations; cells: nsel distinct cell ids.  For each listed
 * cell: Table 1 steps 1-3, N_new = floor(rho * ppc + R) (mass conservation at
 * the coupling site; stochastic rounding with R from counters
 * (0, c, e, RESEED_N)), then steps 4-6 for each new particle with
 * v = sqrt(kT/m) (xi + u), v_z = sqrt(kT/m) z, position uniform in the cell
 * from counters (0, c, e, RESEED_POS|k) and z from (1, c, e, RESEED_POS|k).
 * The cell's old particles are removed; all other cells keep their
 * particles in order.  Every call uses up one event index e.  Returns 0, or
 * -1 (a repeated or out-of-range cell id), -2 (capacity); in both error
 * cases the state is left unchanged. */
int or_lb2dsmc(or_sim *s, int32_t Q, int32_t order, const double *xi, const double *f, const int32_t *cells,
               int32_t nsel)
{
    int32_t nc = s->ncells;
    int32_t *mark = (int32_t *)xalloc((size_t)nc * 4);
    for (int32_t i = 0; i < nsel; ++i) {
        int32_t c = cells[i];
        if (c < 0 || c >= nc || mark[c]) {
            free(mark);
            s->status |= OR_ST_BAD_CELL;
            s->reseed_events += 1;
            return -1;
        }
        mark[c] = i + 1;
    }
    uint32_t e = (uint32_t)s->reseed_events;
    double *prm = (double *)xalloc((size_t)(nsel > 0 ? nsel : 1) * 12 * 8);
    int32_t *nnew = (int32_t *)xalloc((size_t)(nsel > 0 ? nsel : 1) * 4);
    int64_t total = 0;
    uint32_t st = 0;
#pragma omp parallel for schedule(static) reduction(+ : total) reduction(| : st)
    for (int32_t c = 0; c < nc; ++c) {
        if (!mark[c]) { total += s->cell_start[c + 1] - s->cell_start[c]; continue; }
        int32_t i = mark[c] - 1;
        double *pr = &prm[(size_t)i * 12];
        or_grad_params(&f[c], nc, Q, order, xi, pr);
        uint32_t r[4];
        draw(s->seed, 0u, (uint32_t)c, e, OR_TAG_RESEED_N, 0u, r);
        double target = pr[0] * (double)s->ppc + or_u53(r[0], r[1]);
        int32_t nn = 0;
        int finite = 1;
        for (int k = 0; k < 12; ++k) if (!isfinite(pr[k])) finite = 0;
        if (!finite) { st |= OR_ST_NONFINITE; nn = 0; }
        else if (target >= 16777215.0) { st |= OR_ST_NNEW_LIMIT; nn = 16777215; }
        else if (target >= 1.0) nn = (int32_t)floor(target);
        if (!(pr[0] > 0.0)) nn = 0;
        nnew[i] = nn;
        total += nn;
    }
    s->status |= st;
    if (total > s->capacity) {
        s->status |= OR_ST_CAPACITY;
        free(mark); free(prm); free(nnew);
        s->reseed_events += 1;
        return -2;
    }
    /* new cell starts first, then every cell's slots independently */
    int32_t *ncs = (int32_t *)xalloc((size_t)(nc + 1) * 4);
    int64_t d = 0;
    for (int32_t c = 0; c < nc; ++c) {
        ncs[c] = (int32_t)d;
        d += mark[c] ? nnew[mark[c] - 1] : s->cell_start[c + 1] - s->cell_start[c];
    }
    ncs[nc] = (int32_t)d;
    st = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : st)
    for (int32_t c = 0; c < nc; ++c) {
        int64_t d = ncs[c];
        if (!mark[c]) {
            for (int32_t p = s->cell_start[c]; p < s->cell_start[c + 1]; ++p, ++d) {
                s->tx[d] = s->x[p]; s->ty[d] = s->y[p];
                s->tvx[d] = s->vx[p]; s->tvy[d] = s->vy[p]; s->tvz[d] = s->vz[p];
            }
            continue;
        }
        int32_t i = mark[c] - 1;
        const double *pr = &prm[(size_t)i * 12];
        int32_t ix = c % s->nx, iy = c / s->nx;
        for (int32_t k = 0; k < nnew[i]; ++k, ++d) {
            double z[2], zz[2];
            ar_sample(s->seed, pr, (uint32_t)c, e, (uint32_t)k, s->ar_max_tries, z, &st);
            uint32_t a[4], b[4];
            draw(s->seed, 0u, (uint32_t)c, e, OR_TAG_RESEED_POS, (uint32_t)k, a);
            draw(s->seed, 1u, (uint32_t)c, e, OR_TAG_RESEED_POS, (uint32_t)k, b);
            or_box_muller(or_u53(b[0], b[1]), or_u53(b[2], b[3]), zz);
            s->tx[d] = stv(s, inside(ix, or_u53(a[0], a[1])));
            s->ty[d] = stv(s, inside(iy, or_u53(a[2], a[3])));
            s->tvx[d] = stv(s, s->s_th * (z[0] + pr[1]));
            s->tvy[d] = stv(s, s->s_th * (z[1] + pr[2]));
            s->tvz[d] = stv(s, s->s_th * zz[0]);
        }
    }
    s->status |= st;
    s->n = d;
    memcpy(s->cell_start, ncs, (size_t)(nc + 1) * 4);
    double *t;
    t = s->x; s->x = s->tx; s->tx = t;
    t = s->y; s->y = s->ty; s->ty = t;
    t = s->vx; s->vx = s->tvx; s->tvx = t;
    t = s->vy; s->vy = s->tvy; s->tvy = t;
    t = s->vz; s->vz = s->tvz; s->tvz = t;
    s->reseed_events += 1;
    free(mark); free(prm); free(nnew); free(ncs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* BGK lattice Boltzmann step (Section 3.1, relaxation time from Eq. (tau))  */
/* ------------------------------------------------------------------------ */
/* Populations f[a][node], node = iy*nx + ix, pre-collision.  Per node:
 * rho = sum f, u = (sum f xi + rho g / 2) / rho (forcing with the half-step
 * velocity shift), Hermite equilibrium to second order (Q = 9) or third
 * order (otherwise), BGK relaxation, second-order Hermite force term
 * (1 - 1/(2 tau)) w rho [xi.g + (xi.g)(xi.u) - g.u], then push along e_a.
 * x is periodic.  y_mode 0: y periodic.  y_mode 1: the K = max|e_y| rows at
 * each edge hold caller-set populations: they are neither collided nor
 * overwritten, and stream into the interior unchanged.  y_mode 2 (lattices
 * with |e_y| <= 1): diffuse walls half a node below row 0 and above row
 * ny-1; a population that would stream through a wall is taken up by it,
 * and the wall gives back to the same node the populations that point away
 * from it as the rest equilibrium w_a rho_w, with rho_w such that the node
 * gets back the mass it sent into the wall (full accommodation, wall at
 * rest).  x_buffer: the columns 0 .. x_buffer-1 hold caller-set populations
 * like buffer rows (not collided, not overwritten, streamed on into their
 * neighbours, across the periodic seam too); what streams into them is
 * dropped.  Result in f. */
void or_lbm_step(int32_t nx, int32_t ny, int32_t Q, const int32_t *ex, const int32_t *ey, const double *w,
                 const double *xi, double tau, double gx, int32_t y_mode, int32_t x_buffer, double *f, double *ftmp,
                 int32_t nsteps)
{
    int64_t nn = (int64_t)nx * ny;
    if (Q > 64) abort(); /* the per-row population buffer holds D2Q9 and D2Q37 */
    int32_t K = 0;
    for (int32_t a = 0; a < Q; ++a) if (abs(ey[a]) > K) K = abs(ey[a]);
    /* mass each node sends into the lower and the upper wall (y_mode 2) */
    double *wall_lo = (double *)xalloc((size_t)nn * 8);
    double *wall_hi = (double *)xalloc((size_t)nn * 8);
    for (int32_t st = 0; st < nsteps; ++st) {
        for (int64_t node = 0; node < nn; ++node) wall_lo[node] = wall_hi[node] = 0.0;
#pragma omp parallel for schedule(static)
        for (int32_t iy = 0; iy < ny; ++iy) {
            for (int32_t ix = 0; ix < nx; ++ix) {
                int64_t node = (int64_t)iy * nx + ix;
                int held = ((y_mode == 1) && (iy < K || iy >= ny - K)) || ix < x_buffer;
                if (held) {
                    for (int32_t a = 0; a < Q; ++a) ftmp[(size_t)a * nn + node] = f[(size_t)a * nn + node];
                }
            }
        }
        /* every (direction, destination) pair has one source node: the rows
         * are independent */
#pragma omp parallel for schedule(static)
        for (int32_t iy = 0; iy < ny; ++iy) {
            double fe[64];
            for (int32_t ix = 0; ix < nx; ++ix) {
                int64_t node = (int64_t)iy * nx + ix;
                int held = ((y_mode == 1) && (iy < K || iy >= ny - K)) || ix < x_buffer;
                if (held) {
                    for (int32_t a = 0; a < Q; ++a) fe[a] = f[(size_t)a * nn + node];
                } else {
                    double rho = 0.0, jx = 0.0, jy = 0.0;
                    for (int32_t a = 0; a < Q; ++a) {
                        double fa = f[(size_t)a * nn + node];
                        rho += fa;
                        jx += fa * xi[2 * a];
                        jy += fa * xi[2 * a + 1];
                    }
                    double ux = (jx + 0.5 * rho * gx) / rho;
                    double uy = jy / rho;
                    double uu = ux * ux + uy * uy;
                    for (int32_t a = 0; a < Q; ++a) {
                        double cu = xi[2 * a] * ux + xi[2 * a + 1] * uy;
                        double eq = 1.0 + cu + 0.5 * (cu * cu - uu);
                        if (Q != 9) eq += (cu * (cu * cu - 3.0 * uu)) / 6.0;
                        double feq = w[a] * rho * eq;
                        double cg = xi[2 * a] * gx;
                        double F = (1.0 - 0.5 / tau) * w[a] * rho * (cg + cg * cu - gx * ux);
                        double fa = f[(size_t)a * nn + node];
                        fe[a] = fa - (fa - feq) / tau + F;
                    }
                }
                for (int32_t a = 0; a < Q; ++a) {
                    int32_t jx2 = ix + ex[a];
                    int32_t jy2 = iy + ey[a];
                    jx2 = ((jx2 % nx) + nx) % nx;
                    if (y_mode == 1) {
                        if (jy2 < K || jy2 >= ny - K) continue;
                    } else if (y_mode == 2) {
                        if (jy2 < 0) { wall_lo[node] += fe[a]; continue; }
                        if (jy2 >= ny) { wall_hi[node] += fe[a]; continue; }
                    } else {
                        jy2 = ((jy2 % ny) + ny) % ny;
                    }
                    if (jx2 < x_buffer) continue;
                    ftmp[(size_t)a * nn + (int64_t)jy2 * nx + jx2] = fe[a];
                }
            }
        }
        if (y_mode == 2) {
            double wsum_up = 0.0, wsum_dn = 0.0;  /* weight of the directions pointing away from each wall */
            for (int32_t a = 0; a < Q; ++a) {
                if (ey[a] > 0) wsum_up += w[a];
                if (ey[a] < 0) wsum_dn += w[a];
            }
            for (int32_t ix = x_buffer; ix < nx; ++ix) {
                int64_t lo = ix, hi = (int64_t)(ny - 1) * nx + ix;
                double rlo = wall_lo[lo] / wsum_up, rhi = wall_hi[hi] / wsum_dn;
                for (int32_t a = 0; a < Q; ++a) {
                    if (ey[a] > 0) ftmp[(size_t)a * nn + lo] = w[a] * rlo;
                    if (ey[a] < 0) ftmp[(size_t)a * nn + hi] = w[a] * rhi;
                }
            }
        }
        memcpy(f, ftmp, (size_t)Q * nn * 8);
    }
    free(wall_lo);
    free(wall_hi);
}

/* The equilibrium mapping of Section 4, Eq. (feq_dsmc): from each cell's
 * averages only rho = <N>/ppc and u = <sum v>/<N> (in units of sqrt(kT/m))
 * enter, f_a = w_a rho [1 + xi.u + ((xi.u)^2 - u.u)/2], plus
 * xi.u ((xi.u)^2 - 3 u.u)/6 when order is 3 (a lattice that carries it).
 * Empty cells give zero populations.  avg: [11][ncells]; f: [Q][ncells]. */
void or_dsmc2lb_eq(const double *avg, int32_t ncells, int32_t ppc, double kT, int32_t Q, int32_t order,
                   const double *w, const double *xi, double *f)
{
    double s1 = sqrt(kT);
    for (int32_t c = 0; c < ncells; ++c) {
        double m0 = avg[c];
        if (!(m0 > 0.0)) {
            for (int32_t a = 0; a < Q; ++a) f[(size_t)a * ncells + c] = 0.0;
            continue;
        }
        double rho = m0 / (double)ppc;
        double ux = (avg[(size_t)ncells + c] / m0) / s1, uy = (avg[2 * (size_t)ncells + c] / m0) / s1;
        double uu = ux * ux + uy * uy;
        for (int32_t a = 0; a < Q; ++a) {
            double cu = xi[2 * a] * ux + xi[2 * a + 1] * uy;
            double eq = 1.0 + cu + 0.5 * (cu * cu - uu);
            if (order >= 3) eq += cu * (cu * cu - 3.0 * uu) / 6.0;
            f[(size_t)a * ncells + c] = w[a] * rho * eq;
        }
    }
}
