/*
 * dsmc.h -- C ABI of the MI355X (gfx950) DSMC particle step and DSMC<->LBM
 * mapping library (libdsmc.so).
 *
 * Method: Di Staso, Clercx, Succi & Toschi, "DSMC-LBM mapping scheme for
 * rarefied and non-rarefied gas flows", arXiv:1512.08042.
 *
 * Geometry and units (the nondimensionalisation of the paper's appendix
 * "Scaling factors"): a 2-D channel of nx x ny unit cells, periodic in x,
 * walls at y = 0 and y = H = ny with full diffuse reflection at the reference
 * temperature, body force along +x.  Particles carry three velocity
 * components (hard spheres in 3-D velocity space).  Speeds are in units in
 * which kT/m = kT_over_m (1 by default), so the Hermite variable is
 * xi = v / sqrt(kT/m).  Kn is on the channel height: lambda = Kn H, and the
 * hard-sphere relation of Eq. (MFP) fixes F_N sigma_T / V_c = 1/(sqrt(2) lambda ppc).
 *
 * Memory: every device buffer is allocated and owned by the caller and must
 * outlive the context; the library allocates no device memory after
 * dsmc_init (dsmc_init itself allocates none either) and owns only the small
 * host-side context.  All calls that take a stream enqueue asynchronous work
 * on it (NULL = the null stream) and return immediately unless stated.
 *
 * Errors: calls return DSMC_OK (0) or a negative DSMC_E* code; argument
 * errors are detected on the host before anything is enqueued.  Conditions
 * found on the device set bits of a status word read by dsmc_read_status.
 * No exception crosses the ABI and the library prints nothing.
 *
 * Determinism: the same configuration, seed and call sequence give
 * bitwise-identical results on the same build and GPU (the random numbers
 * are counter-based Philox4x32-10 keyed by (draw, entity, step, tag), and
 * no result depends on the order of atomic operations).
 */
#ifndef DSMC_H
#define DSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define DSMC_OK 0
#define DSMC_EINVAL (-1)   /* bad argument (reported before any work is enqueued) */
#define DSMC_ECAPACITY (-2) /* a size exceeds the configured capacity */
#define DSMC_EHIP (-3)     /* a HIP runtime call failed */
#define DSMC_ESTATE (-4)   /* call not valid in the context's current state */

/* device status bits (sticky until dsmc_read_status with clear = 1) */
#define DSMC_ST_WALL_LIMIT 0x1u   /* a particle hit the walls 16 times in one step and was stopped on the wall */
#define DSMC_ST_FAR_OVERFLOW 0x2u /* more long jumps (> 1 cell) in one step than far_capacity: the next step found
                                     them by scanning every cell's long-jump group instead of the list (slower;
                                     results are unchanged) */
#define DSMC_ST_CAPACITY 0x4u     /* a reseed would exceed capacity: it was skipped, state unchanged */
#define DSMC_ST_AR_LIMIT 0x8u     /* acceptance-rejection reached ar_max_tries: the last try was kept */
#define DSMC_ST_NONFINITE 0x10u   /* non-finite populations in a reseeded cell: it received no particles */
#define DSMC_ST_NNEW_LIMIT 0x20u  /* more than 2^24-1 new particles requested for one cell: clamped */
#define DSMC_ST_BAD_CELL 0x40u    /* reseed cell list had an out-of-range or repeated id: reseed skipped */
#define DSMC_ST_INTERNAL 0x80u    /* inconsistent sort tables inside a step (a library fault; never expected) */

#define DSMC_NMOM 11 /* sampled sums per cell, see dsmc_sample_moments */

/* Velocity ordering of lattice populations f[a] (shared by every call that
 * takes populations): shells of increasing |e|, counter-clockwise inside a
 * shell starting from the first-octant representative:
 *   a = 0: (0,0); 1-4: (1,0) (0,1) (-1,0) (0,-1); 5-8: (1,1) (-1,1) (-1,-1) (1,-1);
 *   D2Q37 continues 9-12: (2,0) (0,2) (-2,0) (0,-2);
 *   13-20: (2,1) (1,2) (-1,2) (-2,1) (-2,-1) (-1,-2) (1,-2) (2,-1);
 *   21-24: (2,2) (-2,2) (-2,-2) (2,-2); 25-28: (3,0) (0,3) (-3,0) (0,-3);
 *   29-36: (3,1) (1,3) (-1,3) (-3,1) (-3,-1) (-1,-3) (1,-3) (3,-1).
 * Hermite abscissae xi_a = r e_a with r = sqrt(3) (D2Q9) or the D2Q37 scale
 * obtained by solving the Gauss-Hermite conditions (Section 2.1: the lattice
 * must integrate the Hermite weight exactly to degree >= 2N; D2Q37 is exact
 * to degree 9).  Populations are laid out f[a * ncells + cell]. */

typedef struct dsmc_config {
    int32_t nx;            /* cells along the periodic direction x (>= 1) */
    int32_t ny;            /* cells across the channel, H = ny (>= 1) */
    int32_t ppc;           /* particles per cell at density 1 (>= 1) */
    int32_t nbar_mode;     /* NTC pair factor: 0 = N * running mean of N (Eq. (collisionnumber)), 1 = N (N - 1) */
    int64_t capacity;      /* particles each state buffer can hold (>= nx*ny*ppc for dsmc_init mode 0) */
    double kn;             /* Knudsen number on the channel height (> 0) */
    double dt;             /* time step (> 0) */
    double body_force_x;   /* acceleration along x */
    double kT_over_m;      /* kT/m of the gas and of the walls (> 0; 1 in the default units) */
    double sigcr_max0;     /* initial (sigma_T c_r)_max / sigma_T of every cell, a speed (> 0) */
    uint64_t seed;         /* Philox key */
    int32_t ar_max_tries;  /* acceptance-rejection try limit per particle (<= 0: 65536) */
    int32_t far_capacity;  /* long-jump list entries per step (<= 0: min(capacity, 65536)) */
    int32_t state_bits;    /* particle state precision: 64 (or 0) FP64; 32 FP32 storage with FP64
                              arithmetic (every write of a particle value rounds to the nearest float) */
    int32_t reserved;      /* 0 */
} dsmc_config;

typedef struct dsmc_sizes {
    int64_t ncells;          /* nx * ny */
    int64_t capacity;        /* particles per state array */
    size_t state_array_bytes; /* bytes of each of the 10 state arrays (capacity * 8, or * 4 for FP32 state) */
    size_t workspace_bytes;  /* bytes of the single workspace buffer */
} dsmc_sizes;

typedef struct dsmc_buffers {
    /* two structure-of-arrays particle buffers, [buffer][x, y, vx, vy, vz],
     * each array `capacity` elements of device memory (double, or float when
     * state_bits is 32); the library sorts from one into the other every step
     * (see dsmc_get_views for which is current) */
    void *state[2][5];
    void *workspace;        /* device memory, >= dsmc_sizes.workspace_bytes, 256-byte aligned */
    size_t workspace_bytes;
} dsmc_buffers;

typedef struct dsmc_views {
    int32_t current;          /* index (0/1) of the state buffer that holds the particles, sorted by cell */
    const int32_t *cell_start; /* device, ncells + 1: particles of cell c are slots [cell_start[c], cell_start[c+1]) */
    double *nbar;             /* device, ncells: running mean of N per cell (NTC) */
    double *sigcmax;          /* device, ncells: (sigma_T c_r)_max / sigma_T per cell */
    double *rem;              /* device, ncells: carried fractional candidate count per cell */
    const double *mom_sums;   /* device, [11][ncells]: sums over samples, see dsmc_sample_moments */
    int64_t nsamples;         /* samples in mom_sums */
    int64_t step;             /* DSMC steps taken since dsmc_init */
    int64_t reseed_events;    /* map_lbm_to_dsmc calls so far */
} dsmc_views;

typedef struct dsmc_status {
    uint32_t bits;           /* DSMC_ST_* */
    uint32_t moved;          /* 1: the state is moved for the coming step (see dsmc_step_moved) */
    int64_t n_particles;     /* current particle count */
    uint64_t ncoll;          /* accepted collisions since init */
    uint64_t ncand;          /* collision candidates since init */
    uint64_t nwall;          /* wall hits since init */
    uint64_t nfar;           /* long jumps since init */
} dsmc_status;

typedef struct dsmc_ctx dsmc_ctx;

/* Sizes of the caller-owned buffers for a configuration.  Host only,
 * synchronous.  Returns DSMC_EINVAL for an invalid configuration. */
int dsmc_query_sizes(const dsmc_config *cfg, dsmc_sizes *out);

/* Create a context over caller buffers and set the initial particle state.
 * mode 0: exactly ppc particles in every cell (Section 3.1), uniform in the
 *   cell, Maxwellian velocities at kT_over_m by Box-Muller (Table 1 step 4
 *   names the transformation); particle g = c*ppc + k of cell c.
 * mode 1: adopt n_load particles the caller wrote into state[0] (any order;
 *   positions in [0,nx) x [0,ny]): they are stably sorted by cell.
 * Per-cell NTC state starts at nbar = 0, sigcmax = sigcr_max0, rem = 0.
 * Errors: DSMC_EINVAL (config, buffers, mode), DSMC_ECAPACITY (too many
 * particles), DSMC_EHIP.  On success *out receives the context. */
int dsmc_init(const dsmc_config *cfg, const dsmc_buffers *buf, int32_t mode, int64_t n_load, void *stream,
              dsmc_ctx **out);

/* Advance nsteps DSMC steps.  One step: free flight under the body force
 * with diffuse wall reflection, cell indexing and a stable counting sort by
 * cell, No-Time-Counter hard-sphere collisions per cell
 * (Eq. (collisionnumber)), then, when (step + 1) % sample_every == 0 and
 * sample_every > 0, one sample of the per-cell velocity moments (the
 * cumulative averages that feed DSMC2LB, Section 2.1).  Errors: DSMC_EINVAL. */
int dsmc_step(dsmc_ctx *ctx, int32_t nsteps, int32_t sample_every, void *stream);

/* dsmc_step that leaves the state moved.  Steps are those of dsmc_step
 * (Eq. (collisionnumber) and the cycle of Section 2.1); internally every
 * step ends by moving its particles for the next step and partitioning
 * them by cell and direction, and a dsmc_step call's last step instead
 * writes them settled (sorted into their cells), so that the next call
 * begins with a pass that moves them again.  Here the last step moves as
 * the others do and the next call (either kind) begins without that pass.
 * Every later result is identical to a run of dsmc_step calls, also with
 * a map_lbm_to_dsmc between calls (see there); the wall hits of the coming
 * step's move are counted in this call or in the next one.  In a one-channel
 * context the last step leaves the tiles that hold a particle bound for a
 * wall unmoved (a reseed before the next step changes the cell starts that
 * key its wall draws); the next call (or graph replay) moves them first, in
 * a pass over those cells only.  While moved (dsmc_status.moved = 1) the
 * state buffers do not hold cell-sorted particles, dsmc_graph_launch of a
 * dsmc_graph_create graph returns DSMC_ESTATE, and a dsmc_step call with
 * nsteps >= 1 settles the state again.  Moments, both mappings and the
 * status are available as usual.  nsteps = 0 runs only the moving pass (none
 * on a moved state).  For loops that step, sample and map without reading
 * particles between calls.  Errors: DSMC_EINVAL. */
int dsmc_step_moved(dsmc_ctx *ctx, int32_t nsteps, int32_t sample_every, void *stream);

/* The cumulative averages of the DSMC moments that DSMC2LB projects
 * (Section 2.1: the coupling cells' averaged hydrodynamic variables, scaled
 * as in the appendix, give the coefficients of the truncated expansion).
 * Writes the time averages of the 11 sampled sums per cell to out (device,
 * [11][ncells] doubles; may be NULL to only reset): the mean over samples of
 * N, sum vx, sum vy, sum vx^2, sum vx vy, sum vy^2, sum vx^3, sum vx^2 vy,
 * sum vx vy^2, sum vy^3, sum vz^2 (raw velocities).  reset != 0 zeroes the
 * sums afterwards.  Errors: DSMC_ESTATE if no sample has been taken and out
 * is not NULL. */
int dsmc_sample_moments(dsmc_ctx *ctx, double *out, int32_t reset, void *stream);

/* DSMC2LB projection (Eq. (discretefunctions)) of every cell's cumulative
 * averages: a(0) = rho = <N>/ppc (the appendix's mass scale), a(1..3) the
 * absolute-frame Hermite coefficients of Eq. (nordercoefficients) from the
 * sampled moments, f_a = w_a sum_{n<=order} a(n):H(n)(xi_a)/n!.
 * lattice 9 or 37, order 0..3 (D2Q9 drops H_xxx and H_yyy, which vanish on
 * its nodes).  f_out: device, [Q][ncells].  Errors: DSMC_EINVAL,
 * DSMC_ESTATE (no samples). */
int map_dsmc_to_lbm(dsmc_ctx *ctx, int32_t lattice, int32_t order, double *f_out, void *stream);

/* The same projection from caller-given averages (device, [11][ncells]). */
int dsmc_project_moments(const double *avg, int64_t ncells, int32_t ppc, double kT_over_m, int32_t lattice,
                         int32_t order, double *f_out, void *stream);

/* LB2DSMC reconstruction (Section 2.2, Table 1) of the listed cells.
 * f_in: device, [Q][ncells] populations; cell_ids: device, nsel distinct ids.
 * Per listed cell: rho, u and the comoving, density-normalised a(2), a(3)
 * (Table 1 step 1), M and C = 1 + 30 M (steps 2-3), N_new = floor(rho ppc + R)
 * (mass conservation at the coupling site), then for each new particle
 * Box-Muller tries accepted when C R <= G(xi) (steps 4-5) and
 * v = sqrt(kT/m) (xi + u), v_z = sqrt(kT/m) z, position uniform in the cell.
 * The cell's previous particles are removed; every other cell keeps its
 * particles in order.  order 2 or 3.  A cell list with bad ids, or a result
 * above capacity, skips the whole reseed and sets a status bit.
 * The call writes only the new particles; the other cells' particles move to
 * their new slots in the next dsmc_step's first pass over the state (which
 * reads every particle anyway), or, if another call that reads the state
 * comes first (dsmc_get_views, dsmc_read_status, map_lbm_to_dsmc, the graph
 * calls), in a copy that call enqueues.  On a moved state (dsmc_step_moved)
 * the new particles are written after the state's last slot, and the next
 * step's pass over the listed cells and the unmoved tiles moves them; the
 * results equal those of the same reseed of the settled state, except that
 * the buffer must also hold the replaced particles until that step (a
 * reseed that does not fit is skipped with DSMC_ST_CAPACITY), and a second
 * reseed of the same moved state returns DSMC_ESTATE.  cell_ids is not read
 * after the call's work has run.  Errors: DSMC_EINVAL, DSMC_ESTATE. */
int map_lbm_to_dsmc(dsmc_ctx *ctx, int32_t lattice, int32_t order, const double *f_in, const int32_t *cell_ids,
                    int32_t nsel, void *stream);

typedef struct lbm_config {
    int32_t nx, ny;       /* nodes; x periodic */
    int32_t lattice;      /* 9 or 37 */
    int32_t y_mode;       /* 0: y periodic; 1: the max|e_y| rows at each y edge hold caller-set populations;
                             2 (D2Q9): diffuse walls half a node below row 0 and above row ny-1 (Section 4's
                             kinetic walls: what streams through a wall is taken up and given back to the same
                             node as the rest equilibrium w_a rho_w of the mass it took) */
    double tau;           /* BGK relaxation time in lattice steps (> 1/2), e.g. from Eq. (tau) */
    double body_force_x;  /* velocity gain along x per lattice step, in units of sqrt(kT/m) */
    int32_t x_buffer;     /* held inflow columns 0 .. x_buffer-1 (Section 4's buffer layer): like buffer rows
                             they keep caller-set populations, stream them on into their neighbours (across the
                             periodic seam too) and drop what streams into them; 0 <= x_buffer <= nx */
    int32_t reserved;     /* 0 */
} lbm_config;

/* nsteps BGK steps (Section 3.1) on populations f (device, [Q][nx*ny],
 * pre-collision), with f_tmp (same size) as scratch; the result is in f.
 * Per interior node: rho, u = (sum f xi + rho g/2)/rho, Hermite equilibrium
 * of order 2 (D2Q9) or 3 (D2Q37), BGK relaxation, second-order Hermite force
 * term (1 - 1/(2 tau)) w rho [xi.g + (xi.g)(xi.u) - g.u], streaming along
 * e_a.  Errors: DSMC_EINVAL. */
int lbm_step(const lbm_config *cfg, double *f, double *f_tmp, int32_t nsteps, void *stream);

/* lbm_step that also keeps checkpoints for the adjoint: before steps 0,
 * every, 2 every, ... the populations entering the step are written to
 * ckpt[k] (device, [ceil(nsteps/every)][Q][nx*ny]; ckpt may be NULL).  The
 * result is in f, as for lbm_step.  Errors: DSMC_EINVAL (also every < 1). */
int lbm_step_checkpointed(const lbm_config *cfg, double *f, double *f_tmp, double *ckpt, int32_t nsteps,
                          int32_t every, void *stream);

/* Bytes of device workspace that lbm_adjoint needs for segments of `every`
 * steps (per-block partial sums, one cotangent buffer, every - 1 recomputed
 * states); every = 0 gives the (small) size that lbm_adjoint_step needs.
 * Errors: DSMC_EINVAL. */
int lbm_adjoint_workspace(const lbm_config *cfg, int32_t every, size_t *bytes);

/* Reverse-mode derivative of one lbm_step step (Section 3.1; tau of
 * Eq. (tau)): with f_n the populations entering the step (device,
 * [Q][nx*ny]) and lam_next = dJ/df_{n+1} (same layout), writes
 * lam_out = (df_{n+1}/df_n)^T lam_next and adds this step's dJ/dg and dJ/dtau
 * to grad[0] and grad[1] (device, 2 doubles; g = body_force_x).  Buffer rows
 * (y_mode 1) pass cotangents through; populations streamed into them were
 * dropped and carry none.  The sums are in a fixed order (bitwise
 * reproducible).  lam_out must not alias lam_next or f_n.  work: device,
 * lbm_adjoint_workspace(cfg, 0) bytes, caller-owned.  Errors: DSMC_EINVAL. */
int lbm_adjoint_step(const lbm_config *cfg, const double *f_n, const double *lam_next, double *lam_out,
                     double *grad, void *work, void *stream);

/* lbm_adjoint_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same step and results, with the per-block partial sums
 * kept in a fixed array inside the library instead of a caller workspace.
 * The array (2 doubles per block of 256 nodes, 256 KB) exists once on every
 * GPU the library runs on, from the first call on that device until the
 * process ends; the call itself allocates nothing.  Calls that overlap on
 * one GPU (other streams, other threads) share the array and race: run them
 * one after another.  Errors: DSMC_EINVAL (as lbm_adjoint_step),
 * DSMC_ECAPACITY when nx * ny exceeds 4,194,304 nodes (16,384 blocks),
 * DSMC_EHIP. */
int lbm_adjoint_step_noalloc(const lbm_config *cfg, const double *f_n, const double *lam_next, double *lam_out,
                             double *grad, void *stream);

/* Reverse pass of nsteps lbm_step steps from the checkpoints that
 * lbm_step_checkpointed wrote with the same cfg and every: each segment's
 * states are recomputed into the workspace, then the adjoint steps run from
 * the last step back to the first.  lam: device [Q][nx*ny], on entry
 * dJ/df_N, on return dJ/df_0.  grad[0], grad[1] += dJ/dg, dJ/dtau over all
 * steps.  work: lbm_adjoint_workspace(cfg, every) bytes.  nsteps = 0 leaves
 * lam and grad unchanged.  Errors: DSMC_EINVAL. */
int lbm_adjoint(const lbm_config *cfg, const double *ckpt, int32_t nsteps, int32_t every, double *lam,
                double *grad, void *work, void *stream);

/* Hermite coefficients of populations (the expansion that
 * Eq. (discretefunctions) truncates): a_out[n][i] = sum_q f[q][nodes[i]]
 * H(n)(xi_q) for the (order+1)(order+2)/2 tensors up to `order` (0..3) in the
 * row order 1, x, y, xx, xy, yy, xxx, xxy, xyy, yyy.  f: device
 * [Q][nnodes]; nodes: device, nsel ids; a_out: device [nh][nsel].  An id
 * outside [0, nnodes) gets NaN coefficients.  Errors: DSMC_EINVAL. */
int lbm_hermite_moments(int32_t lattice, int32_t order, const double *f, int64_t nnodes, const int32_t *nodes,
                        int32_t nsel, double *a_out, void *stream);

/* Transpose of lbm_hermite_moments: f_bar[q][nodes[i]] += sum_n H(n)(xi_q)
 * a_bar[n][i].  The ids must be distinct (repeated ids race); ids outside
 * [0, nnodes) are skipped.  Errors: DSMC_EINVAL. */
int lbm_hermite_moments_adjoint(int32_t lattice, int32_t order, const double *a_bar, const int32_t *nodes,
                                int32_t nsel, double *f_bar, int64_t nnodes, void *stream);

/* Transpose of dsmc_project_moments (Eq. (discretefunctions) with the
 * coefficients of Eq. (nordercoefficients)), which is linear in the averages
 * of a cell with <N> > 0: avg_bar[k][c] = sum_q f_bar[q][c] df_q/davg_k.
 * avg (device [11][ncells]) is only read for <N> > 0; empty cells and row 10
 * (vz^2, unused by the projection) get zero.  f_bar: device [Q][ncells];
 * avg_bar: device [11][ncells], overwritten.  Errors: DSMC_EINVAL. */
int dsmc_project_moments_adjoint(const double *f_bar, const double *avg, int64_t ncells, int32_t ppc,
                                 double kT_over_m, int32_t lattice, int32_t order, double *avg_bar, void *stream);

/* The equilibrium mapping of Section 4, Eq. (feq_dsmc), from caller-given
 * averages (device, [11][ncells]): only rho = <N>/ppc and u = <sum v>/<N>
 * enter, f_a = w_a rho [1 + xi.u + ((xi.u)^2 - u.u)/2], plus the third-order
 * equilibrium term xi.u ((xi.u)^2 - 3 u.u)/6 when order is 3 (D2Q37 only).
 * Empty cells give zero populations.  f_out: device [Q][ncells].
 * Errors: DSMC_EINVAL. */
int dsmc_project_equilibrium(const double *avg, int64_t ncells, int32_t ppc, double kT_over_m, int32_t lattice,
                             int32_t order, double *f_out, void *stream);

/* One cycle of the hybrid coupling of Section 4: the context's channel is
 * the DSMC subdomain, f_lb (device, [Q][lbm.nx * lbm.ny], lbm.ny equal to
 * the channel's ny) the lattice subdomain, whose inflow columns
 * 0 .. lbm.x_buffer-1 form the buffer layer.  The cycle runs dsmc_steps DSMC
 * steps sampled every step; projects the averages over those steps of DSMC
 * column dsmc_column onto every buffer column (mapping 0: the equilibrium of
 * Eq. (feq_dsmc); 1: the full projection of Eq. (discretefunctions), with
 * the sampled non-equilibrium moments up to `order`); writes the cycle's
 * averages of every DSMC cell to avg_out (device [11][ncells], may be NULL);
 * resets the sums; and runs lbm_steps lattice steps (f_tmp: scratch of
 * f_lb's size).  flags DSMC_HYBRID_MOVED: the DSMC steps end with the state
 * moved, as dsmc_step_moved leaves it (for loops of cycles that read no
 * particles in between).  Errors: DSMC_EINVAL, DSMC_ESTATE (batch contexts). */
#define DSMC_HYBRID_MOVED 0x1
typedef struct dsmc_hybrid {
    lbm_config lbm;
    int32_t dsmc_steps;
    int32_t lbm_steps;
    int32_t mapping;
    int32_t order;
    int32_t dsmc_column;
    int32_t flags;            /* 0 or DSMC_HYBRID_MOVED */
} dsmc_hybrid;
int dsmc_hybrid_cycle(dsmc_ctx *ctx, const dsmc_hybrid *h, double *f_lb, double *f_tmp, double *avg_out,
                      void *stream);

/* Host copy of a lattice table: e_out int[Q][2], w_out double[Q], r_out. */
int dsmc_lattice(int32_t lattice, int32_t *e_out, double *w_out, double *r_out);

/* ---- batches of independent channels ------------------------------------
 * A batch context holds nrep independent channels (replicas) of a force-
 * driven Poiseuille flow (Section 3.1), each with its own size, particles per
 * cell, Knudsen number, time step, body force and Philox seed, stored one
 * after the other: replica r owns cells [cbase_r, cbase_r + nx_r ny_r) of
 * every per-cell array (cbase_r = sum of the cells of replicas < r, each
 * replica's cells in its own row-major order) and, after every call, the
 * particle slots [cell_start[cbase_r], cell_start[cbase_r + nx_r ny_r]).
 * One launch steps the cell tiles of all replicas together.  Every random
 * draw is keyed by cell and slot indices inside the replica, so replica r
 * evolves bit for bit as a one-channel context with its parameters would.
 * dsmc_step, dsmc_sample_moments (cells in the order above; rho = N/ppc_r is
 * the caller's), dsmc_read_status (totals over all replicas),
 * dsmc_get_views and the profiling calls take batch contexts;
 * map_dsmc_to_lbm and map_lbm_to_dsmc return DSMC_ESTATE for them. */
typedef struct dsmc_replica {
    int32_t nx, ny;        /* cells (>= 1 each) */
    int32_t ppc;           /* particles per cell at density 1 (>= 1) */
    int32_t reserved;      /* 0 */
    double kn;             /* Knudsen number on the replica's height ny (> 0) */
    double dt;             /* time step (> 0) */
    double body_force_x;   /* acceleration along x */
    uint64_t seed;         /* Philox key */
} dsmc_replica;

/* Sizes for a batch: common->capacity must hold every replica's
 * nx ny ppc particles; common's nx, ny, ppc, kn, dt, body_force_x and seed
 * are not used (each replica has its own).  Errors: DSMC_EINVAL. */
int dsmc_batch_query_sizes(const dsmc_config *common, const dsmc_replica *reps, int32_t nrep, dsmc_sizes *out);

/* A batch context, every replica started as dsmc_init mode 0 would start it
 * alone (a Maxwellian at kT/m with exactly ppc particles per cell).  reps is
 * host memory, copied.  Errors: DSMC_EINVAL, DSMC_ECAPACITY, DSMC_EHIP. */
int dsmc_batch_init(const dsmc_config *common, const dsmc_replica *reps, int32_t nrep, const dsmc_buffers *buf,
                    void *stream, dsmc_ctx **out);

/* Step tiling: every replica's cells are cut into tiles of TC consecutive
 * cells (one wavefront each) holding about particles_per_tile particles
 * (0: the default, 200 for FP64 and 400 for FP32 state); tiles of equal shape
 * share a launch.  Particles, cell starts and counters do not depend on the
 * tiling; the moment sums add the same terms in an order that follows the
 * tile shape (agreeing to rounding).  Synchronises the stream.
 * Errors: DSMC_EINVAL, DSMC_EHIP. */
int dsmc_set_tiling(dsmc_ctx *ctx, int32_t particles_per_tile, void *stream);

/* Tiling autotuner: runs steps_per_trial real steps (sampling every
 * sample_every, as dsmc_step) under each candidate particles_per_tile, timed
 * with HIP events, and keeps the fastest.  The trial steps advance the run
 * like any other steps; the trajectory does not depend on the tiling.  out
 * (host, may be NULL) receives the candidates, their times and the choice.
 * Errors: DSMC_EINVAL, DSMC_EHIP. */
typedef struct dsmc_tuning {
    int32_t ncand;                  /* candidates tried */
    int32_t chosen;                 /* index of the one kept */
    int32_t particles_per_tile[8];
    double ms_per_step[8];
} dsmc_tuning;
int dsmc_autotune(dsmc_ctx *ctx, int32_t steps_per_trial, int32_t sample_every, dsmc_tuning *out, void *stream);

/* Per-replica counters since init: out (host, [nrep][3]) = accepted
 * collisions, collision candidates, wall hits.  Synchronises the stream.
 * Errors: DSMC_EINVAL, DSMC_EHIP. */
int dsmc_replica_counters(dsmc_ctx *ctx, uint64_t *out, void *stream);

/* Step graphs: dsmc_graph_create captures one dsmc_step(ctx, nsteps,
 * sample_every) call (nsteps even, a multiple of sample_every when that is
 * > 0) into a HIP graph on `stream`, which must be a created stream (not
 * the null stream); nothing of the step runs and the context is unchanged
 * (a pending reseed is completed first).  Each dsmc_graph_launch replays it
 * on `stream` exactly as that dsmc_step call would run from the current
 * step: the step index comes from device memory, set by one small kernel
 * before the replay.  A replay needs the current step even, aligned with
 * sample_every, and the same current buffer as at capture, counting the
 * buffer switch of completing a pending reseed (DSMC_ESTATE otherwise,
 * before anything is enqueued).  Creating a graph replaces the previous
 * one; dsmc_destroy releases it, and so does a re-tiling (dsmc_set_tiling,
 * dsmc_autotune: the graph holds the old tile shapes), after which
 * dsmc_graph_launch returns DSMC_ESTATE until a graph is created again.  Kernel profiling does not time replays.
 * Batches run their tile groups on side streams forked from `stream`; the
 * fork and join are captured with them.
 * Errors: DSMC_EINVAL, DSMC_ESTATE, DSMC_EHIP. */
int dsmc_graph_create(dsmc_ctx *ctx, int32_t nsteps, int32_t sample_every, void *stream);
int dsmc_graph_launch(dsmc_ctx *ctx, void *stream);

/* The same for dsmc_step_moved calls: the graph replays nsteps steps of a
 * moved state and leaves it moved.  dsmc_graph_launch first runs the moving
 * pass, eagerly, on a settled state; a graph from dsmc_graph_create needs a
 * settled one.  Errors as dsmc_graph_create. */
int dsmc_graph_create_moved(dsmc_ctx *ctx, int32_t nsteps, int32_t sample_every, void *stream);

/* Synchronise the context's last stream and read the status word and
 * counters; clear != 0 resets the status bits.  Completes a pending reseed
 * first (see map_lbm_to_dsmc).  Errors: DSMC_EHIP. */
int dsmc_read_status(dsmc_ctx *ctx, dsmc_status *out, int32_t clear, void *stream);

/* Pointers into the caller's buffers describing the current state.  A
 * pending reseed (see map_lbm_to_dsmc) is completed first, on the stream of
 * the context's last call. */
int dsmc_get_views(dsmc_ctx *ctx, dsmc_views *out);

/* Kernel timing with HIP events on the launch stream.  dsmc_profile_enable
 * starts (enable = 1) or stops recording; dsmc_profile_read synchronises and
 * returns, for kernel id k (DSMC_K_*), the summed duration in ms and the
 * number of timed launches, then clears the records of that kernel. */
#define DSMC_K_CLASSIFY 0   /* moves of a settled state for the coming step (first step of a dsmc_step call) */
#define DSMC_K_CELL_COUNT 1 /* particles arriving per cell */
#define DSMC_K_SCAN 2       /* (not used by dsmc_step: its scan is part of DSMC_K_CELL_FINAL) */
#define DSMC_K_CELL_FINAL 3 /* new cell_start: block offsets and scan in one pass */
#define DSMC_K_STEP 4       /* gather + collide + sample + next move + partitioned write */
#define DSMC_K_PROJECT 5    /* DSMC2LB projection */
#define DSMC_K_RESEED 6     /* LB2DSMC reseed (all of its kernels) */
#define DSMC_K_COUNT 7
int dsmc_profile_enable(dsmc_ctx *ctx, int32_t enable);
int dsmc_profile_read(dsmc_ctx *ctx, int32_t kernel, double *ms_total, int64_t *launches);

void dsmc_destroy(dsmc_ctx *ctx);

/* Text of a return code (static storage). */
const char *dsmc_strerror(int code);

/* What the most recent failing call on ctx reported: the call's name, the
 * reason (the argument or state it rejected, or the HIP runtime's message)
 * and the code's text.  An empty string when no call on ctx has failed; a
 * successful call leaves it unchanged.  The text is owned by ctx and valid
 * until its next failing call or dsmc_destroy.  ctx = NULL gives a static
 * message.  Errors found on the device are status bits, not messages (see
 * dsmc_read_status). */
const char *dsmc_last_error(const dsmc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DSMC_H */
