// Kernel argument blocks and declarations shared by the kernel sources and
// the host side of libdsmc (passed by value; all pointers are device memory).
#pragma once

#include "dsmc_device.hpp"

namespace dsmc {

// NTC constants of one step's collisions
struct NtcParams {
    double K, dt;       // F_N sigma_T / V_c and the time step
    uint32_t k0, k1;    // Philox key
    uint32_t step;      // index of the step whose collisions these are
    int nbar_mode;
};

// Per-cell partition of a moved state: inside every old cell's slot range
// the particles are grouped by direction code 0..9 (the 9 near moves, then
// long jumps), each group in slot order; grp[c][d] holds the group sizes.
constexpr int NGRP = NDIR + 1;

struct StepArgs {
    const double *in[5];     // state of the step: moved and partitioned (k_step), or settled (k_classify)
    double *out[5];          // the state written (k_classify: the same arrays as in)
    const int32_t *cs_old;   // cell_start of in
    const int32_t *cs_new;   // cell_start after the step's sort (k_classify: cs_old)
    const int32_t *grp_in;   // [ncells][NGRP] group sizes of in
    int32_t *grp_out;        // [ncells][NGRP] group sizes of the next step's partition
    const int32_t *far_in;   // the step's long jumps (slot, old cell, new cell, -)
    int32_t *farcnt_in;      // [ncells] long jumps arriving per cell (read and cleared)
    int32_t *far_out;        // the next step's long jumps
    int32_t *farcnt_out;     // [ncells] the next step's long jumps per arrival cell
    double *scr;             // [capacity] scratch of oversized tiles
    int32_t *scr_i;          // [capacity] scratch of oversized tiles
    Counters *ctr;
    unsigned long long *tstat;  // [tiles][3] running collisions, candidates and wall hits of every tile
    double *mom;             // [11][ncells] sums
    double *nbar, *sigcmax, *rem;
    Geometry G;
    MoveParams M1;           // the move done here: the next step's (k_step), the coming step's (k_classify)
    NtcParams N;             // this step's collisions
    int ncells, far_cap, far_in_slot, far_out_slot, sample;
};

struct CellArgs {
    const int32_t *grp;      // [ncells][NGRP] group sizes of the moved state
    const int32_t *farcnt;   // [ncells] long jumps arriving per cell
    int32_t *countnew;
    int32_t *blocksum;
    int nx, ny, ncells;
};

struct InitArgs {
    double *st[5];
    int32_t *cs;
    double *nbar, *sigcmax, *rem;
    int nx, ncells, ppc;
    double s_th, sigcr0;
    uint32_t k0, k1;
};

struct AdoptArgs {
    const double *in[5];
    double *out[5];
    int32_t *cellid, *counts, *cursor, *perm;
    const int32_t *cs;
    Geometry G;
    int64_t n;
};

struct ProjectArgs {
    const double *mom;  // sums [11][ncells]
    double S;           // number of samples the sums hold (1 for averages)
    double *f;          // [Q][ncells]
    Lattice L;
    int ncells, ppc, order;
    double s1;          // sqrt(kT/m)
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
    const double *in[5];
    double *out[5];
    Counters *ctr;
    Lattice L;
    int nx, ncells, ppc, order, ar_max_tries;
    int64_t capacity;
    double s_th;
    uint32_t k0, k1, event;
};

struct LbmArgs {
    const double *f;
    double *ft;
    Lattice L;
    int ex[37], ey[37];
    int nx, ny, y_mode, K;
    double tau, gx;
};

// TC cells per tile (one wave); tiles of up to 64*CH particles are staged in LDS
template <int TC, int CH>
__global__ void k_classify(StepArgs a);
template <int TC, int CH, bool MOVE>
__global__ void k_step(StepArgs a);
__global__ void k_cell_count(CellArgs a);
__global__ void k_scan_blocks(int32_t *blocksum, int nblk, int32_t *cs_out, int ncells, Counters *ctr,
                              int reset_slot);
__global__ void k_average(const double *mom, double *out, size_t n, double S);
__global__ void k_init_maxwell(InitArgs a);
__global__ void k_adopt_count(AdoptArgs a);
__global__ void k_block_sums(const int32_t *counts, int ncells, int32_t *blocksum);
__global__ void k_block_scan(const int32_t *counts, int ncells, const int32_t *blockoff, int32_t *cs);
__global__ void k_adopt_place(AdoptArgs a);
__global__ void k_adopt_sortcell(AdoptArgs a);
__global__ void k_adopt_gather(AdoptArgs a);
__global__ void k_fill_f64(double *p, size_t n, double v);
__global__ void k_fill_i32(int32_t *p, size_t n, int32_t v);
__global__ void k_zero_counters(Counters *c);
__global__ void k_clear_status(Counters *c);
__global__ void k_tile_stats(const unsigned long long *tstat, int ntiles, Counters *c);
__global__ void k_far_reset(Counters *c, int slot);

__global__ void k_project(ProjectArgs a);
__global__ void k_reseed_prep(ReseedArgs a);
__global__ void k_reseed_count(ReseedArgs a);
__global__ void k_reseed_check(ReseedArgs a);
__global__ void k_reseed_copy(ReseedArgs a);
__global__ void k_reseed_gen(ReseedArgs a);
__global__ void k_reseed_unmark(ReseedArgs a);
__global__ void k_lbm(LbmArgs a);

}  // namespace dsmc
