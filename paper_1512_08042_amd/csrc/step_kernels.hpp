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

struct ClassifyArgs {
    double *st[5];        // current sorted state, moved in place
    const int32_t *cs;    // its cell_start
    uint8_t *code;        // direction code per particle
    int32_t *cnt;         // [9][ncells] group counts
    int32_t *farcnt;      // [ncells] long jumps arriving per cell
    int32_t *far;         // long-jump list of the step's parity
    Counters *ctr;
    Geometry G;
    MoveParams M;         // the coming step
    int ncells, far_cap, far_slot;
};

struct InvertArgs {
    const int32_t *cs;      // current cell_start
    const uint8_t *code;    // direction code per particle
    const int32_t *base;    // [9][ncells] first new slot of every group
    int32_t *from;          // source slot of every new slot
    Counters *ctr;
    int ncells;
};

struct StepArgs {
    const double *in[5];    // current sorted state
    double *out[5];         // the state after the step, sorted by the new cells
    const int32_t *cs_old;  // current cell_start
    const int32_t *cs_new;  // cell_start after the step
    const int32_t *from;    // source slot of every new slot
    uint8_t *code_out;      // direction codes of the new state for the next step
    int32_t *far_out;       // the next step's long jumps
    int32_t *cnt;           // [9][ncells] the next step's group counts
    int32_t *farcnt;        // [ncells] the next step's long jumps per arrival cell
    Counters *ctr;
    double *mom;            // [11][ncells] sums
    double *nbar, *sigcmax, *rem;
    Geometry G;
    MoveParams M1;          // the next step (its move is done here unless this is the call's last step)
    NtcParams N;            // this step's collisions
    int ncells, far_cap, far_slot, sample, classify;
};

struct CellArgs {
    int32_t *from;  // inverse map, filled here for long jumps
    const int32_t *cnt;
    int32_t *base;
    int32_t *farcnt;
    int32_t *far;
    int32_t *countnew;
    int32_t *blocksum;
    int32_t *cs_new;
    Counters *ctr;
    int nx, ny, ncells, far_cap, far_slot;
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

__global__ void k_classify(ClassifyArgs a);
__global__ void k_invert(InvertArgs a);
template <int TC>
__global__ void k_step(StepArgs a);
__global__ void k_cell_count(CellArgs a);
__global__ void k_scan_blocks(int32_t *blocksum, int nblk, int32_t *cs_out, int ncells, Counters *ctr,
                              int reset_slot);
__global__ void k_cell_final(CellArgs a);
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
