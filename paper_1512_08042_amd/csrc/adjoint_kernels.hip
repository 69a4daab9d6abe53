// Reverse-mode derivatives of the lattice path: the BGK collide-and-stream
// step (Section 3.1, relaxation time of Eq. (tau)), the Hermite coefficients
// of populations and the DSMC2LB projection (Eq. (discretefunctions) with the
// coefficients of Eq. (nordercoefficients)).  Hand-derived adjoints, one
// thread per node or cell, FP64 throughout.
#include "step_kernels.hpp"

namespace dsmc {

// H(n)(x, y) for n <= 3 in the ABI row order 1, x, y, xx, xy, yy, xxx, xxy,
// xyy, yyy (probabilists' Hermite tensors in units of sqrt(kT/m))
__device__ __forceinline__ void hermite10(double x, double y, double h[10])
{
    h[0] = 1.0;
    h[1] = x;
    h[2] = y;
    h[3] = x * x - 1.0;
    h[4] = x * y;
    h[5] = y * y - 1.0;
    h[6] = x * x * x - 3.0 * x;
    h[7] = x * x * y - y;
    h[8] = x * y * y - x;
    h[9] = y * y * y - 3.0 * y;
}

// Deterministic sum over a 256-thread block (fixed shuffle tree, then the
// four wave sums in order).  Every thread of the block must call it.
__device__ __forceinline__ double block_sum256(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

// ---- adjoint of one lattice step --------------------------------------------
// Forward: f'(x + e_q) = C_q(f(x)) for interior x whose target x + e_q is an
// interior row; buffer rows (y_mode 1) keep f and stream it on uncollided.
// With l*_q(x) = lam'(x + e_q) (zero when x + e_q is a buffer row):
//   buffer node:   lam_q(x) = lam'_q(x) + l*_q(x)
//   interior node: lam_p(x) = sum_q l*_q dC_q/df_p
// C_q = (1 - 1/tau) f_q + G_q(rho, u), G_q = w_q rho [E_q(u)/tau + c P_q(u)],
// c = 1 - 1/(2 tau), P_q = xi_qx g (1 + xi_q.u) - g u_x, E_q the Hermite
// equilibrium polynomial, rho = sum f, u_x = j_x/rho + g/2, u_y = j_y/rho.
// So lam_p = (1 - 1/tau) l*_p + A + Bx (xi_px - j_x/rho) + By (xi_py - u_y),
// A = sum_q l*_q w_q (E_q/tau + c P_q),
// Bx = sum_q l*_q w_q (dE_q/du_x / tau + c (xi_qx^2 g - g)),
// By = sum_q l*_q w_q (dE_q/du_y / tau + c xi_qx xi_qy g);
// dJ/dtau += sum_q l*_q [(f_q - f_eq,q)/tau^2 + w_q rho P_q / (2 tau^2)],
// dJ/dg += rho [c sum_q l*_q w_q (xi_qx (1 + xi_q.u) - u_x) + Bx / 2].
// Every q-sum above is a polynomial of degree <= 3 in xi_q, so the node first
// forms the moments M_a = sum_q w_q l*_q xi_q^a (|a| <= 3, ten of them, with
// the integer velocity components as compile-time coefficients) and then
// evaluates the sums from them.

template <int Q, int q>
__device__ __forceinline__ void adj_moments(double wl, double M[10])
{
    constexpr int x = VelSet<Q>::ex[q], y = VelSet<Q>::ey[q];
    M[0] += wl;
    cmad<x>(M[1], wl);
    cmad<y>(M[2], wl);
    cmad<x * x>(M[3], wl);
    cmad<x * y>(M[4], wl);
    cmad<y * y>(M[5], wl);
    cmad<x * x * x>(M[6], wl);
    cmad<x * x * y>(M[7], wl);
    cmad<x * y * y>(M[8], wl);
    cmad<y * y * y>(M[9], wl);
}

template <int Q, bool YB, bool NARROW>
__device__ __forceinline__ void lbm_adj_node(const LbmAdjArgs &a, int node, double &dg, double &dtau)
{
#pragma clang fp contract(fast)
    using V = VelSet<Q>;
    constexpr int R = V::R;
    const int nx = a.nx, ny = a.ny;
    const size_t nn = (size_t)nx * ny;
    const int ix = node % nx, iy = node / nx;
    const bool buffer = YB && (iy < a.K || iy >= ny - a.K);
    const double r = a.L.r;
    Nbr<R> nb;
    neighbours<R, YB ? 1 : 0, NARROW>(ix, iy, nx, ny, a.K, nb);
    // every address is in the grid (rows clamped), so all Q loads issue
    // together; what streams into a buffer row is then dropped
    double lp[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double v = *plane_ptr(a.lam_in, nn, q, (uint32_t)(nb.row[V::ey[q] + R] + nb.col[V::ex[q] + R]));
        lp[q] = (!YB || nb.in[V::ey[q] + R]) ? v : 0.0;
    }
    dg = 0.0;
    dtau = 0.0;
    if (buffer) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            *plane_ptr(a.lam_out, nn, q, (uint32_t)node) = *plane_ptr(a.lam_in, nn, q, (uint32_t)node) + lp[q];
        return;
    }
    const double *fp[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) fp[q] = plane_ptr(a.f, nn, q, (uint32_t)node);
    double rho = 0.0, ex = 0.0, ey = 0.0, lf = 0.0, M[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) M[k] = 0.0;
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double fq = *fp[q];
        rho += fq;
        cmad<V::ex[q]>(ex, fq);
        cmad<V::ey[q]>(ey, fq);
        lf += lp[q] * fq;
        adj_moments<Q, q>(a.L.ws[V::sh[q]] * lp[q], M);
    });
    const double r2 = r * r, r3 = r2 * r;
    M[1] *= r, M[2] *= r;
    M[3] *= r2, M[4] *= r2, M[5] *= r2;
    M[6] *= r3, M[7] *= r3, M[8] *= r3, M[9] *= r3;
    const double g = a.gx;
    const double itau = 1.0 / a.tau, c = 1.0 - 0.5 * itau;
    const double irho = 1.0 / rho;
    const double jx = r * ex, jy = r * ey;
    const double ux = (jx + 0.5 * rho * g) * irho;
    const double uy = jy * irho;
    const double wx = jx * irho;
    const double uu = ux * ux + uy * uy;
    // sums over q of w l* times: xi.u, xi_x xi.u, xi_y xi.u, (xi.u)^2
    const double C1 = ux * M[1] + uy * M[2];
    const double Dx = ux * M[3] + uy * M[4];
    const double Dy = ux * M[4] + uy * M[5];
    const double C2 = ux * Dx + uy * Dy;
    const double Lg = M[1] + Dx - ux * M[0];
    double Leq = M[0] + C1 + 0.5 * (C2 - uu * M[0]);
    double SEx = Lg;
    double SEy = M[2] + Dy - uy * M[0];
    if (Q != 9) {
        // ... and xi_x (xi.u)^2, xi_y (xi.u)^2, (xi.u)^3
        const double Ex2 = ux * ux * M[6] + 2.0 * ux * uy * M[7] + uy * uy * M[8];
        const double Ey2 = ux * ux * M[7] + 2.0 * ux * uy * M[8] + uy * uy * M[9];
        const double C3 = ux * Ex2 + uy * Ey2;
        Leq += (C3 - 3.0 * uu * C1) * (1.0 / 6.0);
        SEx += 0.5 * (Ex2 - uu * M[1]) - ux * C1;
        SEy += 0.5 * (Ey2 - uu * M[2]) - uy * C1;
    }
    const double Lp = g * Lg;
    const double A = Leq * itau + c * Lp;
    const double Bx = SEx * itau + c * g * (M[3] - M[0]);
    const double By = SEy * itau + c * g * M[4];
    const double k1 = 1.0 - itau;
    const double A0 = A - Bx * wx - By * uy, Bxr = Bx * r, Byr = By * r;
    static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        double v = k1 * lp[q] + A0;
        cmad<V::ex[q]>(v, Bxr);
        cmad<V::ey[q]>(v, Byr);
        *plane_ptr(a.lam_out, nn, q, (uint32_t)node) = v;
    });
    dtau = ((lf - rho * Leq) + 0.5 * rho * Lp) * itau * itau;
    dg = rho * (c * Lg + 0.5 * Bx);
}

// One block of 256 nodes; the block's (dJ/dg, dJ/dtau) go to partial[2 b]
// (added when a.accumulate, else written): one writer per slot, so the sums
// do not depend on scheduling.
template <int Q, bool YB, bool NARROW>
__global__ __launch_bounds__(256, 4) void k_lbm_adjoint(LbmAdjArgs a)
{
    __shared__ double sh[4];
    const int node = blockIdx.x * 256 + threadIdx.x;
    double dg = 0.0, dtau = 0.0;
    if (node < a.nx * a.ny) lbm_adj_node<Q, YB, NARROW>(a, node, dg, dtau);
    const double sg = block_sum256(dg, sh);
    const double st = block_sum256(dtau, sh);
    if (threadIdx.x == 0) {
        double *p = a.partial + 2 * (size_t)blockIdx.x;
        p[0] = a.accumulate ? p[0] + sg : sg;
        p[1] = a.accumulate ? p[1] + st : st;
    }
}

#define DSMC_ADJ_INSTANCES(Q)                                                  \
    template __global__ void k_lbm_adjoint<Q, false, false>(LbmAdjArgs);       \
    template __global__ void k_lbm_adjoint<Q, false, true>(LbmAdjArgs);        \
    template __global__ void k_lbm_adjoint<Q, true, false>(LbmAdjArgs);        \
    template __global__ void k_lbm_adjoint<Q, true, true>(LbmAdjArgs);
DSMC_ADJ_INSTANCES(9)
DSMC_ADJ_INSTANCES(37)
#undef DSMC_ADJ_INSTANCES

// grad[0..1] += sum over the blocks' partials, in a fixed order
__global__ __launch_bounds__(256) void k_adjoint_finish(const double *partial, int nblk, double *grad)
{
    __shared__ double sh[4];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        s0 += partial[2 * (size_t)b];
        s1 += partial[2 * (size_t)b + 1];
    }
    s0 = block_sum256(s0, sh);
    s1 = block_sum256(s1, sh);
    if (threadIdx.x == 0) {
        grad[0] += s0;
        grad[1] += s1;
    }
}

// ---- Hermite coefficients of populations and their adjoint --------------------
// a[n][i] = sum_q f[q][nodes[i]] H(n)(xi_q), n < nh.  An id outside the grid
// gets NaN coefficients.
__global__ __launch_bounds__(256) void k_hermite_moments(HermiteArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.nsel) return;
    const int64_t node = a.nodes[i];
    double acc[10];
#pragma unroll
    for (int n = 0; n < 10; ++n) acc[n] = 0.0;
    if (node < 0 || node >= a.nnodes) {
        for (int n = 0; n < a.nh; ++n) a.a[(size_t)n * a.nsel + i] = __builtin_nan("");
        return;
    }
    for (int q = 0; q < a.L.Q; ++q) {
        const double fq = a.f[(size_t)q * a.nnodes + node];
        double h[10];
        hermite10(a.L.xi[q][0], a.L.xi[q][1], h);
#pragma unroll
        for (int n = 0; n < 10; ++n) acc[n] += fq * h[n];
    }
    for (int n = 0; n < a.nh; ++n) a.a[(size_t)n * a.nsel + i] = acc[n];
}

// f_bar[q][nodes[i]] += sum_n H(n)(xi_q) a_bar[n][i]; ids outside the grid are
// skipped.
__global__ __launch_bounds__(256) void k_hermite_moments_adjoint(HermiteArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.nsel) return;
    const int64_t node = a.nodes[i];
    if (node < 0 || node >= a.nnodes) return;
    double ab[10];
#pragma unroll
    for (int n = 0; n < 10; ++n) ab[n] = n < a.nh ? a.a_bar[(size_t)n * a.nsel + i] : 0.0;
    for (int q = 0; q < a.L.Q; ++q) {
        double h[10];
        hermite10(a.L.xi[q][0], a.L.xi[q][1], h);
        double s = 0.0;
#pragma unroll
        for (int n = 0; n < 10; ++n) s += h[n] * ab[n];
        a.f_bar[(size_t)q * a.nnodes + node] += s;
    }
}

// ---- adjoint of the DSMC2LB projection ---------------------------------------
// For a cell with <N> > 0 the projection is linear in the averages m:
//   rho = m0/ppc, a_x = m1/(ppc s), a_y = m2/(ppc s),
//   a_xx = m3/(ppc s^2) - m0/ppc, a_xy = m4/(ppc s^2), a_yy = m5/(ppc s^2) - m0/ppc,
//   a_xxx = m6/(ppc s^3) - 3 m1/(ppc s), a_xxy = m7/(ppc s^3) - m2/(ppc s),
//   a_xyy = m8/(ppc s^3) - m1/(ppc s), a_yyy = m9/(ppc s^3) - 3 m2/(ppc s),
// and f_q = w_q [rho + a1.xi + a2:H2/2 + a3:H3/6].  The transpose first forms
// the coefficient cotangents sum_q f_bar_q w_q dF_q/da, then maps them back
// to m.  Empty cells (and the unused m10 = <sum vz^2>) get zero.
__global__ __launch_bounds__(256) void k_project_adjoint(ProjectAdjArgs a)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= a.ncells) return;
    const size_t nc = (size_t)a.ncells;
    double mb[NMOM];
#pragma unroll
    for (int k = 0; k < NMOM; ++k) mb[k] = 0.0;
    if (a.avg[c] > 0.0) {
        const int order = a.order, Q = a.L.Q;
        double r = 0.0, b1x = 0.0, b1y = 0.0, b2xx = 0.0, b2xy = 0.0, b2yy = 0.0;
        double b3xxx = 0.0, b3xxy = 0.0, b3xyy = 0.0, b3yyy = 0.0;
        for (int q = 0; q < Q; ++q) {
            const double x = a.L.xi[q][0], y = a.L.xi[q][1];
            const double wf = a.L.w[q] * a.f_bar[(size_t)q * nc + c];
            r += wf;
            if (order >= 1) {
                b1x += wf * x;
                b1y += wf * y;
            }
            if (order >= 2) {
                b2xx += wf * 0.5 * (x * x - 1.0);
                b2xy += wf * (x * y);
                b2yy += wf * 0.5 * (y * y - 1.0);
            }
            if (order >= 3) {
                b3xxy += wf * 0.5 * (x * x * y - y);
                b3xyy += wf * 0.5 * (x * y * y - x);
                if (Q != 9) {
                    b3xxx += wf * (x * x * x - 3.0 * x) / 6.0;
                    b3yyy += wf * (y * y * y - 3.0 * y) / 6.0;
                }
            }
        }
        const double p = (double)a.ppc, s1 = a.s1, s2 = s1 * s1, s3 = s2 * s1;
        mb[0] = (r - b2xx - b2yy) / p;
        mb[1] = (b1x - 3.0 * b3xxx - b3xyy) / (p * s1);
        mb[2] = (b1y - b3xxy - 3.0 * b3yyy) / (p * s1);
        mb[3] = b2xx / (p * s2);
        mb[4] = b2xy / (p * s2);
        mb[5] = b2yy / (p * s2);
        mb[6] = b3xxx / (p * s3);
        mb[7] = b3xxy / (p * s3);
        mb[8] = b3xyy / (p * s3);
        mb[9] = b3yyy / (p * s3);
    }
#pragma unroll
    for (int k = 0; k < NMOM; ++k) a.avg_bar[(size_t)k * nc + c] = mb[k];
}

}  // namespace dsmc
