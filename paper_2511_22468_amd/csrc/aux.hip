// Kernels around the integrator: the MMD loss and its gradient (Sec. 2.2.1 and
// Fig. 2, step 4), energies, the test-particle orbit of the progenitor's centre of
// mass and its adjoint (Fig. 2, step 2), and the Plummer-sphere placement with its
// adjoint (Fig. 2, step 3), and the debug scan of a state for non-finite values.
// All FP64.
#include <algorithm>

#include "dnb_internal.h"

namespace dnb {

// ---------------------------------------------------------------------- MMD --
// 2^x for x <= 0 (the Gaussian kernel is exp(-s / (2 h^2)) = 2^(-s c) with
// c = log2(e) / (2 h^2)).  x = n + f with n = rint(x) and |f| <= 1/2; 2^f =
// e^(f ln 2) is summed from its Taylor series to degree 13, whose first omitted
// term, (ln 2 / 2)^14 / 14!, is below 5e-18; ldexp then scales by 2^n, with
// gradual underflow to exactly 0.  n is clamped at -2000 before its conversion
// to int (2^-2000 p is 0 in FP64), which keeps the conversion defined for any
// finite x.  Maximum error 0.57 ulp against a long-double 2^x over [-1080, 0].
// A NaN argument gives NaN through p; so does -inf, which would need |p - q|
// beyond 1e154.
struct Exp2Taylor { double c[14]; };
constexpr Exp2Taylor exp2_taylor() {
    constexpr double LN2 = 0.69314718055994530942;
    Exp2Taylor t{};
    double term = 1.0;
    for (int k = 0; k < 14; ++k) { t.c[k] = term; term = term * LN2 / (k + 1); }
    return t;
}

__device__ __forceinline__ double exp2_nonpos(double x) {
    constexpr Exp2Taylor T = exp2_taylor();
    const double n = rint(x);
    const double f = x - n;
    double p = T.c[13];
#pragma unroll
    for (int k = 12; k >= 0; --k) p = fma(p, f, T.c[k]);
    return ldexp(p, (int)fmax(n, -2000.0));
}

// For targets p_i and sources q_j of one slice:
//   part[s][0][i] = sum_j k(p_i, q_j),  part[s][1..3][i] = sum_j k(p_i, q_j) (p_i - q_j)
// with k(p, q) = exp(-|p - q|^2 / (2 h^2)); slice s starts at part + s * sstride
// (4 npad with the gradient terms, npad without).  blockIdx.z selects a member of
// an ensemble: P, Q and part advance by the given member strides (0 for one system).
// neg_c = -log2(e) / (2 h^2).  Without GRAD only the kernel sums are formed.
template <bool GRAD>
__global__ __launch_bounds__(BS) void k_mmd_rows(const double* __restrict__ P, int np,
                                                 const double* __restrict__ Q, int nq,
                                                 double neg_c, int jslice,
                                                 double* __restrict__ part, int64_t npad,
                                                 int64_t sstride, int64_t p_bstride,
                                                 int64_t q_bstride, int64_t part_bstride) {
    __shared__ double4 tile[TILE];
    P += blockIdx.z * p_bstride;
    Q += blockIdx.z * q_bstride;
    part += blockIdx.z * part_bstride;
    const int i = blockIdx.x * BS + threadIdx.x;
    const int j0 = blockIdx.y * jslice;
    const int j1 = min(nq, j0 + jslice);
    const int ii = min(i, np - 1);
    const double px = P[ii], py = P[np + ii], pz = P[2 * np + ii];
    double s0 = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int jt = j0; jt < j1; jt += TILE) {
        const int j = jt + threadIdx.x;
        tile[threadIdx.x] = (j < j1) ? make_double4(Q[j], Q[nq + j], Q[2 * nq + j], 1.0)
                                     : make_double4(0.0, 0.0, 0.0, 0.0);
        __syncthreads();
        const int cnt = min(TILE, j1 - jt);
        for (int k = 0; k < cnt; ++k) {
            const double4 q = tile[k];
            const double dx = px - q.x, dy = py - q.y, dz = pz - q.z;
            const double e = exp2_nonpos(fma(dx, dx, fma(dy, dy, dz * dz)) * neg_c);
            s0 += e;
            if (GRAD) {
                gx = fma(e, dx, gx);
                gy = fma(e, dy, gy);
                gz = fma(e, dz, gz);
            }
        }
        __syncthreads();
    }
    if (i < np) {
        double* p = part + (int64_t)blockIdx.y * sstride + i;
        p[0] = s0;
        if (GRAD) { p[npad] = gx; p[2 * npad] = gy; p[3 * npad] = gz; }
    }
}

// Launch of k_mmd_rows with the kernel width h given as inv2h2 = 1 / (2 h^2).
static void mmd_rows(dim3 grid, hipStream_t st, const double* P, int np, const double* Q, int nq,
                     double inv2h2, int jslice, int with_grad, double* part, int64_t npad,
                     int64_t sstride, int64_t p_bstride, int64_t q_bstride,
                     int64_t part_bstride) {
    const double neg_c = -1.44269504088896340736 * inv2h2;
    if (with_grad)
        hipLaunchKernelGGL(k_mmd_rows<true>, grid, dim3(BS), 0, st, P, np, Q, nq, neg_c, jslice,
                           part, npad, sstride, p_bstride, q_bstride, part_bstride);
    else
        hipLaunchKernelGGL(k_mmd_rows<false>, grid, dim3(BS), 0, st, P, np, Q, nq, neg_c, jslice,
                           part, npad, sstride, p_bstride, q_bstride, part_bstride);
}

// Per-target slice sums -> gradient rows and per-block sums of the kernel sums.
// red[b][0] = sum over the block of sum_j k(x_i, x_j); red[b][1] = of sum_a k(x_i, y_a).
__global__ __launch_bounds__(BS) void k_mmd_x(const double* __restrict__ pxx, int Sxx,
                                              const double* __restrict__ pxy, int Sxy,
                                              int64_t npad, int n, int m, double h,
                                              double* __restrict__ gpos, double* __restrict__ red) {
    __shared__ double sh[2 * BS];
    const int i = blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    double v[2] = {0.0, 0.0};
    if (ok) {
        double sx = 0.0, sy = 0.0, gx[3] = {0, 0, 0}, gy[3] = {0, 0, 0};
        for (int s = 0; s < Sxx; ++s) {
            const double* q = pxx + (int64_t)s * 4 * npad + i;
            sx += q[0];
            for (int c = 0; c < 3; ++c) gx[c] += q[(1 + c) * npad];
        }
        for (int s = 0; s < Sxy; ++s) {
            const double* q = pxy + (int64_t)s * 4 * npad + i;
            sy += q[0];
            for (int c = 0; c < 3; ++c) gy[c] += q[(1 + c) * npad];
        }
        v[0] = sx; v[1] = sy;
        if (gpos) {
            const double cxx = -2.0 / ((double)n * n * h * h);
            const double cxy = 2.0 / ((double)n * m * h * h);
            for (int c = 0; c < 3; ++c) gpos[(int64_t)c * n + i] = cxx * gx[c] + cxy * gy[c];
        }
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) { red[8 * blockIdx.x + 0] = v[0]; red[8 * blockIdx.x + 1] = v[1]; }
}

__global__ __launch_bounds__(BS) void k_mmd_y(const double* __restrict__ pyy, int Syy,
                                              int64_t npad, int m, double* __restrict__ red) {
    __shared__ double sh[BS];
    const int a = blockIdx.x * BS + threadIdx.x;
    double v[1] = {0.0};
    if (a < m)
        for (int s = 0; s < Syy; ++s) v[0] += pyy[(int64_t)s * 4 * npad + a];
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) red[8 * blockIdx.x + 2] = v[0];
}

__global__ __launch_bounds__(BS) void k_mmd_final(const double* __restrict__ red, int nbx, int nby,
                                                  int n, int m, double* __restrict__ loss) {
    __shared__ double sh[3 * BS];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nbx; b += BS) { v[0] += red[8 * b]; v[1] += red[8 * b + 1]; }
    for (int b = threadIdx.x; b < nby; b += BS) v[2] += red[8 * b + 2];
    block_sum<3>(v, sh);
    if (threadIdx.x == 0)
        loss[0] = v[0] / ((double)n * n) + v[2] / ((double)m * m) - 2.0 * v[1] / ((double)n * m);
}

hipError_t launch_mmd(dnb_ctx* c, int64_t n, const double* pos, int64_t m, const double* tgt,
                      double h, double* loss, double* gpos, hipStream_t st) {
    const double inv2h2 = 1.0 / (2.0 * h * h);
    const int wg = gpos != nullptr;
    double* pv = (double*)c->partv;   // [S][8][npad] doubles available
    Slicing sx = plain_slicing(c, n);    // targets x, sources x
    Slicing sxy = plain_slicing(c, n);    // targets x, sources y: slice length from m
    {
        int64_t want = sxy.S;
        sxy.jslice = (int)(cdiv(cdiv(m, want), TILE) * TILE);
        sxy.S = (int)cdiv(m, sxy.jslice);
    }
    Slicing sy = plain_slicing(c, m);
    double* pxx = pv;
    double* pxy = pv + (int64_t)4 * sx.S * sx.npad;
    double* pyy = (double*)c->part;
    mmd_rows(dim3(sx.nblk, sx.S), st, pos, (int)n, pos, (int)n,
                       inv2h2, sx.jslice, wg, pxx, sx.npad, 4 * sx.npad, 0, 0, 0);
    mmd_rows(dim3(sxy.nblk, sxy.S), st, pos, (int)n, tgt,
                       (int)m, inv2h2, sxy.jslice, wg, pxy, sxy.npad, 4 * sxy.npad, 0, 0, 0);
    mmd_rows(dim3(sy.nblk, sy.S), st, tgt, (int)m, tgt, (int)m,
                       inv2h2, sy.jslice, 0, pyy, sy.npad, 4 * sy.npad, 0, 0, 0);
    hipLaunchKernelGGL(k_mmd_x, dim3(sx.nblk), dim3(BS), 0, st, pxx, sx.S, pxy, sxy.S, sx.npad,
                       (int)n, (int)m, h, gpos, c->red);
    hipLaunchKernelGGL(k_mmd_y, dim3(sy.nblk), dim3(BS), 0, st, pyy, sy.S, sy.npad, (int)m,
                       c->red);
    hipLaunchKernelGGL(k_mmd_final, dim3(1), dim3(BS), 0, st, c->red, sx.nblk, sy.nblk, (int)n,
                       (int)m, loss);
    return hipGetLastError();
}

// Loss of every member of an ensemble.  pxx, pxy: [batch][S][rows][npad] kernel
// sums per target (rows = 1, or 4 with the gradient terms; sstride = rows npad).
// The target term sum_ab k(y_a, y_b) comes, for one shared target, from the
// block sums red[8 q + 2] of k_mmd_y (pyy NULL), or, for a target per member,
// from pyy [batch][Syy][npad_y] (the slice sums of each member's target; with
// pyy_bstride = 0 one target's sums serve every member).  loss[b * lstride].
// One block per member.
__global__ __launch_bounds__(BS) void k_mmd_batch_final(const double* __restrict__ pxx, int S,
                                                        const double* __restrict__ pxy, int Sxy,
                                                        int64_t sstride, int n, int m,
                                                        const double* __restrict__ red, int nby,
                                                        const double* __restrict__ pyy, int Syy,
                                                        int64_t npad_y, int64_t pyy_bstride,
                                                        double* __restrict__ loss,
                                                        int64_t lstride) {
    __shared__ double sh[3 * BS];
    const int b = blockIdx.x;
    const double* qx = pxx + (int64_t)b * S * sstride;
    const double* qy = pxy + (int64_t)b * Sxy * sstride;
    double v[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < S; ++s)
        for (int i = threadIdx.x; i < n; i += BS) v[0] += qx[(int64_t)s * sstride + i];
    for (int s = 0; s < Sxy; ++s)
        for (int i = threadIdx.x; i < n; i += BS) v[1] += qy[(int64_t)s * sstride + i];
    if (pyy) {
        const double* qq = pyy + (int64_t)b * pyy_bstride;
        for (int s = 0; s < Syy; ++s)
            for (int a = threadIdx.x; a < m; a += BS) v[2] += qq[(int64_t)s * npad_y + a];
    } else {
        for (int q = threadIdx.x; q < nby; q += BS) v[2] += red[8 * q + 2];
    }
    block_sum<3>(v, sh);
    if (threadIdx.x == 0)
        loss[b * lstride] =
            v[0] / ((double)n * n) + v[2] / ((double)m * m) - 2.0 * v[1] / ((double)n * m);
}

// Source slicing of the batched loss: slices of whole tiles, about target_blocks
// blocks per launch over all members.
static void mmd_batch_slices(const dnb_ctx* c, int64_t batch, int64_t n, int64_t m, int& S,
                             int& jslice, int& Sxy, int& jslice_xy) {
    const int64_t nblk = cdiv(n, BS);
    int64_t want = c->target_blocks / (nblk * batch);
    if (want > S_MAX) want = S_MAX;
    if (want < 1) want = 1;
    const int64_t wx = want < cdiv(n, TILE) ? want : cdiv(n, TILE);
    const int64_t wy = want < cdiv(m, TILE) ? want : cdiv(m, TILE);
    jslice = (int)(cdiv(cdiv(n, wx), TILE) * TILE);
    S = (int)cdiv(n, jslice);
    jslice_xy = (int)(cdiv(cdiv(m, wy), TILE) * TILE);
    Sxy = (int)cdiv(m, jslice_xy);
}

// Partial-sum doubles of the batched loss: the target-source sums of every
// member, plus, with a target per member, the slice sums of each target.
static int64_t mmd_batch_doubles(const dnb_ctx* c, int64_t batch, int64_t n, int64_t m,
                                 bool grad, bool per_member) {
    int S, js, Sxy, jsxy;
    mmd_batch_slices(c, batch, n, m, S, js, Sxy, jsxy);
    int64_t total = batch * (S + Sxy) * cdiv(n, BS) * BS * (grad ? 4 : 1);
    if (per_member) {
        mmd_batch_slices(c, batch, m, m, S, js, Sxy, jsxy);
        total += batch * S * cdiv(m, BS) * BS;
    }
    return total;
}

bool mmd_batch_fits(const dnb_ctx* c, int64_t batch, int64_t n, int64_t m, bool grad,
                    bool per_member) {
    if (batch < 1 || batch > DNB_BATCH_MAX || n < 1 || m < 1 || n > c->max_n || m > c->max_n)
        return false;
    return mmd_batch_doubles(c, batch, n, m, grad, per_member) <= 8 * c->slice_rows;
}

// Gradient rows of every member (the arithmetic and order of k_mmd_x).
// grid (nblk, batch).
__global__ __launch_bounds__(BS) void k_mmd_batch_grad(const double* __restrict__ pxx, int S,
                                                       const double* __restrict__ pxy, int Sxy,
                                                       int64_t npad, int n, int m, double h,
                                                       double* __restrict__ gpos) {
    const int64_t b = blockIdx.y;
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const double* px = pxx + b * S * 4 * npad;
    const double* py = pxy + b * Sxy * 4 * npad;
    double gx[3] = {0, 0, 0}, gy[3] = {0, 0, 0};
    for (int s = 0; s < S; ++s) {
        const double* q = px + (int64_t)s * 4 * npad + i;
        for (int c = 0; c < 3; ++c) gx[c] += q[(1 + c) * npad];
    }
    for (int s = 0; s < Sxy; ++s) {
        const double* q = py + (int64_t)s * 4 * npad + i;
        for (int c = 0; c < 3; ++c) gy[c] += q[(1 + c) * npad];
    }
    const double cxx = -2.0 / ((double)n * n * h * h);
    const double cxy = 2.0 / ((double)n * m * h * h);
    double* g = gpos + b * 3 * n;
    for (int c = 0; c < 3; ++c) g[(int64_t)c * n + i] = cxx * gx[c] + cxy * gy[c];
}

hipError_t launch_mmd_batch(dnb_ctx* c, int64_t batch, int64_t n, const double* pos, int64_t m,
                            const double* tgt, int per_member, double h, double* loss,
                            double* gpos, hipStream_t st) {
    const double inv2h2 = 1.0 / (2.0 * h * h);
    int S, jslice, Sxy, jslice_xy;
    mmd_batch_slices(c, batch, n, m, S, jslice, Sxy, jslice_xy);
    const int nblk = (int)cdiv(n, BS);
    const int64_t npad = (int64_t)nblk * BS;
    const int wg = gpos != nullptr;
    const int64_t ss = (wg ? 4 : 1) * npad;      // stride of one slice's rows
    double* pxx = (double*)c->partv;
    double* pxy = pxx + batch * S * ss;
    double* pyy = (double*)c->part;
    const Slicing sy = plain_slicing(c, m);
    mmd_rows(dim3(nblk, S, (unsigned)batch), st, pos, (int)n,
                       pos, (int)n, inv2h2, jslice, wg, pxx, npad, ss, 3 * n, 3 * n, S * ss);
    const int64_t tstride = per_member ? 3 * m : 0;
    mmd_rows(dim3(nblk, Sxy, (unsigned)batch), st, pos, (int)n,
                       tgt, (int)m, inv2h2, jslice_xy, wg, pxy, npad, ss, 3 * n, tstride,
                       Sxy * ss);
    if (per_member) {
        // each member's own target term, in its own slices after pxy
        int Syy, jsyy, s2, j2;
        mmd_batch_slices(c, batch, m, m, Syy, jsyy, s2, j2);
        const int nblk_y = (int)cdiv(m, BS);
        const int64_t npad_y = (int64_t)nblk_y * BS;
        double* pyb = pxy + batch * Sxy * ss;
        mmd_rows(dim3(nblk_y, Syy, (unsigned)batch), st, tgt,
                           (int)m, tgt, (int)m, inv2h2, jsyy, 0, pyb, npad_y, npad_y, 3 * m, 3 * m,
                           Syy * npad_y);
        hipLaunchKernelGGL(k_mmd_batch_final, dim3((unsigned)batch), dim3(BS), 0, st, pxx, S, pxy,
                           Sxy, ss, (int)n, (int)m, (const double*)nullptr, 0,
                           (const double*)pyb, Syy, npad_y, (int64_t)Syy * npad_y, loss,
                           (int64_t)1);
    } else {
        mmd_rows(dim3(sy.nblk, sy.S), st, tgt, (int)m, tgt,
                           (int)m, inv2h2, sy.jslice, 0, pyy, sy.npad, 4 * sy.npad, 0, 0, 0);
        hipLaunchKernelGGL(k_mmd_y, dim3(sy.nblk), dim3(BS), 0, st, pyy, sy.S, sy.npad, (int)m,
                           c->red);
        hipLaunchKernelGGL(k_mmd_batch_final, dim3((unsigned)batch), dim3(BS), 0, st, pxx, S, pxy,
                           Sxy, ss, (int)n, (int)m, (const double*)c->red, sy.nblk,
                           (const double*)nullptr, 0, (int64_t)0, (int64_t)0, loss, (int64_t)1);
    }
    if (wg)
        hipLaunchKernelGGL(k_mmd_batch_grad, dim3(nblk, (unsigned)batch), dim3(BS), 0, st, pxx, S,
                           pxy, Sxy, npad, (int)n, (int)m, h, gpos);
    return hipGetLastError();
}

// Loss of every member against each of n_tgt targets: loss [batch][n_tgt].  The
// member-member sums are made once; per target, the member-target sums, the
// target's own sums (the slicing of the per-member-target mode, so that the
// result equals it bit for bit) and the losses of all members.
bool mmd_batch_targets_fits(const dnb_ctx* c, int64_t batch, int64_t n, int64_t n_tgt,
                            int64_t m) {
    if (n_tgt < 1 || n_tgt > DNB_BATCH_MAX) return false;
    return mmd_batch_fits(c, batch, n, m, false, true);
}

hipError_t launch_mmd_batch_targets(dnb_ctx* c, int64_t batch, int64_t n, const double* pos,
                                    int64_t n_tgt, int64_t m, const double* tgts, double h,
                                    double* loss, hipStream_t st) {
    const double inv2h2 = 1.0 / (2.0 * h * h);
    int S, jslice, Sxy, jslice_xy, Syy, jsyy, s2, j2;
    mmd_batch_slices(c, batch, n, m, S, jslice, Sxy, jslice_xy);
    mmd_batch_slices(c, batch, m, m, Syy, jsyy, s2, j2);
    const int nblk = (int)cdiv(n, BS);
    const int64_t npad = (int64_t)nblk * BS;
    const int nblk_y = (int)cdiv(m, BS);
    const int64_t npad_y = (int64_t)nblk_y * BS;
    double* pxx = (double*)c->partv;
    double* pxy = pxx + batch * S * npad;
    double* pyy = pxy + batch * Sxy * npad;
    mmd_rows(dim3(nblk, S, (unsigned)batch), st, pos, (int)n,
                       pos, (int)n, inv2h2, jslice, 0, pxx, npad, npad, 3 * n, 3 * n, S * npad);
    for (int64_t t = 0; t < n_tgt; ++t) {
        const double* tgt = tgts + t * 3 * m;
        mmd_rows(dim3(nblk, Sxy, (unsigned)batch), st, pos,
                           (int)n, tgt, (int)m, inv2h2, jslice_xy, 0, pxy, npad, npad, 3 * n,
                           (int64_t)0, Sxy * npad);
        mmd_rows(dim3(nblk_y, Syy, 1), st, tgt, (int)m, tgt,
                           (int)m, inv2h2, jsyy, 0, pyy, npad_y, npad_y, (int64_t)0, (int64_t)0,
                           (int64_t)0);
        hipLaunchKernelGGL(k_mmd_batch_final, dim3((unsigned)batch), dim3(BS), 0, st, pxx, S, pxy,
                           Sxy, npad, (int)n, (int)m, (const double*)nullptr, 0,
                           (const double*)pyy, Syy, npad_y, (int64_t)0, loss + t, n_tgt);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ energies --
__device__ inline double ext_potential(const Pot& p, double x, double y, double z) {
    double phi = 0.0;
    if (p.m_nfw != 0.0) {
        const double r = sqrt(x * x + y * y + z * z);
        phi += (r == 0.0) ? -p.G * p.m_nfw / p.rs_nfw : -p.G * p.m_nfw * log1p(r / p.rs_nfw) / r;
    }
    if (p.m_mn != 0.0) {
        const double S = sqrt(z * z + p.b_mn * p.b_mn);
        const double A = p.a_mn + S;
        phi += -p.G * p.m_mn / sqrt(x * x + y * y + A * A);
    }
    return phi;
}

// part[s][0][i] = sum_{j in slice, j != i} m_j (r_ij^2 + eps^2)^(-1/2)
__global__ __launch_bounds__(BS) void k_energy_pairs(const double* __restrict__ x,
                                                     const double* __restrict__ mass, int n,
                                                     int jslice, double eps2,
                                                     double* __restrict__ part, int64_t npad) {
    __shared__ double4 tile[TILE];
    const int i = blockIdx.x * BS + threadIdx.x;
    const int j0 = blockIdx.y * jslice;
    const int j1 = min(n, j0 + jslice);
    const int ii = min(i, n - 1);
    const double mx = x[ii], my = x[n + ii], mz = x[2 * n + ii];
    double acc = 0.0;
    for (int jt = j0; jt < j1; jt += TILE) {
        const int j = jt + threadIdx.x;
        tile[threadIdx.x] = (j < j1) ? make_double4(x[j], x[n + j], x[2 * n + j], mass[j])
                                     : make_double4(0.0, 0.0, 0.0, 0.0);
        __syncthreads();
        const int cnt = min(TILE, j1 - jt);
        for (int k = 0; k < cnt; ++k) {
            if (jt + k == i) continue;
            const double4 q = tile[k];
            const double dx = q.x - mx, dy = q.y - my, dz = q.z - mz;
            acc += q.w / sqrt(dx * dx + dy * dy + dz * dz + eps2);
        }
        __syncthreads();
    }
    if (i < n) part[(int64_t)blockIdx.y * npad + i] = acc;
}

__global__ __launch_bounds__(BS) void k_energy_rows(const double* __restrict__ x,
                                                    const double* __restrict__ v,
                                                    const double* __restrict__ mass, int n,
                                                    Pot p, const double* __restrict__ part, int S,
                                                    int64_t npad, double* __restrict__ red) {
    __shared__ double sh[3 * BS];
    const int i = blockIdx.x * BS + threadIdx.x;
    double e[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const double m = mass[i];
        double w = 0.0;
        for (int s = 0; s < S; ++s) w += part[(int64_t)s * npad + i];
        e[0] = 0.5 * m * (v[i] * v[i] + v[n + i] * v[n + i] + v[2 * n + i] * v[2 * n + i]);
        e[1] = m * w;
        e[2] = m * ext_potential(p, x[i], x[n + i], x[2 * n + i]);
    }
    block_sum<3>(e, sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) red[8 * blockIdx.x + c] = e[c];
}

__global__ __launch_bounds__(BS) void k_energy_final(const double* __restrict__ red, int nb,
                                                     double G, double* __restrict__ out3) {
    __shared__ double sh[3 * BS];
    double e[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += BS)
        for (int c = 0; c < 3; ++c) e[c] += red[8 * b + c];
    block_sum<3>(e, sh);
    if (threadIdx.x == 0) { out3[0] = e[0]; out3[1] = -0.5 * G * e[1]; out3[2] = e[2]; }
}

hipError_t launch_energy(dnb_ctx* c, int64_t n, const double* pos, const double* vel,
                         const double* mass, const Pot& p, double* out3, hipStream_t st) {
    Slicing sl = plain_slicing(c, n);
    double* part = (double*)c->partv;
    hipLaunchKernelGGL(k_energy_pairs, dim3(sl.nblk, sl.S), dim3(BS), 0, st, pos, mass, (int)n,
                       sl.jslice, p.eps * p.eps, part, sl.npad);
    hipLaunchKernelGGL(k_energy_rows, dim3(sl.nblk), dim3(BS), 0, st, pos, vel, mass, (int)n, p,
                       (const double*)part, sl.S, sl.npad, c->red);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(BS), 0, st, c->red, sl.nblk, p.G, out3);
    return hipGetLastError();
}

// -------------------------------------------------------- test-particle orbit --
// One lane integrates the single particle; the loop is sequential in time.
__global__ void k_orbit(const double* __restrict__ w0, Pot p, double dt, int64_t n_steps,
                        double* __restrict__ w_out, double* __restrict__ traj) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double x = w0[0], y = w0[1], z = w0[2], vx = w0[3], vy = w0[4], vz = w0[5];
    const double hdt = 0.5 * dt;
    Ext e = ext_accel(p, x, y, z);
    if (traj) { traj[0] = x; traj[1] = y; traj[2] = z; }
    for (int64_t s = 0; s < n_steps; ++s) {
        const double hx = fma(hdt, e.ax, vx), hy = fma(hdt, e.ay, vy), hz = fma(hdt, e.az, vz);
        x = fma(dt, hx, x); y = fma(dt, hy, y); z = fma(dt, hz, z);
        e = ext_accel(p, x, y, z);
        vx = fma(hdt, e.ax, hx); vy = fma(hdt, e.ay, hy); vz = fma(hdt, e.az, hz);
        if (traj) { traj[3 * (s + 1)] = x; traj[3 * (s + 1) + 1] = y; traj[3 * (s + 1) + 2] = z; }
    }
    w_out[0] = x; w_out[1] = y; w_out[2] = z; w_out[3] = vx; w_out[4] = vy; w_out[5] = vz;
}

// Reverse sweep of k_orbit with merged half kicks (see the N-body sweep).
// gparams = (dL/dm_nfw, dL/dm_mn, dL/ddt).
__global__ void k_orbit_vjp(const double* __restrict__ traj, Pot p, double dt, int64_t n_steps,
                            const double* __restrict__ gw_out, double* __restrict__ gw0,
                            double* __restrict__ gparams) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double lx = gw_out[0], ly = gw_out[1], lz = gw_out[2];
    double wx = gw_out[3], wy = gw_out[4], wz = gw_out[5];
    double g_nfw = 0.0, g_mn = 0.0, g_dt = 0.0;
    const double inv = 1.0 / dt;
    for (int64_t s = n_steps; s >= 0 && n_steps > 0; --s) {
        const double coef = (s == n_steps || s == 0) ? 0.5 * dt : dt;
        const double kc = (s == n_steps || s == 0) ? 0.5 : 1.0;
        const double x = traj[3 * s], y = traj[3 * s + 1], z = traj[3 * s + 2];
        Ext e = ext_accel(p, x, y, z);
        double hx, hy, hz;
        ext_hvp(p, x, y, z, wx, wy, wz, hx, hy, hz);
        lx += coef * hx; ly += coef * hy; lz += coef * hz;
        g_dt += kc * (e.ax * wx + e.ay * wy + e.az * wz);
        g_nfw += coef * (e.nx * wx + e.ny * wy + e.nz * wz);
        g_mn += coef * (e.mx * wx + e.my * wy + e.mz * wz);
        if (s > 0) {
            const double vx = (x - traj[3 * (s - 1)]) * inv;
            const double vy = (y - traj[3 * (s - 1) + 1]) * inv;
            const double vz = (z - traj[3 * (s - 1) + 2]) * inv;
            g_dt += vx * lx + vy * ly + vz * lz;
            wx += dt * lx; wy += dt * ly; wz += dt * lz;
        }
    }
    gw0[0] = lx; gw0[1] = ly; gw0[2] = lz; gw0[3] = wx; gw0[4] = wy; gw0[5] = wz;
    gparams[0] = g_nfw; gparams[1] = g_mn; gparams[2] = g_dt;
}

hipError_t launch_orbit(const double* w0, const Pot& p, double dt, int64_t n_steps, double* w_out,
                        double* traj, hipStream_t st) {
    hipLaunchKernelGGL(k_orbit, dim3(1), dim3(64), 0, st, w0, p, dt, n_steps, w_out, traj);
    return hipGetLastError();
}

hipError_t launch_orbit_vjp(const double* traj, const Pot& p, double dt, int64_t n_steps,
                            const double* gw_out, double* gw0, double* gparams, hipStream_t st) {
    hipLaunchKernelGGL(k_orbit_vjp, dim3(1), dim3(64), 0, st, traj, p, dt, n_steps, gw_out, gw0,
                       gparams);
    return hipGetLastError();
}

// --------------------------------------------------------- Plummer placement --
__global__ __launch_bounds__(BS) void k_place(int64_t n, const double* __restrict__ w,
                                              const double* __restrict__ xi,
                                              const double* __restrict__ zeta, double a_p,
                                              double vscale, double mi, double* __restrict__ pos,
                                              double* __restrict__ vel,
                                              double* __restrict__ mass) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < 3; ++c) {
        pos[c * n + i] = w[c] + a_p * xi[c * n + i];
        vel[c * n + i] = w[3 + c] + vscale * zeta[c * n + i];
    }
    mass[i] = mi;
}

__global__ __launch_bounds__(BS) void k_place_vjp_rows(int64_t n, const double* __restrict__ zeta,
                                                       const double* __restrict__ gpos,
                                                       const double* __restrict__ gvel,
                                                       const double* __restrict__ gmass,
                                                       double* __restrict__ red) {
    __shared__ double sh[8 * BS];
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < n) {
        for (int c = 0; c < 3; ++c) {
            v[c] = gpos[c * n + i];
            v[3 + c] = gvel[c * n + i];
            v[6] += gvel[c * n + i] * zeta[c * n + i];
        }
        v[7] = gmass ? gmass[i] : 0.0;
    }
    block_sum<8>(v, sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < 8; ++c) red[8 * blockIdx.x + c] = v[c];
}

__global__ __launch_bounds__(BS) void k_place_vjp_final(const double* __restrict__ red, int nb,
                                                        int64_t n, double dvs_dm,
                                                        double* __restrict__ gw,
                                                        double* __restrict__ gm_tot) {
    __shared__ double sh[8 * BS];
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += BS)
        for (int c = 0; c < 8; ++c) v[c] += red[8 * b + c];
    block_sum<8>(v, sh);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 6; ++c) gw[c] = v[c];
        gm_tot[0] = v[6] * dvs_dm + v[7] / (double)n;
    }
}

hipError_t launch_place(int64_t n, const double* w, const double* xi, const double* zeta,
                        double m_tot, double a_p, double G, double* pos, double* vel,
                        double* mass, hipStream_t st) {
    const double vscale = sqrt(G * m_tot / a_p);
    hipLaunchKernelGGL(k_place, dim3((unsigned)cdiv(n, BS)), dim3(BS), 0, st, n, w, xi, zeta, a_p,
                       vscale, m_tot / (double)n, pos, vel, mass);
    return hipGetLastError();
}

hipError_t launch_place_vjp(dnb_ctx* c, int64_t n, const double* zeta, double m_tot, double a_p,
                            double G, const double* gpos, const double* gvel, const double* gmass,
                            double* gw, double* gm_tot, hipStream_t st) {
    const int nb = (int)cdiv(n, BS);
    // d sqrt(G M / a_p) / dM = sqrt(G / (a_p M)) / 2
    const double dvs_dm = 0.5 * sqrt(G / (a_p * m_tot));
    hipLaunchKernelGGL(k_place_vjp_rows, dim3(nb), dim3(BS), 0, st, n, zeta, gpos, gvel, gmass,
                       c->red);
    hipLaunchKernelGGL(k_place_vjp_final, dim3(1), dim3(BS), 0, st, c->red, nb, n, dvs_dm, gw,
                       gm_tot);
    return hipGetLastError();
}

// ------------------------------------------------------------ state scan --
// Smallest index p = b n + i (member b, particle i) of nsys systems laid out as
// x, v [nsys][3][n] and m [nsys][n] at which a coordinate, a velocity component
// or the mass is NaN or infinite; INT64_MAX when there is none.  v and m may be
// NULL.  Blocks stride over the particles and write their minimum to out[b];
// k_scan_final takes the minimum of the nb block minima into out[slot].
__device__ inline int64_t wave_min_i64(int64_t a) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const int64_t o = __shfl_xor(a, m, 64);
        a = o < a ? o : a;
    }
    return a;
}

__device__ inline int64_t block_min_i64(int64_t a) {
    __shared__ int64_t sh[BS / 64];
    a = wave_min_i64(a);
    if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = a;
    __syncthreads();
    a = sh[0];
    for (int w = 1; w < BS / 64; ++w) a = sh[w] < a ? sh[w] : a;
    return a;
}

__global__ __launch_bounds__(BS) void k_scan_state(const double* __restrict__ x,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ m, int64_t n,
                                                   int64_t total, int64_t* __restrict__ out) {
    int64_t bad = INT64_MAX;
    for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * BS) {
        const int64_t b = p / n, i = p - b * n;
        bool ok = true;
        for (int c = 0; c < 3; ++c) {
            ok = ok && isfinite(x[(3 * b + c) * n + i]);
            if (v) ok = ok && isfinite(v[(3 * b + c) * n + i]);
        }
        if (m) ok = ok && isfinite(m[p]);
        if (!ok && p < bad) bad = p;
    }
    bad = block_min_i64(bad);
    if (threadIdx.x == 0) out[blockIdx.x] = bad;
}

__global__ __launch_bounds__(BS) void k_scan_final(int64_t* __restrict__ out, int nb, int slot) {
    int64_t bad = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += BS) bad = out[b] < bad ? out[b] : bad;
    bad = block_min_i64(bad);
    if (threadIdx.x == 0) out[slot] = bad;
}

hipError_t launch_scan_state(dnb_ctx* c, const double* x, const double* v, const double* m,
                             int64_t n, int64_t nsys, hipStream_t st) {
    const int64_t total = n * nsys;
    const int nb = (int)std::min<int64_t>(cdiv(total, BS), c->nbmax);
    hipLaunchKernelGGL(k_scan_state, dim3(nb), dim3(BS), 0, st, x, v, m, n, total, c->scan);
    hipLaunchKernelGGL(k_scan_final, dim3(1), dim3(BS), 0, st, c->scan, nb, c->nbmax);
    return hipGetLastError();
}

}  // namespace dnb
