// O(N^2) kernels: the softened pairwise gravity sum (Sec. 1, direct pairwise
// forces with softening) and its vector-Jacobian product (Sec. 2: reverse-mode
// gradients through the simulation).
//
// Layout.  A launch is a grid of (target blocks) x (source slices).  Each
// 256-thread block owns 256 target particles (one per lane) and one contiguous
// slice of sources, which it streams through LDS in tiles of 256.  Every lane
// reads the same source from LDS at the same time (a broadcast read), so LDS
// bandwidth is not a limit; the kernel is bound by VALU issue.  Each block writes
// its per-target partial sums for its slice; the O(N) kernel that consumes the
// sum adds the slices in FP64 in slice order, so results are deterministic and
// independent of scheduling.  No floating-point atomics are used.
//
// FP32C: pair terms in FP32 on positions staged relative to a common centre.
// Within a sub-tile of 128 sources a lane sums in plain FP32; each sub-tile sum
// is then added to a (hi, lo) pair with an error-free TwoSum, so the error of
// the running sum does not grow with N.  The reciprocal square root is the
// hardware v_rsq_f32 (1 ulp).
//
// FP64: the same in double precision on absolute positions; v_rsq_f64 gives
// about 23 correct bits and two Newton steps y <- y (3/2 - s y^2 / 2) bring it
// to full precision.
#include "dnb_internal.h"

namespace dnb {

// Padding source far away with zero mass: contributes exactly zero.
constexpr float FAR32 = 1.0e18f;
constexpr double FAR64 = 1.0e150;

__device__ __forceinline__ void two_sum_acc(float& hi, float& lo, float x) {
    float s = hi + x;
    float bp = s - hi;
    float e = (hi - (s - bp)) + (x - bp);
    hi = s;
    lo += e;
}

__device__ __forceinline__ double rsqrt_f64(double s) {
    double y = __builtin_amdgcn_rsq(s);
    double hs = 0.5 * s;
    y = y * fma(-hs * y, y, 1.5);
    y = y * fma(-hs * y, y, 1.5);
    return y;
}

// ------------------------------------------------------------ forward FP32C --
// js: staged sources (x, y, z, m).  part: [S][6][npad] = (hi_x, hi_y, hi_z,
// lo_x, lo_y, lo_z) of sum_j m_j d_ij s_ij^-3/2 over the block's slice.
template <bool EPS0>
__global__ __launch_bounds__(BS) void k_pair_fwd_f32c(const float4* __restrict__ js, int n,
                                                      int jslice, float eps2,
                                                      float* __restrict__ part, int64_t npad) {
    __shared__ float4 tile[TILE];
    const int i = blockIdx.x * BS + threadIdx.x;
    const int j0 = blockIdx.y * jslice;
    const int j1 = min(n, j0 + jslice);
    const float4 me = js[min(i, n - 1)];
    float hx = 0.f, hy = 0.f, hz = 0.f, lx = 0.f, ly = 0.f, lz = 0.f;
    for (int jt = j0; jt < j1; jt += TILE) {
        const int j = jt + threadIdx.x;
        tile[threadIdx.x] = (j < j1) ? js[j] : make_float4(FAR32, FAR32, FAR32, 0.f);
        __syncthreads();
#pragma unroll
        for (int h = 0; h < TILE / SUBTILE; ++h) {
            float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll 16
            for (int k = 0; k < SUBTILE; ++k) {
                const float4 q = tile[h * SUBTILE + k];
                const float dx = q.x - me.x, dy = q.y - me.y, dz = q.z - me.z;
                const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                const float r = __builtin_amdgcn_rsqf(s);
                float w = (q.w * r) * (r * r);
                if (EPS0) w = (jt + h * SUBTILE + k == i) ? 0.f : w;
                ax = fmaf(w, dx, ax);
                ay = fmaf(w, dy, ay);
                az = fmaf(w, dz, az);
            }
            two_sum_acc(hx, lx, ax);
            two_sum_acc(hy, ly, ay);
            two_sum_acc(hz, lz, az);
        }
        __syncthreads();
    }
    if (i < n) {
        float* p = part + (int64_t)blockIdx.y * 6 * npad + i;
        p[0 * npad] = hx; p[1 * npad] = hy; p[2 * npad] = hz;
        p[3 * npad] = lx; p[4 * npad] = ly; p[5 * npad] = lz;
    }
}

// ------------------------------------------------------------- forward FP64 --
// part: [S][3][npad] doubles.
template <bool EPS0>
__global__ __launch_bounds__(BS) void k_pair_fwd_f64(const double* __restrict__ x,
                                                     const double* __restrict__ mass, int n,
                                                     int jslice, double eps2,
                                                     double* __restrict__ part, int64_t npad) {
    __shared__ double4 tile[TILE];
    const int i = blockIdx.x * BS + threadIdx.x;
    const int j0 = blockIdx.y * jslice;
    const int j1 = min(n, j0 + jslice);
    const int ii = min(i, n - 1);
    const double mx = x[ii], my = x[n + ii], mz = x[2 * n + ii];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int jt = j0; jt < j1; jt += TILE) {
        const int j = jt + threadIdx.x;
        tile[threadIdx.x] = (j < j1) ? make_double4(x[j], x[n + j], x[2 * n + j], mass[j])
                                     : make_double4(FAR64, FAR64, FAR64, 0.0);
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < TILE; ++k) {
            const double4 q = tile[k];
            const double dx = q.x - mx, dy = q.y - my, dz = q.z - mz;
            const double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
            const double r = rsqrt_f64(s);
            double w = (q.w * r) * (r * r);
            if (EPS0) w = (jt + k == i) ? 0.0 : w;
            ax = fma(w, dx, ax);
            ay = fma(w, dy, ay);
            az = fma(w, dz, az);
        }
        __syncthreads();
    }
    if (i < n) {
        double* p = part + (int64_t)blockIdx.y * 3 * npad + i;
        p[0] = ax; p[npad] = ay; p[2 * npad] = az;
    }
}

// --------------------------------------------------------------- VJP FP32C --
// For target k and cotangent w, with d = x_j - x_k, s = |d|^2 + eps^2:
//   (J^T w)_k / G = sum_j [s^-3/2 u - 3 s^-5/2 (d.u) d],  u = m_k w_j - m_j w_k
//   a_int,k / G   = sum_j m_j s^-3/2 d            (needed for the dt and mass terms)
//   gm_k / G      = sum_j (d.w_j) s^-3/2          (mass cotangent, negated later)
// jsv: [0..n) staged (x, y, z, m), [n..2n) staged (wx, wy, wz, 0).
// part: [S][14][npad] floats: JTw hi(3) lo(3), a hi(3) lo(3), gm hi, lo.
template <bool EPS0, bool MASS>
__global__ __launch_bounds__(BS) void k_pair_vjp_f32c(const float4* __restrict__ jsv, int n,
                                                      int jslice, float eps2,
                                                      float* __restrict__ part, int64_t npad) {
    __shared__ float4 tp[TILE];
    __shared__ float4 tw[TILE];
    const int i = blockIdx.x * BS + threadIdx.x;
    const int j0 = blockIdx.y * jslice;
    const int j1 = min(n, j0 + jslice);
    const int ii = min(i, n - 1);
    const float4 me = jsv[ii];
    const float4 mw = jsv[n + ii];
    float h[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float l[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int jt = j0; jt < j1; jt += TILE) {
        const int j = jt + threadIdx.x;
        if (j < j1) {
            tp[threadIdx.x] = jsv[j];
            tw[threadIdx.x] = jsv[n + j];
        } else {
            tp[threadIdx.x] = make_float4(FAR32, FAR32, FAR32, 0.f);
            tw[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int hh = 0; hh < TILE / SUBTILE; ++hh) {
            float gx = 0.f, gy = 0.f, gz = 0.f, ax = 0.f, ay = 0.f, az = 0.f, gm = 0.f;
#pragma unroll 8
            for (int k = 0; k < SUBTILE; ++k) {
                const float4 q = tp[hh * SUBTILE + k];
                const float4 qw = tw[hh * SUBTILE + k];
                const float dx = q.x - me.x, dy = q.y - me.y, dz = q.z - me.z;
                const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                float r = __builtin_amdgcn_rsqf(s);
                if (EPS0) r = (jt + hh * SUBTILE + k == i) ? 0.f : r;
                const float r2 = r * r;
                const float r3 = r2 * r;
                const float r5 = r3 * r2;
                const float ux = fmaf(me.w, qw.x, -(q.w * mw.x));
                const float uy = fmaf(me.w, qw.y, -(q.w * mw.y));
                const float uz = fmaf(me.w, qw.z, -(q.w * mw.z));
                const float du = fmaf(dx, ux, fmaf(dy, uy, dz * uz));
                const float c = -3.f * (r5 * du);
                gx = fmaf(c, dx, fmaf(r3, ux, gx));
                gy = fmaf(c, dy, fmaf(r3, uy, gy));
                gz = fmaf(c, dz, fmaf(r3, uz, gz));
                const float mr3 = q.w * r3;
                ax = fmaf(mr3, dx, ax);
                ay = fmaf(mr3, dy, ay);
                az = fmaf(mr3, dz, az);
                if (MASS) {
                    const float dw = fmaf(dx, qw.x, fmaf(dy, qw.y, dz * qw.z));
                    gm = fmaf(dw, r3, gm);
                }
            }
            two_sum_acc(h[0], l[0], gx);
            two_sum_acc(h[1], l[1], gy);
            two_sum_acc(h[2], l[2], gz);
            two_sum_acc(h[3], l[3], ax);
            two_sum_acc(h[4], l[4], ay);
            two_sum_acc(h[5], l[5], az);
            if (MASS) two_sum_acc(h[6], l[6], gm);
        }
        __syncthreads();
    }
    if (i < n) {
        float* p = part + (int64_t)blockIdx.y * 14 * npad + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            p[c * npad] = h[c];
            p[(3 + c) * npad] = l[c];
            p[(6 + c) * npad] = h[3 + c];
            p[(9 + c) * npad] = l[3 + c];
        }
        if (MASS) {
            p[12 * npad] = h[6];
            p[13 * npad] = l[6];
        }
    }
}

// ---------------------------------------------------------------- VJP FP64 --
// part: [S][7][npad] doubles: JTw(3), a(3), gm.
template <bool EPS0, bool MASS>
__global__ __launch_bounds__(BS) void k_pair_vjp_f64(const double* __restrict__ x,
                                                     const double* __restrict__ mass,
                                                     const double* __restrict__ w, int n,
                                                     int jslice, double eps2,
                                                     double* __restrict__ part, int64_t npad) {
    __shared__ double4 tp[TILE];
    __shared__ double4 tw[TILE];
    const int i = blockIdx.x * BS + threadIdx.x;
    const int j0 = blockIdx.y * jslice;
    const int j1 = min(n, j0 + jslice);
    const int ii = min(i, n - 1);
    const double mx = x[ii], my = x[n + ii], mz = x[2 * n + ii], mm = mass[ii];
    const double wx0 = w[ii], wy0 = w[n + ii], wz0 = w[2 * n + ii];
    double gx = 0, gy = 0, gz = 0, ax = 0, ay = 0, az = 0, gm = 0;
    for (int jt = j0; jt < j1; jt += TILE) {
        const int j = jt + threadIdx.x;
        if (j < j1) {
            tp[threadIdx.x] = make_double4(x[j], x[n + j], x[2 * n + j], mass[j]);
            tw[threadIdx.x] = make_double4(w[j], w[n + j], w[2 * n + j], 0.0);
        } else {
            tp[threadIdx.x] = make_double4(FAR64, FAR64, FAR64, 0.0);
            tw[threadIdx.x] = make_double4(0.0, 0.0, 0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < TILE; ++k) {
            const double4 q = tp[k];
            const double4 qw = tw[k];
            const double dx = q.x - mx, dy = q.y - my, dz = q.z - mz;
            const double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
            double r = rsqrt_f64(s);
            if (EPS0) r = (jt + k == i) ? 0.0 : r;
            const double r2 = r * r;
            const double r3 = r2 * r;
            const double r5 = r3 * r2;
            const double ux = fma(mm, qw.x, -(q.w * wx0));
            const double uy = fma(mm, qw.y, -(q.w * wy0));
            const double uz = fma(mm, qw.z, -(q.w * wz0));
            const double du = fma(dx, ux, fma(dy, uy, dz * uz));
            const double c = -3.0 * (r5 * du);
            gx = fma(c, dx, fma(r3, ux, gx));
            gy = fma(c, dy, fma(r3, uy, gy));
            gz = fma(c, dz, fma(r3, uz, gz));
            const double mr3 = q.w * r3;
            ax = fma(mr3, dx, ax);
            ay = fma(mr3, dy, ay);
            az = fma(mr3, dz, az);
            if (MASS) {
                const double dw = fma(dx, qw.x, fma(dy, qw.y, dz * qw.z));
                gm = fma(dw, r3, gm);
            }
        }
        __syncthreads();
    }
    if (i < n) {
        double* p = part + (int64_t)blockIdx.y * 7 * npad + i;
        p[0] = gx; p[npad] = gy; p[2 * npad] = gz;
        p[3 * npad] = ax; p[4 * npad] = ay; p[5 * npad] = az;
        if (MASS) p[6 * npad] = gm;
    }
}

// ---------------------------------------------------------------- launchers --
hipError_t launch_pair_fwd(dnb_ctx* c, int64_t n, const double* x, const double* mass,
                               double eps, hipStream_t st) {
    Slicing sl = slicing_for(n);
    dim3 grid(sl.nblk, sl.S);
    if (c->prec == DNB_FP32C) {
        const float eps2 = (float)(eps * eps);
        if (eps == 0.0)
            hipLaunchKernelGGL(k_pair_fwd_f32c<true>, grid, dim3(BS), 0, st, c->js, (int)n,
                               sl.jslice, eps2, (float*)c->part, sl.npad);
        else
            hipLaunchKernelGGL(k_pair_fwd_f32c<false>, grid, dim3(BS), 0, st, c->js, (int)n,
                               sl.jslice, eps2, (float*)c->part, sl.npad);
    } else {
        const double eps2 = eps * eps;
        if (eps == 0.0)
            hipLaunchKernelGGL(k_pair_fwd_f64<true>, grid, dim3(BS), 0, st, x, mass, (int)n,
                               sl.jslice, eps2, (double*)c->part, sl.npad);
        else
            hipLaunchKernelGGL(k_pair_fwd_f64<false>, grid, dim3(BS), 0, st, x, mass, (int)n,
                               sl.jslice, eps2, (double*)c->part, sl.npad);
    }
    return hipGetLastError();
}

hipError_t launch_pair_vjp(dnb_ctx* c, int64_t n, const double* x, const double* mass,
                               const double* w, int with_mass, double eps, hipStream_t st) {
    Slicing sl = slicing_for(n);
    dim3 grid(sl.nblk, sl.S);
    if (c->prec == DNB_FP32C) {
        const float eps2 = (float)(eps * eps);
        float* p = (float*)c->partv;
        if (eps == 0.0) {
            if (with_mass)
                hipLaunchKernelGGL((k_pair_vjp_f32c<true, true>), grid, dim3(BS), 0, st, c->jsv,
                                   (int)n, sl.jslice, eps2, p, sl.npad);
            else
                hipLaunchKernelGGL((k_pair_vjp_f32c<true, false>), grid, dim3(BS), 0, st, c->jsv,
                                   (int)n, sl.jslice, eps2, p, sl.npad);
        } else {
            if (with_mass)
                hipLaunchKernelGGL((k_pair_vjp_f32c<false, true>), grid, dim3(BS), 0, st, c->jsv,
                                   (int)n, sl.jslice, eps2, p, sl.npad);
            else
                hipLaunchKernelGGL((k_pair_vjp_f32c<false, false>), grid, dim3(BS), 0, st,
                                   c->jsv, (int)n, sl.jslice, eps2, p, sl.npad);
        }
    } else {
        const double eps2 = eps * eps;
        double* p = (double*)c->partv;
        if (eps == 0.0) {
            if (with_mass)
                hipLaunchKernelGGL((k_pair_vjp_f64<true, true>), grid, dim3(BS), 0, st, x, mass,
                                   w, (int)n, sl.jslice, eps2, p, sl.npad);
            else
                hipLaunchKernelGGL((k_pair_vjp_f64<true, false>), grid, dim3(BS), 0, st, x, mass,
                                   w, (int)n, sl.jslice, eps2, p, sl.npad);
        } else {
            if (with_mass)
                hipLaunchKernelGGL((k_pair_vjp_f64<false, true>), grid, dim3(BS), 0, st, x, mass,
                                   w, (int)n, sl.jslice, eps2, p, sl.npad);
            else
                hipLaunchKernelGGL((k_pair_vjp_f64<false, false>), grid, dim3(BS), 0, st, x,
                                   mass, w, (int)n, sl.jslice, eps2, p, sl.npad);
        }
    }
    return hipGetLastError();
}

}  // namespace dnb
