// Device code shared by the single-system and the batched O(N) kernels of the
// integrator and of its reverse sweep: staging of sources, the staging centre,
// the cotangent scale, and the sums of the pair kernels' slice partials.
#pragma once

#include "dnb_internal.h"

namespace dnb {

constexpr float FAR32 = 1.0e18f;
constexpr double FAR64 = 1.0e150;

// Per-block record of the O(N) kernels (FP32C staging), REC doubles:
//   [0..2] sums of the positions the kernel wrote or staged,
//   [3]    maximum |w| of the cotangent it staged (reverse sweep; 0 otherwise),
//   [4..6] sums of the displacement from the positions before them (x_new - x_old),
//   [7]    0.
// The displacement sums let the next kernel predict where the particles it is
// about to move will be.  A progenitor on its orbit travels 0.1-0.25 kpc per
// step, ten to twenty times its own 0.01 kpc size: staged relative to the mean
// of the previous positions, the FP32 offsets would carry that drift and lose
// the same factor in resolution of the pair separations.  (REC is defined with
// the launch geometry, since the host sizes the record buffers.)

// Staging centre: the mean of the recorded positions, plus, with extrapolate,
// the mean recorded displacement (the centre of the positions one step on).
__device__ inline void centre_from(const double* __restrict__ cpart, int nb, int64_t n, double* sh,
                                   double& cx, double& cy, double& cz, bool extrapolate) {
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += BS) {
        v[0] += cpart[REC * b + 0];
        v[1] += cpart[REC * b + 1];
        v[2] += cpart[REC * b + 2];
        if (extrapolate) {
            v[3] += cpart[REC * b + 4];
            v[4] += cpart[REC * b + 5];
            v[5] += cpart[REC * b + 6];
        }
    }
    block_sum<6>(v, sh);
    const double inv = 1.0 / (double)n;
    cx = (v[0] + v[3]) * inv; cy = (v[1] + v[4]) * inv; cz = (v[2] + v[5]) * inv;
}

// Record of this block: sums of (x, y, z) and of the displacement (dx, dy, dz)
// over its valid lanes; slot 3 is cleared (write_block_max fills it).
__device__ inline void write_block_sums(double x, double y, double z, double dx, double dy,
                                        double dz, bool valid, double* sh,
                                        double* __restrict__ cpart_out) {
    double v[6] = {valid ? x : 0.0, valid ? y : 0.0, valid ? z : 0.0,
                   valid ? dx : 0.0, valid ? dy : 0.0, valid ? dz : 0.0};
    block_sum<6>(v, sh);
    if (threadIdx.x == 0) {
        double* c = cpart_out + REC * blockIdx.x;
        c[0] = v[0]; c[1] = v[1]; c[2] = v[2]; c[3] = 0.0;
        c[4] = v[3]; c[5] = v[4]; c[6] = v[5]; c[7] = 0.0;
    }
}

// Cotangent scaling (FP32C reverse sweep).  Over long horizons the velocity
// cotangent of a chaotic system grows without bound (1e45 after 2000 steps is
// typical) and would overflow FP32.  The cotangent is therefore staged as w * S
// with S a power of two (exact) chosen so that max |w S| is about 1; the pair VJP
// is linear in w, so the consumer divides the slice sums by S in FP64.  S is
// taken from the block maxima of the previous cotangent (slot 3 of the
// block records), which differs from the staged one by one drift update.
__device__ inline double absmax3(double a, double b, double c) {
    return fmax(fabs(a), fmax(fabs(b), fabs(c)));
}

__device__ inline void write_block_max(double v, double* sh, double* __restrict__ cpart_out) {
    const double m = block_max(v, sh);
    if (threadIdx.x == 0) cpart_out[REC * blockIdx.x + 3] = m;
}

// Power-of-two scale from the block maxima in slot 3 of cpart (1 if all zero).
__device__ inline double scale_from(const double* __restrict__ cpart, int nb, double* sh) {
    double m = 0.0;
    for (int b = threadIdx.x; b < nb; b += BS) m = fmax(m, cpart[REC * b + 3]);
    m = block_max(m, sh);
    if (!(m > 0.0) || !isfinite(m)) return 1.0;
    int e;
    (void)frexp(m, &e);
    return ldexp(1.0, -e);
}

// Source record of particle i (i < n) or padding (n <= i < pad_sources(n)).
template <bool F32>
__device__ inline void put_source(void* js, int64_t i, bool real, double x, double y, double z,
                                  double m, double cx, double cy, double cz) {
    if (F32)
        ((float4*)js)[i] = real ? make_float4((float)(x - cx), (float)(y - cy), (float)(z - cz),
                                              (float)m)
                                : make_float4(FAR32, FAR32, FAR32, 0.f);
    else
        ((double4*)js)[i] = real ? make_double4(x, y, z, m) : make_double4(FAR64, FAR64, FAR64, 0.0);
}

template <bool F32>
__device__ inline void put_source_w(void* jsv, int64_t i, bool real, double x, double y, double z,
                                    double m, double cx, double cy, double cz, double wx, double wy,
                                    double wz) {
    if (F32) {
        float4* p = (float4*)jsv + 2 * i;
        p[0] = real ? make_float4((float)(x - cx), (float)(y - cy), (float)(z - cz), (float)m)
                    : make_float4(FAR32, FAR32, FAR32, 0.f);
        p[1] = real ? make_float4((float)wx, (float)wy, (float)wz, 0.f)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        double4* p = (double4*)jsv + 2 * i;
        p[0] = real ? make_double4(x, y, z, m) : make_double4(FAR64, FAR64, FAR64, 0.0);
        p[1] = real ? make_double4(wx, wy, wz, 0.0) : make_double4(0.0, 0.0, 0.0, 0.0);
    }
}

// Sum of the slice partials of the forward pair kernel for particle i (times G):
// FP32C (hi, lo) float2 [S][3][npad], FP64 double [S][3][npad], in slice order.
template <bool F32>
__device__ inline void pair_sum(const void* part, int S, int64_t npad, int64_t i, double G,
                                double& ax, double& ay, double& az) {
    ax = ay = az = 0.0;
    if (F32) {
        const float2* p = (const float2*)part;
#pragma unroll 4
        for (int s = 0; s < S; ++s) {
            const float2* q = p + (int64_t)s * 3 * npad + i;
            const float2 vx = q[0], vy = q[npad], vz = q[2 * npad];
            ax += (double)vx.x; ax += (double)vx.y;
            ay += (double)vy.x; ay += (double)vy.y;
            az += (double)vz.x; az += (double)vz.y;
        }
    } else {
        const double* p = (const double*)part;
#pragma unroll 4
        for (int s = 0; s < S; ++s) {
            const double* q = p + (int64_t)s * 3 * npad + i;
            ax += q[0]; ay += q[npad]; az += q[2 * npad];
        }
    }
    ax *= G; ay *= G; az *= G;
}

// Slice sums of the VJP kernel for particle i: J^T w and the raw mass term
// sum_j (d.w_j) s^-3/2, both times G, in slice order.  The slice loops here and
// in pair_sum are unrolled so that the loads of several slices are in flight
// together: a small system has many slices and few waves to hide their latency
// (at n = 1000 this took a pipeline gradient from 50 to 37 ms).
template <bool F32>
__device__ inline void vjp_sum(const void* part, int S, int64_t npad, int64_t i, double G,
                               bool with_mass, double (&g)[3], double& gm) {
    for (int c = 0; c < 3; ++c) g[c] = 0.0;
    gm = 0.0;
    if (F32) {
        const float2* p = (const float2*)part;
#pragma unroll 4
        for (int s = 0; s < S; ++s) {
            const float2* q = p + (int64_t)s * 4 * npad + i;
            for (int c = 0; c < 3; ++c) {
                const float2 v = q[c * npad];
                g[c] += (double)v.x; g[c] += (double)v.y;
            }
            if (with_mass) {
                const float2 v = q[3 * npad];
                gm += (double)v.x; gm += (double)v.y;
            }
        }
    } else {
        const double* p = (const double*)part;
#pragma unroll 4
        for (int s = 0; s < S; ++s) {
            const double* q = p + (int64_t)s * 4 * npad + i;
            for (int c = 0; c < 3; ++c) g[c] += q[c * npad];
            if (with_mass) gm += q[3 * npad];
        }
    }
    for (int c = 0; c < 3; ++c) g[c] *= G;
    gm *= G;
}

// ------------------------------------------------ FP32C slice reductions --
// Inside the integrator (forward steps and the reverse sweep) the FP32C slice
// partials are summed by a reduction kernel of their own, which also records the
// net internal force of the step: sum_k m_k a_k, zero in exact arithmetic
// (Newton's third law), and for the reverse sweep sum_k (J^T w)_k, zero for the
// same reason (the pair Jacobian's blocks K(d_kj) are even in d_kj).  The
// consumer subtracts the mean that restores these identities.  What it removes
// is the common part of the FP32 rounding of the per-target sums: in exact
// arithmetic it is zero.  That common part matters because the gradients with
// respect to the host masses are small differences (about 1e-4 of their terms)
// between the progenitor's orbit and the response of its particles, and the
// orbit's part follows the sum of the particles' cotangents, which per-target
// FP32 rounding would otherwise shift by ~1e-7 per step.

// Sum of the S slice partials of target i (FP32C (hi, lo) float2, STRIDE rows
// per slice, the first ROWS summed): RG groups of consecutive slices, each
// summed in slice order (hi, then lo) in FP64 by its own wave, the group sums
// added in group order.  Returns the sums in the threads of group 0
// (threadIdx.x < RT).  sh: [RG * ROWS * RT].
template <int ROWS, int STRIDE>
__device__ inline void slice_reduce(const float2* __restrict__ part, int S, int64_t npad,
                                    int64_t i, bool valid, double (&out)[ROWS], double* sh) {
    const int t = threadIdx.x % RT, g = threadIdx.x / RT;
    const int per = (S + RG - 1) / RG;
    const int s0 = g * per;
    const int s1 = min(S, s0 + per);
    double v[ROWS];
#pragma unroll
    for (int c = 0; c < ROWS; ++c) v[c] = 0.0;
    if (valid) {
#pragma unroll 4
        for (int s = s0; s < s1; ++s) {
            const float2* q = part + (int64_t)s * STRIDE * npad + i;
#pragma unroll
            for (int c = 0; c < ROWS; ++c) {
                const float2 x = q[c * npad];
                v[c] += (double)x.x;
                v[c] += (double)x.y;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < ROWS; ++c) sh[(g * ROWS + c) * RT + t] = v[c];
    __syncthreads();
    if (g == 0) {
#pragma unroll
        for (int c = 0; c < ROWS; ++c) {
            double a = sh[c * RT + t];
            for (int q = 1; q < RG; ++q) a += sh[(q * ROWS + c) * RT + t];
            out[c] = a;
        }
    }
    __syncthreads();
}

// Butterfly sum over the RT = 64 lanes of each wave of NV values (every lane of
// a wave gets its wave's sum; group 0, the first wave, holds the block's).
template <int NV>
__device__ inline void rt_sum(double (&v)[NV]) {
    static_assert(RT == 64, "one wave per group");
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], m, 64);
    }
}

// Forward reduction for targets [blockIdx.x RT, +RT) of one system: ared [3][n]
// = G x (slice sums), rec [4] = (sum m a_x, sum m a_y, sum m a_z, sum m) over
// the block's targets.  sh: at least 3 RG RT doubles.
__device__ inline void fwd_reduce_block(const float2* __restrict__ part, int S, int64_t npad,
                                        int64_t n, double G, const double* __restrict__ mass,
                                        double* __restrict__ ared, double* __restrict__ rec,
                                        double* sh) {
    const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x % RT;
    const bool valid = i < n;
    double a[3] = {0.0, 0.0, 0.0};
    slice_reduce<3, 3>(part, S, npad, i, valid, a, sh);
    double m = 0.0;
    if (threadIdx.x < RT && valid) {
        for (int c = 0; c < 3; ++c) {
            a[c] *= G;
            ared[c * n + i] = a[c];
        }
        m = mass[i];
    } else {
        a[0] = a[1] = a[2] = 0.0;
    }
    double v[4] = {m * a[0], m * a[1], m * a[2], m};
    rt_sum<4>(v);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) rec[4 * blockIdx.x + c] = v[c];
}

// Reverse reduction: gred [4][n] = (J^T w (3 rows), raw mass term) x G / S_w
// (S_w: the power-of-two scale the cotangent was staged with), rec [4] =
// (sum of the three J^T w rows over the block's targets, 0).
__device__ inline void vjp_reduce_block(const float2* __restrict__ part, int S, int64_t npad,
                                        int64_t n, double G, bool with_mass, double inv_s,
                                        double* __restrict__ gred, double* __restrict__ rec,
                                        double* sh) {
    const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x % RT;
    const bool valid = i < n;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (with_mass) {
        slice_reduce<4, 4>(part, S, npad, i, valid, g, sh);
    } else {
        double g3[3] = {0.0, 0.0, 0.0};
        slice_reduce<3, 4>(part, S, npad, i, valid, g3, sh);
        g[0] = g3[0]; g[1] = g3[1]; g[2] = g3[2];
    }
    if (threadIdx.x < RT && valid) {
        for (int c = 0; c < 4; ++c) {
            g[c] = (g[c] * G) * inv_s;
            if (c < 3 || with_mass) gred[c * n + i] = g[c];
        }
    } else {
        g[0] = g[1] = g[2] = 0.0;
    }
    double v[3] = {g[0], g[1], g[2]};
    rt_sum<3>(v);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) rec[4 * blockIdx.x + c] = v[c];
        rec[4 * blockIdx.x + 3] = 0.0;
    }
}

// The staging centre (as centre_from with extrapolation) and the sums of the nr
// net-force records (as rec_total) in one block reduction.
__device__ inline void centre_and_total(const double* __restrict__ cpart, int nb, int64_t n,
                                        const double* __restrict__ rec, int nr, double* sh,
                                        double& cx, double& cy, double& cz, double (&tot)[4]) {
    double v[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) v[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += BS) {
        v[0] += cpart[REC * b + 0];
        v[1] += cpart[REC * b + 1];
        v[2] += cpart[REC * b + 2];
        v[3] += cpart[REC * b + 4];
        v[4] += cpart[REC * b + 5];
        v[5] += cpart[REC * b + 6];
    }
    for (int b = threadIdx.x; b < nr; b += BS)
        for (int c = 0; c < 4; ++c) v[6 + c] += rec[4 * b + c];
    block_sum<10>(v, sh);
    const double inv = 1.0 / (double)n;
    cx = (v[0] + v[3]) * inv; cy = (v[1] + v[4]) * inv; cz = (v[2] + v[5]) * inv;
    for (int c = 0; c < 4; ++c) tot[c] = v[6 + c];
}

// Sum of the nr reduction records (fixed order; every thread gets it).
__device__ inline void rec_total(const double* __restrict__ rec, int nr, double* sh,
                                 double (&tot)[4]) {
    for (int c = 0; c < 4; ++c) tot[c] = 0.0;
    for (int b = threadIdx.x; b < nr; b += BS)
        for (int c = 0; c < 4; ++c) tot[c] += rec[4 * b + c];
    block_sum<4>(tot, sh);
}

}  // namespace dnb
