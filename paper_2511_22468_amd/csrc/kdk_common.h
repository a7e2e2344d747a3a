// Device code shared by the single-system and the batched O(N) kernels of the
// integrator and of its reverse sweep: staging of sources, the staging centre,
// the cotangent scale, and the sums of the pair kernels' slice partials.
#pragma once

#include "dnb_internal.h"

namespace dnb {

constexpr float FAR32 = 1.0e18f;
constexpr double FAR64 = 1.0e150;

__device__ inline void centre_from(const double* __restrict__ cpart, int nb, int64_t n, double* sh,
                                   double& cx, double& cy, double& cz) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += BS) {
        v[0] += cpart[4 * b + 0];
        v[1] += cpart[4 * b + 1];
        v[2] += cpart[4 * b + 2];
    }
    block_sum<3>(v, sh);
    const double inv = 1.0 / (double)n;
    cx = v[0] * inv; cy = v[1] * inv; cz = v[2] * inv;
}

__device__ inline void write_block_sums(double x, double y, double z, bool valid, double* sh,
                                        double* __restrict__ cpart_out) {
    double v[3] = {valid ? x : 0.0, valid ? y : 0.0, valid ? z : 0.0};
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        cpart_out[4 * blockIdx.x + 0] = v[0];
        cpart_out[4 * blockIdx.x + 1] = v[1];
        cpart_out[4 * blockIdx.x + 2] = v[2];
        cpart_out[4 * blockIdx.x + 3] = 0.0;
    }
}

// Cotangent scaling (FP32C reverse sweep).  Over long horizons the velocity
// cotangent of a chaotic system grows without bound (1e45 after 2000 steps is
// typical) and would overflow FP32.  The cotangent is therefore staged as w * S
// with S a power of two (exact) chosen so that max |w S| is about 1; the pair VJP
// is linear in w, so the consumer divides the slice sums by S in FP64.  S is
// taken from the block maxima of the previous cotangent (slot 3 of the
// block-sum records), which differs from the staged one by one drift update.
__device__ inline double absmax3(double a, double b, double c) {
    return fmax(fabs(a), fmax(fabs(b), fabs(c)));
}

__device__ inline void write_block_max(double v, double* sh, double* __restrict__ cpart_out) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) cpart_out[4 * blockIdx.x + 3] = sh[0];
    __syncthreads();
}

// Power-of-two scale from the block maxima in slot 3 of cpart (1 if all zero).
__device__ inline double scale_from(const double* __restrict__ cpart, int nb, double* sh) {
    double m = 0.0;
    for (int b = threadIdx.x; b < nb; b += BS) m = fmax(m, cpart[4 * b + 3]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    m = sh[0];
    __syncthreads();
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

}  // namespace dnb
