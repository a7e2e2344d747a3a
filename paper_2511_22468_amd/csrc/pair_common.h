// Device code shared by the single-system and the batched pair kernels.
#pragma once

#include "dnb_internal.h"

namespace dnb {

// Error-free addition of x to the (hi, lo) pair (Knuth's TwoSum).
__device__ __forceinline__ void two_sum_acc(float& hi, float& lo, float x) {
    float s = hi + x;
    float bp = s - hi;
    float e = (hi - (s - bp)) + (x - bp);
    hi = s;
    lo += e;
}

// Start index of the batch loaded ahead of batch k of a sub-tile starting at jt;
// on the last batch of the slice it re-reads the slice's last batch (in bounds).
__device__ __forceinline__ int next_batch(int jt, int k, int PB, int j1) {
    return (k + PB < SUBTILE) ? jt + k + PB : min(jt + SUBTILE, j1 - PB);
}

// Sum over the slice [j0, j1) of the staged sources js for target i (position
// me) into the (hi, lo) pairs: plain FP32 within sub-tiles of 128 sources, TwoSum
// across them.  Sources are read with wave-uniform addresses (scalar loads), one
// batch of 4 ahead of use.  With UNI (all masses equal) the mass is left out of
// the pair term and applied once by the caller: 11 VALU operations and one
// v_rsq_f32 per pair instead of 12.
template <bool EPS0, bool UNI>
__device__ __forceinline__ void fwd_f32c_slice(const float4* __restrict__ js, int i, int j0,
                                               int j1, float eps2, float4 me, float (&h)[3],
                                               float (&l)[3]) {
    constexpr int PB = 4;
    float4 qa[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) qa[u] = js[j0 + u];
    for (int jt = j0; jt < j1; jt += SUBTILE) {
        float ax = 0.f, ay = 0.f, az = 0.f;
        for (int k = 0; k < SUBTILE; k += PB) {
            const int nx = next_batch(jt, k, PB, j1);
            float4 qb[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) qb[u] = js[nx + u];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const float4 q = qa[u];
                const float dx = q.x - me.x, dy = q.y - me.y, dz = q.z - me.z;
                const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                const float r = __builtin_amdgcn_rsqf(s);
                float w = UNI ? (r * r) * r : (q.w * r) * (r * r);
                if (EPS0) w = (jt + k + u == i) ? 0.f : w;
                ax = fmaf(w, dx, ax);
                ay = fmaf(w, dy, ay);
                az = fmaf(w, dz, az);
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) qa[u] = qb[u];
        }
        two_sum_acc(h[0], l[0], ax);
        two_sum_acc(h[1], l[1], ay);
        two_sum_acc(h[2], l[2], az);
    }
}

}  // namespace dnb
