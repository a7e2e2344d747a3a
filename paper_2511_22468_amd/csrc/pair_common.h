// Device code shared by the single-system and the batched pair kernels: the
// slice sums of the forward pair kernel and of the pair VJP.
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

// Stores one slice partial (hi, lo).  With NT the store is non-temporal: the
// partial streams out to memory instead of staying dirty in L2 until the kernel
// ends, when the whole launch's partials would be written back at once (that
// drain cost 3-5 us per launch at n = 8192).  A small launch keeps plain stores:
// its partials are few, and the reduction that follows reads them from L2.
// (A compile-time choice: with a run-time flag the compiler merges the two
// stores into one plain store.)
template <bool NT>
__device__ __forceinline__ void put_partial(float2* p, float h, float l) {
    if (NT) {
        __builtin_nontemporal_store(h, &p->x);
        __builtin_nontemporal_store(l, &p->y);
    } else {
        *p = make_float2(h, l);
    }
}

// Launch-wide bytes of slice partials from which the stores are non-temporal.
constexpr int64_t NT_PARTIAL_BYTES = int64_t(2) << 20;

// Start index of the batch loaded ahead of batch k of a sub-tile that starts at
// jt and holds kend sources (SUBTILE, or fewer at the end of a short slice); on
// the last batch of the slice it re-reads the slice's last batch (in bounds).
__device__ __forceinline__ int next_batch(int jt, int k, int PB, int kend, int j1) {
    return (k + PB < kend) ? jt + k + PB : min(jt + SUBTILE, j1 - PB);
}

// One pair of the forward slice sum: source q (position, mass) at index j onto
// target i at me, accumulated into (ax, ay, az).
template <bool EPS0, bool UNI>
__device__ __forceinline__ void fwd_f32c_pair(float4 q, int j, int i, float eps2, float4 me,
                                              float& ax, float& ay, float& az) {
    const float dx = q.x - me.x, dy = q.y - me.y, dz = q.z - me.z;
    const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float r = __builtin_amdgcn_rsqf(s);
    float w = UNI ? (r * r) * r : (q.w * r) * (r * r);
    if (EPS0) w = (j == i) ? 0.f : w;
    ax = fmaf(w, dx, ax);
    ay = fmaf(w, dy, ay);
    az = fmaf(w, dz, az);
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
        const int kend = min(SUBTILE, j1 - jt);
        for (int k = 0; k < kend; k += PB) {
            const int nx = next_batch(jt, k, PB, kend, j1);
            float4 qb[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) qb[u] = js[nx + u];
#pragma unroll
            for (int u = 0; u < PB; ++u)
                fwd_f32c_pair<EPS0, UNI>(qa[u], jt + k + u, i, eps2, me, ax, ay, az);
#pragma unroll
            for (int u = 0; u < PB; ++u) qa[u] = qb[u];
        }
        two_sum_acc(h[0], l[0], ax);
        two_sum_acc(h[1], l[1], ay);
        two_sum_acc(h[2], l[2], az);
    }
}

// The same sum with the slice's sources held in LDS (lds[j - j0] is source j):
// the same pairs in the same order, so the result is bit for bit that of
// fwd_f32c_slice.  The reads are LDS broadcasts issued at the top of each batch
// of 4; other waves cover their latency, so no batch is held in registers ahead
// of use.
template <bool EPS0, bool UNI>
__device__ __forceinline__ void fwd_f32c_slice_lds(const float4* lds, int i, int j0, int j1,
                                                   float eps2, float4 me, float (&h)[3],
                                                   float (&l)[3]) {
    constexpr int PB = 4;
    for (int jt = j0; jt < j1; jt += SUBTILE) {
        float ax = 0.f, ay = 0.f, az = 0.f;
        const int kend = min(SUBTILE, j1 - jt);
        for (int k = 0; k < kend; k += PB) {
            float4 q[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) q[u] = lds[jt - j0 + k + u];
#pragma unroll
            for (int u = 0; u < PB; ++u)
                fwd_f32c_pair<EPS0, UNI>(q[u], jt + k + u, i, eps2, me, ax, ay, az);
        }
        two_sum_acc(h[0], l[0], ax);
        two_sum_acc(h[1], l[1], ay);
        two_sum_acc(h[2], l[2], az);
    }
}

// For target k and cotangent w, with d = x_j - x_k, s = |d|^2 + eps^2:
//   (J^T w)_k / G = sum_j [s^-3/2 u - 3 s^-5/2 (d.u) d],  u = m_k w_j - m_j w_k
//   gm_k / G      = sum_j (d.w_j) s^-3/2          (mass cotangent, negated later)
// Without FORCE the internal acceleration the dt and mass-scale terms need is not
// summed here: the forward pass stores it with the tape.
// jsv: interleaved [2 j] = (x, y, z, m), [2 j + 1] = (wx, wy, wz, 0), padded.
// part: [S][4][npad] float2 = (hi, lo) of the three J^T w components and of gm.
// The two terms of J^T w are accumulated apart (A = sum s^-3/2 u,
// B = sum s^-5/2 (d.u) d) and combined as A - 3 B once per sub-tile, which takes
// the factor -3 out of the pair loop.  With UNI (all masses equal to m)
// u = m (w_j - w_k): the mass leaves the pair term and is applied once per
// target, 22 VALU operations and one v_rsq_f32 per pair.
//
// With FORCE the pair term of the internal acceleration at the same positions,
// m_j d s^-3/2 (m_j left out with UNI), is summed into F as well: three more FMA
// operations on the s^-3/2 the VJP already has.  The reverse sweep that rebuilds
// the trajectory by stepping backward needs a(x_k) exactly where it evaluates
// J(x_k)^T w.
template <bool EPS0, bool MASS, bool UNI, bool FORCE = false>
__device__ __forceinline__ void vjp_f32c_pair(float4 q, float4 qw, int j, int i, float eps2,
                                              float4 me, float4 mw, float (&A)[3],
                                              float (&B)[3], float& gm, float (&F)[3]) {
    const float dx = q.x - me.x, dy = q.y - me.y, dz = q.z - me.z;
    const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    float r = __builtin_amdgcn_rsqf(s);
    if (EPS0) r = (j == i) ? 0.f : r;
    const float r2 = r * r;
    const float r3 = r2 * r;
    const float r5 = r3 * r2;
    const float ux = UNI ? qw.x - mw.x : fmaf(me.w, qw.x, -(q.w * mw.x));
    const float uy = UNI ? qw.y - mw.y : fmaf(me.w, qw.y, -(q.w * mw.y));
    const float uz = UNI ? qw.z - mw.z : fmaf(me.w, qw.z, -(q.w * mw.z));
    const float t = r5 * fmaf(dx, ux, fmaf(dy, uy, dz * uz));
    A[0] = fmaf(r3, ux, A[0]);
    A[1] = fmaf(r3, uy, A[1]);
    A[2] = fmaf(r3, uz, A[2]);
    B[0] = fmaf(t, dx, B[0]);
    B[1] = fmaf(t, dy, B[1]);
    B[2] = fmaf(t, dz, B[2]);
    if (MASS) gm = fmaf(fmaf(dx, qw.x, fmaf(dy, qw.y, dz * qw.z)), r3, gm);
    if (FORCE) {
        const float wf = UNI ? r3 : q.w * r3;
        F[0] = fmaf(wf, dx, F[0]);
        F[1] = fmaf(wf, dy, F[1]);
        F[2] = fmaf(wf, dz, F[2]);
    }
}

// h, l: (hi, lo) of J^T w (0..2), gm (3) and, with FORCE, the acceleration
// (4..6).
template <bool EPS0, bool MASS, bool UNI, bool FORCE = false, int NH>
__device__ __forceinline__ void vjp_f32c_slice(const float4* __restrict__ jsv, int i, int j0,
                                               int j1, float eps2, float4 me, float4 mw,
                                               float (&h)[NH], float (&l)[NH]) {
    static_assert(NH >= (FORCE ? 7 : 4), "slice sums need 4 (hi, lo) pairs, 7 with FORCE");
    constexpr int PB = 4;
    float4 pa[PB], wa[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) { pa[u] = jsv[2 * (j0 + u)]; wa[u] = jsv[2 * (j0 + u) + 1]; }
    for (int jt = j0; jt < j1; jt += SUBTILE) {
        float A[3] = {0.f, 0.f, 0.f}, B[3] = {0.f, 0.f, 0.f}, gm = 0.f;
        float F[3] = {0.f, 0.f, 0.f};
        const int kend = min(SUBTILE, j1 - jt);
        for (int k = 0; k < kend; k += PB) {
            const int nx = next_batch(jt, k, PB, kend, j1);
            float4 pb[PB], wb[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) { pb[u] = jsv[2 * (nx + u)]; wb[u] = jsv[2 * (nx + u) + 1]; }
#pragma unroll
            for (int u = 0; u < PB; ++u)
                vjp_f32c_pair<EPS0, MASS, UNI, FORCE>(pa[u], wa[u], jt + k + u, i, eps2, me, mw,
                                                      A, B, gm, F);
#pragma unroll
            for (int u = 0; u < PB; ++u) { pa[u] = pb[u]; wa[u] = wb[u]; }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) two_sum_acc(h[c], l[c], fmaf(-3.f, B[c], A[c]));
        if (MASS) two_sum_acc(h[3], l[3], gm);
        if (FORCE) {
#pragma unroll
            for (int c = 0; c < 3; ++c) two_sum_acc(h[4 + c], l[4 + c], F[c]);
        }
    }
}

// The same sum with the slice's interleaved sources held in LDS (lds[2 (j - j0)]
// and lds[2 (j - j0) + 1] are those of source j): the same pairs in the same
// order, bit for bit the result of vjp_f32c_slice, with the reads issued at the
// top of each batch rather than one batch ahead.
template <bool EPS0, bool MASS, bool UNI, bool FORCE = false, int NH>
__device__ __forceinline__ void vjp_f32c_slice_lds(const float4* lds, int i, int j0, int j1,
                                                   float eps2, float4 me, float4 mw,
                                                   float (&h)[NH], float (&l)[NH]) {
    static_assert(NH >= (FORCE ? 7 : 4), "slice sums need 4 (hi, lo) pairs, 7 with FORCE");
    constexpr int PB = 4;
    for (int jt = j0; jt < j1; jt += SUBTILE) {
        float A[3] = {0.f, 0.f, 0.f}, B[3] = {0.f, 0.f, 0.f}, gm = 0.f;
        float F[3] = {0.f, 0.f, 0.f};
        const int kend = min(SUBTILE, j1 - jt);
        for (int k = 0; k < kend; k += PB) {
            float4 q[PB], qw[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                q[u] = lds[2 * (jt - j0 + k + u)];
                qw[u] = lds[2 * (jt - j0 + k + u) + 1];
            }
#pragma unroll
            for (int u = 0; u < PB; ++u)
                vjp_f32c_pair<EPS0, MASS, UNI, FORCE>(q[u], qw[u], jt + k + u, i, eps2, me, mw, A,
                                                      B, gm, F);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) two_sum_acc(h[c], l[c], fmaf(-3.f, B[c], A[c]));
        if (MASS) two_sum_acc(h[3], l[3], gm);
        if (FORCE) {
#pragma unroll
            for (int c = 0; c < 3; ++c) two_sum_acc(h[4 + c], l[4 + c], F[c]);
        }
    }
}

}  // namespace dnb
