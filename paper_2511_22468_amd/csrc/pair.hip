// O(N^2) kernels: the softened pairwise gravity sum (Sec. 1, direct pairwise
// forces with softening) and its vector-Jacobian product (Sec. 2: reverse-mode
// gradients through the simulation).
//
// Layout.  A launch is a grid of (target blocks) x (source slices).  Each
// 256-thread block owns 256 targets (one per lane) and one contiguous slice of
// sources.  Every lane of a wave needs the same source at the same time, so the
// sources are read with wave-uniform addresses: the compiler turns these into
// scalar loads (s_load_dwordx8/x16 through the scalar cache) and the VALU
// instructions take the source coordinates straight from SGPRs.  No LDS, no
// barriers, and the source data costs no VGPRs.  Sources are read in batches,
// one batch ahead of use, so the scalar-load latency overlaps the arithmetic of
// the current batch.  The staged source arrays are padded with far-away
// zero-mass particles to a multiple of 128, so every batch is whole and in
// bounds.
//
// Each block writes per-target partial sums for its slice; the O(N) kernel that
// consumes them adds the slices in FP64 in slice order, so results are
// deterministic and independent of scheduling.  No floating-point atomics.
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
#include "pair_common.h"

namespace dnb {


__device__ __forceinline__ double rsqrt_f64(double s) {
    double y = __builtin_amdgcn_rsq(s);
    double hs = 0.5 * s;
    y = y * fma(-hs * y, y, 1.5);
    y = y * fma(-hs * y, y, 1.5);
    return y;
}


// ------------------------------------------------------- external-field row --
// The row is added only if the launch's blocks still fit in one round of
// resident blocks (256 CUs x 8 blocks of 256 threads): a launch that fills the
// chip (n = 8192: 32 x 64 blocks) would push pair blocks into a second round and
// lose more than the kick saves.
constexpr int RESIDENT_BLOCKS = 256 * 8;
inline bool ext_row_fits(const Slicing& sl) {
    return (int64_t)sl.nblk * (sl.S + 1) <= RESIDENT_BLOCKS;
}

// The blocks of an ExtRow (see dnb_internal.h), the launch's first row of blocks
// (blockIdx.y = 0; the slices follow), so that their FP64 work starts with the
// launch instead of waiting for a free slot behind the pair blocks: particles
// [blockIdx.x BS, +BS).
__device__ inline void ext_row_fwd(const ExtRow& er, int n, double* __restrict__ out) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const double* x = er.x;
    const Ext e = ext_accel(er.pot, x[i], x[n + i], x[2 * n + i]);
    out[i] = e.ax; out[n + i] = e.ay; out[2 * n + i] = e.az;
}

__device__ inline void ext_row_vjp(const ExtRow& er, int n, double* __restrict__ out) {
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const double* x = er.x;
    const double* w = er.w;
    const double wx = w[i], wy = w[n + i], wz = w[2 * n + i];
    Ext e;
    double hx, hy, hz, shp[3];
    ext_accel_hvp(er.pot, x[i], x[n + i], x[2 * n + i], wx, wy, wz, e, hx, hy, hz, shp);
    const double r[9] = {hx, hy, hz, e.ax * wx + e.ay * wy + e.az * wz,
                         e.nx * wx + e.ny * wy + e.nz * wz, e.mx * wx + e.my * wy + e.mz * wz,
                         shp[0], shp[1], shp[2]};
#pragma unroll
    for (int c = 0; c < 9; ++c) out[(int64_t)c * n + i] = r[c];
}

// ------------------------------------------------------------ forward FP32C --
// js: staged sources (x, y, z, m), padded to nj = roundup(n, 128).
// part: [S][3][npad] float2 = (hi, lo) of the x, y and z components of
// sum_j m_j d_ij s_ij^-3/2 over the block's slice (one 8-byte store per
// component, one 8-byte load for the consumer).
// muni: [flag, m] -- flag != 0 when every particle has mass m (set per call by
// k_mass_info); the branch on it is uniform over the grid.
//
// Short slices (a system of up to some 16k particles, cut into many slices so
// that the launch still fills the chip) are latency-bound: a block runs a few
// hundred pairs per lane, and each scalar-load batch waits on the scalar
// cache.  With LDS the block first copies its slice into LDS (one coalesced
// load per lane), and every batch is then an LDS broadcast.  A long slice keeps
// the scalar loads: an LDS broadcast of 16 bytes to 64 lanes takes the LDS
// several cycles, which at full occupancy competes with the arithmetic, while
// scalar loads cost the vector units nothing.  Both give the same bits.
constexpr int FWD_LDS_SLICE = 256;   // longest slice that takes the LDS kernel

template <bool EPS0, bool LDS, bool NT, bool ROW>
__global__ __launch_bounds__(BS) void k_pair_fwd_f32c(const float4* __restrict__ js, int n,
                                                      int i0, int iend, int nj, int jslice,
                                                      float eps2, float* __restrict__ part,
                                                      int64_t npad,
                                                      const float* __restrict__ muni,
                                                      ExtRow er, double* __restrict__ aext,
                                                      int smaj) {
    if (ROW && blockIdx.y == 0) {   // the external-field row, first so it starts at once
        ext_row_fwd(er, n, aext);
        return;
    }
    // smaj: the grid is (slices, target blocks), so that consecutive blocks, which
    // the dispatcher spreads over the compute units, share their sources
    const int tb = smaj ? blockIdx.y : blockIdx.x;
    const int i = i0 + tb * BS + threadIdx.x;
    const int sy = smaj ? blockIdx.x : blockIdx.y - (ROW ? 1 : 0);   // source slice
    const int j0 = sy * jslice;
    const int j1 = min(nj, j0 + jslice);
    const float4 me = js[min(i, n - 1)];
    float h[3] = {0.f, 0.f, 0.f}, l[3] = {0.f, 0.f, 0.f};
    if (LDS) {
        __shared__ float4 lds[FWD_LDS_SLICE];
        const int jl = min(j1, j0 + FWD_LDS_SLICE);   // the launcher keeps j1 - j0 within it
        for (int t = threadIdx.x; t < jl - j0; t += BS) lds[t] = js[j0 + t];
        __syncthreads();
        if (muni[0] != 0.f) {
            fwd_f32c_slice_lds<EPS0, true>(lds, i, j0, jl, eps2, me, h, l);
            const float m = muni[1];
#pragma unroll
            for (int c = 0; c < 3; ++c) { h[c] *= m; l[c] *= m; }
        } else {
            fwd_f32c_slice_lds<EPS0, false>(lds, i, j0, jl, eps2, me, h, l);
        }
    } else if (muni[0] != 0.f) {
        fwd_f32c_slice<EPS0, true>(js, i, j0, j1, eps2, me, h, l);
        const float m = muni[1];
#pragma unroll
        for (int c = 0; c < 3; ++c) { h[c] *= m; l[c] *= m; }
    } else {
        fwd_f32c_slice<EPS0, false>(js, i, j0, j1, eps2, me, h, l);
    }
    if (i < iend) {
        float2* p = (float2*)part + (int64_t)sy * 3 * npad + (i - i0);
#pragma unroll
        for (int c = 0; c < 3; ++c) put_partial<NT>(p + c * npad, h[c], l[c]);
    }
}

// ------------------------------------------------------------- forward FP64 --
// js: staged sources (x, y, z, m) in FP64, padded like the FP32C array.
// part: [S][3][npad] doubles.
template <bool EPS0>
__global__ __launch_bounds__(BS) void k_pair_fwd_f64(const double4* __restrict__ js, int n,
                                                     int i0, int iend, int nj, int jslice,
                                                     double eps2, double* __restrict__ part,
                                                     int64_t npad, int smaj) {
    constexpr int PB = 4;
    const int tb = smaj ? blockIdx.y : blockIdx.x;   // grid (slices, target blocks) with smaj
    const int sy = smaj ? blockIdx.x : blockIdx.y;
    const int i = i0 + tb * BS + threadIdx.x;
    const int j0 = sy * jslice;
    const int j1 = min(nj, j0 + jslice);
    const double4 me = js[min(i, n - 1)];
    double ax = 0.0, ay = 0.0, az = 0.0;
    double4 qa[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) qa[u] = js[j0 + u];
    for (int jt = j0; jt < j1; jt += SUBTILE) {
        const int kend = min(SUBTILE, j1 - jt);
        for (int k = 0; k < kend; k += PB) {
            const int nx = next_batch(jt, k, PB, kend, j1);
            double4 qb[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) qb[u] = js[nx + u];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const double4 q = qa[u];
                const double dx = q.x - me.x, dy = q.y - me.y, dz = q.z - me.z;
                const double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                const double r = rsqrt_f64(s);
                double w = (q.w * r) * (r * r);
                if (EPS0) w = (jt + k + u == i) ? 0.0 : w;
                ax = fma(w, dx, ax);
                ay = fma(w, dy, ay);
                az = fma(w, dz, az);
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) qa[u] = qb[u];
        }
    }
    if (i < iend) {
        double* p = part + (int64_t)sy * 3 * npad + (i - i0);
        p[0] = ax; p[npad] = ay; p[2 * npad] = az;
    }
}

// --------------------------------------------------------------- VJP FP32C --
// The slice sum is vjp_f32c_slice (pair_common.h); with LDS the block first
// copies its slice (two float4 per source) into LDS, as in the forward kernel.
constexpr int VJP_LDS_SLICE = 64;    // longest slice that takes the LDS kernel

//
// With FORCE the launch also sums the internal acceleration at the staged
// positions (the reverse sweep that steps the trajectory backward): its slice
// partials go to partf in the layout of the forward pair kernel's, [S][3][npad]
// float2, so that the forward reduction sums them.
template <bool EPS0, bool MASS, bool LDS, bool NT, bool ROW, bool FORCE>
__global__ __launch_bounds__(BS) void k_pair_vjp_f32c(const float4* __restrict__ jsv, int n,
                                                      int i0, int iend, int nj, int jslice,
                                                      float eps2, float* __restrict__ part,
                                                      int64_t npad,
                                                      const float* __restrict__ muni,
                                                      ExtRow er, double* __restrict__ aext,
                                                      float* __restrict__ partf, int smaj) {
    static_assert(!(ROW && FORCE), "the external-field row and FORCE are not combined");
    if (ROW && blockIdx.y == 0) {   // the external-field row, first so it starts at once
        ext_row_vjp(er, n, aext);
        return;
    }
    constexpr int NH = FORCE ? 7 : 4;
    const int tb = smaj ? blockIdx.y : blockIdx.x;   // grid (slices, target blocks) with smaj
    const int i = i0 + tb * BS + threadIdx.x;
    const int sy = smaj ? blockIdx.x : blockIdx.y - (ROW ? 1 : 0);   // source slice
    const int j0 = sy * jslice;
    const int j1 = min(nj, j0 + jslice);
    const int ii = min(i, n - 1);
    const float4 me = jsv[2 * ii];
    const float4 mw = jsv[2 * ii + 1];
    float h[NH], l[NH];
#pragma unroll
    for (int c = 0; c < NH; ++c) { h[c] = 0.f; l[c] = 0.f; }
    bool uni = false;
    if (LDS) {
        __shared__ float4 lds[2 * VJP_LDS_SLICE];
        const int jl = min(j1, j0 + VJP_LDS_SLICE);   // the launcher keeps j1 - j0 within it
        for (int t = threadIdx.x; t < 2 * (jl - j0); t += BS) lds[t] = jsv[2 * j0 + t];
        __syncthreads();
        if (muni[0] != 0.f) {
            vjp_f32c_slice_lds<EPS0, MASS, true, FORCE>(lds, i, j0, jl, eps2, me, mw, h, l);
            uni = true;
        } else {
            vjp_f32c_slice_lds<EPS0, MASS, false, FORCE>(lds, i, j0, jl, eps2, me, mw, h, l);
        }
    } else if (muni[0] != 0.f) {
        vjp_f32c_slice<EPS0, MASS, true, FORCE>(jsv, i, j0, j1, eps2, me, mw, h, l);
        uni = true;
    } else {
        vjp_f32c_slice<EPS0, MASS, false, FORCE>(jsv, i, j0, j1, eps2, me, mw, h, l);
    }
    if (uni) {   // the common mass left out of the pair terms
        const float m = muni[1];
#pragma unroll
        for (int c = 0; c < 3; ++c) { h[c] *= m; l[c] *= m; }
        if (FORCE) {
#pragma unroll
            for (int c = 4; c < 7; ++c) { h[c] *= m; l[c] *= m; }
        }
    }
    if (i < iend) {
        float2* p = (float2*)part + (int64_t)sy * 4 * npad + (i - i0);
#pragma unroll
        for (int c = 0; c < 3; ++c) put_partial<NT>(p + c * npad, h[c], l[c]);
        if (MASS) put_partial<NT>(p + 3 * npad, h[3], l[3]);
        if (FORCE) {
            float2* pf = (float2*)partf + (int64_t)sy * 3 * npad + (i - i0);
#pragma unroll
            for (int c = 0; c < 3; ++c) put_partial<NT>(pf + c * npad, h[4 + c], l[4 + c]);
        }
    }
}

// ---------------------------------------------------------------- VJP FP64 --
// jsv: interleaved double4 [2 j] = (x, y, z, m), [2 j + 1] = (w, 0), padded.
// part: [S][4][npad] doubles: JTw(3), gm.
// FORCE: the internal acceleration at the staged positions as well, into partf
// [S][3][npad] doubles (the forward pair kernel's layout), with the forward
// kernel's expressions in its source order, so that at the same positions the
// partials are those of the forward kernel bit for bit.
template <bool EPS0, bool MASS, bool FORCE>
__global__ __launch_bounds__(BS) void k_pair_vjp_f64(const double4* __restrict__ jsv, int n,
                                                     int i0, int iend, int nj, int jslice,
                                                     double eps2, double* __restrict__ part,
                                                     int64_t npad, double* __restrict__ partf,
                                                     int smaj) {
    constexpr int PB = 2;
    const int tb = smaj ? blockIdx.y : blockIdx.x;   // grid (slices, target blocks) with smaj
    const int sy = smaj ? blockIdx.x : blockIdx.y;
    const int i = i0 + tb * BS + threadIdx.x;
    const int j0 = sy * jslice;
    const int j1 = min(nj, j0 + jslice);
    const int ii = min(i, n - 1);
    const double4 me = jsv[2 * ii];
    const double4 mw = jsv[2 * ii + 1];
    double acc[4] = {0, 0, 0, 0};
    double f[3] = {0, 0, 0};
    double4 pa[PB], wa[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) { pa[u] = jsv[2 * (j0 + u)]; wa[u] = jsv[2 * (j0 + u) + 1]; }
    for (int jt = j0; jt < j1; jt += SUBTILE) {
        const int kend = min(SUBTILE, j1 - jt);
        for (int k = 0; k < kend; k += PB) {
            const int nx = next_batch(jt, k, PB, kend, j1);
            double4 pb[PB], wb[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) { pb[u] = jsv[2 * (nx + u)]; wb[u] = jsv[2 * (nx + u) + 1]; }
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const double4 q = pa[u];
                const double4 qw = wa[u];
                const double dx = q.x - me.x, dy = q.y - me.y, dz = q.z - me.z;
                const double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                double r = rsqrt_f64(s);
                if (EPS0) r = (jt + k + u == i) ? 0.0 : r;
                const double r2 = r * r;
                const double r3 = r2 * r;
                const double r5 = r3 * r2;
                const double ux = fma(me.w, qw.x, -(q.w * mw.x));
                const double uy = fma(me.w, qw.y, -(q.w * mw.y));
                const double uz = fma(me.w, qw.z, -(q.w * mw.z));
                const double du = fma(dx, ux, fma(dy, uy, dz * uz));
                const double c3 = -3.0 * (r5 * du);
                acc[0] = fma(c3, dx, fma(r3, ux, acc[0]));
                acc[1] = fma(c3, dy, fma(r3, uy, acc[1]));
                acc[2] = fma(c3, dz, fma(r3, uz, acc[2]));
                if (MASS) {
                    const double dw = fma(dx, qw.x, fma(dy, qw.y, dz * qw.z));
                    acc[3] = fma(dw, r3, acc[3]);
                }
                if (FORCE) {
                    const double wf = (q.w * r) * r2;
                    f[0] = fma(wf, dx, f[0]);
                    f[1] = fma(wf, dy, f[1]);
                    f[2] = fma(wf, dz, f[2]);
                }
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) { pa[u] = pb[u]; wa[u] = wb[u]; }
        }
    }
    if (i < iend) {
        double* p = part + (int64_t)sy * 4 * npad + (i - i0);
#pragma unroll
        for (int c = 0; c < 3; ++c) p[c * npad] = acc[c];
        if (MASS) p[3 * npad] = acc[3];
        if (FORCE) {
            double* pf = partf + (int64_t)sy * 3 * npad + (i - i0);
#pragma unroll
            for (int c = 0; c < 3; ++c) pf[c * npad] = f[c];
        }
    }
}

// ---------------------------------------------------------------- launchers --
// Targets [i0, i0 + ni) against all n staged sources with the slicing sl; slice
// partials of target i at row i - i0 (the whole system: i0 = 0, ni = n).
static hipError_t launch_pair_fwd_sliced(dnb_ctx* c, int64_t n, int64_t i0, int64_t ni,
                                         const Slicing& sl, double eps, hipStream_t st,
                                         const ExtRow& er = ExtRow{}, bool* ext_done = nullptr) {
    if (ext_done) *ext_done = false;
    const int nj = (int)pad_sources(n);
    const int a = (int)i0, e = (int)(i0 + ni);
    dim3 grid(sl.nblk, sl.S);
    if (c->prec == DNB_FP32C) {
        const float eps2 = (float)(eps * eps);
        const float4* js = (const float4*)c->js;
        float* part = (float*)c->part;
        const bool lds = sl.jslice <= FWD_LDS_SLICE;
        const bool nt = (int64_t)sl.S * sl.npad * 3 * 8 >= NT_PARTIAL_BYTES;
        // the external-field row (whole-system launches, so the row blocks cover n;
        // the LDS instances, those of small systems, only; and only while the launch
        // stays within one round of resident blocks)
        const bool row = c->ext_row && er.x && i0 == 0 && ni == n && lds && ext_row_fits(sl);
        if (row) grid.y += 1;
        if (ext_done) *ext_done = row;
        // (slices, target blocks) order, see dnb_ctx::slice_major
        const int smaj = (c->slice_major && !row && sl.nblk <= 65535) ? 1 : 0;
        const dim3 grid32 = smaj ? dim3(sl.S, sl.nblk) : grid;
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, grid32, dim3(BS), 0, st, js, (int)n, a, e, nj, sl.jslice,
                               eps2, part, sl.npad, c->muni, row ? er : ExtRow{}, c->aext_f,
                               smaj);
        };
        const int which = (eps == 0.0 ? 8 : 0) + (lds ? 4 : 0) + (nt ? 2 : 0) + (row ? 1 : 0);
        switch (which) {
            case 0: go(k_pair_fwd_f32c<false, false, false, false>); break;
            case 2: go(k_pair_fwd_f32c<false, false, true, false>); break;
            case 4: go(k_pair_fwd_f32c<false, true, false, false>); break;
            case 5: go(k_pair_fwd_f32c<false, true, false, true>); break;
            case 6: go(k_pair_fwd_f32c<false, true, true, false>); break;
            case 7: go(k_pair_fwd_f32c<false, true, true, true>); break;
            case 8: go(k_pair_fwd_f32c<true, false, false, false>); break;
            case 10: go(k_pair_fwd_f32c<true, false, true, false>); break;
            case 12: go(k_pair_fwd_f32c<true, true, false, false>); break;
            case 13: go(k_pair_fwd_f32c<true, true, false, true>); break;
            case 14: go(k_pair_fwd_f32c<true, true, true, false>); break;
            default: go(k_pair_fwd_f32c<true, true, true, true>); break;   // 15
        }
    } else {
        const double eps2 = eps * eps;
        const double4* js = (const double4*)c->js;
        const int smaj = (c->slice_major && sl.nblk <= 65535) ? 1 : 0;
        const dim3 grid64 = smaj ? dim3(sl.S, sl.nblk) : grid;
        if (eps == 0.0)
            hipLaunchKernelGGL(k_pair_fwd_f64<true>, grid64, dim3(BS), 0, st, js, (int)n, a, e,
                               nj, sl.jslice, eps2, (double*)c->part, sl.npad, smaj);
        else
            hipLaunchKernelGGL(k_pair_fwd_f64<false>, grid64, dim3(BS), 0, st, js, (int)n, a, e,
                               nj, sl.jslice, eps2, (double*)c->part, sl.npad, smaj);
    }
    return hipGetLastError();
}

hipError_t launch_pair_fwd(dnb_ctx* c, int64_t n, double eps, hipStream_t st,
                           const ExtRow& ext, bool* ext_done) {
    return launch_pair_fwd_sliced(c, n, 0, n, fwd_slicing(c, n), eps, st, ext, ext_done);
}

hipError_t launch_pair_fwd_rows(dnb_ctx* c, int64_t n, int64_t i0, int64_t ni, double eps,
                                hipStream_t st) {
    return launch_pair_fwd_sliced(c, n, i0, ni, rows_slicing(c, ni, n), eps, st);
}

template <bool EPS0, bool MASS>
static void vjp_dispatch(dnb_ctx* c, const Slicing& sl, int64_t n, int i0, int iend, int nj,
                         double eps2, hipStream_t st, const ExtRow& er, bool* ext_done,
                         bool force) {
    dim3 grid(sl.nblk, sl.S);
    const int comps = (MASS ? 4 : 3) + (force ? 3 : 0);
    const bool nt = (int64_t)sl.S * sl.npad * comps * 8 >= NT_PARTIAL_BYTES;
    const bool lds = sl.jslice <= VJP_LDS_SLICE;
    // the external-field row (whole-system launches, so the row blocks cover n;
    // the LDS instances, those of small systems, only; and only while the launch
    // stays within one round of resident blocks); not with the acceleration sum,
    // whose caller needs the external acceleration itself, which the row does not
    // return
    const bool row = !force && c->prec == DNB_FP32C && c->ext_row && er.x && i0 == 0 &&
                     iend == n && lds && ext_row_fits(sl);
    if (row) grid.y += 1;
    if (ext_done) *ext_done = row;
    // (slices, target blocks) order, see dnb_ctx::slice_major (not with the row,
    // which is the grid's first row of blocks)
    const int smaj = (c->slice_major && !row && sl.nblk <= 65535) ? 1 : 0;
    const dim3 grid32 = smaj ? dim3(sl.S, sl.nblk) : grid;
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid32, dim3(BS), 0, st, (const float4*)c->jsv, (int)n, i0,
                           iend, nj, sl.jslice, (float)eps2, (float*)c->partv, sl.npad, c->muni,
                           row ? er : ExtRow{}, c->aext_v, (float*)c->part, smaj);
    };
    if (c->prec == DNB_FP32C) {
        if (force) {
            if (lds && nt) go(k_pair_vjp_f32c<EPS0, MASS, true, true, false, true>);
            else if (lds) go(k_pair_vjp_f32c<EPS0, MASS, true, false, false, true>);
            else if (nt) go(k_pair_vjp_f32c<EPS0, MASS, false, true, false, true>);
            else go(k_pair_vjp_f32c<EPS0, MASS, false, false, false, true>);
        }
        else if (lds && nt && row) go(k_pair_vjp_f32c<EPS0, MASS, true, true, true, false>);
        else if (lds && nt) go(k_pair_vjp_f32c<EPS0, MASS, true, true, false, false>);
        else if (lds && row) go(k_pair_vjp_f32c<EPS0, MASS, true, false, true, false>);
        else if (lds) go(k_pair_vjp_f32c<EPS0, MASS, true, false, false, false>);
        else if (nt) go(k_pair_vjp_f32c<EPS0, MASS, false, true, false, false>);
        else go(k_pair_vjp_f32c<EPS0, MASS, false, false, false, false>);
    } else if (force) {
        hipLaunchKernelGGL((k_pair_vjp_f64<EPS0, MASS, true>), grid32, dim3(BS), 0, st,
                           (const double4*)c->jsv, (int)n, i0, iend, nj, sl.jslice, eps2,
                           (double*)c->partv, sl.npad, (double*)c->part, smaj);
    } else {
        hipLaunchKernelGGL((k_pair_vjp_f64<EPS0, MASS, false>), grid32, dim3(BS), 0, st,
                           (const double4*)c->jsv, (int)n, i0, iend, nj, sl.jslice, eps2,
                           (double*)c->partv, sl.npad, (double*)nullptr, smaj);
    }
}

static hipError_t launch_pair_vjp_sliced(dnb_ctx* c, int64_t n, int64_t i0, int64_t ni,
                                         const Slicing& sl, int with_mass, double eps,
                                         hipStream_t st, const ExtRow& er = ExtRow{},
                                         bool* ext_done = nullptr, bool force = false) {
    if (ext_done) *ext_done = false;
    const int nj = (int)pad_sources(n);
    const int a = (int)i0, e = (int)(i0 + ni);
    const double eps2 = eps * eps;
    if (eps == 0.0) {
        if (with_mass) vjp_dispatch<true, true>(c, sl, n, a, e, nj, eps2, st, er, ext_done, force);
        else vjp_dispatch<true, false>(c, sl, n, a, e, nj, eps2, st, er, ext_done, force);
    } else {
        if (with_mass) vjp_dispatch<false, true>(c, sl, n, a, e, nj, eps2, st, er, ext_done, force);
        else vjp_dispatch<false, false>(c, sl, n, a, e, nj, eps2, st, er, ext_done, force);
    }
    return hipGetLastError();
}

hipError_t launch_pair_vjp(dnb_ctx* c, int64_t n, int with_mass, double eps, hipStream_t st,
                           const ExtRow& ext, bool* ext_done) {
    return launch_pair_vjp_sliced(c, n, 0, n, vjp_slicing(c, n), with_mass, eps, st, ext,
                                  ext_done);
}

// The pair VJP of the whole system together with the internal acceleration at
// the same staged positions: the VJP partials as launch_pair_vjp writes them, the
// acceleration partials in the forward pair kernel's buffer and layout (the
// forward and VJP slicings are the same), for launch_fwd_reduce (FP32C) or the
// kernel that sums them (FP64).
hipError_t launch_pair_vjp_force(dnb_ctx* c, int64_t n, int with_mass, double eps,
                                 hipStream_t st) {
    return launch_pair_vjp_sliced(c, n, 0, n, vjp_slicing(c, n), with_mass, eps, st, ExtRow{},
                                  nullptr, true);
}

hipError_t launch_pair_vjp_rows(dnb_ctx* c, int64_t n, int64_t i0, int64_t ni, int with_mass,
                                double eps, hipStream_t st) {
    return launch_pair_vjp_sliced(c, n, i0, ni, rows_slicing(c, ni, n), with_mass, eps, st);
}

}  // namespace dnb
