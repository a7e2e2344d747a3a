// Batched ensembles: many independent small systems advanced together.
//
// The paper relies on automatic vectorisation to run many simulations of one
// small system at once (Sec. 2), which is what a training set for the surrogate
// or a parameter grid needs.  A single system of a few thousand particles is far
// too small to fill 256 compute units; here every O(N^2) and O(N) launch carries
// a third grid dimension over the members of the ensemble, so one launch per step
// advances all of them.  Each member has its own potential parameters and step
// size (a row of the parameter table).  Pair terms are FP32 with compensated
// accumulation (the FP32C path), drift FP64, exactly as for a single system; the
// per-target slice sums reuse the single-system device code.
#include "dnb_internal.h"
#include "kdk_common.h"
#include "pair_common.h"

namespace dnb {

struct BatchGeom {
    int n;            // particles per member
    int nj;           // padded sources per member
    int S, jslice;    // source slicing per member
    int nblk;         // target blocks per member (BS targets each)
    int64_t npad;     // partial row stride per member
    int nb;           // O(N) blocks per member
};

// Tape of a batched run (every step kept): the states (x, v) of steps
// 0 .. T-1 as [T][batch][6][n], then the internal accelerations of steps 0 .. T
// as [T+1][batch][3][n].
struct BatchTape {
    double* base;
    int64_t batch, n, T;
    double* state(int64_t s) const { return base + s * batch * 6 * n; }
    double* aint(int64_t s) const { return base + T * batch * 6 * n + s * batch * 3 * n; }
};

constexpr float BFAR32 = 1.0e18f;

// Parameter row: (G, eps, m_nfw, rs_nfw, m_mn, a_mn, b_mn, dt).
__device__ inline Pot pot_row(const double* __restrict__ P) {
    return Pot{P[0], P[1], P[2], P[3], P[4], P[5], P[6]};
}


__global__ __launch_bounds__(BS) void k_batch_mass_info(const double* __restrict__ mass, int n,
                                                        float* __restrict__ muni) {
    __shared__ double sh[BS];
    const double* m = mass + (int64_t)blockIdx.x * n;
    const double m0 = m[0];
    double diff = 0.0;
    for (int i = threadIdx.x; i < n; i += BS) diff = fmax(diff, fabs(m[i] - m0));
    sh[threadIdx.x] = diff;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool uni = sh[0] == 0.0 && isfinite(m0);
        muni[2 * blockIdx.x] = uni ? 1.f : 0.f;
        muni[2 * blockIdx.x + 1] = uni ? (float)m0 : 0.f;
    }
}

// Block records of member positions with the displacement dt v of the first
// drift (for the staging centre, as k_block_sums).  grid (nb, batch).
__global__ __launch_bounds__(BS) void k_batch_block_sums(const double* __restrict__ pos,
                                                         const double* __restrict__ vel,
                                                         const double* __restrict__ params,
                                                         int n, int nb,
                                                         double* __restrict__ cpart) {
    __shared__ double sh[3 * BS];
    const int b = blockIdx.y;
    const double* x = pos + (int64_t)b * 3 * n;
    const double* v = vel + (int64_t)b * 3 * n;
    const double dt = params[8 * b + 7];
    const int i = blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int k = ok ? i : 0;
    write_block_sums(x[k], x[n + k], x[2 * n + k], dt * v[k], dt * v[n + k], dt * v[2 * n + k],
                     ok, sh, cpart + (int64_t)b * nb * REC);
}

// Stage member positions relative to their centre.  grid (cdiv(nj, BS), batch).
__global__ __launch_bounds__(BS) void k_batch_stage(const double* __restrict__ pos,
                                                    const double* __restrict__ mass, BatchGeom g,
                                                    const double* __restrict__ cpart,
                                                    float4* __restrict__ js) {
    __shared__ double sh[3 * BS];
    const int b = blockIdx.y;
    double cx, cy, cz;
    centre_from(cpart + (int64_t)b * g.nb * REC, g.nb, g.n, sh, cx, cy, cz, false);
    const double* x = pos + (int64_t)b * 3 * g.n;
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i < g.nj) {
        float4* o = js + (int64_t)b * g.nj + i;
        if (i < g.n)
            *o = make_float4((float)(x[i] - cx), (float)(x[g.n + i] - cy),
                             (float)(x[2 * g.n + i] - cz), (float)mass[(int64_t)b * g.n + i]);
        else
            *o = make_float4(BFAR32, BFAR32, BFAR32, 0.f);
    }
}

// Target block x, source slice y and member b of a block of a batched pair
// launch (grid (nblk, S, batch)); with remap, read from the linear block index by
// batch_block_index (host_logic.h) so that the blocks one compute unit holds at a
// time share their sources.
struct BatchBlock {
    int x, y;
    int64_t b;
};
__device__ inline BatchBlock batch_block(const BatchGeom& g, int remap) {
    if (!remap) return BatchBlock{(int)blockIdx.x, (int)blockIdx.y, (int64_t)blockIdx.z};
    const int64_t L =
        blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    const BatchBlockIdx t = batch_block_index(L, g.nblk, g.S, gridDim.z);
    return BatchBlock{(int)t.x, (int)t.y, t.b};
}

// Pair sums of every member.  grid (nblk, S, batch).
template <bool NT>
__global__ __launch_bounds__(BS) void k_batch_pair_fwd(const float4* __restrict__ js, BatchGeom g,
                                                       const double* __restrict__ params,
                                                       const float* __restrict__ muni,
                                                       float* __restrict__ part, int remap) {
    const BatchBlock bb = batch_block(g, remap);
    const int b = (int)bb.b;
    const float4* jb = js + (int64_t)b * g.nj;
    const int i = bb.x * BS + threadIdx.x;
    const int j0 = bb.y * g.jslice;
    const int j1 = min(g.nj, j0 + g.jslice);
    const double eps = params[8 * b + 1];
    const float eps2 = (float)(eps * eps);
    const float4 me = jb[min(i, g.n - 1)];
    float h[3] = {0.f, 0.f, 0.f}, l[3] = {0.f, 0.f, 0.f};
    if (muni[2 * b] != 0.f) {
        fwd_f32c_slice<false, true>(jb, i, j0, j1, eps2, me, h, l);
        const float m = muni[2 * b + 1];
        for (int c = 0; c < 3; ++c) { h[c] *= m; l[c] *= m; }
    } else {
        fwd_f32c_slice<false, false>(jb, i, j0, j1, eps2, me, h, l);
    }
    if (i < g.n) {
        float2* p = (float2*)part + ((int64_t)b * g.S + bb.y) * 3 * g.npad + i;
        for (int c = 0; c < 3; ++c) put_partial<NT>(p + c * g.npad, h[c], l[c]);
    }
}

// Kick-drift-kick of every member (same arithmetic as k_kdk), staging the new
// positions.  grid (cdiv(nj, BS), batch).  mode 0: first (v is full-step), 1: mid,
// 2: last (closing kick only).
template <int MODE>
__global__ __launch_bounds__(BS) void k_batch_kdk(double* __restrict__ pos,
                                                  double* __restrict__ vel,
                                                  double* __restrict__ vh,
                                                  const double* __restrict__ mass, BatchGeom g,
                                                  const double* __restrict__ params,
                                                  const float* __restrict__ part,
                                                  const double* __restrict__ cp_in,
                                                  double* __restrict__ cp_out,
                                                  float4* __restrict__ js,
                                                  double* __restrict__ tape_state,
                                                  double* __restrict__ aint_out,
                                                  const double* __restrict__ ared,
                                                  const double* __restrict__ arec) {
    __shared__ double sh[4 * BS];
    const int b = blockIdx.y;
    const int n = g.n;
    const double* P = params + 8 * b;
    const Pot pot = pot_row(P);
    const double dt = P[7], hdt = 0.5 * dt;
    double* x = pos + (int64_t)b * 3 * n;
    double* v = vel + (int64_t)b * 3 * n;
    double* w = vh + (int64_t)b * 3 * n;
    const int i = blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int k = ok ? i : 0;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (MODE != 2) centre_from(cp_in + (int64_t)b * g.nb * REC, g.nb, n, sh, cx, cy, cz, true);
    // the member's reduced internal acceleration minus its net internal force
    // per unit mass (as k_kdk in FP32C)
    const int nr = red_blocks(n);
    double tot[4];
    rec_total(arec + (int64_t)b * nr * 4, nr, sh, tot);
    const double inv_m = 1.0 / tot[3];
    const double* ar = ared + (int64_t)b * 3 * n;
    double ax = ar[k] - tot[0] * inv_m;
    double ay = ar[n + k] - tot[1] * inv_m;
    double az = ar[2 * n + k] - tot[2] * inv_m;
    if (aint_out && ok) {
        double* t = aint_out + (int64_t)b * 3 * n;
        t[i] = ax; t[n + i] = ay; t[2 * n + i] = az;
    }
    const double x0 = x[k], y0 = x[n + k], z0 = x[2 * n + k];
    const Ext e = ext_accel(pot, x0, y0, z0);
    ax += e.ax; ay += e.ay; az += e.az;
    double xn = x0, yn = y0, zn = z0;
    if (ok) {
        if (MODE == 2) {
            v[i] = fma(hdt, ax, w[i]);
            v[n + i] = fma(hdt, ay, w[n + i]);
            v[2 * n + i] = fma(hdt, az, w[2 * n + i]);
        } else {
            double vx, vy, vz;
            if (MODE == 0) { vx = v[i]; vy = v[n + i]; vz = v[2 * n + i]; }
            else { vx = fma(hdt, ax, w[i]); vy = fma(hdt, ay, w[n + i]); vz = fma(hdt, az, w[2 * n + i]); }
            if (tape_state) {
                double* t = tape_state + (int64_t)b * 6 * n;
                t[i] = x0; t[n + i] = y0; t[2 * n + i] = z0;
                t[3 * n + i] = vx; t[4 * n + i] = vy; t[5 * n + i] = vz;
            }
            const double hx = fma(hdt, ax, vx), hy = fma(hdt, ay, vy), hz = fma(hdt, az, vz);
            xn = fma(dt, hx, x0); yn = fma(dt, hy, y0); zn = fma(dt, hz, z0);
            w[i] = hx; w[n + i] = hy; w[2 * n + i] = hz;
            x[i] = xn; x[n + i] = yn; x[2 * n + i] = zn;
        }
    }
    if (MODE != 2) {
        if (i < g.nj) {
            float4* o = js + (int64_t)b * g.nj + i;
            *o = ok ? make_float4((float)(xn - cx), (float)(yn - cy), (float)(zn - cz),
                                  (float)mass[(int64_t)b * n + i])
                    : make_float4(BFAR32, BFAR32, BFAR32, 0.f);
        }
        write_block_sums(xn, yn, zn, xn - x0, yn - y0, zn - z0, ok, sh,
                         cp_out + (int64_t)b * g.nb * REC);
    }
}

// Slice reductions of every member (the batched forms of k_fwd_reduce and
// k_vjp_reduce, same arithmetic).  grid (cdiv(n, RT), batch).
__global__ __launch_bounds__(BS) void k_batch_fwd_reduce(const float* __restrict__ part,
                                                         BatchGeom g,
                                                         const double* __restrict__ params,
                                                         const double* __restrict__ mass,
                                                         double* __restrict__ ared,
                                                         double* __restrict__ arec) {
    __shared__ double sh[3 * RG * RT];
    const int64_t b = blockIdx.y;
    const int64_t n = g.n;
    const int nr = red_blocks(n);
    fwd_reduce_block((const float2*)part + b * g.S * 3 * g.npad, g.S, g.npad, n, params[8 * b],
                     mass + b * n, ared + b * 3 * n, arec + b * nr * 4, sh);
}

__global__ __launch_bounds__(BS) void k_batch_vjp_reduce(const float* __restrict__ part,
                                                         BatchGeom g,
                                                         const double* __restrict__ params,
                                                         const double* __restrict__ wscale,
                                                         int wq, double* __restrict__ gred,
                                                         double* __restrict__ grec) {
    __shared__ double sh[4 * RG * RT];
    const int64_t b = blockIdx.y;
    const int64_t n = g.n;
    const int nr = red_blocks(n);
    vjp_reduce_block((const float2*)part + b * g.S * 4 * g.npad, g.S, g.npad, n, params[8 * b],
                     false, 1.0 / wscale[2 * b + wq], gred + b * 4 * n, grec + b * nr * 4, sh);
}

// Test-particle orbits of every member, one lane each (the batched form of k_orbit);
// traj (nullable) receives member b's positions x_0 .. x_T at traj + b (T+1) 3.
__global__ void k_batch_orbit(const double* __restrict__ w0, const double* __restrict__ params,
                              int batch, int64_t n_steps, double* __restrict__ w_out,
                              double* __restrict__ traj) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double* P = params + 8 * b;
    const Pot p = pot_row(P);
    const double dt = P[7], hdt = 0.5 * dt;
    const double* w = w0 + 6 * b;
    double* tr = traj ? traj + (int64_t)b * (n_steps + 1) * 3 : nullptr;
    double x = w[0], y = w[1], z = w[2], vx = w[3], vy = w[4], vz = w[5];
    Ext e = ext_accel(p, x, y, z);
    if (tr) { tr[0] = x; tr[1] = y; tr[2] = z; }
    for (int64_t s = 0; s < n_steps; ++s) {
        const double hx = fma(hdt, e.ax, vx), hy = fma(hdt, e.ay, vy), hz = fma(hdt, e.az, vz);
        x = fma(dt, hx, x); y = fma(dt, hy, y); z = fma(dt, hz, z);
        e = ext_accel(p, x, y, z);
        vx = fma(hdt, e.ax, hx); vy = fma(hdt, e.ay, hy); vz = fma(hdt, e.az, hz);
        if (tr) { tr[3 * (s + 1)] = x; tr[3 * (s + 1) + 1] = y; tr[3 * (s + 1) + 2] = z; }
    }
    double* o = w_out + 6 * b;
    o[0] = x; o[1] = y; o[2] = z; o[3] = vx; o[4] = vy; o[5] = vz;
}

// Reverse sweep of every member's orbit (the batched form of k_orbit_vjp, same
// arithmetic): gw0 [batch][6], gparams [batch][3] = (dL/dm_nfw, dL/dm_mn, dL/ddt).
__global__ void k_batch_orbit_vjp(const double* __restrict__ traj, const double* __restrict__ params,
                                  int batch, int64_t n_steps, const double* __restrict__ gw_out,
                                  double* __restrict__ gw0, double* __restrict__ gparams) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double* P = params + 8 * b;
    const Pot p = pot_row(P);
    const double dt = P[7];
    const double* tr = traj + (int64_t)b * (n_steps + 1) * 3;
    const double* go = gw_out + 6 * b;
    double lx = go[0], ly = go[1], lz = go[2];
    double wx = go[3], wy = go[4], wz = go[5];
    double g_nfw = 0.0, g_mn = 0.0, g_dt = 0.0;
    const double inv = 1.0 / dt;
    for (int64_t s = n_steps; s >= 0 && n_steps > 0; --s) {
        const double coef = (s == n_steps || s == 0) ? 0.5 * dt : dt;
        const double kc = (s == n_steps || s == 0) ? 0.5 : 1.0;
        const double x = tr[3 * s], y = tr[3 * s + 1], z = tr[3 * s + 2];
        Ext e = ext_accel(p, x, y, z);
        double hx, hy, hz;
        ext_hvp(p, x, y, z, wx, wy, wz, hx, hy, hz);
        lx += coef * hx; ly += coef * hy; lz += coef * hz;
        g_dt += kc * (e.ax * wx + e.ay * wy + e.az * wz);
        g_nfw += coef * (e.nx * wx + e.ny * wy + e.nz * wz);
        g_mn += coef * (e.mx * wx + e.my * wy + e.mz * wz);
        if (s > 0) {
            const double vx = (x - tr[3 * (s - 1)]) * inv;
            const double vy = (y - tr[3 * (s - 1) + 1]) * inv;
            const double vz = (z - tr[3 * (s - 1) + 2]) * inv;
            g_dt += vx * lx + vy * ly + vz * lz;
            wx += dt * lx; wy += dt * ly; wz += dt * lz;
        }
    }
    double* o = gw0 + 6 * b;
    o[0] = lx; o[1] = ly; o[2] = lz; o[3] = wx; o[4] = wy; o[5] = wz;
    gparams[3 * b] = g_nfw; gparams[3 * b + 1] = g_mn; gparams[3 * b + 2] = g_dt;
}

// Adjoint of the batched Plummer placement: per member the sums over particles of
// gpos, gvel and gvel . zeta (the order of k_place_vjp_rows / k_place_vjp_final).
__global__ __launch_bounds__(BS) void k_batch_place_vjp_rows(int64_t n, const double* __restrict__ zeta,
                                                             const double* __restrict__ gpos,
                                                             const double* __restrict__ gvel,
                                                             double* __restrict__ red) {
    __shared__ double sh[8 * BS];
    const int64_t b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const double* gp = gpos + b * 3 * n;
    const double* gv = gvel + b * 3 * n;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < n) {
        for (int c = 0; c < 3; ++c) {
            v[c] = gp[c * n + i];
            v[3 + c] = gv[c * n + i];
            v[6] += gv[c * n + i] * zeta[c * n + i];
        }
    }
    block_sum<8>(v, sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < 8; ++c) red[(b * gridDim.x + blockIdx.x) * 8 + c] = v[c];
}

__global__ __launch_bounds__(BS) void k_batch_place_vjp_final(const double* __restrict__ red,
                                                              int nb, int64_t n,
                                                              const double* __restrict__ m_tot,
                                                              double a_p, double G,
                                                              double* __restrict__ gw,
                                                              double* __restrict__ gm_tot) {
    __shared__ double sh[8 * BS];
    const int64_t b = blockIdx.x;
    const double* r = red + b * nb * 8;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = threadIdx.x; q < nb; q += BS)
        for (int c = 0; c < 8; ++c) v[c] += r[8 * q + c];
    block_sum<8>(v, sh);
    if (threadIdx.x == 0) {
        // d sqrt(G M / a_p) / dM = sqrt(G / (a_p M)) / 2
        const double dvs_dm = 0.5 * sqrt(G / (a_p * m_tot[b]));
        for (int c = 0; c < 6; ++c) gw[6 * b + c] = v[c];
        gm_tot[b] = v[6] * dvs_dm + v[7] / (double)n;
    }
}

hipError_t launch_place_batch_vjp(dnb_ctx* c, int64_t batch, int64_t n, const double* zeta,
                                  const double* m_tot, double a_p, double G, const double* gpos,
                                  const double* gvel, double* gw, double* gm_tot,
                                  hipStream_t st) {
    const int nb = (int)cdiv(n, BS);
    hipLaunchKernelGGL(k_batch_place_vjp_rows, dim3((unsigned)nb, (unsigned)batch), dim3(BS), 0,
                       st, n, zeta, gpos, gvel, c->red);
    hipLaunchKernelGGL(k_batch_place_vjp_final, dim3((unsigned)batch), dim3(BS), 0, st, c->red, nb,
                       n, m_tot, a_p, G, gw, gm_tot);
    return hipGetLastError();
}

hipError_t launch_orbit_batch_vjp(int64_t batch, const double* traj, const double* params_dev,
                                  int64_t n_steps, const double* gw_out, double* gw0,
                                  double* gparams, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_orbit_vjp, dim3((unsigned)cdiv(batch, 64)), dim3(64), 0, st, traj,
                       params_dev, (int)batch, n_steps, gw_out, gw0, gparams);
    return hipGetLastError();
}

// Plummer spheres of every member placed at their own phase-space points (the
// batched form of k_place): the unit samples xi, zeta [3][n] are shared, member b
// has centre w[b] [6] and total mass m_tot[b].  grid (cdiv(n, BS), batch).
__global__ __launch_bounds__(BS) void k_batch_place(int64_t n, const double* __restrict__ w,
                                                    const double* __restrict__ xi,
                                                    const double* __restrict__ zeta,
                                                    const double* __restrict__ m_tot, double a_p,
                                                    double G, double* __restrict__ pos,
                                                    double* __restrict__ vel,
                                                    double* __restrict__ mass) {
    const int64_t b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const double M = m_tot[b];
    const double vscale = sqrt(G * M / a_p);
    const double* wb = w + 6 * b;
    double* x = pos + b * 3 * n;
    double* v = vel + b * 3 * n;
    for (int c = 0; c < 3; ++c) {
        x[c * n + i] = wb[c] + a_p * xi[c * n + i];
        v[c * n + i] = wb[3 + c] + vscale * zeta[c * n + i];
    }
    mass[b * n + i] = M / (double)n;
}

hipError_t launch_place_batch(int64_t batch, int64_t n, const double* w, const double* xi,
                              const double* zeta, const double* m_tot, double a_p, double G,
                              double* pos, double* vel, double* mass, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_place, dim3((unsigned)cdiv(n, BS), (unsigned)batch), dim3(BS), 0,
                       st, n, w, xi, zeta, m_tot, a_p, G, pos, vel, mass);
    return hipGetLastError();
}

BatchGeom batch_geom(const dnb_ctx* c, int64_t batch, int64_t n) {
    BatchGeom g;
    g.n = (int)n;
    g.nj = (int)pad_sources(n);
    g.nblk = (int)cdiv(n, BS);
    g.npad = (int64_t)g.nblk * BS;
    g.nb = (int)cdiv(g.nj, BS);
    // The single-system slicing with the launch's blocks shared by all members;
    // every slice adds a row of partial sums per particle that the O(N) step
    // kernels read, so a large ensemble keeps to at most max(8, 512 / batch)
    // slices (measured at n = 1000: 16, 64 and 256 members).
    int64_t smax = 512 / batch;
    if (smax < 8) smax = 8;
    if (smax > S_MAX) smax = S_MAX;
    const Slicing sl = pair_slicing(n, n, (int)(c->target_blocks / batch), (int)smax);
    g.jslice = sl.jslice;
    g.S = sl.S;
    return g;
}

// Whether a launch's slice partials (rows of float2 per member, slice and
// target) are many enough for non-temporal stores (put_partial).
static bool nt_partials(const BatchGeom& g, int64_t batch, int rows) {
    return batch * g.S * g.npad * rows * 8 >= NT_PARTIAL_BYTES;
}

// Capacity of the context for a batch (checked before anything is enqueued).
bool batch_fits(const dnb_ctx* c, int64_t batch, int64_t n) {
    const BatchGeom g = batch_geom(c, batch, n);
    const int64_t npadmax = (int64_t)c->nbmax * BS;
    return batch <= DNB_BATCH_MAX && batch * g.nj <= 2 * npadmax && batch * n <= npadmax &&
           batch * g.S * g.npad * 6 <= 8 * c->slice_rows && batch * g.nb <= c->nbmax;
}

hipError_t launch_simulate_batch(dnb_ctx* c, int64_t batch, int64_t n, double* pos, double* vel,
                                 const double* mass, const double* params_dev, int64_t n_steps,
                                 double* tape, hipStream_t st) {
    if (n_steps == 0) return hipSuccess;
    const BatchGeom g = batch_geom(c, batch, n);
    float4* js = (float4*)c->js;
    float* part = (float*)c->part;
    double* cp[2] = {c->cpart, c->cpart + REC * c->nbmax};
    const dim3 on(g.nb, (unsigned)batch);
    hipLaunchKernelGGL(k_batch_mass_info, dim3((unsigned)batch), dim3(BS), 0, st, mass, g.n,
                       c->muni);
    hipLaunchKernelGGL(k_batch_block_sums, on, dim3(BS), 0, st, pos, vel, params_dev, g.n, g.nb,
                       cp[0]);
    hipLaunchKernelGGL(k_batch_stage, on, dim3(BS), 0, st, pos, mass, g, cp[0], js);
    const BatchTape tp{tape, batch, n, n_steps};
    const dim3 red((unsigned)red_blocks(n), (unsigned)batch);
    int q = 0;
    for (int64_t s = 0; s <= n_steps; ++s) {
        hipLaunchKernelGGL(nt_partials(g, batch, 3) ? k_batch_pair_fwd<true>
                                                    : k_batch_pair_fwd<false>,
                           dim3(g.nblk, g.S, (unsigned)batch), dim3(BS), 0, st, js, g,
                           params_dev, c->muni, part, c->slice_major);
        hipLaunchKernelGGL(k_batch_fwd_reduce, red, dim3(BS), 0, st, (const float*)part, g,
                           params_dev, mass, c->ared, c->arec);
        double* ts = (tape && s < n_steps) ? tp.state(s) : nullptr;
        double* ta = tape ? tp.aint(s) : nullptr;
        if (s == 0)
            hipLaunchKernelGGL(k_batch_kdk<0>, on, dim3(BS), 0, st, pos, vel, c->vh, mass, g,
                               params_dev, part, cp[q], cp[1 - q], js, ts, ta, c->ared, c->arec);
        else if (s == n_steps)
            hipLaunchKernelGGL(k_batch_kdk<2>, on, dim3(BS), 0, st, pos, vel, c->vh, mass, g,
                               params_dev, part, cp[q], cp[1 - q], js, ts, ta, c->ared, c->arec);
        else
            hipLaunchKernelGGL(k_batch_kdk<1>, on, dim3(BS), 0, st, pos, vel, c->vh, mass, g,
                               params_dev, part, cp[q], cp[1 - q], js, ts, ta, c->ared, c->arec);
        q = 1 - q;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ batched VJP --
// The reverse sweep of dnb_simulate_vjp (every step on the tape, FP32C), member by
// member with the same arithmetic and reduction order, so a member's gradient
// equals that of a single-system run with the same source slicing bit for bit.

// Stage the final positions and the velocity cotangent.  grid (nb, batch).
__global__ __launch_bounds__(BS) void k_batch_rev_stage(const double* __restrict__ pos,
                                                        const double* __restrict__ mass,
                                                        const double* __restrict__ w, BatchGeom g,
                                                        const double* __restrict__ cpart,
                                                        float4* __restrict__ jsv,
                                                        double* __restrict__ cpart_out,
                                                        double* __restrict__ wscale,
                                                        const double* __restrict__ xprev_base,
                                                        int64_t xprev_stride) {
    __shared__ double sh[3 * BS];
    const int64_t b = blockIdx.y;
    const int64_t n = g.n;
    const double* cp = cpart + b * g.nb * REC;
    double cx, cy, cz;
    centre_from(cp, g.nb, n, sh, cx, cy, cz, false);
    const double S = scale_from(cp, g.nb, sh);
    const double* x = pos + b * 3 * n;
    const double* wb = w + b * 3 * n;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    const double x0 = x[k], y0 = x[n + k], z0 = x[2 * n + k];
    const double wx = wb[k], wy = wb[n + k], wz = wb[2 * n + k];
    if (i < g.nj)
        put_source_w<true>(jsv + b * g.nj * 2, i, ok, x0, y0, z0, mass[b * n + k], cx, cy, cz,
                           wx * S, wy * S, wz * S);
    double* co = cpart_out + b * g.nb * REC;
    double dx = 0.0, dy = 0.0, dz = 0.0;
    if (xprev_base) {
        const double* xp = xprev_base + b * xprev_stride;
        dx = xp[k] - x0; dy = xp[n + k] - y0; dz = xp[2 * n + k] - z0;
    }
    write_block_sums(x0, y0, z0, dx, dy, dz, ok, sh, co);
    write_block_max(ok ? absmax3(wx, wy, wz) : 0.0, sh, co);
    if (blockIdx.x == 0 && threadIdx.x == 0) wscale[2 * b] = S;
}

// Block sums of positions with the block maxima of w (slot 3).  grid (nb, batch).
__global__ __launch_bounds__(BS) void k_batch_block_sums_w(const double* __restrict__ pos,
                                                           const double* __restrict__ w,
                                                           BatchGeom g,
                                                           double* __restrict__ cpart) {
    __shared__ double sh[3 * BS];
    const int64_t b = blockIdx.y;
    const int64_t n = g.n;
    const double* x = pos + b * 3 * n;
    const double* wb = w + b * 3 * n;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    double* co = cpart + b * g.nb * REC;
    write_block_sums(x[k], x[n + k], x[2 * n + k], 0.0, 0.0, 0.0, ok, sh, co);
    write_block_max(ok ? absmax3(wb[k], wb[n + k], wb[2 * n + k]) : 0.0, sh, co);
}

// Pair VJP of every member.  grid (nblk, S, batch).
template <bool NT>
__global__ __launch_bounds__(BS) void k_batch_pair_vjp(const float4* __restrict__ jsv,
                                                       BatchGeom g,
                                                       const double* __restrict__ params,
                                                       const float* __restrict__ muni,
                                                       float* __restrict__ part, int remap) {
    const BatchBlock bb = batch_block(g, remap);
    const int64_t b = bb.b;
    const float4* jb = jsv + b * g.nj * 2;
    const int i = bb.x * BS + threadIdx.x;
    const int j0 = bb.y * g.jslice;
    const int j1 = min(g.nj, j0 + g.jslice);
    const int ii = min(i, g.n - 1);
    const float4 me = jb[2 * ii];
    const float4 mw = jb[2 * ii + 1];
    const double eps = params[8 * b + 1];
    const float eps2 = (float)(eps * eps);
    float h[4] = {0.f, 0.f, 0.f, 0.f};
    float l[4] = {0.f, 0.f, 0.f, 0.f};
    if (muni[2 * b] != 0.f) {
        vjp_f32c_slice<false, false, true>(jb, i, j0, j1, eps2, me, mw, h, l);
        const float m = muni[2 * b + 1];
        for (int c = 0; c < 3; ++c) { h[c] *= m; l[c] *= m; }
    } else {
        vjp_f32c_slice<false, false, false>(jb, i, j0, j1, eps2, me, mw, h, l);
    }
    if (i < g.n) {
        float2* p = (float2*)part + (b * g.S + bb.y) * 4 * g.npad + i;
        for (int c = 0; c < 3; ++c) put_partial<NT>(p + c * g.npad, h[c], l[c]);
    }
}

// One merged kick of the reverse sweep for every member (k_rev_kick, FP32C,
// without per-particle mass cotangents).  x_n / x_prev / aint are the positions,
// the previous positions (null: the last reverse step) and the internal
// accelerations of the step, each with its own member stride.  half: the kick
// coefficient is dt/2 (first and last steps) rather than dt.  grid (nb, batch).
__global__ __launch_bounds__(BS) void k_batch_rev_kick(
    BatchGeom g, const double* __restrict__ params, const double* __restrict__ mass,
    const float* __restrict__ part, const double* __restrict__ xn_base, int64_t xn_stride,
    const double* __restrict__ xp_base, int64_t xp_stride, const double* __restrict__ aint_base,
    int half, double* __restrict__ lx_base, double* __restrict__ lv_base,
    double* __restrict__ accum_base, const double* __restrict__ cpart_in,
    double* __restrict__ cpart_out, double* __restrict__ wscale, int wq,
    float4* __restrict__ jsv, const double* __restrict__ gred, const double* __restrict__ grec) {
    __shared__ double sh[4 * BS];
    const int64_t b = blockIdx.y;
    const int64_t n = g.n;
    const double* P = params + 8 * b;
    const Pot pot = pot_row(P);
    const double dt = P[7];
    const double coef = half ? 0.5 * dt : dt;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    const bool drift = xp_base != nullptr;
    const double* cpi = cpart_in + b * g.nb * REC;
    const double* xnb = xn_base + b * xn_stride;
    const double* ai_b = aint_base + b * 3 * n;
    double* lx = lx_base + b * 3 * n;
    double* lv = lv_base + b * 3 * n;
    double* accum = accum_base + b * 4 * n;

    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (drift) centre_from(cpi, g.nb, n, sh, cx, cy, cz, true);
    // the member's reduced J^T w minus its mean (as k_rev_kick in FP32C)
    const int nr = red_blocks(n);
    double tot[4];
    rec_total(grec + b * nr * 4, nr, sh, tot);
    const double inv_n = 1.0 / (double)n;
    const double* gr = gred + b * 4 * n;
    double gg[3] = {gr[k] - tot[0] * inv_n, gr[n + k] - tot[1] * inv_n,
                    gr[2 * n + k] - tot[2] * inv_n};
    const double ai[3] = {ai_b[k], ai_b[n + k], ai_b[2 * n + k]};
    const double x = xnb[k], y = xnb[n + k], z = xnb[2 * n + k];
    const double wx = lv[k], wy = lv[n + k], wz = lv[2 * n + k];
    Ext e = ext_accel(pot, x, y, z);
    double hx, hy, hz;
    ext_hvp(pot, x, y, z, wx, wy, wz, hx, hy, hz);

    const double lxx = fma(coef, gg[0] + hx, lx[k]);
    const double lxy = fma(coef, gg[1] + hy, lx[n + k]);
    const double lxz = fma(coef, gg[2] + hz, lx[2 * n + k]);
    const double kc = coef / dt;
    const double aw_int = ai[0] * wx + ai[1] * wy + ai[2] * wz;
    const double aw_ext = e.ax * wx + e.ay * wy + e.az * wz;
    double d_dt = kc * (aw_int + aw_ext);
    const double d_nfw = coef * (e.nx * wx + e.ny * wy + e.nz * wz);
    const double d_mn = coef * (e.mx * wx + e.my * wy + e.mz * wz);
    const double d_ms = coef * aw_int;

    double px = 0.0, py = 0.0, pz = 0.0;
    double nwx = wx, nwy = wy, nwz = wz;
    if (drift) {
        const double* xpb = xp_base + b * xp_stride;
        px = xpb[k]; py = xpb[n + k]; pz = xpb[2 * n + k];
        const double inv = 1.0 / dt;
        const double vx = (x - px) * inv, vy = (y - py) * inv, vz = (z - pz) * inv;
        d_dt += vx * lxx + vy * lxy + vz * lxz;
        nwx = fma(dt, lxx, wx); nwy = fma(dt, lxy, wy); nwz = fma(dt, lxz, wz);
    }
    if (ok) {
        lx[i] = lxx; lx[n + i] = lxy; lx[2 * n + i] = lxz;
        accum[i] += d_nfw;
        accum[n + i] += d_mn;
        accum[2 * n + i] += d_dt;
        accum[3 * n + i] += d_ms;
        if (drift) { lv[i] = nwx; lv[n + i] = nwy; lv[2 * n + i] = nwz; }
    }
    if (drift) {
        const double Sn = scale_from(cpi, g.nb, sh);
        if (i < g.nj)
            put_source_w<true>(jsv + b * g.nj * 2, i, ok, px, py, pz, mass[b * n + k], cx, cy,
                               cz, nwx * Sn, nwy * Sn, nwz * Sn);
        double* co = cpart_out + b * g.nb * REC;
        write_block_sums(px, py, pz, px - x, py - y, pz - z, ok, sh, co);
        write_block_max(ok ? absmax3(nwx, nwy, nwz) : 0.0, sh, co);
        if (blockIdx.x == 0 && threadIdx.x == 0) wscale[2 * b + (1 - wq)] = Sn;
    }
}

// Per-member sums of the four per-particle cotangent accumulators (the order of
// k_reduce_rows).  One block per member.
__global__ __launch_bounds__(BS) void k_batch_reduce4(const double* __restrict__ accum, int64_t n,
                                                      double* __restrict__ out) {
    __shared__ double sh[5 * BS];
    const double* v = accum + (int64_t)blockIdx.x * 4 * n;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += BS)
        for (int t = 0; t < 4; ++t) s[t] += v[t * n + i];
    block_sum<5>(s, sh);
    if (threadIdx.x == 0)
        for (int t = 0; t < 4; ++t) out[4 * blockIdx.x + t] = s[t];
}

hipError_t launch_simulate_batch_vjp(dnb_ctx* c, int64_t batch, int64_t n, const double* mass,
                                     const double* params_dev, int64_t T, const double* tape,
                                     const double* pos_T, double* accum, double* lx, double* lv,
                                     double* gparams, hipStream_t st) {
    const BatchGeom g = batch_geom(c, batch, n);
    const BatchTape tp{const_cast<double*>(tape), batch, n, T};
    float4* jsv = (float4*)c->jsv;
    float* part = (float*)c->partv;
    double* cpv[2] = {c->cpartv, c->cpartv + REC * c->nbmax};
    const dim3 on(g.nb, (unsigned)batch);
    hipLaunchKernelGGL(k_batch_mass_info, dim3((unsigned)batch), dim3(BS), 0, st, mass, g.n,
                       c->muni);
    hipLaunchKernelGGL(k_batch_block_sums_w, on, dim3(BS), 0, st, pos_T, lv, g, cpv[0]);
    hipLaunchKernelGGL(k_batch_rev_stage, on, dim3(BS), 0, st, pos_T, mass, lv, g, cpv[0], jsv,
                       cpv[1], c->bwscale, T > 0 ? tp.state(T - 1) : nullptr, (int64_t)6 * n);
    int q = 1, wq = 0;
    for (int64_t m = T; m >= 0; --m) {
        hipLaunchKernelGGL(nt_partials(g, batch, 3) ? k_batch_pair_vjp<true>
                                                    : k_batch_pair_vjp<false>,
                           dim3(g.nblk, g.S, (unsigned)batch), dim3(BS), 0, st,
                           (const float4*)jsv, g, params_dev, c->muni, part, c->slice_major);
        hipLaunchKernelGGL(k_batch_vjp_reduce, dim3((unsigned)red_blocks(n), (unsigned)batch),
                           dim3(BS), 0, st, (const float*)part, g, params_dev, c->bwscale, wq,
                           c->gred, c->grec);
        const double* xn = (m == T) ? pos_T : tp.state(m);
        const int64_t xs = (m == T) ? 3 * n : 6 * n;
        const double* xp = (m > 0) ? tp.state(m - 1) : nullptr;
        hipLaunchKernelGGL(k_batch_rev_kick, on, dim3(BS), 0, st, g, params_dev, mass,
                           (const float*)part, xn, xs, xp, (int64_t)6 * n, tp.aint(m),
                           (int)(m == T || m == 0), lx, lv, accum, cpv[q], cpv[1 - q], c->bwscale,
                           wq, jsv, c->gred, c->grec);
        q = 1 - q;
        wq = 1 - wq;
    }
    hipLaunchKernelGGL(k_batch_reduce4, dim3((unsigned)batch), dim3(BS), 0, st, accum, n,
                       gparams);
    return hipGetLastError();
}

hipError_t launch_orbit_batch(int64_t batch, const double* w0, const double* params_dev,
                              int64_t n_steps, double* w_out, double* traj, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_orbit, dim3((unsigned)cdiv(batch, 64)), dim3(64), 0, st, w0,
                       params_dev, (int)batch, n_steps, w_out, traj);
    return hipGetLastError();
}

}  // namespace dnb
