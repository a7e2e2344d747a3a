// O(N) kernels of the integrator and of its reverse sweep.
//
// Forward (Sec. 2.2.1: Velocity-Verlet with fixed steps, i.e. kick-drift-kick).
// One step n -> n+1 is two launches: the pair kernel at x_n, then k_kdk, which
// adds the slice partials in FP64, adds the FP64 host-galaxy acceleration, and
// performs, in the unmerged textbook order,
//     v_n      = v_half + dt/2 a(x_n)          (closing kick of step n-1)
//     v_half'  = v_n + dt/2 a(x_n)             (opening kick of step n)
//     x_{n+1}  = x_n + dt v_half'              (drift, FP64)
// It then stages x_{n+1} for the next pair kernel (FP32C mode) and writes the
// block sums of x_{n+1}, from which the next launch takes its staging centre.
//
// Staging centre.  Positions x_{n+1} are staged relative to the mean of x_n (the
// centre lags one step; it only has to lie near the particles).  Because the
// centre is a deterministic function of x_n, a recomputation started from a
// checkpoint reproduces the forward run bit for bit once the checkpoint also
// stores the centre its positions were staged with.
//
// Reverse (the exact discrete adjoint).  With the two half kicks that meet at x_n
// merged, the sweep newest-first is, for n = T .. 0,
//     lambda_x += c_n J(x_n)^T lambda_v            c_n = dt (dt/2 at n = 0, T)
//     then, for n > 0, the adjoint of the drift of step n-1:
//     lambda_v += dt lambda_x
// together with the cotangents of dt, the two host masses and the particle masses.
#include "dnb_internal.h"

namespace dnb {

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

__global__ __launch_bounds__(BS) void k_block_sums(const double* __restrict__ x, int64_t n,
                                                   double* __restrict__ cpart) {
    __shared__ double sh[3 * BS];
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    write_block_sums(x[k], x[n + k], x[2 * n + k], ok, sh, cpart);
}

__global__ __launch_bounds__(BS) void k_stage(const double* __restrict__ x,
                                              const double* __restrict__ mass, int64_t n,
                                              const double* __restrict__ cpart, int nb,
                                              const double* __restrict__ centre_override,
                                              float4* __restrict__ js,
                                              double* __restrict__ centre_out) {
    __shared__ double sh[3 * BS];
    double cx, cy, cz;
    if (centre_override) {
        cx = centre_override[0]; cy = centre_override[1]; cz = centre_override[2];
    } else {
        centre_from(cpart, nb, n, sh, cx, cy, cz);
    }
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i < n)
        js[i] = make_float4((float)(x[i] - cx), (float)(x[n + i] - cy), (float)(x[2 * n + i] - cz),
                            (float)mass[i]);
    if (centre_out && blockIdx.x == 0 && threadIdx.x == 0) {
        centre_out[0] = cx; centre_out[1] = cy; centre_out[2] = cz; centre_out[3] = 0.0;
    }
}

// Sum of the slice partials of the forward pair kernel for particle i (times G).
template <bool F32>
__device__ inline void pair_sum(const void* part, int S, int64_t npad, int64_t i, double G,
                                double& ax, double& ay, double& az) {
    ax = ay = az = 0.0;
    if (F32) {
        const float* p = (const float*)part;
        for (int s = 0; s < S; ++s) {
            const float* q = p + (int64_t)s * 6 * npad + i;
            ax += (double)q[0]; ax += (double)q[3 * npad];
            ay += (double)q[npad]; ay += (double)q[4 * npad];
            az += (double)q[2 * npad]; az += (double)q[5 * npad];
        }
    } else {
        const double* p = (const double*)part;
        for (int s = 0; s < S; ++s) {
            const double* q = p + (int64_t)s * 3 * npad + i;
            ax += q[0]; ay += q[npad]; az += q[2 * npad];
        }
    }
    ax *= G; ay *= G; az *= G;
}

template <int MODE, bool F32>
__global__ __launch_bounds__(BS) void k_kdk(FwdArgs a, const void* __restrict__ part, int S,
                                            int64_t npad, float4* __restrict__ js) {
    __shared__ double sh[3 * BS];
    const int64_t n = a.n;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    const bool drift = (MODE == KDK_FIRST || MODE == KDK_MID);

    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (F32 && drift) centre_from(a.cpart_in, a.nb_in, n, sh, cx, cy, cz);

    double ax, ay, az;
    pair_sum<F32>(part, S, npad, k, a.pot.G, ax, ay, az);
    const double x = a.x[k], y = a.x[n + k], z = a.x[2 * n + k];
    if (a.with_ext) {
        Ext e = ext_accel(a.pot, x, y, z);
        ax += e.ax; ay += e.ay; az += e.az;
    }
    const double hdt = 0.5 * a.dt;
    double xn = x, yn = y, zn = z;
    if (ok) {
        if (MODE == KDK_ACC) {
            a.acc_out[i] = ax; a.acc_out[n + i] = ay; a.acc_out[2 * n + i] = az;
        } else if (MODE == KDK_LAST) {
            a.v[i] = a.vh[i] + hdt * ax;
            a.v[n + i] = a.vh[n + i] + hdt * ay;
            a.v[2 * n + i] = a.vh[2 * n + i] + hdt * az;
        } else {
            double vx, vy, vz;
            if (MODE == KDK_FIRST) {
                vx = a.v[i]; vy = a.v[n + i]; vz = a.v[2 * n + i];
            } else {
                vx = a.vh[i] + hdt * ax; vy = a.vh[n + i] + hdt * ay; vz = a.vh[2 * n + i] + hdt * az;
            }
            if (a.tape_state) {
                double* t = a.tape_state;
                t[i] = x; t[n + i] = y; t[2 * n + i] = z;
                t[3 * n + i] = vx; t[4 * n + i] = vy; t[5 * n + i] = vz;
            }
            const double hx = vx + hdt * ax, hy = vy + hdt * ay, hz = vz + hdt * az;
            xn = x + a.dt * hx; yn = y + a.dt * hy; zn = z + a.dt * hz;
            a.vh[i] = hx; a.vh[n + i] = hy; a.vh[2 * n + i] = hz;
            a.x_out[i] = xn; a.x_out[n + i] = yn; a.x_out[2 * n + i] = zn;
            if (F32)
                js[i] = make_float4((float)(xn - cx), (float)(yn - cy), (float)(zn - cz),
                                    (float)a.mass[i]);
        }
    }
    if (F32 && drift) {
        write_block_sums(xn, yn, zn, ok, sh, a.cpart_out);
        if (a.tape_centre_next && blockIdx.x == 0 && threadIdx.x == 0) {
            a.tape_centre_next[0] = cx; a.tape_centre_next[1] = cy;
            a.tape_centre_next[2] = cz; a.tape_centre_next[3] = 0.0;
        }
    }
}

hipError_t launch_block_sums(const double* x, int64_t n, double* cpart, hipStream_t st) {
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)cdiv(n, BS)), dim3(BS), 0, st, x, n, cpart);
    return hipGetLastError();
}

hipError_t launch_stage(const double* x, const double* mass, int64_t n, const double* cpart,
                        int nb, const double* centre_override, float4* js, double* centre_out,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_stage, dim3((unsigned)cdiv(n, BS)), dim3(BS), 0, st, x, mass, n, cpart,
                       nb, centre_override, js, centre_out);
    return hipGetLastError();
}

template <int MODE>
static void kdk_dispatch(dnb_ctx* c, const FwdArgs& a, const Slicing& sl, hipStream_t st) {
    dim3 grid((unsigned)cdiv(a.n, BS));
    if (c->prec == DNB_FP32C)
        hipLaunchKernelGGL((k_kdk<MODE, true>), grid, dim3(BS), 0, st, a, (const void*)c->part,
                           sl.S, sl.npad, c->js);
    else
        hipLaunchKernelGGL((k_kdk<MODE, false>), grid, dim3(BS), 0, st, a, (const void*)c->part,
                           sl.S, sl.npad, c->js);
}

hipError_t launch_kdk(dnb_ctx* c, KdkMode mode, const FwdArgs& a, hipStream_t st) {
    Slicing sl = slicing_for(a.n);
    switch (mode) {
        case KDK_FIRST: kdk_dispatch<KDK_FIRST>(c, a, sl, st); break;
        case KDK_MID: kdk_dispatch<KDK_MID>(c, a, sl, st); break;
        case KDK_LAST: kdk_dispatch<KDK_LAST>(c, a, sl, st); break;
        case KDK_ACC: kdk_dispatch<KDK_ACC>(c, a, sl, st); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ reverse --

__global__ __launch_bounds__(BS) void k_rev_stage(const double* __restrict__ x,
                                                  const double* __restrict__ mass,
                                                  const double* __restrict__ w, int64_t n,
                                                  const double* __restrict__ cpart, int nb,
                                                  float4* __restrict__ jsv,
                                                  double* __restrict__ cpart_out) {
    __shared__ double sh[3 * BS];
    double cx, cy, cz;
    centre_from(cpart, nb, n, sh, cx, cy, cz);
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    const double x0 = x[k], y0 = x[n + k], z0 = x[2 * n + k];
    if (ok) {
        jsv[i] = make_float4((float)(x0 - cx), (float)(y0 - cy), (float)(z0 - cz), (float)mass[i]);
        jsv[n + i] = make_float4((float)w[i], (float)w[n + i], (float)w[2 * n + i], 0.f);
    }
    write_block_sums(x0, y0, z0, ok, sh, cpart_out);
}

// Slice sums of the VJP kernel for particle i: J^T w, a_int (both times G) and the
// raw mass term sum_j (d.w_j) s^-3/2 (times G).
template <bool F32>
__device__ inline void vjp_sum(const void* part, int S, int64_t npad, int64_t i, double G,
                               bool with_mass, double (&g)[3], double (&a)[3], double& gm) {
    for (int c = 0; c < 3; ++c) g[c] = a[c] = 0.0;
    gm = 0.0;
    if (F32) {
        const float* p = (const float*)part;
        for (int s = 0; s < S; ++s) {
            const float* q = p + (int64_t)s * 14 * npad + i;
            for (int c = 0; c < 3; ++c) {
                g[c] += (double)q[c * npad]; g[c] += (double)q[(3 + c) * npad];
                a[c] += (double)q[(6 + c) * npad]; a[c] += (double)q[(9 + c) * npad];
            }
            if (with_mass) { gm += (double)q[12 * npad]; gm += (double)q[13 * npad]; }
        }
    } else {
        const double* p = (const double*)part;
        for (int s = 0; s < S; ++s) {
            const double* q = p + (int64_t)s * 7 * npad + i;
            for (int c = 0; c < 3; ++c) {
                g[c] += q[c * npad];
                a[c] += q[(3 + c) * npad];
            }
            if (with_mass) gm += q[6 * npad];
        }
    }
    for (int c = 0; c < 3; ++c) { g[c] *= G; a[c] *= G; }
    gm *= G;
}

template <bool F32>
__global__ __launch_bounds__(BS) void k_rev_kick(RevArgs a, const void* __restrict__ part, int S,
                                                 int64_t npad, float4* __restrict__ jsv) {
    __shared__ double sh[3 * BS];
    const int64_t n = a.n;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    const bool drift = a.x_prev != nullptr;

    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (F32 && drift) centre_from(a.cpart_in, a.nb_in, n, sh, cx, cy, cz);

    double g[3], ai[3], gm;
    vjp_sum<F32>(part, S, npad, k, a.pot.G, a.with_mass != 0, g, ai, gm);
    const double x = a.x_n[k], y = a.x_n[n + k], z = a.x_n[2 * n + k];
    const double wx = a.lv[k], wy = a.lv[n + k], wz = a.lv[2 * n + k];
    Ext e = ext_accel(a.pot, x, y, z);
    double hx, hy, hz;
    ext_hvp(a.pot, x, y, z, wx, wy, wz, hx, hy, hz);

    double lx = a.lx[k] + a.coef * (g[0] + hx);
    double ly = a.lx[n + k] + a.coef * (g[1] + hy);
    double lz = a.lx[2 * n + k] + a.coef * (g[2] + hz);
    const double kc = a.coef / a.dt;
    const double aw_int = ai[0] * wx + ai[1] * wy + ai[2] * wz;
    const double aw_ext = e.ax * wx + e.ay * wy + e.az * wz;
    double d_dt = kc * (aw_int + aw_ext);
    const double d_nfw = a.coef * (e.nx * wx + e.ny * wy + e.nz * wz);
    const double d_mn = a.coef * (e.mx * wx + e.my * wy + e.mz * wz);
    const double d_ms = a.coef * aw_int;

    double px = 0.0, py = 0.0, pz = 0.0;
    double nwx = wx, nwy = wy, nwz = wz;
    if (drift) {
        px = a.x_prev[k]; py = a.x_prev[n + k]; pz = a.x_prev[2 * n + k];
        const double inv = 1.0 / a.dt;
        const double vx = (x - px) * inv, vy = (y - py) * inv, vz = (z - pz) * inv;
        d_dt += vx * lx + vy * ly + vz * lz;
        nwx = wx + a.dt * lx; nwy = wy + a.dt * ly; nwz = wz + a.dt * lz;
    }
    if (ok) {
        a.lx[i] = lx; a.lx[n + i] = ly; a.lx[2 * n + i] = lz;
        a.accum[i] += d_nfw;
        a.accum[n + i] += d_mn;
        a.accum[2 * n + i] += d_dt;
        a.accum[3 * n + i] += d_ms;
        if (a.with_mass) a.accum[4 * n + i] -= a.coef * gm;
        if (drift) {
            a.lv[i] = nwx; a.lv[n + i] = nwy; a.lv[2 * n + i] = nwz;
            if (F32) {
                jsv[i] = make_float4((float)(px - cx), (float)(py - cy), (float)(pz - cz),
                                     (float)a.mass[i]);
                jsv[n + i] = make_float4((float)nwx, (float)nwy, (float)nwz, 0.f);
            }
        }
    }
    if (F32 && drift) write_block_sums(px, py, pz, ok, sh, a.cpart_out);
}

hipError_t launch_rev_stage(dnb_ctx* c, int64_t n, const double* x, const double* mass,
                            const double* w, const double* cpart, int nb, double* cpart_out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_rev_stage, dim3((unsigned)cdiv(n, BS)), dim3(BS), 0, st, x, mass, w, n,
                       cpart, nb, c->jsv, cpart_out);
    return hipGetLastError();
}

hipError_t launch_rev_kick(dnb_ctx* c, const RevArgs& a, hipStream_t st) {
    Slicing sl = slicing_for(a.n);
    dim3 grid((unsigned)cdiv(a.n, BS));
    if (c->prec == DNB_FP32C)
        hipLaunchKernelGGL((k_rev_kick<true>), grid, dim3(BS), 0, st, a, (const void*)c->partv,
                           sl.S, sl.npad, c->jsv);
    else
        hipLaunchKernelGGL((k_rev_kick<false>), grid, dim3(BS), 0, st, a, (const void*)c->partv,
                           sl.S, sl.npad, c->jsv);
    return hipGetLastError();
}

// Sum of nterms per-particle arrays [nterms][n] -> out[nterms]; one block,
// fixed order.
__global__ __launch_bounds__(BS) void k_reduce_rows5(const double* __restrict__ v, int64_t n,
                                                     int nterms, double* __restrict__ out) {
    __shared__ double sh[5 * BS];
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += BS)
        for (int t = 0; t < nterms; ++t) s[t] += v[t * n + i];
    block_sum<5>(s, sh);
    if (threadIdx.x == 0)
        for (int t = 0; t < nterms; ++t) out[t] = s[t];
}

hipError_t launch_reduce_accum(const double* accum, int64_t n, int nterms, double* out,
                               double* scratch, hipStream_t st) {
    (void)scratch;
    hipLaunchKernelGGL(k_reduce_rows5, dim3(1), dim3(BS), 0, st, accum, n, nterms, out);
    return hipGetLastError();
}

}  // namespace dnb
