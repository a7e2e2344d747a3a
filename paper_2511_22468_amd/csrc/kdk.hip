// O(N) kernels of the integrator and of its reverse sweep.
//
// Forward (Sec. 2.2.1: Velocity-Verlet with fixed steps, i.e. kick-drift-kick).
// One step n -> n+1 is two launches: the pair kernel at x_n, then k_kdk, which
// adds the slice partials in FP64, adds the FP64 host-galaxy acceleration, and
// performs, in the unmerged textbook order,
//     v_n      = v_half + dt/2 a(x_n)          (closing kick of step n-1)
//     v_half'  = v_n + dt/2 a(x_n)             (opening kick of step n)
//     x_{n+1}  = x_n + dt v_half'              (drift, FP64)
// It then stages x_{n+1} as the sources of the next pair kernel and, in FP32C
// mode, writes the block sums of x_{n+1}, from which the next launch takes its
// staging centre.
//
// Staging centre (FP32C).  Positions x_{n+1} are staged relative to the mean of
// x_n plus the mean displacement of the drift that produced x_n, i.e. the
// centre of x_n carried one step on (it only has to lie near the particles, but
// the closer it lies the more FP32 resolution the pair separations keep; the
// first step extrapolates with dt v_0).  The centre is a deterministic function
// of x_n and x_{n-1}, so a recomputation started from a checkpoint reproduces
// the forward run bit for bit once the checkpoint also stores the two centres
// that the run staged the checkpoint's positions and the step after with.
//
// Reverse (the exact discrete adjoint).  With the two half kicks that meet at x_n
// merged, the sweep newest-first is, for n = T .. 0,
//     lambda_x += c_n J(x_n)^T lambda_v            c_n = dt (dt/2 at n = 0, T)
//     then, for n > 0, the adjoint of the drift of step n-1:
//     lambda_v += dt lambda_x
// together with the cotangents of dt, the two host masses and the particle masses.
#include "dnb_internal.h"
#include "kdk_common.h"

namespace dnb {

__global__ __launch_bounds__(BS) void k_block_sums(const double* __restrict__ x, int64_t n,
                                                   double* __restrict__ cpart,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ v, double dt) {
    __shared__ double sh[3 * BS];
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    double dx = 0.0, dy = 0.0, dz = 0.0;
    if (v) { dx = dt * v[k]; dy = dt * v[n + k]; dz = dt * v[2 * n + k]; }
    write_block_sums(x[k], x[n + k], x[2 * n + k], dx, dy, dz, ok, sh, cpart);
    if (w) write_block_max(ok ? absmax3(w[k], w[n + k], w[2 * n + k]) : 0.0, sh, cpart);
}

template <bool F32>
__global__ __launch_bounds__(BS) void k_stage(const double* __restrict__ x,
                                              const double* __restrict__ mass, int64_t n,
                                              int64_t nj, const double* __restrict__ cpart,
                                              int nb, const double* __restrict__ centre_override,
                                              void* __restrict__ js,
                                              double* __restrict__ centre_out) {
    __shared__ double sh[3 * BS];
    double cx = 0.0, cy = 0.0, cz = 0.0;
    if (F32) {
        if (centre_override) {
            cx = centre_override[0]; cy = centre_override[1]; cz = centre_override[2];
        } else {
            centre_from(cpart, nb, n, sh, cx, cy, cz, false);
        }
    }
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i < nj) {
        const bool real = i < n;
        const int64_t k = real ? i : 0;
        put_source<F32>(js, i, real, x[k], x[n + k], x[2 * n + k], mass[k], cx, cy, cz);
    }
    if (F32 && centre_out && blockIdx.x == 0 && threadIdx.x == 0) {
        centre_out[0] = cx; centre_out[1] = cy; centre_out[2] = cz; centre_out[3] = 0.0;
    }
}

template <int MODE, bool F32>
__global__ __launch_bounds__(BS) void k_kdk(FwdArgs a, const void* __restrict__ part, int S,
                                            int64_t npad, int64_t nj, void* __restrict__ js) {
    __shared__ double sh[10 * BS / 64];
    const int64_t n = a.n;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    const bool drift = (MODE == KDK_FIRST || MODE == KDK_MID);
    const bool reduced = F32 && a.ared;

    // every load that does not wait for the block reductions, issued first
    const double x = a.x[k], y = a.x[n + k], z = a.x[2 * n + k];
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (reduced) { ax = a.ared[k]; ay = a.ared[n + k]; az = a.ared[2 * n + k]; }
    double ux = 0.0, uy = 0.0, uz = 0.0;     // v (FIRST) or v_half (MID, LAST)
    if (MODE == KDK_FIRST) { ux = a.v[k]; uy = a.v[n + k]; uz = a.v[2 * n + k]; }
    if (MODE == KDK_MID || MODE == KDK_LAST) { ux = a.vh[k]; uy = a.vh[n + k]; uz = a.vh[2 * n + k]; }
    const double mk = drift ? a.mass[k] : 0.0;
    const bool pre = a.with_ext && a.aext;   // external field from the pair launch's extra row
    double ex = 0.0, ey = 0.0, ez = 0.0;
    if (pre) { ex = a.aext[k]; ey = a.aext[n + k]; ez = a.aext[2 * n + k]; }

    // staging centre and net internal force (FP32C), one block reduction
    double cx = 0.0, cy = 0.0, cz = 0.0;
    double tot[4] = {0.0, 0.0, 0.0, 1.0};
    if (F32) {
        const bool centre = drift && !a.centre_override;
        if (centre && reduced) {
            centre_and_total(a.cpart_in, a.nb_in, n, a.arec, a.nr, sh, cx, cy, cz, tot);
        } else {
            if (centre) centre_from(a.cpart_in, a.nb_in, n, sh, cx, cy, cz, true);
            if (reduced) rec_total(a.arec, a.nr, sh, tot);
        }
        if (drift && a.centre_override) {
            cx = a.centre_override[0]; cy = a.centre_override[1]; cz = a.centre_override[2];
        }
    }

    if (reduced) {
        // the reduced internal acceleration minus the net internal force per unit mass
        const double inv_m = 1.0 / tot[3];
        ax -= tot[0] * inv_m;
        ay -= tot[1] * inv_m;
        az -= tot[2] * inv_m;
    } else {
        pair_sum<F32>(part, S, npad, k, a.pot.G, ax, ay, az);
    }
    if (a.aint_out && ok) {
        a.aint_out[i] = ax; a.aint_out[n + i] = ay; a.aint_out[2 * n + i] = az;
    }
    if (pre) {
        ax += ex; ay += ey; az += ez;
    } else if (a.with_ext) {
        Ext e = ext_accel(a.pot, x, y, z);
        ax += e.ax; ay += e.ay; az += e.az;
    }
    const double hdt = 0.5 * a.dt;
    double xn = x, yn = y, zn = z;
    if (ok) {
        if (MODE == KDK_ACC) {
            if (a.acc_out) { a.acc_out[i] = ax; a.acc_out[n + i] = ay; a.acc_out[2 * n + i] = az; }
        } else if (MODE == KDK_LAST) {
            a.v[i] = fma(hdt, ax, ux);
            a.v[n + i] = fma(hdt, ay, uy);
            a.v[2 * n + i] = fma(hdt, az, uz);
        } else {
            double vx, vy, vz;
            if (MODE == KDK_FIRST) {
                vx = ux; vy = uy; vz = uz;
            } else {
                vx = fma(hdt, ax, ux);
                vy = fma(hdt, ay, uy);
                vz = fma(hdt, az, uz);
            }
            if (a.tape_state) {
                double* t = a.tape_state;
                t[i] = x; t[n + i] = y; t[2 * n + i] = z;
                t[3 * n + i] = vx; t[4 * n + i] = vy; t[5 * n + i] = vz;
            }
            const double hx = fma(hdt, ax, vx), hy = fma(hdt, ay, vy), hz = fma(hdt, az, vz);
            xn = fma(a.dt, hx, x); yn = fma(a.dt, hy, y); zn = fma(a.dt, hz, z);
            a.vh[i] = hx; a.vh[n + i] = hy; a.vh[2 * n + i] = hz;
            a.x_out[i] = xn; a.x_out[n + i] = yn; a.x_out[2 * n + i] = zn;
        }
    }
    if (drift) {
        if (i < nj) put_source<F32>(js, i, ok, xn, yn, zn, mk, cx, cy, cz);
        if (F32) {
            write_block_sums(xn, yn, zn, xn - x, yn - y, zn - z, ok, sh, a.cpart_out);
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                for (double* t : {a.tape_centre_next, a.tape_centre_cur}) {
                    if (!t) continue;
                    t[0] = cx; t[1] = cy; t[2] = cz; t[3] = 0.0;
                }
            }
        }
    }
}

// Uniform-mass detection for the FP32C fast path: (1, m) when every mass equals
// mass[0] exactly (and is finite), else (0, 0).  One block, fixed reduction order.
__global__ __launch_bounds__(BS) void k_mass_info(const double* __restrict__ mass, int64_t n,
                                                  float* __restrict__ muni) {
    __shared__ double sh[BS];
    const double m0 = mass[0];
    double diff = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += BS) diff = fmax(diff, fabs(mass[i] - m0));
    sh[threadIdx.x] = diff;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool uni = sh[0] == 0.0 && isfinite(m0);
        muni[0] = uni ? 1.f : 0.f;
        muni[1] = uni ? (float)m0 : 0.f;
    }
}

hipError_t launch_mass_info(dnb_ctx* c, const double* mass, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_mass_info, dim3(1), dim3(BS), 0, st, mass, n, c->muni);
    return hipGetLastError();
}

// Blocks of an O(N) kernel that also writes the padded source array.
static inline unsigned onblocks(int64_t n) { return (unsigned)cdiv(pad_sources(n), BS); }

hipError_t launch_block_sums(const double* x, int64_t n, double* cpart, hipStream_t st,
                             const double* w, const double* v, double dt) {
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)cdiv(n, BS)), dim3(BS), 0, st, x, n, cpart, w,
                       v, dt);
    return hipGetLastError();
}

hipError_t launch_stage(dnb_ctx* c, const double* x, const double* mass, int64_t n,
                        const double* cpart, int nb, const double* centre_override,
                        double* centre_out, hipStream_t st) {
    const int64_t nj = pad_sources(n);
    if (c->prec == DNB_FP32C)
        hipLaunchKernelGGL(k_stage<true>, dim3(onblocks(n)), dim3(BS), 0, st, x, mass, n, nj,
                           cpart, nb, centre_override, c->js, centre_out);
    else
        hipLaunchKernelGGL(k_stage<false>, dim3(onblocks(n)), dim3(BS), 0, st, x, mass, n, nj,
                           cpart, nb, centre_override, c->js, centre_out);
    return hipGetLastError();
}

template <int MODE>
static void kdk_dispatch(dnb_ctx* c, const FwdArgs& a, const Slicing& sl, hipStream_t st) {
    dim3 grid(onblocks(a.n));
    const int64_t nj = pad_sources(a.n);
    if (c->prec == DNB_FP32C)
        hipLaunchKernelGGL((k_kdk<MODE, true>), grid, dim3(BS), 0, st, a, (const void*)c->part,
                           sl.S, sl.npad, nj, c->js);
    else
        hipLaunchKernelGGL((k_kdk<MODE, false>), grid, dim3(BS), 0, st, a, (const void*)c->part,
                           sl.S, sl.npad, nj, c->js);
}

hipError_t launch_kdk(dnb_ctx* c, KdkMode mode, const FwdArgs& a, hipStream_t st) {
    Slicing sl = fwd_slicing(c, a.n);
    switch (mode) {
        case KDK_FIRST: kdk_dispatch<KDK_FIRST>(c, a, sl, st); break;
        case KDK_MID: kdk_dispatch<KDK_MID>(c, a, sl, st); break;
        case KDK_LAST: kdk_dispatch<KDK_LAST>(c, a, sl, st); break;
        case KDK_ACC: kdk_dispatch<KDK_ACC>(c, a, sl, st); break;
    }
    return hipGetLastError();
}

// Accelerations of targets [i0, i0 + ni) from the partials of launch_pair_fwd_rows
// (the arithmetic of the KDK_ACC mode): acc [3][ni].
template <bool F32>
__global__ __launch_bounds__(BS) void k_acc_rows(const double* __restrict__ x, int64_t n,
                                                 int64_t i0, int64_t ni, Pot pot, int with_ext,
                                                 const void* __restrict__ part, int S,
                                                 int64_t npad, double* __restrict__ acc) {
    const int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (r >= ni) return;
    const int64_t i = i0 + r;
    double ax, ay, az;
    pair_sum<F32>(part, S, npad, r, pot.G, ax, ay, az);
    if (with_ext) {
        Ext e = ext_accel(pot, x[i], x[n + i], x[2 * n + i]);
        ax += e.ax; ay += e.ay; az += e.az;
    }
    acc[r] = ax; acc[ni + r] = ay; acc[2 * ni + r] = az;
}

hipError_t launch_acc_rows(dnb_ctx* c, const double* x, int64_t n, int64_t i0, int64_t ni,
                           const Pot& pot, int with_ext, double* acc, hipStream_t st) {
    const Slicing sl = rows_slicing(c, ni, n);
    if (c->prec == DNB_FP32C)
        hipLaunchKernelGGL(k_acc_rows<true>, dim3(sl.nblk), dim3(BS), 0, st, x, n, i0, ni, pot,
                           with_ext, (const void*)c->part, sl.S, sl.npad, acc);
    else
        hipLaunchKernelGGL(k_acc_rows<false>, dim3(sl.nblk), dim3(BS), 0, st, x, n, i0, ni, pot,
                           with_ext, (const void*)c->part, sl.S, sl.npad, acc);
    return hipGetLastError();
}

// ------------------------------------------------------------------ reverse --

template <bool F32>
__global__ __launch_bounds__(BS) void k_rev_stage(const double* __restrict__ x,
                                                  const double* __restrict__ mass,
                                                  const double* __restrict__ w, int64_t n,
                                                  int64_t nj, const double* __restrict__ cpart,
                                                  int nb, void* __restrict__ jsv,
                                                  double* __restrict__ cpart_out,
                                                  double* __restrict__ wscale_out,
                                                  const double* __restrict__ xprev,
                                                  const double* __restrict__ vback,
                                                  double dtback) {
    __shared__ double sh[3 * BS];
    double cx = 0.0, cy = 0.0, cz = 0.0;
    double S = 1.0;
    if (F32) {
        centre_from(cpart, nb, n, sh, cx, cy, cz, false);
        S = scale_from(cpart, nb, sh);
    }
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    const double x0 = x[k], y0 = x[n + k], z0 = x[2 * n + k];
    const double wx = w[k], wy = w[n + k], wz = w[2 * n + k];
    if (i < nj)
        put_source_w<F32>(jsv, i, ok, x0, y0, z0, mass[k], cx, cy, cz, wx * S, wy * S, wz * S);
    if (F32) {
        // the displacement to the positions the reverse sweep stages next
        double dx = 0.0, dy = 0.0, dz = 0.0;
        if (xprev) {
            dx = xprev[k] - x0; dy = xprev[n + k] - y0; dz = xprev[2 * n + k] - z0;
        } else if (vback) {   // positions not known yet: one drift back at velocity vback
            dx = -dtback * vback[k]; dy = -dtback * vback[n + k]; dz = -dtback * vback[2 * n + k];
        }
        write_block_sums(x0, y0, z0, dx, dy, dz, ok, sh, cpart_out);
        write_block_max(ok ? absmax3(wx, wy, wz) : 0.0, sh, cpart_out);
        if (blockIdx.x == 0 && threadIdx.x == 0) wscale_out[0] = S;
    }
}

template <bool F32>
__global__ __launch_bounds__(BS) void k_rev_kick(RevArgs a, const void* __restrict__ part, int S,
                                                 int64_t npad, int64_t nj,
                                                 void* __restrict__ jsv) {
    __shared__ double sh[10 * BS / 64];
    const int64_t n = a.n;
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const bool ok = i < n;
    const int64_t k = ok ? i : 0;
    const bool rev = a.rev != 0;
    const bool drift = a.x_prev != nullptr || (rev && a.x_rec != nullptr);
    const bool rebuild = rev && a.x_rec != nullptr;   // x_{n-1} from the step undone

    // every load that does not wait for the block reductions, issued first
    const double x = a.x_n[k], y = a.x_n[n + k], z = a.x_n[2 * n + k];
    const double wx = a.lv[k], wy = a.lv[n + k], wz = a.lv[2 * n + k];
    const double lx0 = a.lx[k], ly0 = a.lx[n + k], lz0 = a.lx[2 * n + k];
    double ai[3] = {0.0, 0.0, 0.0};
    if (!rev) { ai[0] = a.aint[k]; ai[1] = a.aint[n + k]; ai[2] = a.aint[2 * n + k]; }
    if (rev && F32) { ai[0] = a.ared[k]; ai[1] = a.ared[n + k]; ai[2] = a.ared[2 * n + k]; }
    double vs[3] = {0.0, 0.0, 0.0};
    if (rev && drift) { vs[0] = a.rv_src[k]; vs[1] = a.rv_src[n + k]; vs[2] = a.rv_src[2 * n + k]; }
    double g[3] = {0.0, 0.0, 0.0}, gm = 0.0;
    if (F32) {
        g[0] = a.gred[k]; g[1] = a.gred[n + k]; g[2] = a.gred[2 * n + k];
        if (a.with_mass) gm = a.gred[3 * n + k];
    }
    double px = 0.0, py = 0.0, pz = 0.0, mk = 0.0;
    if (drift) {
        if (!rebuild) { px = a.x_prev[k]; py = a.x_prev[n + k]; pz = a.x_prev[2 * n + k]; }
        mk = a.mass[k];
    }
    const double acc0[8] = {a.accum[k], a.accum[n + k], a.accum[2 * n + k], a.accum[3 * n + k],
                            a.accum[4 * n + k], a.accum[5 * n + k], a.accum[6 * n + k],
                            a.with_mass ? a.accum[7 * n + k] : 0.0};
    // the external-field terms from the pair launch's extra row, if it ran
    double xt[9];
    if (a.aext) {
#pragma unroll
        for (int c = 0; c < 9; ++c) xt[c] = a.aext[(int64_t)c * n + k];
    }

    // staging centre, cotangent scale and sum of J^T w (FP32C)
    double cx = 0.0, cy = 0.0, cz = 0.0, Sn = 1.0;
    if (F32) {
        double tot[4];
        if (drift) {
            centre_and_total(a.cpart_in, a.nb_in, n, a.grec, a.nr, sh, cx, cy, cz, tot);
            Sn = scale_from(a.cpart_in, a.nb_in, sh);
        } else {
            rec_total(a.grec, a.nr, sh, tot);
        }
        // the reduced J^T w (cotangent scale undone) minus its mean over the particles
        const double inv_n = 1.0 / (double)n;
        g[0] -= tot[0] * inv_n;
        g[1] -= tot[1] * inv_n;
        g[2] -= tot[2] * inv_n;
        if (rev) {
            // the internal acceleration summed with the VJP, minus the net internal
            // force per unit mass, as the forward kick takes it
            double tota[4];
            rec_total(a.arec, a.nr, sh, tota);
            const double inv_m = 1.0 / tota[3];
            ai[0] -= tota[0] * inv_m;
            ai[1] -= tota[1] * inv_m;
            ai[2] -= tota[2] * inv_m;
        }
    } else {
        vjp_sum<F32>(part, S, npad, k, a.pot.G, a.with_mass != 0, g, gm);
        if (rev) pair_sum<F32>(a.fpart, S, npad, k, a.pot.G, ai[0], ai[1], ai[2]);
    }
    double hx, hy, hz, aw_ext, nw, mw, shp[3];
    double ex = 0.0, ey = 0.0, ez = 0.0;   // external acceleration (reversal only)
    if (a.aext) {
        hx = xt[0]; hy = xt[1]; hz = xt[2];
        aw_ext = xt[3]; nw = xt[4]; mw = xt[5];
        shp[0] = xt[6]; shp[1] = xt[7]; shp[2] = xt[8];
    } else {
        Ext e;
        ext_accel_hvp(a.pot, x, y, z, wx, wy, wz, e, hx, hy, hz, shp);
        aw_ext = e.ax * wx + e.ay * wy + e.az * wz;
        nw = e.nx * wx + e.ny * wy + e.nz * wz;
        mw = e.mx * wx + e.my * wy + e.mz * wz;
        ex = e.ax; ey = e.ay; ez = e.az;
    }
    // the step that led to x_n undone, in the forward kick's expressions with -dt
    double vhx = 0.0, vhy = 0.0, vhz = 0.0;
    if (rev && drift) {
        const double fx = ai[0] + ex, fy = ai[1] + ey, fz = ai[2] + ez;
        const double mhdt = -0.5 * a.dt;
        double vx = vs[0], vy = vs[1], vz = vs[2];
        if (a.rv_half) { vx = fma(mhdt, fx, vx); vy = fma(mhdt, fy, vy); vz = fma(mhdt, fz, vz); }
        vhx = fma(mhdt, fx, vx); vhy = fma(mhdt, fy, vy); vhz = fma(mhdt, fz, vz);
        if (rebuild) { px = fma(-a.dt, vhx, x); py = fma(-a.dt, vhy, y); pz = fma(-a.dt, vhz, z); }
    }

    const double lx = fma(a.coef, g[0] + hx, lx0);
    const double ly = fma(a.coef, g[1] + hy, ly0);
    const double lz = fma(a.coef, g[2] + hz, lz0);
    const double kc = a.coef / a.dt;
    const double aw_int = ai[0] * wx + ai[1] * wy + ai[2] * wz;
    double d_dt = kc * (aw_int + aw_ext);
    const double d_nfw = a.coef * nw;
    const double d_mn = a.coef * mw;
    const double d_ms = a.coef * aw_int;

    double nwx = wx, nwy = wy, nwz = wz;
    if (drift) {
        const double inv = 1.0 / a.dt;
        const double vx = (x - px) * inv, vy = (y - py) * inv, vz = (z - pz) * inv;
        d_dt += vx * lx + vy * ly + vz * lz;
        nwx = fma(a.dt, lx, wx); nwy = fma(a.dt, ly, wy); nwz = fma(a.dt, lz, wz);
    }
    if (ok) {
        a.lx[i] = lx; a.lx[n + i] = ly; a.lx[2 * n + i] = lz;
        a.accum[i] = acc0[0] + d_nfw;
        a.accum[n + i] = acc0[1] + d_mn;
        a.accum[2 * n + i] = acc0[2] + d_dt;
        a.accum[3 * n + i] = acc0[3] + d_ms;
        a.accum[4 * n + i] = acc0[4] + a.coef * shp[0];
        a.accum[5 * n + i] = acc0[5] + a.coef * shp[1];
        a.accum[6 * n + i] = acc0[6] + a.coef * shp[2];
        if (a.with_mass) a.accum[7 * n + i] = acc0[7] - a.coef * gm;
        if (drift) { a.lv[i] = nwx; a.lv[n + i] = nwy; a.lv[2 * n + i] = nwz; }
        if (rev && drift) {
            a.rv_out[i] = vhx; a.rv_out[n + i] = vhy; a.rv_out[2 * n + i] = vhz;
            if (rebuild) { a.x_rec[i] = px; a.x_rec[n + i] = py; a.x_rec[2 * n + i] = pz; }
        }
    }
    if (drift) {
        if (i < nj)
            put_source_w<F32>(jsv, i, ok, px, py, pz, mk, cx, cy, cz, nwx * Sn, nwy * Sn,
                              nwz * Sn);
        if (F32) {
            write_block_sums(px, py, pz, px - x, py - y, pz - z, ok, sh, a.cpart_out);
            write_block_max(ok ? absmax3(nwx, nwy, nwz) : 0.0, sh, a.cpart_out);
            if (blockIdx.x == 0 && threadIdx.x == 0) a.wscale_out[0] = Sn;
        }
    }
}

__global__ __launch_bounds__(BS) void k_fwd_reduce(const float2* __restrict__ part, int S,
                                                   int64_t npad, int64_t n, double G,
                                                   const double* __restrict__ mass,
                                                   double* __restrict__ ared,
                                                   double* __restrict__ rec) {
    __shared__ double sh[3 * RG * RT];
    fwd_reduce_block(part, S, npad, n, G, mass, ared, rec, sh);
}

__global__ __launch_bounds__(BS) void k_vjp_reduce(const float2* __restrict__ part, int S,
                                                   int64_t npad, int64_t n, double G,
                                                   int with_mass,
                                                   const double* __restrict__ wscale,
                                                   double* __restrict__ gred,
                                                   double* __restrict__ rec) {
    __shared__ double sh[4 * RG * RT];
    vjp_reduce_block(part, S, npad, n, G, with_mass != 0, 1.0 / wscale[0], gred, rec, sh);
}

// Both reductions of the reverse sweep that steps the trajectory backward, in
// one launch: the VJP partials into gred as k_vjp_reduce, then the acceleration
// partials the same pair launch summed into ared as k_fwd_reduce (the same device
// code, so the same bits as the two launches).
__global__ __launch_bounds__(BS) void k_vjp_force_reduce(const float2* __restrict__ partv,
                                                         const float2* __restrict__ partf,
                                                         int S, int64_t npad, int64_t n,
                                                         double G, int with_mass,
                                                         const double* __restrict__ wscale,
                                                         const double* __restrict__ mass,
                                                         double* __restrict__ gred,
                                                         double* __restrict__ grec,
                                                         double* __restrict__ ared,
                                                         double* __restrict__ arec) {
    __shared__ double sh[4 * RG * RT];
    vjp_reduce_block(partv, S, npad, n, G, with_mass != 0, 1.0 / wscale[0], gred, grec, sh);
    __syncthreads();
    fwd_reduce_block(partf, S, npad, n, G, mass, ared, arec, sh);
}

hipError_t launch_vjp_force_reduce(dnb_ctx* c, int64_t n, const double* mass, double G,
                                   int with_mass, const double* wscale, hipStream_t st) {
    const Slicing sl = vjp_slicing(c, n);
    hipLaunchKernelGGL(k_vjp_force_reduce, dim3((unsigned)red_blocks(n)), dim3(BS), 0, st,
                       (const float2*)c->partv, (const float2*)c->part, sl.S, sl.npad, n, G,
                       with_mass, wscale, mass, c->gred, c->grec, c->ared, c->arec);
    return hipGetLastError();
}

hipError_t launch_fwd_reduce(dnb_ctx* c, int64_t n, const double* mass, double G,
                             hipStream_t st) {
    const Slicing sl = fwd_slicing(c, n);
    hipLaunchKernelGGL(k_fwd_reduce, dim3((unsigned)red_blocks(n)), dim3(BS), 0, st,
                       (const float2*)c->part, sl.S, sl.npad, n, G, mass, c->ared, c->arec);
    return hipGetLastError();
}

hipError_t launch_vjp_reduce(dnb_ctx* c, int64_t n, double G, int with_mass,
                             const double* wscale, hipStream_t st) {
    const Slicing sl = vjp_slicing(c, n);
    hipLaunchKernelGGL(k_vjp_reduce, dim3((unsigned)red_blocks(n)), dim3(BS), 0, st,
                       (const float2*)c->partv, sl.S, sl.npad, n, G, with_mass, wscale, c->gred,
                       c->grec);
    return hipGetLastError();
}

hipError_t launch_rev_stage(dnb_ctx* c, int64_t n, const double* x, const double* mass,
                            const double* w, const double* cpart, int nb, double* cpart_out,
                            double* wscale_out, hipStream_t st, const double* xprev,
                            const double* vback, double dtback) {
    const int64_t nj = pad_sources(n);
    if (c->prec == DNB_FP32C)
        hipLaunchKernelGGL(k_rev_stage<true>, dim3(onblocks(n)), dim3(BS), 0, st, x, mass, w, n,
                           nj, cpart, nb, c->jsv, cpart_out, wscale_out, xprev, vback, dtback);
    else
        hipLaunchKernelGGL(k_rev_stage<false>, dim3(onblocks(n)), dim3(BS), 0, st, x, mass, w, n,
                           nj, cpart, nb, c->jsv, cpart_out, wscale_out, xprev, vback, dtback);
    return hipGetLastError();
}

// Vector-Jacobian product of the accelerations for targets [i0, i0 + ni): with
// the cotangent w [3][n] of all accelerations, gpos[r] = (J^T w)_k (pair part
// from the partials of launch_pair_vjp_rows, plus H_ext(x_k) w_k) and
// gmass[r] = d(w . a)/dm_k, for k = i0 + r.
template <bool F32>
__global__ __launch_bounds__(BS) void k_acc_vjp_rows(const double* __restrict__ x,
                                                     const double* __restrict__ w, int64_t n,
                                                     int64_t i0, int64_t ni, Pot pot,
                                                     int with_ext, const void* __restrict__ part,
                                                     int S, int64_t npad,
                                                     const double* __restrict__ wscale,
                                                     double* __restrict__ gpos,
                                                     double* __restrict__ gmass) {
    const int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (r >= ni) return;
    const int64_t k = i0 + r;
    double g[3], gm;
    vjp_sum<F32>(part, S, npad, r, pot.G, gmass != nullptr, g, gm);
    if (F32) {
        const double inv_s = 1.0 / wscale[0];
        g[0] *= inv_s; g[1] *= inv_s; g[2] *= inv_s;
        gm *= inv_s;
    }
    if (with_ext) {
        double hx, hy, hz;
        ext_hvp(pot, x[k], x[n + k], x[2 * n + k], w[k], w[n + k], w[2 * n + k], hx, hy, hz);
        g[0] += hx; g[1] += hy; g[2] += hz;
    }
    gpos[r] = g[0]; gpos[ni + r] = g[1]; gpos[2 * ni + r] = g[2];
    if (gmass) gmass[r] = -gm;
}

hipError_t launch_acc_vjp_rows(dnb_ctx* c, const double* x, const double* w, int64_t n,
                               int64_t i0, int64_t ni, const Pot& pot, int with_ext,
                               double* gpos, double* gmass, hipStream_t st) {
    const Slicing sl = rows_slicing(c, ni, n);
    if (c->prec == DNB_FP32C)
        hipLaunchKernelGGL(k_acc_vjp_rows<true>, dim3(sl.nblk), dim3(BS), 0, st, x, w, n, i0, ni,
                           pot, with_ext, (const void*)c->partv, sl.S, sl.npad,
                           (const double*)c->wscale, gpos, gmass);
    else
        hipLaunchKernelGGL(k_acc_vjp_rows<false>, dim3(sl.nblk), dim3(BS), 0, st, x, w, n, i0,
                           ni, pot, with_ext, (const void*)c->partv, sl.S, sl.npad,
                           (const double*)c->wscale, gpos, gmass);
    return hipGetLastError();
}

hipError_t launch_rev_kick(dnb_ctx* c, const RevArgs& a, hipStream_t st) {
    Slicing sl = vjp_slicing(c, a.n);
    dim3 grid(onblocks(a.n));
    const int64_t nj = pad_sources(a.n);
    if (c->prec == DNB_FP32C)
        hipLaunchKernelGGL((k_rev_kick<true>), grid, dim3(BS), 0, st, a, (const void*)c->partv,
                           sl.S, sl.npad, nj, c->jsv);
    else
        hipLaunchKernelGGL((k_rev_kick<false>), grid, dim3(BS), 0, st, a, (const void*)c->partv,
                           sl.S, sl.npad, nj, c->jsv);
    return hipGetLastError();
}

// Sum of nterms per-particle arrays [nterms][n] -> out[nterms]; one block,
// fixed order.
// Sums over the particles of up to 7 rows [nterms][n] (one block, fixed order).
__global__ __launch_bounds__(BS) void k_reduce_rows(const double* __restrict__ v, int64_t n,
                                                    int nterms, double* __restrict__ out) {
    __shared__ double sh[7 * BS];
    double s[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += BS)
        for (int t = 0; t < nterms; ++t) s[t] += v[t * n + i];
    block_sum<7>(s, sh);
    if (threadIdx.x == 0)
        for (int t = 0; t < nterms; ++t) out[t] = s[t];
}

hipError_t launch_reduce_accum(const double* accum, int64_t n, int nterms, double* out,
                               double* scratch, hipStream_t st) {
    (void)scratch;
    hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(BS), 0, st, accum, n, nterms, out);
    return hipGetLastError();
}

}  // namespace dnb
