// Internal declarations of libdnb: context layout, launch geometry and the FP64
// device functions of the host-galaxy potential.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dnb.h"
#include "host_logic.h"

namespace dnb {

// Launch geometry, buffer sizes, the host-galaxy parameter check and the tape
// descriptors are in host_logic.h (no HIP in it).

// Number of reduction blocks (and net-force records) of a system of n particles.
__host__ __device__ inline int red_blocks(int64_t n) { return (int)((n + RT - 1) / RT); }

// ------------------------------------------------------------- potential ---
struct Pot {
    double G, eps, m_nfw, rs_nfw, m_mn, a_mn, b_mn;
};

inline Pot to_pot(const dnb_pot& p) {
    return Pot{p.G, p.eps, p.m_nfw, p.rs_nfw, p.m_mn, p.a_mn, p.b_mn};
}

// mu(x) = ln(1+x) - x/(1+x): NFW enclosed-mass profile in units of the scale mass.
__device__ inline double nfw_mu(double x) {
    if (x < 1e-4) return x * x * (0.5 + x * (-2.0 / 3.0 + x * (0.75 - x * 0.8)));
    return log1p(x) - x / (1.0 + x);
}

// Acceleration of a unit-mass NFW halo (multiply by m_nfw): -G mu(r/rs) r_vec / r^3.
__device__ inline void nfw_unit(double G, double rs, double x, double y, double z,
                                double& ax, double& ay, double& az) {
    double r2 = x * x + y * y + z * z;
    if (r2 == 0.0) { ax = ay = az = 0.0; return; }
    double r = sqrt(r2);
    double g = G * nfw_mu(r / rs) / (r2 * r);
    ax = -g * x; ay = -g * y; az = -g * z;
}

// Acceleration of a unit-mass Miyamoto-Nagai disk.
__device__ inline void mn_unit(double G, double a, double b, double x, double y, double z,
                               double& ax, double& ay, double& az) {
    double S = sqrt(z * z + b * b);
    double A = a + S;
    double D2 = x * x + y * y + A * A;
    double k = G / (D2 * sqrt(D2));
    ax = -k * x; ay = -k * y;
    az = (S == 0.0) ? 0.0 : -k * z * A / S;
}

// Hessian of -Phi_NFW (unit mass) applied to w:  -g w - (g'/r)(r.w) r_vec,
// g = G mu / r^3, g' = G (1/(r^2 (r+rs)^2) - 3 mu / r^4).
__device__ inline void nfw_unit_hvp(double G, double rs, double x, double y, double z,
                                    double wx, double wy, double wz,
                                    double& hx, double& hy, double& hz) {
    double r2 = x * x + y * y + z * z;
    if (r2 == 0.0) { hx = hy = hz = 0.0; return; }
    double r = sqrt(r2);
    double mu = nfw_mu(r / rs);
    double g = G * mu / (r2 * r);
    double rp = r + rs;
    double gp = G * (1.0 / (r2 * rp * rp) - 3.0 * mu / (r2 * r2));
    double c = gp / r * (x * wx + y * wy + z * wz);
    hx = -g * wx - c * x; hy = -g * wy - c * y; hz = -g * wz - c * z;
}

// Hessian of -Phi_MN (unit mass) applied to w.  With S = sqrt(z^2+b^2),
// A = a + S, D^2 = R^2 + A^2 the matrix entries are
//   xx: -G (1/D^3 - 3x^2/D^5)    xy: 3G xy/D^5    xz: 3G x z A/(S D^5)
//   yy: -G (1/D^3 - 3y^2/D^5)    yz: 3G y z A/(S D^5)
//   zz: -G ((1 + a b^2/S^3)/D^3 - 3 z^2 A^2/(S^2 D^5)).
__device__ inline void mn_unit_hvp(double G, double a, double b, double x, double y, double z,
                                   double wx, double wy, double wz,
                                   double& hx, double& hy, double& hz) {
    double S = sqrt(z * z + b * b);
    double A = a + S;
    double D2 = x * x + y * y + A * A;
    double D = sqrt(D2);
    double iD3 = 1.0 / (D2 * D);
    double iD5 = iD3 / D2;
    double hxx = -G * (iD3 - 3.0 * x * x * iD5);
    double hyy = -G * (iD3 - 3.0 * y * y * iD5);
    double hxy = 3.0 * G * x * y * iD5;
    double hxz = 0.0, hyz = 0.0, hzz = -G * iD3;
    if (S != 0.0) {
        double zA_S = z * A / S;
        hxz = 3.0 * G * x * zA_S * iD5;
        hyz = 3.0 * G * y * zA_S * iD5;
        hzz = -G * ((1.0 + a * b * b / (S * S * S)) * iD3 - 3.0 * zA_S * zA_S * iD5);
    }
    hx = hxx * wx + hxy * wy + hxz * wz;
    hy = hxy * wx + hyy * wy + hyz * wz;
    hz = hxz * wx + hyz * wy + hzz * wz;
}

// Full external acceleration, and its two unit-mass parts (for the mass cotangents).
struct Ext {
    double ax, ay, az;        // total
    double nx, ny, nz;        // NFW per unit m_nfw
    double mx, my, mz;        // MN per unit m_mn
};

__device__ inline Ext ext_accel(const Pot& p, double x, double y, double z) {
    Ext e{};
    if (p.m_nfw != 0.0) nfw_unit(p.G, p.rs_nfw, x, y, z, e.nx, e.ny, e.nz);
    if (p.m_mn != 0.0) mn_unit(p.G, p.a_mn, p.b_mn, x, y, z, e.mx, e.my, e.mz);
    e.ax = p.m_nfw * e.nx + p.m_mn * e.mx;
    e.ay = p.m_nfw * e.ny + p.m_mn * e.my;
    e.az = p.m_nfw * e.nz + p.m_mn * e.mz;
    return e;
}

__device__ inline void ext_hvp(const Pot& p, double x, double y, double z, double wx, double wy,
                               double wz, double& hx, double& hy, double& hz) {
    hx = hy = hz = 0.0;
    double tx, ty, tz;
    if (p.m_nfw != 0.0) {
        nfw_unit_hvp(p.G, p.rs_nfw, x, y, z, wx, wy, wz, tx, ty, tz);
        hx += p.m_nfw * tx; hy += p.m_nfw * ty; hz += p.m_nfw * tz;
    }
    if (p.m_mn != 0.0) {
        mn_unit_hvp(p.G, p.a_mn, p.b_mn, x, y, z, wx, wy, wz, tx, ty, tz);
        hx += p.m_mn * tx; hy += p.m_mn * ty; hz += p.m_mn * tz;
    }
}

// ext_accel and ext_hvp at one point in one pass: the square roots, the NFW
// enclosed-mass profile and the shared quotients are formed once, with the same
// expressions as in those functions, so both results are the same bits.
// shape (nullable) receives the derivatives of the acceleration with respect to
// the three shape parameters, each dotted with w: (da/drs_nfw . w, da/da_mn . w,
// da/db_mn . w).  With x = r / rs, mu'(x) = x / (1 + x)^2 and dx/drs = -x / rs:
//   da_NFW/drs = G m_nfw x^2 / ((1 + x)^2 rs) r_vec / r^3.
// With S = sqrt(z^2 + b^2), A = a + S, D^2 = R^2 + A^2 (dD^2/da = 2 A,
// dS/db = b / S):
//   da_x/da = 3 G M x A / D^5 (likewise y),  da_z/da = -G M (z / S)(1/D^3 - 3 A^2/D^5),
//   da_x/db = (b / S) da_x/da,  da_z/db = G M z b (a / (S^3 D^3) + 3 A^2 / (S^2 D^5)),
// the z-derivatives (and b / S) taken as 0 where S = 0, as the acceleration's z
// component is.
__device__ inline void ext_accel_hvp(const Pot& p, double x, double y, double z, double wx,
                                     double wy, double wz, Ext& e, double& hx, double& hy,
                                     double& hz, double* shape = nullptr) {
    e = Ext{};
    hx = hy = hz = 0.0;
    double s_rs = 0.0, s_a = 0.0, s_b = 0.0;
    if (p.m_nfw != 0.0) {
        double r2 = x * x + y * y + z * z;
        double tx = 0.0, ty = 0.0, tz = 0.0;
        if (r2 != 0.0) {
            const double G = p.G, rs = p.rs_nfw;
            double r = sqrt(r2);
            double mu = nfw_mu(r / rs);
            double g = G * mu / (r2 * r);
            e.nx = -g * x; e.ny = -g * y; e.nz = -g * z;
            double rp = r + rs;
            double gp = G * (1.0 / (r2 * rp * rp) - 3.0 * mu / (r2 * r2));
            double c = gp / r * (x * wx + y * wy + z * wz);
            tx = -g * wx - c * x; ty = -g * wy - c * y; tz = -g * wz - c * z;
            if (shape) {
                const double xr = r / rs;
                const double q = xr / (1.0 + xr);
                s_rs = p.m_nfw * (G * (q * q / rs) / (r2 * r)) * (x * wx + y * wy + z * wz);
            }
        }
        hx += p.m_nfw * tx; hy += p.m_nfw * ty; hz += p.m_nfw * tz;
    }
    if (p.m_mn != 0.0) {
        const double G = p.G, a = p.a_mn, b = p.b_mn;
        double S = sqrt(z * z + b * b);
        double A = a + S;
        double D2 = x * x + y * y + A * A;
        double D = sqrt(D2);
        double k = G / (D2 * D);
        e.mx = -k * x; e.my = -k * y;
        e.mz = (S == 0.0) ? 0.0 : -k * z * A / S;
        double iD3 = 1.0 / (D2 * D);
        double iD5 = iD3 / D2;
        double hxx = -G * (iD3 - 3.0 * x * x * iD5);
        double hyy = -G * (iD3 - 3.0 * y * y * iD5);
        double hxy = 3.0 * G * x * y * iD5;
        double hxz = 0.0, hyz = 0.0, hzz = -G * iD3;
        if (S != 0.0) {
            double zA_S = z * A / S;
            hxz = 3.0 * G * x * zA_S * iD5;
            hyz = 3.0 * G * y * zA_S * iD5;
            hzz = -G * ((1.0 + a * b * b / (S * S * S)) * iD3 - 3.0 * zA_S * zA_S * iD5);
        }
        double tx = hxx * wx + hxy * wy + hxz * wz;
        double ty = hxy * wx + hyy * wy + hyz * wz;
        double tz = hxz * wx + hyz * wy + hzz * wz;
        hx += p.m_mn * tx; hy += p.m_mn * ty; hz += p.m_mn * tz;
        if (shape) {
            const double xyw = x * wx + y * wy;
            const double dxa = 3.0 * G * A * iD5;
            double bS = 0.0, dza = 0.0, dzb = 0.0;
            if (S != 0.0) {
                bS = b / S;
                dza = -G * (z / S) * (iD3 - 3.0 * A * A * iD5);
                dzb = G * z * b * (a / (S * S * S) * iD3 + 3.0 * A * A / (S * S) * iD5);
            }
            s_a = p.m_mn * (dxa * xyw + dza * wz);
            s_b = p.m_mn * (dxa * bS * xyw + dzb * wz);
        }
    }
    e.ax = p.m_nfw * e.nx + p.m_mn * e.mx;
    e.ay = p.m_nfw * e.ny + p.m_mn * e.my;
    e.az = p.m_nfw * e.nz + p.m_mn * e.mz;
    if (shape) { shape[0] = s_rs; shape[1] = s_a; shape[2] = s_b; }
}

// Deterministic sum over a block of BS threads of NV doubles per thread: a
// butterfly across the lanes of each wave (lane i adds lane i ^ m for m = 32 ..
// 1; x + y == y + x exactly, so every lane of a wave holds the same bits), then
// the BS / 64 wave sums in wave order.  Every thread gets the block's sums.
// sh: at least NV * BS / 64 doubles.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* sh) {
    constexpr int NW = BS / 64;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], m, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k * NW + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = sh[k * NW];
#pragma unroll
        for (int q = 1; q < NW; ++q) a += sh[k * NW + q];
        v[k] = a;
    }
    __syncthreads();
}

// Largest value over a block of BS threads (every thread gets it).  sh: at
// least BS / 64 doubles.
__device__ inline double block_max(double v, double* sh) {
    constexpr int NW = BS / 64;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double a = sh[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) a = fmax(a, sh[q]);
    __syncthreads();
    return a;
}
// ------------------------------------------------------------------ context --
}  // namespace dnb

struct dnb_ctx {
    int device;
    int64_t max_n;
    dnb_prec prec;
    int64_t slice_rows;      // capacity of S * npad
    int nbmax;               // max blocks of the O(N) kernels
    int target_blocks;       // pair-kernel blocks wanted per launch
    int smax;                // cap on the source slices of the square pair launches
    // forward path
    void* js;                // staged sources: FP32C float4 (x, y, z relative to a centre; m),
                             // FP64 double4 (x, y, z, m); padded to pad_sources(n)
    void* part;              // slice partials: FP32C float2 (hi, lo) [S][3][npad], FP64 double [S][3][npad]
    double* cpart;           // [2][nbmax][8] block records (positions and displacements, for the
                             // staging centre), double buffered
    double* vh;              // [3][max_n] half-step velocities of the running integration
    // reverse path
    void* jsv;               // staged VJP sources, interleaved per particle:
                             // [2 j] = (x, y, z, m), [2 j + 1] = (w, 0); float4 or double4
    void* partv;             // VJP partials: FP32C float2 (hi, lo) [S][4][npad], FP64 double [S][4][npad]
    double* cpartv;          // [2][nbmax][8]
    double* wscale;          // [2] cotangent staging scales of the reverse sweep
    float* muni;             // [DNB_BATCH_MAX][2] (flag, m): all masses of the system (or of
                             // ensemble member b) equal m (FP32C fast path)
    double* bparams;         // [DNB_BATCH_MAX][8] parameter table of a batched ensemble
    double* bwscale;         // [DNB_BATCH_MAX][2] cotangent staging scales of a batched sweep
    double* red;             // [nbmax][8] reduction scratch
    double* ared;            // [3][npadmax] FP32C internal accelerations reduced from the slices
    double* gred;            // [4][npadmax] FP32C J^T w (3 rows) and mass term reduced likewise
    double* aext_f;          // [3][npadmax] external acceleration at the staged positions, from the
                             // forward pair kernel's extra block row (FP32C), for the kick
    double* aext_v;          // [9][npadmax] the reverse kick's external-field terms, from the VJP
                             // pair kernel's extra block row (FP32C; see ExtRow)
    double* arec;            // [cdiv(npadmax, RT) + DNB_BATCH_MAX][4] net-force records
    double* grec;            // the same for J^T w
    int64_t* scan;           // [nbmax + 1] block minima and result of the state scan
    int checks;              // nonzero: the integrators scan their initial state first
    int ext_row;             // nonzero: small FP32C pair launches carry the external-field row
    int slice_major;         // nonzero: pair grids ordered (slices, target blocks)
    void* prof;              // host-side event pool of dnb_profile (null when off)
    // The reverse sweep recomputes checkpoint segments on a second stream of
    // its own (created on first use, default priority) while the caller's stream
    // sweeps the previous one; events: [0..1] segment buffer b recomputed,
    // [2..3] segment buffer b released by the sweep, [4] start of the sweep.
    hipStream_t rstream;
    hipEvent_t revents[5];
    // Descriptors of the tapes written by the most recent dnb_simulate calls:
    // dnb_simulate_vjp accepts only a tape, with its final positions and the
    // arguments it was written with, listed here.
    dnb::TapeRing tapes;
};

namespace dnb {

// Message returned by dnb_last_error() on this host thread.
void set_error(const char* msg);
// Host-side argument checks shared by the entry points (DNB_OK or DNB_ERR_ARG
// with the message set).
dnb_status check_pot_args(const dnb_pot* p, const char* fn);
dnb_status check_device_ptr(const void* p, const char* name, const char* fn);

// Geometry of the forward and VJP pair kernels for this context (FP64 uses one
// target per lane).
inline Slicing fwd_slicing(const dnb_ctx* c, int64_t n) {
    return pair_slicing(n, n, c->target_blocks, c->smax);
}
inline Slicing vjp_slicing(const dnb_ctx* c, int64_t n) {
    return pair_slicing(n, n, c->target_blocks, c->smax);
}
inline Slicing plain_slicing(const dnb_ctx* c, int64_t n) {
    return slicing_for(n, BS, c->target_blocks);
}
// Rectangular block: ni targets against n sources.  A block of few targets
// against many sources (one device's share of a split system) needs more slices
// than a square launch to fill the chip, so the cap is S_MAX_ROWS; S * npad stays
// below target_blocks * BS (the partial buffer's bound).
constexpr int S_MAX_ROWS = 256;
inline Slicing rows_slicing(const dnb_ctx* c, int64_t ni, int64_t n) {
    return pair_slicing(ni, n, c->target_blocks, S_MAX_ROWS);
}

// Kernel launchers (defined in the .hip files).  All return hipError_t of the launch.
enum KdkMode { KDK_FIRST = 0, KDK_MID = 1, KDK_LAST = 2, KDK_ACC = 3 };

// An extra row of blocks in a pair launch (blockIdx.y == 0, the source slices
// following in rows 1 .. S) that evaluates the external field at the FP64
// positions x[3][n] for the kick that follows, beside the pair sums (at small n
// the pair launch leaves most compute units idle):
//   forward (w null): the acceleration, rows 0-2;
//   reverse (w = the velocity cotangent): H w (rows 0-2), a_ext . w (3),
//   (da/dm_nfw) . w (4), (da/dm_mn) . w (5) and (da/dp) . w for the three shape
//   parameters (6-8), with the expressions of ext_accel_hvp and k_rev_kick, so
//   the kick gets the same bits as evaluating them itself.
struct ExtRow {
    const double* x;   // null: no extra row
    const double* w;
    Pot pot;
};

struct FwdArgs {
    int64_t n;
    const double* mass;
    Pot pot;
    double dt;
    // state
    const double* x;    // [3][n] positions read (x_n) ...
    double* x_out;      // ... and written (x_{n+1}); may equal x
    double* v;          // [3][n] full-step velocity (FIRST reads, MID/LAST write)
    double* vh;         // [3][n] half-step velocity
    double* acc_out;    // KDK_ACC: [3][n] output accelerations (nullable)
    double* aint_out;   // [3][n] internal (pair) acceleration at x, any mode (nullable)
    int with_ext;
    // centre bookkeeping
    const double* cpart_in;   // block sums of x (positions being kicked at)
    double* cpart_out;        // block sums of x_out
    int nb_in;                // number of blocks that wrote cpart_in
    // checkpoint: write (x, v) of this step to tape_state, and the centre used
    // for staging x_out to tape_centre_next and tape_centre_cur (each if non-null:
    // the first record of the next checkpoint, the second of this one)
    double* tape_state;
    double* tape_centre_next;
    double* tape_centre_cur;
    const double* centre_override;   // if non-null: centre to stage x_out with
    // FP32C inside the integrator: the internal accelerations reduced by
    // launch_fwd_reduce ([3][n]) and its net-force records (nr of them), from
    // which the kernel removes the net internal force; null: sum the slice
    // partials directly, no correction (dnb_accelerations)
    const double* ared;
    const double* arec;
    int nr;
    const double* aext;   // [3][n] external acceleration at x from an ExtRow (null: evaluate)
};

// Block records of x into cpart (layout REC of kdk_common.h): sums of x in
// [b][0..2]; with w non-null the block maximum of the |w| components in [b][3]
// (the cotangent scale of the reverse sweep); with v non-null the sums of the
// displacement dt v in [b][4..6] (the first drift of a run).
hipError_t launch_block_sums(const double* x, int64_t n, double* cpart, hipStream_t st,
                             const double* w = nullptr, const double* v = nullptr,
                             double dt = 0.0);
// Stage x (and mass) into ctx->js: FP32C relative to the centre (from the block
// sums cpart over nb blocks, or centre_override), FP64 as absolute positions.
// Pads the tail to pad_sources(n).  centre_out (nullable) receives the centre.
hipError_t launch_stage(dnb_ctx* c, const double* x, const double* mass, int64_t n,
                        const double* cpart, int nb, const double* centre_override,
                        double* centre_out, hipStream_t st);
// ext: the external-field row to add if the launch takes one (small FP32C
// systems); *ext_done (nullable) says whether it did, i.e. whether the kick may
// read ctx->aext_f (aext_v) instead of evaluating the field itself.
hipError_t launch_pair_fwd(dnb_ctx* c, int64_t n, double eps, hipStream_t st,
                           const ExtRow& ext = ExtRow{}, bool* ext_done = nullptr);
hipError_t launch_pair_fwd_rows(dnb_ctx* c, int64_t n, int64_t i0, int64_t ni, double eps,
                                hipStream_t st);
hipError_t launch_acc_rows(dnb_ctx* c, const double* x, int64_t n, int64_t i0, int64_t ni,
                           const Pot& pot, int with_ext, double* acc, hipStream_t st);
// Sets c->muni = (1, m) if all n masses equal m, else (0, 0); one block.
hipError_t launch_mass_info(dnb_ctx* c, const double* mass, int64_t n, hipStream_t st);
hipError_t launch_kdk(dnb_ctx* c, KdkMode mode, const FwdArgs& a, hipStream_t st);
// FP32C: reduce the forward slice partials of the last pair launch into c->ared
// and c->arec (records of cdiv(n, RT) target blocks).
hipError_t launch_fwd_reduce(dnb_ctx* c, int64_t n, const double* mass, double G,
                             hipStream_t st);
// FP32C: reduce the VJP slice partials into c->gred and c->grec, undoing the
// cotangent scale wscale[0].
hipError_t launch_vjp_reduce(dnb_ctx* c, int64_t n, double G, int with_mass,
                             const double* wscale, hipStream_t st);

struct RevArgs {
    int64_t n;
    const double* mass;
    Pot pot;
    double dt;
    double coef;            // dt or dt/2 for this kick
    const double* x_n;      // positions of the kick
    const double* x_prev;   // positions x_{n-1} (null: no drift, last reverse step)
    const double* aint;     // [3][n] internal acceleration at x_n (from the forward pass)
    double* lx;             // [3][n] position cotangent (in/out)
    double* lv;             // [3][n] velocity cotangent (in/out)
    double* accum;          // [8][n] per-particle running sums: m_nfw, m_mn, dt, mass scale,
                            // rs_nfw, a_mn, b_mn, mass
    int with_mass;
    const double* cpart_in; int nb_in; double* cpart_out;
    const double* wscale_in;   // scale the consumed cotangent was staged with (FP32C)
    double* wscale_out;        // scale of the cotangent staged by this kernel (FP32C)
    // FP32C: J^T w and the mass term reduced by launch_vjp_reduce ([4][n], scale
    // undone) and its records (nr), from which the kernel removes sum_k (J^T w)_k
    const double* gred;
    const double* grec;
    int nr;
    const double* aext;   // [9][n] the external-field terms of an ExtRow (null: evaluate)
    // Reverse sweep that steps the trajectory backward (rev != 0).  The kernel
    // takes the internal acceleration at x_n from the pair launch that summed it
    // with the VJP (FP32C: ared and its net-force records arec as the forward
    // reduction writes them; FP64: the slice partials fpart) instead of aint, and
    // undoes the step that led to x_n:
    //   v_n     = v_{n+1/2} - dt/2 a(x_n)     (rv_half; else rv_src holds v_n)
    //   v_{n-1/2} = v_n - dt/2 a(x_n),  x_{n-1} = x_n - dt v_{n-1/2}
    // writing v_{n-1/2} to rv_out and, when x_rec is set, x_{n-1} to x_rec (which
    // is then also x_prev); with x_rec null, x_prev holds x_{n-1} (a checkpoint).
    int rev;
    const double* rv_src;
    int rv_half;
    double* rv_out;
    double* x_rec;
    const double* ared;
    const double* arec;
    const void* fpart;
};

// xprev (nullable): the positions the sweep stages next, whose displacement from
// x the records in cpart_out carry for the next staging centre; without them,
// vback (nullable) stands in with the displacement -dtback vback.
hipError_t launch_rev_stage(dnb_ctx* c, int64_t n, const double* x, const double* mass,
                            const double* w, const double* cpart, int nb, double* cpart_out,
                            double* wscale_out, hipStream_t st, const double* xprev = nullptr,
                            const double* vback = nullptr, double dtback = 0.0);
hipError_t launch_pair_vjp(dnb_ctx* c, int64_t n, int with_mass, double eps, hipStream_t st,
                           const ExtRow& ext = ExtRow{}, bool* ext_done = nullptr);
hipError_t launch_pair_vjp_rows(dnb_ctx* c, int64_t n, int64_t i0, int64_t ni, int with_mass,
                                double eps, hipStream_t st);
hipError_t launch_pair_vjp_force(dnb_ctx* c, int64_t n, int with_mass, double eps,
                                 hipStream_t st);
hipError_t launch_vjp_force_reduce(dnb_ctx* c, int64_t n, const double* mass, double G,
                                   int with_mass, const double* wscale, hipStream_t st);
hipError_t launch_acc_vjp_rows(dnb_ctx* c, const double* x, const double* w, int64_t n,
                               int64_t i0, int64_t ni, const Pot& pot, int with_ext,
                               double* gpos, double* gmass, hipStream_t st);
hipError_t launch_rev_kick(dnb_ctx* c, const RevArgs& a, hipStream_t st);
hipError_t launch_reduce_accum(const double* accum, int64_t n, int nterms, double* out,
                               double* scratch, hipStream_t st);

hipError_t launch_mmd(dnb_ctx* c, int64_t n, const double* pos, int64_t m, const double* tgt,
                      double h, double* loss, double* gpos, hipStream_t st);
hipError_t launch_energy(dnb_ctx* c, int64_t n, const double* pos, const double* vel,
                         const double* mass, const Pot& p, double* out3, hipStream_t st);
hipError_t launch_orbit(const double* w0, const Pot& p, double dt, int64_t n_steps, double* w_out,
                        double* traj, hipStream_t st);
hipError_t launch_orbit_vjp(const double* traj, const Pot& p, double dt, int64_t n_steps,
                            const double* gw_out, double* gw0, double* gparams, hipStream_t st);
hipError_t launch_place(int64_t n, const double* w, const double* xi, const double* zeta,
                        double m_tot, double a_p, double G, double* pos, double* vel,
                        double* mass, hipStream_t st);
hipError_t launch_place_vjp(dnb_ctx* c, int64_t n, const double* zeta, double m_tot, double a_p,
                            double G, const double* gpos, const double* gvel, const double* gmass,
                            double* gw, double* gm_tot, hipStream_t st);

// Batched ensembles (batch.hip).  params_dev is the [batch][8] table on the device.
bool batch_fits(const dnb_ctx* c, int64_t batch, int64_t n);
hipError_t launch_simulate_batch(dnb_ctx* c, int64_t batch, int64_t n, double* pos, double* vel,
                                 const double* mass, const double* params_dev, int64_t n_steps,
                                 double* tape, hipStream_t st);
hipError_t launch_simulate_batch_vjp(dnb_ctx* c, int64_t batch, int64_t n, const double* mass,
                                     const double* params_dev, int64_t T, const double* tape,
                                     const double* pos_T, double* accum, double* lx, double* lv,
                                     double* gparams, hipStream_t st);
hipError_t launch_orbit_batch(int64_t batch, const double* w0, const double* params_dev,
                              int64_t n_steps, double* w_out, double* traj, hipStream_t st);
hipError_t launch_orbit_batch_vjp(int64_t batch, const double* traj, const double* params_dev,
                                  int64_t n_steps, const double* gw_out, double* gw0,
                                  double* gparams, hipStream_t st);
hipError_t launch_place_batch_vjp(dnb_ctx* c, int64_t batch, int64_t n, const double* zeta,
                                  const double* m_tot, double a_p, double G, const double* gpos,
                                  const double* gvel, double* gw, double* gm_tot,
                                  hipStream_t st);
hipError_t launch_place_batch(int64_t batch, int64_t n, const double* w, const double* xi,
                              const double* zeta, const double* m_tot, double a_p, double G,
                              double* pos, double* vel, double* mass, hipStream_t st);
bool mmd_batch_fits(const dnb_ctx* c, int64_t batch, int64_t n, int64_t m, bool grad,
                    bool per_member);
bool mmd_batch_targets_fits(const dnb_ctx* c, int64_t batch, int64_t n, int64_t n_tgt,
                            int64_t m);
hipError_t launch_mmd_batch_targets(dnb_ctx* c, int64_t batch, int64_t n, const double* pos,
                                    int64_t n_tgt, int64_t m, const double* tgts, double h,
                                    double* loss, hipStream_t st);

// Orbit fit (orbitfit.hip).  The model struct is declared in dnb_orbitfit.h.
}  // namespace dnb
struct dnb_track_model;
namespace dnb {
hipError_t launch_track_observe(const dnb_track_model& md, int K, const double* phi1,
                                const double* p, double* y, hipStream_t st);
hipError_t launch_track_eval(const dnb_track_model& md, const double* trk, int K, int batch,
                             const double* p, double* chi2, double* jtr, double* jtj,
                             hipStream_t st);
hipError_t launch_track_hessian(const dnb_track_model& md, const double* trk, int K, int batch,
                                const double* p, double* hess, double* cov, hipStream_t st);
size_t lm_workspace_bytes(int64_t batch);
hipError_t launch_track_lm(const dnb_track_model& md, const double* trk, int K, int batch,
                           double* p, int64_t n_iter, double lam0, double* chi2, void* work,
                           hipStream_t st);
// Debug scan: the index of the first non-finite particle of nsys systems (or
// INT64_MAX) into c->scan[nbmax]; see aux.hip.
hipError_t launch_scan_state(dnb_ctx* c, const double* x, const double* v, const double* m,
                             int64_t n, int64_t nsys, hipStream_t st);
hipError_t launch_mmd_batch(dnb_ctx* c, int64_t batch, int64_t n, const double* pos, int64_t m,
                            const double* tgt, int per_member, double h, double* loss,
                            double* gpos, hipStream_t st);

}  // namespace dnb
