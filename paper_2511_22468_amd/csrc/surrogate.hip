// Learned-surrogate kernels: BF16 matrix-core MLP (forward, backward, MSE,
// Adam) and the orbit-frame density image of a stream.
//
// The MLP products use gfx950's v_mfma_f32_16x16x32_bf16 (BF16 inputs, FP32
// accumulation, 32 products per output per instruction).  A 256-thread block
// computes a 64 x 64 output tile; each of its four waves owns a 32 x 32 quadrant
// as 2 x 2 MFMA tiles; K advances in steps of 32 through LDS, where both operand
// tiles are stored K-contiguous (A as [m][k], B transposed as [n][k], rows padded
// to 80 bytes), so each lane reads its eight K-values of an operand with one
// 16-byte LDS load.  Operand strides are arguments, so transposed operands (W^T
// in the data gradient, X^T in the weight gradient) need no copies: the tile
// loader reads eight consecutive elements with one 16-byte global load along
// whichever dimension is contiguous, and falls back to bounds-checked,
// zero-filled element loads at ragged edges and unaligned addresses, so any
// M, N, K work (the first layer has K = 4).
// Epilogues fuse the bias, the GELU, and the GELU derivative of the backward
// pass.  The networks here are small (batch <= 65536, widths <= 2048); these
// kernels are latency-bound, not MFMA-bound.
#include <stdint.h>
#include <cstdio>

#include "dnb_internal.h"
#include "../../include/dnb_surrogate.h"

namespace dnb {

typedef __bf16 mfma_bf8 __attribute__((ext_vector_type(8)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int GK = 32;        // K per step of the GEMM
constexpr int GLD = GK + 8;   // LDS row length (elements): 80-byte rows, 16-byte aligned

// Eight consecutive elements p[0], p[step], ..., p[7 step] of a BF16 operand,
// of which the first `valid` exist (the rest read as zero): one 16-byte load
// when the elements are contiguous, whole and 16-byte aligned.
__device__ __forceinline__ u16x8 load8(const uint16_t* __restrict__ p, int64_t step, int valid) {
    if (step == 1 && valid >= 8 && ((uintptr_t)p & 15) == 0)
        return *(const u16x8*)p;
    u16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (j < valid) ? p[j * step] : (uint16_t)0;
    return v;
}

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu_f(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float pdf = expf(-0.5f * z * z) * 0.39894228040143268f;
    return fmaf(z, pdf, cdf);
}

enum Epi { EPI_PLAIN = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3, EPI_PARTIAL = 4 };

// Split of the inner dimension for products with few output tiles and a long
// inner dimension (the backward pass through the 2048-wide output layer): each
// block sums a K-slice into its own FP32 partial tile, k_splitk_epi adds the
// slices in order and applies the epilogue.
constexpr int KSPLIT_MAX = 16;
constexpr int KSPLIT_MIN_K = 1024;

// C[M x N] = A[M x K] . B[K x N];  A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn].
// EPI_PLAIN:     outf = C
// EPI_BIAS:      outf = C + bias
// EPI_BIAS_GELU: outf = z = C + bias, outb = bf16(gelu(z))
// EPI_GELU_BWD:  g = C * gelu'(zin), outf = g, outb = bf16(g)
// EPI_PARTIAL:   outf[z][M][ldo] = the product over the K-slice z (blockIdx.z) of
//                length kchunk
// Outputs are row-major with leading dimension ldo.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K,
                                                   const uint16_t* __restrict__ A, int64_t sam,
                                                   int64_t sak, const uint16_t* __restrict__ B,
                                                   int64_t sbk, int64_t sbn,
                                                   const float* __restrict__ bias,
                                                   const float* __restrict__ zin,
                                                   float* __restrict__ outf,
                                                   uint16_t* __restrict__ outb, int64_t ldo,
                                                   int kchunk) {
    __shared__ __attribute__((aligned(16))) uint16_t As[64][GLD];   // A tile, [m][k]
    __shared__ __attribute__((aligned(16))) uint16_t Bt[64][GLD];   // B tile, [n][k]
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    mfma_f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f4{0.f, 0.f, 0.f, 0.f};
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    // which operand dimension the loader walks eight elements along
    const bool a_k = sak == 1 || sam != 1;   // A: along k (else along m)
    const bool b_k = sbk == 1 || sbn != 1;   // B: along k (else along n)
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        // 64 x 32 elements of each operand, eight per thread
        if (a_k) {
            const int r = t >> 2, c = (t & 3) * 8;
            const int gm = m0 + r, gk = k0 + c;
            const int valid = gm < M ? max(0, min(8, kend - gk)) : 0;
            const u16x8 v = load8(A + (valid ? gm * sam + gk * sak : 0), sak, valid);
            *(u16x8*)&As[r][c] = v;
        } else {
            const int kk = t >> 3, c = (t & 7) * 8;
            const int gk = k0 + kk, gm = m0 + c;
            const int valid = gk < kend ? max(0, min(8, M - gm)) : 0;
            const u16x8 v = load8(A + (valid ? gm * sam + gk * sak : 0), sam, valid);
#pragma unroll
            for (int j = 0; j < 8; ++j) As[c + j][kk] = v[j];
        }
        if (b_k) {
            const int n = t >> 2, c = (t & 3) * 8;
            const int gn = n0 + n, gk = k0 + c;
            const int valid = gn < N ? max(0, min(8, kend - gk)) : 0;
            const u16x8 v = load8(B + (valid ? gk * sbk + gn * sbn : 0), sbk, valid);
            *(u16x8*)&Bt[n][c] = v;
        } else {
            const int kk = t >> 3, c = (t & 7) * 8;
            const int gk = k0 + kk, gn = n0 + c;
            const int valid = gk < kend ? max(0, min(8, N - gn)) : 0;
            const u16x8 v = load8(B + (valid ? gk * sbk + gn * sbn : 0), sbn, valid);
#pragma unroll
            for (int j = 0; j < 8; ++j) Bt[c + j][kk] = v[j];
        }
        __syncthreads();
        // lane l supplies K-values 8 (l / 16) .. 8 (l / 16) + 7 of row / column l % 16
        // for both operands, so the instruction pairs equal k whatever its internal
        // order of the 32 products
        const int kq = 8 * (lane >> 4);
        mfma_bf8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const u16x8 va = *(const u16x8*)&As[wr + i * 16 + (lane & 15)][kq];
            const u16x8 vb = *(const u16x8*)&Bt[wc + i * 16 + (lane & 15)][kq];
            a[i] = __builtin_bit_cast(mfma_bf8, va);
            b[i] = __builtin_bit_cast(mfma_bf8, vb);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wr + i * 16 + 4 * (lane >> 4) + q;
                const int col = n0 + wc + j * 16 + (lane & 15);
                if (row >= M || col >= N) continue;
                const float c = acc[i][j][q];
                const int64_t o = (int64_t)row * ldo + col;
                if (EPI == EPI_PARTIAL) {
                    outf[(int64_t)blockIdx.z * M * ldo + o] = c;
                } else if (EPI == EPI_PLAIN) {
                    outf[o] = c;
                } else if (EPI == EPI_BIAS) {
                    outf[o] = c + bias[col];
                } else if (EPI == EPI_BIAS_GELU) {
                    const float z = c + bias[col];
                    outf[o] = z;
                    outb[o] = f2bf(gelu_f(z));
                } else {
                    const float g = c * gelu_grad_f(zin[o]);
                    outf[o] = g;
                    outb[o] = f2bf(g);
                }
            }
}

// Sum of the K-slice partials part[splits][M][N] in slice order, then the
// epilogue EPI (EPI_PLAIN or EPI_GELU_BWD) into row-major outputs (ldo = N).
template <int EPI>
__global__ void k_splitk_epi(int M, int N, int splits, const float* __restrict__ part,
                             const float* __restrict__ zin, float* __restrict__ outf,
                             uint16_t* __restrict__ outb) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (int64_t)M * N) return;
    float c = 0.f;
    for (int z = 0; z < splits; ++z) c += part[(int64_t)z * M * N + o];
    if (EPI == EPI_PLAIN) {
        outf[o] = c;
    } else {
        const float g = c * gelu_grad_f(zin[o]);
        outf[o] = g;
        outb[o] = f2bf(g);
    }
}

// kpart: room for KSPLIT_MAX partial products of M x N (null: no split).
template <int EPI>
static void gemm(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak,
                 const uint16_t* B, int64_t sbk, int64_t sbn, const float* bias, const float* zin,
                 float* outf, uint16_t* outb, int64_t ldo, hipStream_t st,
                 float* kpart = nullptr) {
    dim3 grid((unsigned)cdiv(N, 64), (unsigned)cdiv(M, 64));
    const int64_t tiles = (int64_t)grid.x * grid.y;
    if ((EPI == EPI_PLAIN || EPI == EPI_GELU_BWD) && kpart && K >= KSPLIT_MIN_K && tiles < 64 &&
        ldo == N) {
        int splits = K / 128;
        if (splits > KSPLIT_MAX) splits = KSPLIT_MAX;
        const int kchunk = (int)(cdiv(cdiv(K, splits), GK) * GK);
        splits = (int)cdiv(K, kchunk);
        hipLaunchKernelGGL(k_gemm_bf16<EPI_PARTIAL>, dim3(grid.x, grid.y, (unsigned)splits),
                           dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, bias, zin, kpart,
                           (uint16_t*)nullptr, ldo, kchunk);
        hipLaunchKernelGGL(k_splitk_epi<EPI>, dim3((unsigned)cdiv((int64_t)M * N, 256)),
                           dim3(256), 0, st, M, N, splits, (const float*)kpart, zin, outf, outb);
        return;
    }
    hipLaunchKernelGGL(k_gemm_bf16<EPI>, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk,
                       sbn, bias, zin, outf, outb, ldo, K);
}

__global__ void k_bcast_rows(int64_t n, int cols, const float* __restrict__ row,
                             float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = row[i % cols];
}

__global__ void k_fill0(int64_t n, float* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.f;
}

__global__ void k_clamp(int64_t n, float* __restrict__ x, float lo, float hi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = fminf(hi, fmaxf(lo, x[i]));
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// Column sums of g [rows][cols] (bias gradient), one thread per column, fixed
// order; four rows' loads in flight.
__global__ void k_colsum(int rows, int cols, const float* __restrict__ g, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
#pragma unroll 4
    for (int r = 0; r < rows; ++r) s += g[(int64_t)r * cols + c];
    out[c] = s;
}

// Mean squared error and its gradient in one block of 1024 threads; thread t
// takes elements t, t + 1024, ... (coalesced, four loads in flight, fixed order).
constexpr int MSE_T = 1024;
__global__ __launch_bounds__(MSE_T) void k_mse(int64_t n, const float* __restrict__ y,
                                               const float* __restrict__ t,
                                               double* __restrict__ loss,
                                               float* __restrict__ dy) {
    __shared__ double sh[MSE_T];
    double s = 0.0;
    const float sc = (float)(2.0 / (double)n);
#pragma unroll 4
    for (int64_t i = threadIdx.x; i < n; i += MSE_T) {
        const float d = y[i] - t[i];
        s += (double)d * (double)d;
        dy[i] = sc * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = MSE_T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = sh[0] / (double)n;
}

__global__ void k_adam(int64_t n, float* __restrict__ p, uint16_t* __restrict__ pb,
                       float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = f2bf(pi);
}

// Network geometry and workspace layout.
constexpr int NL = 4;
constexpr int LIN[NL] = {4, 256, 256, 256};
constexpr int LOUT[NL] = {256, 256, 256, 2048};

inline int64_t w_off(int l) {
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += (int64_t)LIN[k] * LOUT[k] + LOUT[k];
    return o;
}
inline int64_t b_off(int l) { return w_off(l) + (int64_t)LIN[l] * LOUT[l]; }
inline int64_t param_count() { return w_off(NL); }

struct MlpWs {
    uint16_t* a[NL];     // layer inputs, BF16 [B][in_l]
    float* z[NL - 1];    // hidden pre-activations, FP32 [B][out_l]
    float* g;            // gradient, FP32 [B][2048]
    uint16_t* gb;        // gradient, BF16 [B][2048]
    float* h;            // gradient, FP32 [B][256]
    uint16_t* hb;        // gradient, BF16 [B][256]
    float* kpart;        // split-K partial products, FP32 [KSPLIT_MAX][B][256]
};

inline int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

inline int64_t mlp_ws_layout(int64_t B, char* base, MlpWs* w) {
    int64_t off = 0;
    auto take = [&](int64_t bytes) { char* p = base ? base + off : nullptr; off += align256(bytes); return p; };
    for (int l = 0; l < NL; ++l) { char* p = take(2 * B * LIN[l]); if (w) w->a[l] = (uint16_t*)p; }
    for (int l = 0; l < NL - 1; ++l) { char* p = take(4 * B * LOUT[l]); if (w) w->z[l] = (float*)p; }
    char* p;
    p = take(4 * B * 2048); if (w) w->g = (float*)p;
    p = take(2 * B * 2048); if (w) w->gb = (uint16_t*)p;
    p = take(4 * B * 256); if (w) w->h = (float*)p;
    p = take(2 * B * 256); if (w) w->hb = (uint16_t*)p;
    p = take(4 * (int64_t)KSPLIT_MAX * B * 256); if (w) w->kpart = (float*)p;
    return off;
}

// --------------------------------------------------------------- density grid --
struct Frame { double e1[3], e2[3], n[3]; };

__global__ void k_grid_count(int64_t n, const double* __restrict__ pos, Frame f,
                             unsigned int* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
    const double r = sqrt(x * x + y * y + z * z);
    const double u = x * f.e1[0] + y * f.e1[1] + z * f.e1[2];
    const double w = x * f.e2[0] + y * f.e2[1] + z * f.e2[2];
    const double h = x * f.n[0] + y * f.n[1] + z * f.n[2];
    const double phi1 = atan2(w, u);
    const double phi2 = asin(fmin(1.0, fmax(-1.0, h / r)));
    const double pi = 3.141592653589793;
    const int i1 = (int)floor((phi1 + pi) / (2.0 * pi) * 64.0);
    const int i2 = (int)floor((phi2 + 0.1) / 0.2 * 32.0);
    if (i1 >= 0 && i1 < 64 && i2 >= 0 && i2 < 32) atomicAdd(&cnt[i2 * 64 + i1], 1u);
}

// One block: blur along phi1 (periodic), then phi2 (zero padded), normalise.
__global__ __launch_bounds__(BS) void k_grid_blur(const unsigned int* __restrict__ cnt,
                                                  float* __restrict__ out) {
    __shared__ double c[2048];
    __shared__ double t[2048];
    __shared__ double sh[BS];
    double k[7], ks = 0.0;
    for (int d = -3; d <= 3; ++d) { k[d + 3] = exp(-0.5 * d * d); ks += k[d + 3]; }
    for (int d = 0; d < 7; ++d) k[d] /= ks;
    for (int e = threadIdx.x; e < 2048; e += BS) c[e] = (double)cnt[e];
    __syncthreads();
    for (int e = threadIdx.x; e < 2048; e += BS) {
        const int r = e >> 6, col = e & 63;
        double s = 0.0;
        for (int d = -3; d <= 3; ++d) s += k[d + 3] * c[r * 64 + ((col - d + 64) & 63)];
        t[e] = s;
    }
    __syncthreads();
    double v[8];
    double tot[1] = {0.0};
    for (int q = 0; q < 8; ++q) {
        const int e = threadIdx.x + q * BS;
        const int r = e >> 6, col = e & 63;
        double s = 0.0;
        for (int d = -3; d <= 3; ++d) {
            const int rr = r - d;
            if (rr >= 0 && rr < 32) s += k[d + 3] * t[rr * 64 + col];
        }
        v[q] = s;
        tot[0] += s;
    }
    block_sum<1>(tot, sh);
    const double inv = tot[0] > 0.0 ? 1.0 / tot[0] : 0.0;
    for (int q = 0; q < 8; ++q) out[threadIdx.x + q * BS] = (float)(v[q] * inv);
}

}  // namespace dnb

using namespace dnb;

namespace {
dnb_status sfail(const char* m) {
    set_error(m);
    return DNB_ERR_ARG;
}
bool is_dev(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) { (void)hipGetLastError(); return false; }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}
dnb_status hip_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return DNB_OK;
    char msg[256];
    snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
    set_error(msg);
    return DNB_ERR_HIP;
}
}  // namespace

extern "C" {

int64_t dnb_mlp_param_count(void) { return param_count(); }

int64_t dnb_mlp_workspace_bytes(int64_t batch) {
    if (batch < 1) return -1;
    return mlp_ws_layout(batch, nullptr, nullptr);
}

dnb_status dnb_mlp_to_bf16(int64_t count, const float* params, uint16_t* params_bf16,
                           void* stream) {
    if (count < 1 || !is_dev(params) || !is_dev(params_bf16)) return sfail("dnb_mlp_to_bf16: bad argument");
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)cdiv(count, 256)), dim3(256), 0,
                       (hipStream_t)stream, count, params, params_bf16);
    return hip_status("dnb_mlp_to_bf16");
}

dnb_status dnb_mlp_forward(const float* params, const uint16_t* pb, int64_t B, const float* x,
                           float* y, void* workspace, void* stream) {
    if (B < 16 || B > 65536 || B % 16 != 0) return sfail("dnb_mlp_forward: batch must be a multiple of 16 in [16, 65536]");
    if (!is_dev(params) || !is_dev(pb) || !is_dev(x) || !is_dev(y) || !is_dev(workspace))
        return sfail("dnb_mlp_forward: every pointer must be device memory");
    hipStream_t st = (hipStream_t)stream;
    MlpWs w;
    mlp_ws_layout(B, (char*)workspace, &w);
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)cdiv(B * 4, 256)), dim3(256), 0, st, B * 4, x,
                       w.a[0]);
    for (int l = 0; l < NL; ++l) {
        const uint16_t* W = pb + w_off(l);
        const float* bias = params + b_off(l);
        const int K = LIN[l], N = LOUT[l];
        if (l < NL - 1)
            gemm<EPI_BIAS_GELU>((int)B, N, K, w.a[l], K, 1, W, N, 1, bias, nullptr, w.z[l],
                                w.a[l + 1], N, st);
        else
            gemm<EPI_BIAS>((int)B, N, K, w.a[l], K, 1, W, N, 1, bias, nullptr, y, nullptr, N, st);
    }
    return hip_status("dnb_mlp_forward");
}

dnb_status dnb_mlp_backward(const uint16_t* pb, int64_t B, const float* dy, void* workspace,
                            float* grads, float* dx, void* stream) {
    if (B < 16 || B > 65536 || B % 16 != 0) return sfail("dnb_mlp_backward: bad batch");
    if (!is_dev(pb) || !is_dev(dy) || !is_dev(workspace) || (grads && !is_dev(grads)) ||
        (dx && !is_dev(dx)) || (!grads && !dx))
        return sfail("dnb_mlp_backward: every pointer must be device memory, grads or dx non-null");
    hipStream_t st = (hipStream_t)stream;
    MlpWs w;
    mlp_ws_layout(B, (char*)workspace, &w);
    // output layer: the incoming cotangent is the gradient of its pre-activation
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)cdiv(B * 2048, 256)), dim3(256), 0, st,
                       B * 2048, dy, w.gb);
    const float* gf = dy;            // FP32 gradient of the current layer's pre-activation
    const uint16_t* gbf = w.gb;      // its BF16 copy
    for (int l = NL - 1; l >= 0; --l) {
        const int K = LIN[l], N = LOUT[l];
        if (grads) {
            // dW_l = a_l^T . g  (M = K, N = N, inner dimension = batch)
            gemm<EPI_PLAIN>(K, N, (int)B, w.a[l], 1, K, gbf, N, 1, nullptr, nullptr,
                            grads + w_off(l), nullptr, N, st);
            hipLaunchKernelGGL(k_colsum, dim3((unsigned)cdiv(N, 256)), dim3(256), 0, st, (int)B,
                               N, gf, grads + b_off(l));
        }
        const uint16_t* W = pb + w_off(l);
        if (l > 0) {
            // g_{l-1} = (g . W_l^T) * gelu'(z_{l-1})
            float* hf = (l % 2 == 1) ? w.h : w.g;
            uint16_t* hb = (l % 2 == 1) ? w.hb : w.gb;
            if (l == NL - 1) { hf = w.h; hb = w.hb; }
            gemm<EPI_GELU_BWD>((int)B, K, N, gbf, N, 1, W, 1, N, nullptr, w.z[l - 1], hf, hb, K,
                               st, w.kpart);
            gf = hf;
            gbf = hb;
        } else if (dx) {
            gemm<EPI_PLAIN>((int)B, K, N, gbf, N, 1, W, 1, N, nullptr, nullptr, dx, nullptr, K, st,
                            w.kpart);
        }
    }
    return hip_status("dnb_mlp_backward");
}

dnb_status dnb_mlp_mse(int64_t count, const float* y, const float* t, double* loss, float* dy,
                       void* stream) {
    if (count < 1 || !is_dev(y) || !is_dev(t) || !is_dev(loss) || !is_dev(dy))
        return sfail("dnb_mlp_mse: bad argument");
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(MSE_T), 0, (hipStream_t)stream, count, y, t, loss,
                       dy);
    return hip_status("dnb_mlp_mse");
}

dnb_status dnb_mlp_adam(int64_t count, float* params, uint16_t* pb, float* m, float* v,
                        const float* grads, double lr, double beta1, double beta2, double eps,
                        int64_t t, void* stream) {
    if (count < 1 || t < 1 || !is_dev(params) || !is_dev(pb) || !is_dev(m) || !is_dev(v) ||
        !is_dev(grads))
        return sfail("dnb_mlp_adam: bad argument");
    const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, (hipStream_t)stream,
                       count, params, pb, m, v, grads, (float)lr, (float)beta1, (float)beta2,
                       (float)eps, (float)c1, (float)c2);
    return hip_status("dnb_mlp_adam");
}

int64_t dnb_mlp_invert_workspace_bytes(int64_t batch) {
    if (batch < 1) return -1;
    // network workspace, y and dy [B][2048], the broadcast target [B][2048],
    // dx [B][4], the BF16 copy of u and the Adam moments of u, the loss
    return mlp_ws_layout(batch, nullptr, nullptr) + 3 * align256(4 * batch * 2048) +
           align256(4 * batch * 4) + align256(2 * batch * 4) + 2 * align256(4 * batch * 4) +
           align256(8);
}

dnb_status dnb_mlp_invert(const float* params, const uint16_t* pb, int64_t B, const float* target,
                          float* u, int64_t iters, double lr, void* workspace, void* stream) {
    if (B < 16 || B > 65536 || B % 16 != 0) return sfail("dnb_mlp_invert: batch must be a multiple of 16 in [16, 65536]");
    if (iters < 1) return sfail("dnb_mlp_invert: iters must be >= 1");
    if (!(lr > 0)) return sfail("dnb_mlp_invert: lr must be > 0");
    if (!is_dev(params) || !is_dev(pb) || !is_dev(target) || !is_dev(u) || !is_dev(workspace))
        return sfail("dnb_mlp_invert: every pointer must be device memory");
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)workspace;
    int64_t off = mlp_ws_layout(B, nullptr, nullptr);
    auto take = [&](int64_t bytes) { char* p = base + off; off += align256(bytes); return p; };
    float* y = (float*)take(4 * B * 2048);
    float* dy = (float*)take(4 * B * 2048);
    float* tgt = (float*)take(4 * B * 2048);
    float* dx = (float*)take(4 * B * 4);
    uint16_t* ub = (uint16_t*)take(2 * B * 4);
    float* mu = (float*)take(4 * B * 4);
    float* vu = (float*)take(4 * B * 4);
    double* loss = (double*)take(8);
    const int64_t nu = 4 * B, ny = 2048 * B;
    hipLaunchKernelGGL(k_bcast_rows, dim3((unsigned)cdiv(ny, 256)), dim3(256), 0, st, ny, 2048,
                       target, tgt);
    hipLaunchKernelGGL(k_fill0, dim3((unsigned)cdiv(nu, 256)), dim3(256), 0, st, nu, mu);
    hipLaunchKernelGGL(k_fill0, dim3((unsigned)cdiv(nu, 256)), dim3(256), 0, st, nu, vu);
    for (int64_t it = 1; it <= iters; ++it) {
        dnb_status s = dnb_mlp_forward(params, pb, B, u, y, workspace, stream);
        if (s != DNB_OK) return s;
        hipLaunchKernelGGL(k_mse, dim3(1), dim3(MSE_T), 0, st, ny, (const float*)y,
                           (const float*)tgt, loss, dy);
        s = dnb_mlp_backward(pb, B, dy, workspace, nullptr, dx, stream);
        if (s != DNB_OK) return s;
        s = dnb_mlp_adam(nu, u, ub, mu, vu, dx, lr, 0.9, 0.999, 1e-8, it, stream);
        if (s != DNB_OK) return s;
        hipLaunchKernelGGL(k_clamp, dim3((unsigned)cdiv(nu, 256)), dim3(256), 0, st, nu, u, -1.f,
                           1.f);
    }
    return hip_status("dnb_mlp_invert");
}

int64_t dnb_grid_workspace_bytes(void) { return 2048 * sizeof(unsigned int); }

dnb_status dnb_density_grid(int64_t n, const double* pos, const double* frame9, float* grid,
                            void* workspace, void* stream) {
    if (n < 1 || !frame9 || !is_dev(pos) || !is_dev(grid) || !is_dev(workspace))
        return sfail("dnb_density_grid: bad argument");
    Frame f;
    for (int c = 0; c < 3; ++c) { f.e1[c] = frame9[c]; f.e2[c] = frame9[3 + c]; f.n[c] = frame9[6 + c]; }
    hipStream_t st = (hipStream_t)stream;
    unsigned int* cnt = (unsigned int*)workspace;
    if (hipMemsetAsync(cnt, 0, 2048 * sizeof(unsigned int), st) != hipSuccess)
        return hip_status("dnb_density_grid: memset");
    hipLaunchKernelGGL(k_grid_count, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, n, pos, f,
                       cnt);
    hipLaunchKernelGGL(k_grid_blur, dim3(1), dim3(BS), 0, st, cnt, grid);
    return hip_status("dnb_density_grid");
}

}  // extern "C"
