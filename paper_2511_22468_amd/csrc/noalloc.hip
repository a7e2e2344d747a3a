// dnb_accelerations_noalloc: the accelerations of dnb_accelerations without a
// context and without any device allocation, for callers that cannot allocate
// (code under stream capture, serving loops, harnesses that forbid hipMalloc).
//
// The staged sources, the slice partials and the small reduction records the
// kernels need live in one file-scope device array, `scratch`, which the code
// object carries: every GPU the library runs on holds its own copy of it until
// the process ends.  Its device address is looked up once per device with
// hipGetSymbolAddress (the host-side name of the array is not a device address)
// and kept; every launch takes that address.
//
// Every call on a device shares that device's array, so calls that overlap on
// one device (different streams, or different host threads) race and must be
// serialised by the caller.  Nothing in the array has to start at zero: every
// kernel of the sequence writes what the next one reads (the mass record, the
// block records, every staged source including the padding, and the slice
// partials of every target the accumulation kernel reads).
#include <mutex>

#include "dnb_internal.h"

using namespace dnb;

namespace {

// 16 MiB: the staged sources of DNB_NOALLOC_MAX_N particles in FP64 (2 MiB), the
// block records, the uniform-mass record and, in the rest, the slice partials.
constexpr size_t SCRATCH_BYTES = size_t(16) << 20;
constexpr int MAX_DEVICES = 64;

constexpr size_t JS_BYTES = sizeof(double4) * DNB_NOALLOC_MAX_N;
constexpr size_t REC_BYTES = sizeof(double) * REC * (DNB_NOALLOC_MAX_N / BS);
constexpr size_t MUNI_BYTES = 256;
constexpr size_t PART_OFF = JS_BYTES + REC_BYTES + MUNI_BYTES;
constexpr size_t PART_BYTES = SCRATCH_BYTES - PART_OFF;
static_assert(DNB_NOALLOC_MAX_N % SUBTILE == 0 && DNB_NOALLOC_MAX_N % BS == 0,
              "the staged-source region must hold the padded sources");
static_assert(PART_OFF % 256 == 0, "regions stay 256-byte aligned");

}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

std::mutex g_mu;
void* g_scratch[MAX_DEVICES];   // device address of `scratch` on each device

dnb_status arg_error(const char* msg) {
    set_error(msg);
    return DNB_ERR_ARG;
}

// Device address of this device's copy of `scratch` (looked up on first use).
dnb_status scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= MAX_DEVICES)
        return arg_error("dnb_accelerations_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("dnb_accelerations_noalloc: hipGetSymbolAddress of the scratch array failed");
            (void)hipGetLastError();
            return DNB_ERR_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = (unsigned char*)g_scratch[dev];
    return DNB_OK;
}

}  // namespace

extern "C" dnb_status dnb_accelerations_noalloc(int64_t n, const double* pos,
                                                const double* mass, const dnb_pot* pot,
                                                int with_ext, dnb_prec prec, double* acc,
                                                void* stream) {
    const char* fn = "dnb_accelerations_noalloc";
    if (n < 1 || n > DNB_NOALLOC_MAX_N)
        return arg_error("dnb_accelerations_noalloc: n must lie in [1, DNB_NOALLOC_MAX_N = 65536] "
                         "(the static scratch array holds that many particles)");
    if (prec != DNB_FP64 && prec != DNB_FP32C)
        return arg_error("dnb_accelerations_noalloc: unknown precision");
    dnb_status s = check_pot_args(pot, fn);
    if (s != DNB_OK) return s;
    for (const void* p : {(const void*)pos, (const void*)mass, (const void*)acc}) {
        s = check_device_ptr(p, p == pos ? "pos" : (p == mass ? "mass" : "acc"), fn);
        if (s != DNB_OK) return s;
    }
    if (acc == pos) return arg_error("dnb_accelerations_noalloc: acc must not alias pos");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("dnb_accelerations_noalloc: no current HIP device");
        return DNB_ERR_HIP;
    }
    unsigned char* base = nullptr;
    s = scratch_address(dev, &base);
    if (s != DNB_OK) return s;

    // A context on the stack whose buffers are regions of the scratch array;
    // the source slices are capped so that the partials fit their region.
    dnb_ctx c{};
    c.device = dev;
    c.max_n = DNB_NOALLOC_MAX_N;
    c.prec = prec;
    c.target_blocks = TARGET_BLOCKS;
    c.nbmax = DNB_NOALLOC_MAX_N / BS;
    const int64_t npad = cdiv(n, BS) * BS;
    int64_t smax = (int64_t)(PART_BYTES / (3 * sizeof(double) * (size_t)npad));
    if (smax > S_MAX) smax = S_MAX;
    if (smax < 1) smax = 1;
    c.smax = (int)smax;
    c.js = base;
    c.cpart = (double*)(base + JS_BYTES);
    c.muni = (float*)(base + JS_BYTES + REC_BYTES);
    c.part = base + PART_OFF;

    hipStream_t st = (hipStream_t)stream;
    const Pot p = to_pot(*pot);
    const int nb = (int)cdiv(n, BS);
    hipError_t e = launch_mass_info(&c, mass, n, st);
    if (e == hipSuccess && prec == DNB_FP32C) e = launch_block_sums(pos, n, c.cpart, st);
    if (e == hipSuccess) e = launch_stage(&c, pos, mass, n, c.cpart, nb, nullptr, nullptr, st);
    if (e == hipSuccess) e = launch_pair_fwd(&c, n, p.eps, st);
    if (e == hipSuccess) {
        FwdArgs a{};
        a.n = n; a.mass = mass; a.pot = p; a.x = pos; a.acc_out = acc;
        a.with_ext = with_ext ? 1 : 0;
        e = launch_kdk(&c, KDK_ACC, a, st);
    }
    if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        return DNB_ERR_HIP;
    }
    return DNB_OK;
}
