// C ABI of libdnb: argument validation, context management and the host-side
// sequencing of the kernels for each entry point declared in include/dnb.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <new>
#include <string>
#include <vector>

#include "dnb_internal.h"
#include "../../include/dnb_orbitfit.h"

using namespace dnb;

namespace {

thread_local std::string g_err;

dnb_status fail(dnb_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(DNB_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)


bool is_fin(double v) { return std::isfinite(v); }

int env_int(const char* name, int dflt, std::initializer_list<int> allowed) {
    const char* s = std::getenv(name);
    if (!s || !*s) return dflt;
    const int v = std::atoi(s);
    for (int a : allowed)
        if (a == v) return v;
    return dflt;
}

dnb_status check_ctx(dnb_ctx* c, int64_t n, const char* fn) {
    if (!c) return fail(DNB_ERR_ARG, "%s: ctx is NULL", fn);
    if (n < 1 || n > c->max_n)
        return fail(DNB_ERR_ARG, "%s: n = %lld outside [1, max_n = %lld]", fn, (long long)n,
                    (long long)c->max_n);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
        return fail(DNB_ERR_ARG, "%s: current device %d is not the context's device %d", fn, dev,
                    c->device);
    return DNB_OK;
}

dnb_status check_pot(const dnb_pot* p, const char* fn) {
    if (!p) return fail(DNB_ERR_ARG, "%s: pot is NULL", fn);
    if (const char* why = pot_error(*p)) return fail(DNB_ERR_ARG, "%s: %s", fn, why);
    return DNB_OK;
}

// A pointer must be device memory (or managed) of the current device.
dnb_status check_dev(const void* p, const char* name, const char* fn, bool nullable = false) {
    if (!p) {
        if (nullable) return DNB_OK;
        return fail(DNB_ERR_ARG, "%s: %s is NULL", fn, name);
    }
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DNB_ERR_ARG, "%s: %s is not a HIP device pointer", fn, name);
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return fail(DNB_ERR_ARG, "%s: %s is not device memory", fn, name);
    return DNB_OK;
}

// A device buffer must hold `bytes` bytes from p to the end of its allocation.
// The allocation's range is known to the HIP runtime; a pointer it does not know
// (for instance managed memory) is not checked.
dnb_status check_extent(const void* p, size_t bytes, const char* name, const char* fn) {
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return DNB_OK;
    }
    const size_t avail = size - (size_t)((const char*)p - (const char*)base);
    if (bytes > avail)
        return fail(DNB_ERR_STATE, "%s: %s needs %zu bytes but only %zu remain in its allocation",
                    fn, name, bytes, avail);
    return DNB_OK;
}

// Tape descriptors (dnb_ctx::tapes, see TapeRing).
void forget_tapes(dnb_ctx* c, const double* pos, const double* tape, int64_t tape_len,
                  const double* vel) {
    c->tapes.forget(pos, tape, tape_len, vel);
}

void remember_tape(dnb_ctx* c, const TapeDesc& d) { c->tapes.remember(d); }

TapeDesc single_desc(const double* tape, const double* pos, const double* vel,
                     const double* mass, int64_t n, int64_t T, int64_t K, double dt,
                     const dnb_pot& p) {
    return TapeDesc{tape, pos, mass, n, T, K, dt,
                    {p.G, p.eps, p.m_nfw, p.rs_nfw, p.m_mn, p.a_mn, p.b_mn}, 0, 0, vel};
}

// The descriptor of a batched tape, checked against the arguments of
// dnb_simulate_batch_vjp.
dnb_status match_batch_tape(dnb_ctx* c, const double* tape, const double* pos_T,
                            const double* mass, int64_t batch, int64_t n, int64_t T,
                            const double* params, const char* fn) {
    if (const TapeDesc* dp = c->tapes.find(tape)) {
        const TapeDesc& d = *dp;
        if (d.batch != batch || d.n != n || d.n_steps != T)
            return fail(DNB_ERR_STATE,
                        "%s: the tape was written for batch = %lld, n = %lld, n_steps = %lld "
                        "(called with %lld, %lld, %lld)", fn, (long long)d.batch, (long long)d.n,
                        (long long)d.n_steps, (long long)batch, (long long)n, (long long)T);
        if (d.pos != pos_T)
            return fail(DNB_ERR_STATE, "%s: pos_T is not the position array the tape's forward "
                        "run moved", fn);
        if (d.mass != mass || d.table != table_hash(params, batch))
            return fail(DNB_ERR_STATE, "%s: mass or the parameter table differ from the tape's "
                        "forward run", fn);
        return DNB_OK;
    }
    return fail(DNB_ERR_STATE, "%s: no current tape at this address (no dnb_simulate_batch wrote "
                "it on this context, or a later call moved its final positions or overwrote it)",
                fn);
}

// The descriptor of `tape`, checked against the arguments of a reverse sweep
// (vel_T: the final velocities a sweep that steps backward starts from; null for
// the sweep that recomputes segments).
dnb_status match_tape(dnb_ctx* c, const double* tape, const double* pos_T, const double* mass,
                      int64_t n, int64_t T, int64_t K, double dt, const dnb_pot& p,
                      const char* fn, const double* vel_T = nullptr) {
    const double pv[7] = {p.G, p.eps, p.m_nfw, p.rs_nfw, p.m_mn, p.a_mn, p.b_mn};
    if (const TapeDesc* dp = c->tapes.find(tape)) {
        const TapeDesc& d = *dp;
        if (d.batch != 0)
            return fail(DNB_ERR_STATE, "%s: the tape was written by dnb_simulate_batch", fn);
        if (d.n != n || d.n_steps != T || d.ckpt_every != K)
            return fail(DNB_ERR_STATE,
                        "%s: the tape was written for n = %lld, n_steps = %lld, ckpt_every = %lld "
                        "(called with %lld, %lld, %lld)", fn, (long long)d.n,
                        (long long)d.n_steps, (long long)d.ckpt_every, (long long)n,
                        (long long)T, (long long)K);
        if (d.pos != pos_T)
            return fail(DNB_ERR_STATE, "%s: pos_T is not the position array the tape's forward "
                        "run moved", fn);
        if (vel_T && d.vel != vel_T)
            return fail(DNB_ERR_STATE, "%s: vel_T is not the velocity array the tape's forward "
                        "run moved", fn);
        if (d.mass != mass || d.dt != dt || std::memcmp(d.pot, pv, sizeof pv) != 0)
            return fail(DNB_ERR_STATE, "%s: mass, dt or pot differ from the tape's forward run",
                        fn);
        return DNB_OK;
    }
    return fail(DNB_ERR_STATE, "%s: no current tape at this address (no dnb_simulate wrote it on "
                "this context, or a later dnb_simulate/dnb_step moved its final positions or "
                "overwrote it)", fn);
}

// Event pool of dnb_profile: one (start, stop) pair per profiled launch.
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;           // reusable events
    std::vector<hipEvent_t> ev[2];          // recorded pairs: [0] forward, [1] VJP
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

// Launch one O(N^2) kernel (kind 0: forward pair sum, 1: VJP), bracketed by
// events when profiling is on.
template <class F>
hipError_t profiled(dnb_ctx* c, int kind, hipStream_t st, F launch) {
    Prof* pf = (Prof*)c->prof;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (pf && pf->on) {
        e0 = pf->get();
        e1 = pf->get();
        if (e0 && e1) (void)hipEventRecord(e0, st);
    }
    hipError_t err = launch();
    if (e0 && e1) {
        (void)hipEventRecord(e1, st);
        pf->ev[kind].push_back(e0);
        pf->ev[kind].push_back(e1);
    }
    return err;
}

#define CHECK(x)                          \
    do {                                  \
        dnb_status s_ = (x);              \
        if (s_ != DNB_OK) return s_;      \
    } while (0)

// Tape of one integration, in order: the states (x, v) at the checkpoints
// [n_ckpt][6][n], the staging centres [n_ckpt][8], the internal accelerations
// at the checkpoints [n_ckpt][3][n], and the internal acceleration at the final
// positions [3][n].  The reverse sweep reads the accelerations instead of
// summing them again in the pair VJP.  A checkpoint's two centres (4 doubles
// each) are the ones the run staged the checkpoint's positions with and the
// positions one step later: with them a recomputation from the checkpoint
// repeats the run's FP32 staging exactly.
struct Tape {
    double* base;
    int64_t n, n_ckpt;
    double* state(int64_t c) const { return base + c * 6 * n; }
    double* centre(int64_t c) const { return base + n_ckpt * 6 * n + 8 * c; }
    double* centre_next(int64_t c) const { return centre(c) + 4; }
    double* aint(int64_t c) const { return base + n_ckpt * (6 * n + 8) + c * 3 * n; }
    double* aint_final() const { return aint(n_ckpt); }
};

// Forward integration from (x, v) for n_steps; tape optional.  Positions and
// velocities are updated in place.  centres (nullable): the two FP32C staging
// centres a checkpoint stored (those of its positions and of the positions one
// step later), which a run resumed from that checkpoint takes instead of the
// ones a fresh start computes, so that it continues bit for bit.
dnb_status run_forward(dnb_ctx* c, int64_t n, double* pos, double* vel, const double* mass,
                       const Pot& p, double dt, int64_t T, int64_t K, const Tape* tape,
                       hipStream_t st, const double* centres = nullptr) {
    if (T == 0) return DNB_OK;
    const int nb = (int)cdiv(n, BS);
    double* cp[2] = {c->cpart, c->cpart + REC * c->nbmax};
    HIP_TRY(launch_mass_info(c, mass, n, st));
    if (c->prec == DNB_FP32C && !centres)
        HIP_TRY(launch_block_sums(pos, n, cp[0], st, nullptr, vel, dt));
    HIP_TRY(launch_stage(c, pos, mass, n, cp[0], nb, centres, tape ? tape->centre(0) : nullptr,
                         st));
    int q = 0;
    const bool f32 = c->prec == DNB_FP32C;
    for (int64_t s = 0; s <= T; ++s) {
        // FP32C: the pair launch's extra row evaluates the external field at pos
        const ExtRow row = f32 ? ExtRow{pos, nullptr, p} : ExtRow{};
        bool row_done = false;
        HIP_TRY(profiled(c, 0, st,
                         [&] { return launch_pair_fwd(c, n, p.eps, st, row, &row_done); }));
        if (f32) HIP_TRY(launch_fwd_reduce(c, n, mass, p.G, st));
        FwdArgs a{};
        a.n = n; a.mass = mass; a.pot = p; a.dt = dt;
        if (f32) { a.ared = c->ared; a.arec = c->arec; a.nr = red_blocks(n); }
        if (row_done) a.aext = c->aext_f;
        a.x = pos; a.x_out = pos; a.v = vel; a.vh = c->vh; a.with_ext = 1;
        a.cpart_in = cp[q]; a.cpart_out = cp[1 - q]; a.nb_in = nb;
        if (tape && s < T && s % K == 0) {
            a.tape_state = tape->state(s / K);
            a.aint_out = tape->aint(s / K);
        }
        if (tape && s == T) a.aint_out = tape->aint_final();
        if (tape && s + 1 < T && (s + 1) % K == 0) a.tape_centre_next = tape->centre((s + 1) / K);
        if (tape && s < T && s % K == 0) a.tape_centre_cur = tape->centre_next(s / K);
        if (s == 0 && centres) a.centre_override = centres + 4;
        KdkMode mode = (s == 0) ? KDK_FIRST : (s == T ? KDK_LAST : KDK_MID);
        HIP_TRY(launch_kdk(c, mode, a, st));
        q = 1 - q;
    }
    return DNB_OK;
}

}  // namespace

void dnb::set_error(const char* msg) { g_err = msg; }
dnb_status dnb::check_pot_args(const dnb_pot* p, const char* fn) { return check_pot(p, fn); }
dnb_status dnb::check_device_ptr(const void* p, const char* name, const char* fn) {
    return check_dev(p, name, fn);
}

extern "C" {

const char* dnb_last_error(void) { return g_err.c_str(); }

const char* dnb_version(void) { return "dnb 0.1.0 (gfx950)"; }

dnb_status dnb_create(dnb_ctx** out, int64_t max_n, dnb_prec prec) {
    if (!out) return fail(DNB_ERR_ARG, "dnb_create: out is NULL");
    *out = nullptr;
    if (max_n < 1 || max_n > MAX_N)
        return fail(DNB_ERR_ARG, "dnb_create: max_n = %lld outside [1, 2^26]", (long long)max_n);
    if (prec != DNB_FP64 && prec != DNB_FP32C)
        return fail(DNB_ERR_ARG, "dnb_create: unknown precision %d", (int)prec);
    dnb_ctx* c = new (std::nothrow) dnb_ctx();
    if (!c) return fail(DNB_ERR_NOMEM, "dnb_create: host allocation failed");
    c->max_n = max_n;
    c->prec = prec;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(DNB_ERR_HIP, "dnb_create: no HIP device");
    }
    // Blocks per pair-kernel launch; DNB_TARGET_BLOCKS overrides the tuned
    // default for experiments.
    c->target_blocks = env_int("DNB_TARGET_BLOCKS", TARGET_BLOCKS, {1024, 2048, 4096, 8192, 16384});
    // DNB_EXT_ROW=0: the kicks evaluate the external field themselves (the same
    // bits; for comparisons)
    c->ext_row = env_int("DNB_EXT_ROW", 1, {0, 1});
    // Pair grids in (slices, target blocks) order: the dispatcher spreads
    // consecutive blocks over the compute units, so each unit then runs blocks of
    // one slice, whose sources its scalar cache keeps (DNB_SLICE_MAJOR=0: the
    // (target blocks, slices) order, the same bits; for comparisons)
    c->slice_major = env_int("DNB_SLICE_MAJOR", 1, {0, 1});
    c->slice_rows = max_slice_rows(max_n, BS, c->target_blocks);
    c->smax = S_MAX;
    c->nbmax = (int)cdiv(max_n, BS);
    const int64_t npadmax = (int64_t)c->nbmax * BS;
    struct A { void** p; size_t bytes; } allocs[] = {
        {&c->js, sizeof(double4) * npadmax},
        {&c->part, 32 * (size_t)c->slice_rows},
        {(void**)&c->cpart, sizeof(double) * 2 * REC * c->nbmax},
        {(void**)&c->vh, sizeof(double) * 3 * npadmax},
        {&c->jsv, sizeof(double4) * 2 * npadmax},
        {&c->partv, 64 * (size_t)c->slice_rows},
        {(void**)&c->cpartv, sizeof(double) * 2 * REC * c->nbmax},
        {(void**)&c->wscale, sizeof(double) * 2},
        {(void**)&c->muni, sizeof(float) * 2 * DNB_BATCH_MAX},
        {(void**)&c->bparams, sizeof(double) * 8 * DNB_BATCH_MAX},
        {(void**)&c->bwscale, sizeof(double) * 2 * DNB_BATCH_MAX},
        {(void**)&c->red, sizeof(double) * 8 * (c->nbmax + 8)},
        {(void**)&c->ared, sizeof(double) * 3 * npadmax},
        {(void**)&c->gred, sizeof(double) * 4 * npadmax},
        {(void**)&c->arec, sizeof(double) * 4 * (cdiv(npadmax, RT) + DNB_BATCH_MAX)},
        {(void**)&c->grec, sizeof(double) * 4 * (cdiv(npadmax, RT) + DNB_BATCH_MAX)},
        {(void**)&c->scan, sizeof(int64_t) * (c->nbmax + 1)},
        {(void**)&c->aext_f, sizeof(double) * 3 * npadmax},
        {(void**)&c->aext_v, sizeof(double) * 9 * npadmax},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            (void)hipGetLastError();
            dnb_destroy(c);
            return fail(DNB_ERR_NOMEM, "dnb_create: device allocation of %zu bytes failed", a.bytes);
        }
    }
    *out = c;
    return DNB_OK;
}

void dnb_destroy(dnb_ctx* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    if (c->prof) {
        Prof* pf = (Prof*)c->prof;
        for (auto* v : {&pf->pool, &pf->ev[0], &pf->ev[1]})
            for (hipEvent_t e : *v) (void)hipEventDestroy(e);
        delete pf;
    }
    for (hipEvent_t e : c->revents)
        if (e) (void)hipEventDestroy(e);
    if (c->rstream) (void)hipStreamDestroy(c->rstream);
    void* ps[] = {c->js, c->part, c->cpart, c->vh, c->jsv, c->partv, c->cpartv, c->wscale, c->muni,
                  c->bparams, c->bwscale, c->red, c->ared, c->gred, c->arec, c->grec,
                  c->scan, c->aext_f, c->aext_v};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    delete c;
}

dnb_status dnb_accelerations(dnb_ctx* c, int64_t n, const double* pos, const double* mass,
                             const dnb_pot* pot, int with_ext, double* acc, void* stream) {
    const char* fn = "dnb_accelerations";
    CHECK(check_ctx(c, n, fn));
    CHECK(check_pot(pot, fn));
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(mass, "mass", fn));
    CHECK(check_dev(acc, "acc", fn));
    if (acc == pos) return fail(DNB_ERR_ARG, "%s: acc must not alias pos", fn);
    hipStream_t st = (hipStream_t)stream;
    Pot p = to_pot(*pot);
    const int nb = (int)cdiv(n, BS);
    HIP_TRY(launch_mass_info(c, mass, n, st));
    if (c->prec == DNB_FP32C) HIP_TRY(launch_block_sums(pos, n, c->cpart, st));
    HIP_TRY(launch_stage(c, pos, mass, n, c->cpart, nb, nullptr, nullptr, st));
    HIP_TRY(profiled(c, 0, st, [&] { return launch_pair_fwd(c, n, p.eps, st); }));
    FwdArgs a{};
    a.n = n; a.mass = mass; a.pot = p; a.x = pos; a.acc_out = acc; a.with_ext = with_ext ? 1 : 0;
    HIP_TRY(launch_kdk(c, KDK_ACC, a, st));
    return DNB_OK;
}

dnb_status dnb_accelerations_rows(dnb_ctx* c, int64_t n, const double* pos, const double* mass,
                                  const dnb_pot* pot, int with_ext, int64_t i_begin,
                                  int64_t i_count, double* acc, void* stream) {
    const char* fn = "dnb_accelerations_rows";
    CHECK(check_ctx(c, n, fn));
    CHECK(check_pot(pot, fn));
    if (i_begin < 0 || i_count < 1 || i_begin > n - i_count)
        return fail(DNB_ERR_ARG, "%s: rows [%lld, %lld + %lld) are not inside [0, %lld)", fn,
                    (long long)i_begin, (long long)i_begin, (long long)i_count, (long long)n);
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(mass, "mass", fn));
    CHECK(check_dev(acc, "acc", fn));
    if (acc == pos) return fail(DNB_ERR_ARG, "%s: acc must not alias pos", fn);
    hipStream_t st = (hipStream_t)stream;
    Pot p = to_pot(*pot);
    const int nb = (int)cdiv(n, BS);
    HIP_TRY(launch_mass_info(c, mass, n, st));
    if (c->prec == DNB_FP32C) HIP_TRY(launch_block_sums(pos, n, c->cpart, st));
    HIP_TRY(launch_stage(c, pos, mass, n, c->cpart, nb, nullptr, nullptr, st));
    HIP_TRY(profiled(c, 0, st, [&] {
        return launch_pair_fwd_rows(c, n, i_begin, i_count, p.eps, st);
    }));
    HIP_TRY(launch_acc_rows(c, pos, n, i_begin, i_count, p, with_ext ? 1 : 0, acc, st));
    return DNB_OK;
}

dnb_status dnb_accelerations_vjp(dnb_ctx* c, int64_t n, const double* pos, const double* mass,
                                 const dnb_pot* pot, int with_ext, const double* w,
                                 int64_t i_begin, int64_t i_count, double* gpos, double* gmass,
                                 void* stream) {
    const char* fn = "dnb_accelerations_vjp";
    CHECK(check_ctx(c, n, fn));
    CHECK(check_pot(pot, fn));
    if (i_begin < 0 || i_count < 1 || i_begin > n - i_count)
        return fail(DNB_ERR_ARG, "%s: rows [%lld, %lld + %lld) are not inside [0, %lld)", fn,
                    (long long)i_begin, (long long)i_begin, (long long)i_count, (long long)n);
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(mass, "mass", fn));
    CHECK(check_dev(w, "w", fn));
    CHECK(check_dev(gpos, "gpos", fn));
    CHECK(check_dev(gmass, "gmass", fn, true));
    if (gpos == pos || gpos == w || (gmass && gmass == mass))
        return fail(DNB_ERR_ARG, "%s: outputs must not alias inputs", fn);
    hipStream_t st = (hipStream_t)stream;
    Pot p = to_pot(*pot);
    const int nb = (int)cdiv(n, BS);
    double* cpv[2] = {c->cpartv, c->cpartv + REC * c->nbmax};
    HIP_TRY(launch_mass_info(c, mass, n, st));
    if (c->prec == DNB_FP32C) HIP_TRY(launch_block_sums(pos, n, cpv[0], st, w));
    HIP_TRY(launch_rev_stage(c, n, pos, mass, w, cpv[0], nb, cpv[1], c->wscale, st));
    HIP_TRY(profiled(c, 1, st, [&] {
        return launch_pair_vjp_rows(c, n, i_begin, i_count, gmass != nullptr, p.eps, st);
    }));
    HIP_TRY(launch_acc_vjp_rows(c, pos, w, n, i_begin, i_count, p, with_ext ? 1 : 0, gpos, gmass,
                                st));
    return DNB_OK;
}

int64_t dnb_tape_doubles(int64_t n, int64_t n_steps, int64_t ckpt_every) {
    return tape_doubles(n, n_steps, ckpt_every);
}

int64_t dnb_vjp_workspace_doubles(int64_t n, int64_t ckpt_every) {
    return vjp_workspace_doubles(n, ckpt_every);
}

int64_t dnb_vjp_reversed_workspace_doubles(int64_t n) {
    return vjp_reversed_workspace_doubles(n);
}

// The state scan: *first = index of the first particle (b n + i for member b)
// with a non-finite position, velocity or mass, -1 when there is none.  Waits
// for the stream.
static dnb_status scan_state(dnb_ctx* c, const double* x, const double* v, const double* m,
                             int64_t n, int64_t nsys, hipStream_t st, int64_t* first) {
    int64_t r = 0;
    HIP_TRY(launch_scan_state(c, x, v, m, n, nsys, st));
    HIP_TRY(hipMemcpyAsync(&r, c->scan + c->nbmax, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *first = (r == INT64_MAX) ? -1 : r;
    return DNB_OK;
}

// With checks on (dnb_set_checks): refuse an initial state that holds a
// non-finite value, naming the first such particle.
static dnb_status checked_state(dnb_ctx* c, const double* x, const double* v, const double* m,
                                int64_t n, int64_t nsys, hipStream_t st, const char* fn) {
    if (!c->checks) return DNB_OK;
    int64_t first = -1;
    CHECK(scan_state(c, x, v, m, n, nsys, st, &first));
    if (first < 0) return DNB_OK;
    if (nsys > 1)
        return fail(DNB_ERR_ARG, "%s: initial state of member %lld, particle %lld holds a "
                    "non-finite position, velocity or mass", fn, (long long)(first / n),
                    (long long)(first % n));
    return fail(DNB_ERR_ARG, "%s: initial state of particle %lld holds a non-finite position, "
                "velocity or mass", fn, (long long)first);
}

static dnb_status check_sim_args(dnb_ctx* c, int64_t n, const void* pos, const void* vel,
                                 const void* mass, const dnb_pot* pot, double dt, int64_t T,
                                 int64_t K, const char* fn) {
    CHECK(check_ctx(c, n, fn));
    CHECK(check_pot(pot, fn));
    if (!is_fin(dt)) return fail(DNB_ERR_ARG, "%s: dt is not finite", fn);
    if (T < 0) return fail(DNB_ERR_ARG, "%s: n_steps < 0", fn);
    if (K < 1) return fail(DNB_ERR_ARG, "%s: ckpt_every must be >= 1", fn);
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(vel, "vel", fn));
    CHECK(check_dev(mass, "mass", fn));
    return DNB_OK;
}

dnb_status dnb_step(dnb_ctx* c, int64_t n, double* pos, double* vel, const double* mass,
                    const dnb_pot* pot, double dt, void* stream) {
    CHECK(check_sim_args(c, n, pos, vel, mass, pot, dt, 1, 1, "dnb_step"));
    forget_tapes(c, pos, nullptr, 0, vel);
    return run_forward(c, n, pos, vel, mass, to_pot(*pot), dt, 1, 1, nullptr, (hipStream_t)stream);
}

dnb_status dnb_simulate(dnb_ctx* c, int64_t n, double* pos, double* vel, const double* mass,
                        const dnb_pot* pot, double dt, int64_t n_steps, int64_t ckpt_every,
                        double* tape, void* stream) {
    const char* fn = "dnb_simulate";
    CHECK(check_sim_args(c, n, pos, vel, mass, pot, dt, n_steps, ckpt_every, fn));
    CHECK(check_dev(tape, "tape", fn, true));
    const int64_t tl = dnb_tape_doubles(n, n_steps, ckpt_every);
    if (tape && n_steps > 0) CHECK(check_extent(tape, sizeof(double) * tl, "tape", fn));
    CHECK(checked_state(c, pos, vel, mass, n, 1, (hipStream_t)stream, fn));
    forget_tapes(c, pos, tape, tape ? tl : 0, vel);
    Tape tp{tape, n, cdiv(n_steps, ckpt_every)};
    CHECK(run_forward(c, n, pos, vel, mass, to_pot(*pot), dt, n_steps, ckpt_every,
                      tape ? &tp : nullptr, (hipStream_t)stream));
    if (tape && n_steps > 0)
        remember_tape(c, single_desc(tape, pos, vel, mass, n, n_steps, ckpt_every, dt, *pot));
    return DNB_OK;
}

dnb_status dnb_set_checks(dnb_ctx* c, int on) {
    if (!c) return fail(DNB_ERR_ARG, "dnb_set_checks: ctx is NULL");
    c->checks = on ? 1 : 0;
    return DNB_OK;
}

dnb_status dnb_check_state(dnb_ctx* c, int64_t n, const double* pos, const double* vel,
                           const double* mass, int64_t* first_bad, void* stream) {
    const char* fn = "dnb_check_state";
    CHECK(check_ctx(c, n, fn));
    if (!first_bad) return fail(DNB_ERR_ARG, "%s: first_bad is NULL", fn);
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(vel, "vel", fn, true));
    CHECK(check_dev(mass, "mass", fn, true));
    return scan_state(c, pos, vel, mass, n, 1, (hipStream_t)stream, first_bad);
}

dnb_status dnb_simulate_resume(dnb_ctx* c, int64_t n, const double* tape, int64_t tape_steps,
                               int64_t tape_ckpt_every, int64_t ckpt, double* pos, double* vel,
                               const double* mass, const dnb_pot* pot, double dt,
                               int64_t n_steps, int64_t ckpt_every, double* tape_out,
                               void* stream) {
    const char* fn = "dnb_simulate_resume";
    CHECK(check_sim_args(c, n, pos, vel, mass, pot, dt, n_steps, ckpt_every, fn));
    if (tape_steps < 1 || tape_ckpt_every < 1)
        return fail(DNB_ERR_ARG, "%s: tape_steps and tape_ckpt_every must be >= 1", fn);
    const int64_t n_ckpt = cdiv(tape_steps, tape_ckpt_every);
    if (ckpt < 0 || ckpt >= n_ckpt)
        return fail(DNB_ERR_ARG, "%s: ckpt = %lld outside [0, %lld), the tape's checkpoints", fn,
                    (long long)ckpt, (long long)n_ckpt);
    CHECK(check_dev(tape, "tape", fn));
    CHECK(check_dev(tape_out, "tape_out", fn, true));
    const int64_t tl = dnb_tape_doubles(n, tape_steps, tape_ckpt_every);
    CHECK(check_extent(tape, sizeof(double) * tl, "tape", fn));
    const int64_t tlo = dnb_tape_doubles(n, n_steps, ckpt_every);
    if (tape_out && n_steps > 0)
        CHECK(check_extent(tape_out, sizeof(double) * tlo, "tape_out", fn));
    auto overlaps = [](const double* a, int64_t na, const double* b, int64_t nb_) {
        return a && b && a < b + nb_ && b < a + na;
    };
    if (overlaps(pos, 3 * n, tape, tl) || overlaps(vel, 3 * n, tape, tl) ||
        overlaps(tape_out, tape_out && n_steps > 0 ? tlo : 0, tape, tl) || pos == vel)
        return fail(DNB_ERR_ARG, "%s: pos, vel and tape_out must not overlap the source tape "
                    "or each other", fn);
    hipStream_t st = (hipStream_t)stream;
    const Tape src{const_cast<double*>(tape), n, n_ckpt};
    const double* x0 = src.state(ckpt);
    const size_t vec = sizeof(double) * 3 * n;
    forget_tapes(c, pos, tape_out, tape_out ? tlo : 0, vel);
    HIP_TRY(hipMemcpyAsync(pos, x0, vec, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(vel, x0 + 3 * n, vec, hipMemcpyDeviceToDevice, st));
    CHECK(checked_state(c, pos, vel, mass, n, 1, st, fn));
    Tape tp{tape_out, n, cdiv(n_steps, ckpt_every)};
    CHECK(run_forward(c, n, pos, vel, mass, to_pot(*pot), dt, n_steps, ckpt_every,
                      tape_out ? &tp : nullptr, st, src.centre(ckpt)));
    if (tape_out && n_steps > 0)
        remember_tape(c, single_desc(tape_out, pos, vel, mass, n, n_steps, ckpt_every, dt, *pot));
    return DNB_OK;
}

dnb_status dnb_simulate_vjp(dnb_ctx* c, int64_t n, const double* mass, const dnb_pot* pot,
                            double dt, int64_t n_steps, int64_t ckpt_every, const double* tape,
                            const double* pos_T, const double* gpos_T, const double* gvel_T,
                            double* workspace, double* gpos_0, double* gvel_0, double* gmass,
                            double* gparams, void* stream) {
    const char* fn = "dnb_simulate_vjp";
    CHECK(check_sim_args(c, n, pos_T, gpos_0, mass, pot, dt, n_steps, ckpt_every, fn));
    if (dt == 0.0) return fail(DNB_ERR_ARG, "%s: dt must be non-zero", fn);
    CHECK(check_dev(gpos_T, "gpos_T", fn));
    CHECK(check_dev(gvel_T, "gvel_T", fn, true));
    CHECK(check_dev(workspace, "workspace", fn));
    CHECK(check_dev(gvel_0, "gvel_0", fn));
    CHECK(check_dev(gmass, "gmass", fn, true));
    CHECK(check_dev(gparams, "gparams", fn));
    if (n_steps > 0) CHECK(check_dev(tape, "tape", fn));
    if (gpos_0 == gpos_T || gvel_0 == gvel_T || gpos_0 == gvel_0)
        return fail(DNB_ERR_ARG, "%s: outputs must not alias inputs", fn);
    CHECK(check_extent(workspace, sizeof(double) * dnb_vjp_workspace_doubles(n, ckpt_every),
                       "workspace", fn));
    CHECK(check_extent(gparams, sizeof(double) * 7, "gparams", fn));
    if (n_steps > 0) {
        CHECK(check_extent(tape, sizeof(double) * dnb_tape_doubles(n, n_steps, ckpt_every), "tape",
                           fn));
        CHECK(match_tape(c, tape, pos_T, mass, n, n_steps, ckpt_every, dt, *pot, fn));
    }
    hipStream_t st = (hipStream_t)stream;
    const Pot p = to_pot(*pot);
    const int64_t T = n_steps, K = ckpt_every;
    const int nb = (int)cdiv(n, BS);
    const size_t vec = sizeof(double) * 3 * n;
    double* lx = gpos_0;
    double* lv = gvel_0;
    double* vrec = workspace;                        // [3][n]
    double* accum = workspace + 3 * n;               // [8][n]
    // two buffers of a recomputed segment (K > 1): positions [(K+1)][3][n],
    // then accelerations [K][3][n]; segment cs uses buffer cs & 1
    double* seg[2] = {nullptr, nullptr};
    double* seg_a[2] = {nullptr, nullptr};
    if (K > 1) {
        for (int b = 0; b < 2; ++b) {
            seg[b] = workspace + vjp_segment_offset(n, K, b);
            seg_a[b] = seg[b] + vjp_segment_accel_offset(n, K);
        }
    }
    HIP_TRY(hipMemcpyAsync(lx, gpos_T, vec, hipMemcpyDeviceToDevice, st));
    if (gvel_T) HIP_TRY(hipMemcpyAsync(lv, gvel_T, vec, hipMemcpyDeviceToDevice, st));
    else HIP_TRY(hipMemsetAsync(lv, 0, vec, st));
    HIP_TRY(hipMemsetAsync(accum, 0, sizeof(double) * 8 * n, st));
    HIP_TRY(launch_mass_info(c, mass, n, st));
    const int with_mass = gmass != nullptr;
    if (T > 0) {
        Tape tp{const_cast<double*>(tape), n, cdiv(T, K)};
        auto get_pos = [&](int64_t m) -> const double* {
            if (m == T) return pos_T;
            if (m % K == 0) return tp.state(m / K);
            return seg[(m / K) & 1] + (m % K) * 3 * n;
        };
        auto get_aint = [&](int64_t m) -> const double* {
            if (m == T) return tp.aint_final();
            if (m % K == 0) return tp.aint(m / K);
            return seg_a[(m / K) & 1] + (m % K) * 3 * n;
        };
        // Segment cs spans steps n0 = cs K .. n1 = min(n0 + K, T); the sweep
        // needs its interior positions recomputed when it has more than one step.
        auto needs = [&](int64_t cs) { return (cs * K + K < T ? K : T - cs * K) >= 2; };
        // The recomputation runs on a stream of its own: while the caller's
        // stream sweeps segment cs, segment cs - 1 is recomputed into the other
        // buffer.  The two share no scratch (the recomputation uses the forward
        // staging, partials and reductions, the sweep the VJP ones), so this
        // changes no result, only what overlaps: each one's latency-bound O(N)
        // kernels and launch gaps run beside the other one's pair kernels.
        hipStream_t rs = st;
        hipEvent_t* ev = c->revents;
        if (K > 1) {
            if (!c->rstream) {
                HIP_TRY(hipStreamCreateWithFlags(&c->rstream, hipStreamNonBlocking));
                for (hipEvent_t& e : c->revents)
                    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            }
            rs = c->rstream;
            HIP_TRY(hipEventRecord(ev[4], st));
            HIP_TRY(hipStreamWaitEvent(rs, ev[4], 0));
        }
        double* cpf[2] = {c->cpart, c->cpart + REC * c->nbmax};
        // Positions x_{n0+1} .. x_{n1-1} of segment cs and their internal
        // accelerations, from its checkpoint, bitwise as in the forward run (the
        // first two stagings take the centres the run stored with the checkpoint;
        // from then on the centres follow from the recomputed positions as they
        // did in the run), then the event that the buffer is ready.
        auto recompute = [&](int64_t cs) -> dnb_status {
            if (!needs(cs)) return DNB_OK;
            const int64_t n0 = cs * K, n1 = (n0 + K < T) ? n0 + K : T;
            double* sx = seg[cs & 1];
            double* sa = seg_a[cs & 1];
            double* x0 = tp.state(cs);
            HIP_TRY(launch_stage(c, x0, mass, n, nullptr, 0, tp.centre(cs), nullptr, rs));
            int q = 0;
            for (int64_t s = n0; s <= n1 - 1; ++s) {
                double* xc = (s == n0) ? x0 : sx + (s - n0) * 3 * n;
                const ExtRow row = c->prec == DNB_FP32C ? ExtRow{xc, nullptr, p} : ExtRow{};
                bool row_done = false;
                HIP_TRY(profiled(c, 0, rs, [&] {
                    return launch_pair_fwd(c, n, p.eps, rs, row, &row_done);
                }));
                FwdArgs a{};
                if (c->prec == DNB_FP32C) {
                    HIP_TRY(launch_fwd_reduce(c, n, mass, p.G, rs));
                    a.ared = c->ared; a.arec = c->arec; a.nr = red_blocks(n);
                }
                if (row_done) a.aext = c->aext_f;
                a.n = n; a.mass = mass; a.pot = p; a.dt = dt; a.with_ext = 1;
                a.x = xc;
                a.aint_out = (s == n0) ? nullptr : sa + (s - n0) * 3 * n;
                if (s == n1 - 1) {   // last position of the segment: acceleration only
                    HIP_TRY(launch_kdk(c, KDK_ACC, a, rs));
                    break;
                }
                a.x_out = sx + (s - n0 + 1) * 3 * n;
                a.v = (s == n0) ? x0 + 3 * n : nullptr;
                a.vh = vrec;
                a.cpart_in = cpf[q]; a.cpart_out = cpf[1 - q]; a.nb_in = nb;
                if (s == n0) a.centre_override = tp.centre_next(cs);
                HIP_TRY(launch_kdk(c, s == n0 ? KDK_FIRST : KDK_MID, a, rs));
                q = 1 - q;
            }
            HIP_TRY(hipEventRecord(ev[cs & 1], rs));
            return DNB_OK;
        };
        int64_t waited = -1;   // the segment whose buffer the sweep has waited for
        auto wait_for = [&](int64_t cs) -> dnb_status {
            if (K > 1 && needs(cs) && waited != cs) {
                HIP_TRY(hipStreamWaitEvent(st, ev[cs & 1], 0));
                waited = cs;
            }
            return DNB_OK;
        };
        const int64_t c_last = (T - 1) / K;
        if (K > 1) {   // the two newest segments, one per buffer
            CHECK(recompute(c_last));
            if (c_last >= 1) CHECK(recompute(c_last - 1));
        }
        double* cpv[2] = {c->cpartv, c->cpartv + REC * c->nbmax};
        // x_{T-1} first: its displacement from x_T centres the first staging of
        // the sweep
        CHECK(wait_for(c_last));
        if (c->prec == DNB_FP32C) HIP_TRY(launch_block_sums(pos_T, n, cpv[0], st, lv));
        HIP_TRY(launch_rev_stage(c, n, pos_T, mass, lv, cpv[0], nb, cpv[1], c->wscale, st,
                                 get_pos(T - 1)));
        int q = 1;
        int wq = 0;   // c->wscale[wq]: scale of the currently staged cotangent
        for (int64_t m = T; m >= 0; --m) {
            // step m reads x_m, x_{m-1} and the acceleration at x_m: the buffer of
            // segment (m - 1) / K for m >= 1
            const int64_t cs = m > 0 ? (m - 1) / K : -1;
            if (m > 0) CHECK(wait_for(cs));
            const double* xm = get_pos(m);
            // FP32C: the pair launch's extra row evaluates the reverse kick's
            // external-field terms at x_m for the cotangent lv
            const ExtRow row = c->prec == DNB_FP32C ? ExtRow{xm, lv, p} : ExtRow{};
            bool row_done = false;
            HIP_TRY(profiled(c, 1, st, [&] {
                return launch_pair_vjp(c, n, with_mass, p.eps, st, row, &row_done);
            }));
            RevArgs r{};
            if (c->prec == DNB_FP32C) {
                HIP_TRY(launch_vjp_reduce(c, n, p.G, with_mass, c->wscale + wq, st));
                r.gred = c->gred; r.grec = c->grec; r.nr = red_blocks(n);
            }
            if (row_done) r.aext = c->aext_v;
            r.n = n; r.mass = mass; r.pot = p; r.dt = dt;
            r.coef = (m == T || m == 0) ? 0.5 * dt : dt;
            r.x_n = xm;
            r.x_prev = m > 0 ? get_pos(m - 1) : nullptr;
            r.aint = get_aint(m);
            r.lx = lx; r.lv = lv; r.accum = accum; r.with_mass = with_mass;
            r.cpart_in = cpv[q]; r.nb_in = nb; r.cpart_out = cpv[1 - q];
            r.wscale_in = c->wscale + wq; r.wscale_out = c->wscale + (1 - wq);
            HIP_TRY(launch_rev_kick(c, r, st));
            q = 1 - q;
            wq = 1 - wq;
            // step cs K + 1 is the last to read segment cs: its buffer goes to
            // segment cs - 2
            if (K > 1 && m > 0 && m == cs * K + 1 && cs >= 2) {
                HIP_TRY(hipEventRecord(ev[2 + (cs & 1)], st));
                HIP_TRY(hipStreamWaitEvent(rs, ev[2 + (cs & 1)], 0));
                CHECK(recompute(cs - 2));
            }
        }
    }
    HIP_TRY(launch_reduce_accum(accum, n, 7, gparams, c->red, st));
    if (gmass) HIP_TRY(hipMemcpyAsync(gmass, accum + 7 * n, sizeof(double) * n,
                                      hipMemcpyDeviceToDevice, st));
    return DNB_OK;
}

// Reverse sweep that rebuilds the trajectory by stepping it backward.  Each
// step m (newest first) runs one pair launch at x_m that sums both J(x_m)^T w
// and the internal acceleration a(x_m); the reverse kick then takes the adjoint
// step and undoes the forward step that led to x_m (the kick-drift-kick map
// with -dt: v_{m-1/2} = v_m - dt/2 a(x_m), x_{m-1} = x_m - dt v_{m-1/2}, and
// v_{m-1} = v_{m-1/2} - dt/2 a(x_{m-1}) in the next step).  The sweep starts from
// the final state and takes the stored state in place of the rebuilt one at
// every checkpoint, so the rebuilt positions drift from the run's by at most
// K steps of rounding, grown by the dynamics over those steps.  One pair launch
// per step instead of two (a recomputed forward sum and the VJP), and no
// segment buffers.
dnb_status dnb_simulate_vjp_reversed(dnb_ctx* c, int64_t n, const double* mass,
                                     const dnb_pot* pot, double dt, int64_t n_steps,
                                     int64_t ckpt_every, const double* tape,
                                     const double* pos_T, const double* vel_T,
                                     const double* gpos_T, const double* gvel_T,
                                     double* workspace, double* gpos_0, double* gvel_0,
                                     double* gmass, double* gparams, void* stream) {
    const char* fn = "dnb_simulate_vjp_reversed";
    CHECK(check_sim_args(c, n, pos_T, gpos_0, mass, pot, dt, n_steps, ckpt_every, fn));
    if (dt == 0.0) return fail(DNB_ERR_ARG, "%s: dt must be non-zero", fn);
    CHECK(check_dev(vel_T, "vel_T", fn));
    CHECK(check_dev(gpos_T, "gpos_T", fn));
    CHECK(check_dev(gvel_T, "gvel_T", fn, true));
    CHECK(check_dev(workspace, "workspace", fn));
    CHECK(check_dev(gvel_0, "gvel_0", fn));
    CHECK(check_dev(gmass, "gmass", fn, true));
    CHECK(check_dev(gparams, "gparams", fn));
    if (n_steps > 0) CHECK(check_dev(tape, "tape", fn));
    if (gpos_0 == gpos_T || gvel_0 == gvel_T || gpos_0 == gvel_0 || gpos_0 == vel_T ||
        gvel_0 == vel_T)
        return fail(DNB_ERR_ARG, "%s: outputs must not alias inputs", fn);
    CHECK(check_extent(vel_T, sizeof(double) * 3 * n, "vel_T", fn));
    CHECK(check_extent(workspace, sizeof(double) * dnb_vjp_reversed_workspace_doubles(n),
                       "workspace", fn));
    CHECK(check_extent(gparams, sizeof(double) * 7, "gparams", fn));
    if (n_steps > 0) {
        CHECK(check_extent(tape, sizeof(double) * dnb_tape_doubles(n, n_steps, ckpt_every), "tape",
                           fn));
        CHECK(match_tape(c, tape, pos_T, mass, n, n_steps, ckpt_every, dt, *pot, fn, vel_T));
    }
    hipStream_t st = (hipStream_t)stream;
    const Pot p = to_pot(*pot);
    const int64_t T = n_steps, K = ckpt_every;
    const int nb = (int)cdiv(n, BS);
    const size_t vec = sizeof(double) * 3 * n;
    double* lx = gpos_0;
    double* lv = gvel_0;
    double* rv = workspace;                          // [3][n] velocity stepped back
    double* accum = workspace + 3 * n;               // [8][n]
    double* xb[2] = {workspace + 11 * n, workspace + 14 * n};   // rebuilt positions
    HIP_TRY(hipMemcpyAsync(lx, gpos_T, vec, hipMemcpyDeviceToDevice, st));
    if (gvel_T) HIP_TRY(hipMemcpyAsync(lv, gvel_T, vec, hipMemcpyDeviceToDevice, st));
    else HIP_TRY(hipMemsetAsync(lv, 0, vec, st));
    HIP_TRY(hipMemsetAsync(accum, 0, sizeof(double) * 8 * n, st));
    HIP_TRY(launch_mass_info(c, mass, n, st));
    const int with_mass = gmass != nullptr;
    const bool f32 = c->prec == DNB_FP32C;
    if (T > 0) {
        Tape tp{const_cast<double*>(tape), n, cdiv(T, K)};
        // positions of step m: the final ones, a checkpoint's, or rebuilt
        auto pos_of = [&](int64_t m) -> const double* {
            if (m == T) return pos_T;
            if (m % K == 0) return tp.state(m / K);
            return xb[m & 1];
        };
        double* cpv[2] = {c->cpartv, c->cpartv + REC * c->nbmax};
        // x_{T-1} is not known before the first step: its staging centre is
        // predicted one drift back at the final velocities
        if (f32) HIP_TRY(launch_block_sums(pos_T, n, cpv[0], st, lv));
        HIP_TRY(launch_rev_stage(c, n, pos_T, mass, lv, cpv[0], nb, cpv[1], c->wscale, st,
                                 nullptr, vel_T, dt));
        int q = 1;
        int wq = 0;   // c->wscale[wq]: scale of the currently staged cotangent
        for (int64_t m = T; m >= 0; --m) {
            HIP_TRY(profiled(c, 1, st, [&] {
                return launch_pair_vjp_force(c, n, with_mass, p.eps, st);
            }));
            RevArgs r{};
            if (f32) {
                HIP_TRY(launch_vjp_force_reduce(c, n, mass, p.G, with_mass, c->wscale + wq, st));
                r.gred = c->gred; r.grec = c->grec; r.nr = red_blocks(n);
                r.ared = c->ared; r.arec = c->arec;
            } else {
                r.fpart = c->part;
            }
            r.rev = 1;
            r.n = n; r.mass = mass; r.pot = p; r.dt = dt;
            r.coef = (m == T || m == 0) ? 0.5 * dt : dt;
            r.x_n = pos_of(m);
            if (m > 0) {
                // x_{m-1}: a checkpoint's (exact) or rebuilt into the other buffer
                if ((m - 1) % K == 0) r.x_prev = tp.state((m - 1) / K);
                else r.x_rec = xb[(m - 1) & 1];
                // the velocity at x_m: exact at the end and at checkpoints, else the
                // half-step velocity the previous step left
                if (m == T) { r.rv_src = vel_T; r.rv_half = 0; }
                else if (m % K == 0) { r.rv_src = tp.state(m / K) + 3 * n; r.rv_half = 0; }
                else { r.rv_src = rv; r.rv_half = 1; }
                r.rv_out = rv;
            }
            r.lx = lx; r.lv = lv; r.accum = accum; r.with_mass = with_mass;
            r.cpart_in = cpv[q]; r.nb_in = nb; r.cpart_out = cpv[1 - q];
            r.wscale_in = c->wscale + wq; r.wscale_out = c->wscale + (1 - wq);
            HIP_TRY(launch_rev_kick(c, r, st));
            q = 1 - q;
            wq = 1 - wq;
        }
    }
    HIP_TRY(launch_reduce_accum(accum, n, 7, gparams, c->red, st));
    if (gmass) HIP_TRY(hipMemcpyAsync(gmass, accum + 7 * n, sizeof(double) * n,
                                      hipMemcpyDeviceToDevice, st));
    return DNB_OK;
}

dnb_status dnb_mmd(dnb_ctx* c, int64_t n, const double* pos, int64_t m, const double* tgt,
                   double h, double* loss, double* gpos, void* stream) {
    const char* fn = "dnb_mmd";
    CHECK(check_ctx(c, n, fn));
    if (m < 1 || m > c->max_n) return fail(DNB_ERR_ARG, "%s: m outside [1, max_n]", fn);
    if (!(h > 0) || !is_fin(h)) return fail(DNB_ERR_ARG, "%s: h must be finite and > 0", fn);
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(tgt, "tgt", fn));
    CHECK(check_dev(loss, "loss", fn));
    CHECK(check_dev(gpos, "gpos", fn, true));
    HIP_TRY(launch_mmd(c, n, pos, m, tgt, h, loss, gpos, (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_energy(dnb_ctx* c, int64_t n, const double* pos, const double* vel,
                      const double* mass, const dnb_pot* pot, double* out3, void* stream) {
    const char* fn = "dnb_energy";
    CHECK(check_ctx(c, n, fn));
    CHECK(check_pot(pot, fn));
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(vel, "vel", fn));
    CHECK(check_dev(mass, "mass", fn));
    CHECK(check_dev(out3, "out3", fn));
    HIP_TRY(launch_energy(c, n, pos, vel, mass, to_pot(*pot), out3, (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_orbit(dnb_ctx* c, const double* w0, const dnb_pot* pot, double dt, int64_t n_steps,
                     double* w_out, double* traj, void* stream) {
    const char* fn = "dnb_orbit";
    CHECK(check_ctx(c, 1, fn));
    CHECK(check_pot(pot, fn));
    if (!is_fin(dt) || n_steps < 0) return fail(DNB_ERR_ARG, "%s: bad dt or n_steps", fn);
    CHECK(check_dev(w0, "w0", fn));
    CHECK(check_dev(w_out, "w_out", fn));
    CHECK(check_dev(traj, "traj", fn, true));
    HIP_TRY(launch_orbit(w0, to_pot(*pot), dt, n_steps, w_out, traj, (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_orbit_vjp(dnb_ctx* c, const double* traj, const dnb_pot* pot, double dt,
                         int64_t n_steps, const double* gw_out, double* gw0, double* gparams,
                         void* stream) {
    const char* fn = "dnb_orbit_vjp";
    CHECK(check_ctx(c, 1, fn));
    CHECK(check_pot(pot, fn));
    if (!is_fin(dt) || dt == 0.0 || n_steps < 0)
        return fail(DNB_ERR_ARG, "%s: bad dt or n_steps", fn);
    CHECK(check_dev(traj, "traj", fn));
    CHECK(check_dev(gw_out, "gw_out", fn));
    CHECK(check_dev(gw0, "gw0", fn));
    CHECK(check_dev(gparams, "gparams", fn));
    HIP_TRY(launch_orbit_vjp(traj, to_pot(*pot), dt, n_steps, gw_out, gw0, gparams,
                             (hipStream_t)stream));
    return DNB_OK;
}

// Validates the host parameter table of a batch and copies it to c->bparams.
static dnb_status put_batch_params(dnb_ctx* c, int64_t batch, const double* params,
                                   bool need_eps, hipStream_t st, const char* fn,
                                   bool need_dt = false) {
    if (batch < 1 || batch > DNB_BATCH_MAX)
        return fail(DNB_ERR_ARG, "%s: batch = %lld outside [1, %d]", fn, (long long)batch,
                    DNB_BATCH_MAX);
    if (!params) return fail(DNB_ERR_ARG, "%s: params is NULL", fn);
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, params) == hipSuccess && at.type == hipMemoryTypeDevice)
        return fail(DNB_ERR_ARG, "%s: params must be a host array", fn);
    (void)hipGetLastError();
    for (int64_t b = 0; b < batch; ++b) {
        const double* r = params + 8 * b;
        const dnb_pot p{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
        const dnb_status s = check_pot(&p, fn);
        if (s != DNB_OK) return s;
        if (!is_fin(r[7])) return fail(DNB_ERR_ARG, "%s: member %lld: dt is not finite", fn, (long long)b);
        if (need_eps && !(r[1] > 0))
            return fail(DNB_ERR_ARG, "%s: member %lld: eps must be > 0", fn, (long long)b);
        if (need_dt && r[7] == 0.0)
            return fail(DNB_ERR_ARG, "%s: member %lld: dt must be non-zero", fn, (long long)b);
    }
    HIP_TRY(hipMemcpyAsync(c->bparams, params, sizeof(double) * 8 * batch, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return DNB_OK;
}

int64_t dnb_batch_tape_doubles(int64_t batch, int64_t n, int64_t n_steps) {
    return batch_tape_doubles(batch, n, n_steps);
}

dnb_status dnb_simulate_batch(dnb_ctx* c, int64_t batch, int64_t n, double* pos, double* vel,
                              const double* mass, const double* params, int64_t n_steps,
                              double* tape, void* stream) {
    const char* fn = "dnb_simulate_batch";
    CHECK(check_ctx(c, 1, fn));
    if (n < 1) return fail(DNB_ERR_ARG, "%s: n must be >= 1", fn);
    if (n_steps < 0) return fail(DNB_ERR_ARG, "%s: n_steps < 0", fn);
    if (batch >= 1 && batch <= DNB_BATCH_MAX && !batch_fits(c, batch, n))
        return fail(DNB_ERR_ARG, "%s: batch %lld x n %lld does not fit a context of max_n = %lld",
                    fn, (long long)batch, (long long)n, (long long)c->max_n);
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(vel, "vel", fn));
    CHECK(check_dev(mass, "mass", fn));
    CHECK(check_dev(tape, "tape", fn, true));
    hipStream_t st = (hipStream_t)stream;
    CHECK(put_batch_params(c, batch, params, true, st, fn));
    const int64_t tl = dnb_batch_tape_doubles(batch, n, n_steps);
    if (tape && n_steps > 0) CHECK(check_extent(tape, sizeof(double) * tl, "tape", fn));
    CHECK(checked_state(c, pos, vel, mass, n, batch, st, fn));
    forget_tapes(c, pos, tape, tape ? tl : 0, vel);
    HIP_TRY(launch_simulate_batch(c, batch, n, pos, vel, mass, c->bparams, n_steps, tape, st));
    if (tape && n_steps > 0)
        remember_tape(c, TapeDesc{tape, pos, mass, n, n_steps, 1, 0.0, {}, batch,
                                  table_hash(params, batch), vel});
    return DNB_OK;
}

dnb_status dnb_simulate_batch_vjp(dnb_ctx* c, int64_t batch, int64_t n, const double* mass,
                                  const double* params, int64_t n_steps, const double* tape,
                                  const double* pos_T, const double* gpos_T, const double* gvel_T,
                                  double* workspace, double* gpos_0, double* gvel_0,
                                  double* gparams, void* stream) {
    const char* fn = "dnb_simulate_batch_vjp";
    CHECK(check_ctx(c, 1, fn));
    if (n < 1) return fail(DNB_ERR_ARG, "%s: n must be >= 1", fn);
    if (n_steps < 1) return fail(DNB_ERR_ARG, "%s: n_steps must be >= 1", fn);
    if (batch >= 1 && batch <= DNB_BATCH_MAX && !batch_fits(c, batch, n))
        return fail(DNB_ERR_ARG, "%s: batch %lld x n %lld does not fit a context of max_n = %lld",
                    fn, (long long)batch, (long long)n, (long long)c->max_n);
    CHECK(check_dev(mass, "mass", fn));
    CHECK(check_dev(tape, "tape", fn));
    CHECK(check_dev(pos_T, "pos_T", fn));
    CHECK(check_dev(gpos_T, "gpos_T", fn));
    CHECK(check_dev(gvel_T, "gvel_T", fn, true));
    CHECK(check_dev(workspace, "workspace", fn));
    CHECK(check_dev(gpos_0, "gpos_0", fn));
    CHECK(check_dev(gvel_0, "gvel_0", fn));
    CHECK(check_dev(gparams, "gparams", fn));
    if (gpos_0 == gpos_T || gvel_0 == gvel_T || gpos_0 == gvel_0)
        return fail(DNB_ERR_ARG, "%s: outputs must not alias inputs", fn);
    hipStream_t st = (hipStream_t)stream;
    CHECK(put_batch_params(c, batch, params, true, st, fn, true));
    CHECK(check_extent(workspace, sizeof(double) * 4 * n * batch, "workspace", fn));
    CHECK(check_extent(tape, sizeof(double) * dnb_batch_tape_doubles(batch, n, n_steps), "tape",
                       fn));
    CHECK(match_batch_tape(c, tape, pos_T, mass, batch, n, n_steps, params, fn));
    const size_t vec = sizeof(double) * 3 * n * batch;
    HIP_TRY(hipMemcpyAsync(gpos_0, gpos_T, vec, hipMemcpyDeviceToDevice, st));
    if (gvel_T) HIP_TRY(hipMemcpyAsync(gvel_0, gvel_T, vec, hipMemcpyDeviceToDevice, st));
    else HIP_TRY(hipMemsetAsync(gvel_0, 0, vec, st));
    HIP_TRY(hipMemsetAsync(workspace, 0, sizeof(double) * 4 * n * batch, st));
    HIP_TRY(launch_simulate_batch_vjp(c, batch, n, mass, c->bparams, n_steps, tape, pos_T,
                                      workspace, gpos_0, gvel_0, gparams, st));
    return DNB_OK;
}

dnb_status dnb_mmd_batch(dnb_ctx* c, int64_t batch, int64_t n, const double* pos, int64_t m,
                         const double* tgt, int tgt_per_member, double h, double* loss,
                         double* gpos, void* stream) {
    const char* fn = "dnb_mmd_batch";
    CHECK(check_ctx(c, 1, fn));
    if (!(h > 0) || !is_fin(h)) return fail(DNB_ERR_ARG, "%s: h must be finite and > 0", fn);
    if (tgt_per_member != 0 && tgt_per_member != 1)
        return fail(DNB_ERR_ARG, "%s: tgt_per_member must be 0 or 1", fn);
    if (!mmd_batch_fits(c, batch, n, m, gpos != nullptr, tgt_per_member != 0))
        return fail(DNB_ERR_ARG, "%s: batch %lld, n %lld, m %lld do not fit a context of max_n = %lld",
                    fn, (long long)batch, (long long)n, (long long)m, (long long)c->max_n);
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(tgt, "tgt", fn));
    CHECK(check_dev(loss, "loss", fn));
    CHECK(check_dev(gpos, "gpos", fn, true));
    if (gpos && gpos == pos) return fail(DNB_ERR_ARG, "%s: gpos must not alias pos", fn);
    HIP_TRY(launch_mmd_batch(c, batch, n, pos, m, tgt, tgt_per_member, h, loss, gpos,
                             (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_mmd_batch_targets(dnb_ctx* c, int64_t batch, int64_t n, const double* pos,
                                 int64_t n_tgt, int64_t m, const double* tgts, double h,
                                 double* loss, void* stream) {
    const char* fn = "dnb_mmd_batch_targets";
    CHECK(check_ctx(c, 1, fn));
    if (!(h > 0) || !is_fin(h)) return fail(DNB_ERR_ARG, "%s: h must be finite and > 0", fn);
    if (!mmd_batch_targets_fits(c, batch, n, n_tgt, m))
        return fail(DNB_ERR_ARG,
                    "%s: batch %lld, n %lld, %lld targets of m %lld do not fit a context of "
                    "max_n = %lld",
                    fn, (long long)batch, (long long)n, (long long)n_tgt, (long long)m,
                    (long long)c->max_n);
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(tgts, "tgts", fn));
    CHECK(check_dev(loss, "loss", fn));
    HIP_TRY(launch_mmd_batch_targets(c, batch, n, pos, n_tgt, m, tgts, h, loss,
                                     (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_place_plummer_batch_vjp(dnb_ctx* c, int64_t batch, int64_t n, const double* zeta,
                                       const double* m_tot, double a_p, double G,
                                       const double* gpos, const double* gvel, double* gw,
                                       double* gm_tot, void* stream) {
    const char* fn = "dnb_place_plummer_batch_vjp";
    CHECK(check_ctx(c, 1, fn));
    if (batch < 1 || batch > DNB_BATCH_MAX || n < 1)
        return fail(DNB_ERR_ARG, "%s: batch or n out of range", fn);
    if (batch * cdiv(n, BS) > c->nbmax)
        return fail(DNB_ERR_ARG, "%s: batch %lld x n %lld does not fit a context of max_n = %lld",
                    fn, (long long)batch, (long long)n, (long long)c->max_n);
    if (!(a_p > 0) || !(G > 0) || !is_fin(a_p) || !is_fin(G))
        return fail(DNB_ERR_ARG, "%s: a_p and G must be finite and > 0", fn);
    CHECK(check_dev(zeta, "zeta", fn));
    CHECK(check_dev(m_tot, "m_tot", fn));
    CHECK(check_dev(gpos, "gpos", fn));
    CHECK(check_dev(gvel, "gvel", fn));
    CHECK(check_dev(gw, "gw", fn));
    CHECK(check_dev(gm_tot, "gm_tot", fn));
    HIP_TRY(launch_place_batch_vjp(c, batch, n, zeta, m_tot, a_p, G, gpos, gvel, gw, gm_tot,
                                   (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_place_plummer_batch(dnb_ctx* c, int64_t batch, int64_t n, const double* w,
                                   const double* xi, const double* zeta, const double* m_tot,
                                   double a_p, double G, double* pos, double* vel, double* mass,
                                   void* stream) {
    const char* fn = "dnb_place_plummer_batch";
    CHECK(check_ctx(c, 1, fn));
    if (batch < 1 || batch > DNB_BATCH_MAX)
        return fail(DNB_ERR_ARG, "%s: batch = %lld outside [1, %d]", fn, (long long)batch,
                    DNB_BATCH_MAX);
    if (n < 1) return fail(DNB_ERR_ARG, "%s: n must be >= 1", fn);
    if (!(a_p > 0) || !(G > 0) || !is_fin(a_p) || !is_fin(G))
        return fail(DNB_ERR_ARG, "%s: a_p and G must be finite and > 0", fn);
    CHECK(check_dev(w, "w", fn));
    CHECK(check_dev(xi, "xi", fn));
    CHECK(check_dev(zeta, "zeta", fn));
    CHECK(check_dev(m_tot, "m_tot", fn));
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(vel, "vel", fn));
    CHECK(check_dev(mass, "mass", fn));
    forget_tapes(c, pos, nullptr, 0, vel);
    HIP_TRY(launch_place_batch(batch, n, w, xi, zeta, m_tot, a_p, G, pos, vel, mass,
                               (hipStream_t)stream));
    return DNB_OK;
}

int64_t dnb_batch_capacity(const dnb_ctx* c, int64_t n) {
    if (!c || n < 1) return 0;
    int64_t b = c->max_n / n + 1;
    if (b > DNB_BATCH_MAX) b = DNB_BATCH_MAX;
    while (b > 0 && !batch_fits(c, b, n)) --b;
    return b;
}

dnb_status dnb_orbit_batch(dnb_ctx* c, int64_t batch, const double* w0, const double* params,
                           int64_t n_steps, double* w_out, double* traj, void* stream) {
    const char* fn = "dnb_orbit_batch";
    CHECK(check_ctx(c, 1, fn));
    if (n_steps < 0) return fail(DNB_ERR_ARG, "%s: n_steps < 0", fn);
    CHECK(check_dev(w0, "w0", fn));
    CHECK(check_dev(w_out, "w_out", fn));
    CHECK(check_dev(traj, "traj", fn, true));
    hipStream_t st = (hipStream_t)stream;
    CHECK(put_batch_params(c, batch, params, false, st, fn));
    HIP_TRY(launch_orbit_batch(batch, w0, c->bparams, n_steps, w_out, traj, st));
    return DNB_OK;
}

dnb_status dnb_orbit_batch_vjp(dnb_ctx* c, int64_t batch, const double* traj, const double* params,
                               int64_t n_steps, const double* gw_out, double* gw0, double* gparams,
                               void* stream) {
    const char* fn = "dnb_orbit_batch_vjp";
    CHECK(check_ctx(c, 1, fn));
    if (n_steps < 0) return fail(DNB_ERR_ARG, "%s: n_steps < 0", fn);
    CHECK(check_dev(traj, "traj", fn));
    CHECK(check_dev(gw_out, "gw_out", fn));
    CHECK(check_dev(gw0, "gw0", fn));
    CHECK(check_dev(gparams, "gparams", fn));
    hipStream_t st = (hipStream_t)stream;
    CHECK(put_batch_params(c, batch, params, false, st, fn, true));
    HIP_TRY(launch_orbit_batch_vjp(batch, traj, c->bparams, n_steps, gw_out, gw0, gparams, st));
    return DNB_OK;
}

dnb_status dnb_place_plummer(dnb_ctx* c, int64_t n, const double* w, const double* xi,
                             const double* zeta, double m_tot, double a_p, double G, double* pos,
                             double* vel, double* mass, void* stream) {
    const char* fn = "dnb_place_plummer";
    CHECK(check_ctx(c, n, fn));
    if (!(m_tot > 0) || !(a_p > 0) || !(G > 0) || !is_fin(m_tot) || !is_fin(a_p) || !is_fin(G))
        return fail(DNB_ERR_ARG, "%s: m_tot, a_p and G must be finite and > 0", fn);
    CHECK(check_dev(w, "w", fn));
    CHECK(check_dev(xi, "xi", fn));
    CHECK(check_dev(zeta, "zeta", fn));
    CHECK(check_dev(pos, "pos", fn));
    CHECK(check_dev(vel, "vel", fn));
    CHECK(check_dev(mass, "mass", fn));
    forget_tapes(c, pos, nullptr, 0, vel);
    HIP_TRY(launch_place(n, w, xi, zeta, m_tot, a_p, G, pos, vel, mass, (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_place_plummer_vjp(dnb_ctx* c, int64_t n, const double* zeta, double m_tot,
                                 double a_p, double G, const double* gpos, const double* gvel,
                                 const double* gmass, double* gw, double* gm_tot, void* stream) {
    const char* fn = "dnb_place_plummer_vjp";
    CHECK(check_ctx(c, n, fn));
    if (!(m_tot > 0) || !(a_p > 0) || !(G > 0) || !is_fin(m_tot) || !is_fin(a_p) || !is_fin(G))
        return fail(DNB_ERR_ARG, "%s: m_tot, a_p and G must be finite and > 0", fn);
    CHECK(check_dev(zeta, "zeta", fn));
    CHECK(check_dev(gpos, "gpos", fn));
    CHECK(check_dev(gvel, "gvel", fn));
    CHECK(check_dev(gmass, "gmass", fn, true));
    CHECK(check_dev(gw, "gw", fn));
    CHECK(check_dev(gm_tot, "gm_tot", fn));
    HIP_TRY(launch_place_vjp(c, n, zeta, m_tot, a_p, G, gpos, gvel, gmass, gw, gm_tot,
                             (hipStream_t)stream));
    return DNB_OK;
}

// ------------------------------------------------------------- orbit fit --
static dnb_status check_track(dnb_ctx* c, const dnb_track_model* md, int64_t K,
                              const double* pts, const char* what, const char* fn) {
    CHECK(check_ctx(c, 1, fn));
    if (!md) return fail(DNB_ERR_ARG, "%s: model is NULL", fn);
    for (double w : md->w_now)
        if (!is_fin(w)) return fail(DNB_ERR_ARG, "%s: w_now is not finite", fn);
    const double* x = md->w_now;
    const double* v = md->w_now + 3;
    const double n[3] = {x[1] * v[2] - x[2] * v[1], x[2] * v[0] - x[0] * v[2],
                         x[0] * v[1] - x[1] * v[0]};
    if (!(n[0] * n[0] + n[1] * n[1] + n[2] * n[2] > 0))
        return fail(DNB_ERR_ARG, "%s: w_now has no angular momentum (no orbital frame)", fn);
    if (!(md->G > 0) || !is_fin(md->G)) return fail(DNB_ERR_ARG, "%s: G must be > 0", fn);
    if (!(md->dt_total > 0) || !is_fin(md->dt_total))
        return fail(DNB_ERR_ARG, "%s: dt_total must be finite and > 0", fn);
    if (md->n_steps < 1) return fail(DNB_ERR_ARG, "%s: n_steps must be >= 1", fn);
    for (double s : md->sigma)
        if (!(s > 0) || !is_fin(s)) return fail(DNB_ERR_ARG, "%s: sigma must be finite and > 0", fn);
    if (K < 1 || K > DNB_TRACK_MAX)
        return fail(DNB_ERR_ARG, "%s: K = %lld outside [1, %d]", fn, (long long)K, DNB_TRACK_MAX);
    return check_dev(pts, what, fn);
}

static dnb_status check_batch(int64_t batch, const char* fn) {
    if (batch < 1 || batch > DNB_BATCH_MAX)
        return fail(DNB_ERR_ARG, "%s: batch = %lld outside [1, %d]", fn, (long long)batch,
                    DNB_BATCH_MAX);
    return DNB_OK;
}

dnb_status dnb_track_observe(dnb_ctx* c, const dnb_track_model* md, int64_t K, const double* phi1,
                             const double* p, double* y, void* stream) {
    const char* fn = "dnb_track_observe";
    CHECK(check_track(c, md, K, phi1, "phi1", fn));
    CHECK(check_dev(p, "p", fn));
    CHECK(check_dev(y, "y", fn));
    HIP_TRY(launch_track_observe(*md, (int)K, phi1, p, y, (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_track_chi2(dnb_ctx* c, const dnb_track_model* md, int64_t K, const double* track,
                          int64_t batch, const double* p, double* chi2, double* jtr, double* jtj,
                          void* stream) {
    const char* fn = "dnb_track_chi2";
    CHECK(check_track(c, md, K, track, "track", fn));
    CHECK(check_batch(batch, fn));
    CHECK(check_dev(p, "p", fn));
    CHECK(check_dev(chi2, "chi2", fn));
    CHECK(check_dev(jtr, "jtr", fn, true));
    CHECK(check_dev(jtj, "jtj", fn, true));
    HIP_TRY(launch_track_eval(*md, track, (int)K, (int)batch, p, chi2, jtr, jtj,
                              (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_track_hessian(dnb_ctx* c, const dnb_track_model* md, int64_t K,
                             const double* track, int64_t batch, const double* p, double* hess,
                             double* cov, void* stream) {
    const char* fn = "dnb_track_hessian";
    CHECK(check_track(c, md, K, track, "track", fn));
    CHECK(check_batch(batch, fn));
    CHECK(check_dev(p, "p", fn));
    CHECK(check_dev(hess, "hess", fn));
    CHECK(check_dev(cov, "cov", fn, true));
    if (cov == hess) return fail(DNB_ERR_ARG, "%s: cov must not alias hess", fn);
    HIP_TRY(launch_track_hessian(*md, track, (int)K, (int)batch, p, hess, cov,
                                 (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_track_lm(dnb_ctx* c, const dnb_track_model* md, int64_t K, const double* track,
                        int64_t batch, double* p, int64_t n_iter, double lambda0, double* chi2,
                        void* stream) {
    const char* fn = "dnb_track_lm";
    CHECK(check_track(c, md, K, track, "track", fn));
    CHECK(check_batch(batch, fn));
    if (n_iter < 0) return fail(DNB_ERR_ARG, "%s: n_iter < 0", fn);
    if (!(lambda0 > 0) || !is_fin(lambda0)) return fail(DNB_ERR_ARG, "%s: lambda0 must be > 0", fn);
    CHECK(check_dev(p, "p", fn));
    CHECK(check_dev(chi2, "chi2", fn));
    // workspace: the VJP partial buffer, 64 * slice_rows >= 64 * 2^21 bytes
    if (lm_workspace_bytes(batch) > 64 * (size_t)c->slice_rows)
        return fail(DNB_ERR_ARG, "%s: batch too large for the context workspace", fn);
    HIP_TRY(launch_track_lm(*md, track, (int)K, (int)batch, p, n_iter, lambda0, chi2, c->partv,
                            (hipStream_t)stream));
    return DNB_OK;
}

dnb_status dnb_profile(dnb_ctx* c, int enable) {
    if (!c) return fail(DNB_ERR_ARG, "dnb_profile: ctx is NULL");
    if (!c->prof) {
        c->prof = new (std::nothrow) Prof();
        if (!c->prof) return fail(DNB_ERR_NOMEM, "dnb_profile: host allocation failed");
    }
    ((Prof*)c->prof)->on = enable != 0;
    return DNB_OK;
}

dnb_status dnb_profile_read(dnb_ctx* c, double* out4) {
    if (!c || !out4) return fail(DNB_ERR_ARG, "dnb_profile_read: NULL argument");
    for (int k = 0; k < 4; ++k) out4[k] = 0.0;
    Prof* pf = (Prof*)c->prof;
    if (!pf) return DNB_OK;
    for (int kind = 0; kind < 2; ++kind) {
        auto& v = pf->ev[kind];
        double tot = 0.0;
        for (size_t k = 0; k + 1 < v.size(); k += 2) {
            HIP_TRY(hipEventSynchronize(v[k + 1]));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, v[k], v[k + 1]));
            tot += ms;
        }
        out4[2 * kind] = tot;
        out4[2 * kind + 1] = (double)(v.size() / 2);
        for (hipEvent_t e : v) pf->pool.push_back(e);
        v.clear();
    }
    return DNB_OK;
}

}  // extern "C"
