// The host-side logic of libdnb (paper_2511_22468_amd/csrc/host_logic.h), built
// with a host compiler under AddressSanitizer and UndefinedBehaviorSanitizer and
// run on the CPU: launch geometry invariants over many sizes, buffer-size
// formulas against the buffer layouts and at the edge of int64 overflow, the
// host-galaxy parameter check, and the ring of tape descriptors.  Prints
// "host logic ok" and exits 0 when every check holds; any failed check or
// sanitizer report exits non-zero.
#include <stdio.h>
#include <stdlib.h>

#include <cmath>

#include <vector>

#include "../../paper_2511_22468_amd/csrc/host_logic.h"

using namespace dnb;

static int g_fail = 0;
#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            if (++g_fail > 20) exit(1);                                       \
        }                                                                     \
    } while (0)

// Every source in exactly one slice, every slice non-empty and whole grains,
// S within its cap, every target in a block, and the partial buffer large enough.
static void check_pair_slicing(int64_t ni, int64_t n, int target, int smax, int64_t rows_cap) {
    const Slicing s = pair_slicing(ni, n, target, smax);
    EXPECT(s.S >= 1 && s.S <= (smax < 1 ? 1 : smax));
    EXPECT(s.jslice > 0 && s.jslice % SLICE_GRAIN == 0);
    EXPECT((int64_t)s.S * s.jslice >= n);
    EXPECT((int64_t)(s.S - 1) * s.jslice < n);
    EXPECT((int64_t)s.nblk * BS >= ni && (int64_t)(s.nblk - 1) * BS < ni);
    EXPECT(s.npad == (int64_t)s.nblk * BS);
    if (rows_cap > 0) EXPECT((int64_t)s.S * s.npad <= rows_cap);
}

static void check_slicing_for(int64_t n, int tpb, int target) {
    const Slicing s = slicing_for(n, tpb, target);
    EXPECT(s.S >= 1 && s.S <= S_MAX);
    EXPECT(s.jslice > 0 && s.jslice % TILE == 0);
    EXPECT((int64_t)s.S * s.jslice >= n && (int64_t)(s.S - 1) * s.jslice < n);
    EXPECT((int64_t)s.S * s.npad <= max_slice_rows(n, tpb, target));
}

static void geometry() {
    const int targets[] = {1024, 2048, 4096, 8192, 16384};
    std::vector<int64_t> sizes;
    for (int64_t n = 1; n <= 1100; ++n) sizes.push_back(n);
    for (int64_t n = 1101; n <= 300000; n = n * 21 / 20 + 1) sizes.push_back(n);
    for (int64_t n : {int64_t(65536), int64_t(131072), int64_t(262144), MAX_N - 1, MAX_N})
        sizes.push_back(n);
    for (int t : targets) {
        for (int64_t n : sizes) {
            // square launches of a context of max_n = n: the partials fit
            check_pair_slicing(n, n, t, S_MAX, max_slice_rows(n, BS, t));
            check_slicing_for(n, BS, t);
            EXPECT(pad_sources(n) % SUBTILE == 0 && pad_sources(n) >= n &&
                   pad_sources(n) - n < SUBTILE);
            // a row block of an 8-way split against the whole system (cap 256)
            const int64_t ni = cdiv(n, 8);
            const Slicing r = pair_slicing(ni, n, t, 256);
            EXPECT((int64_t)r.S * r.npad <= max_slice_rows(n, BS, t));
            check_pair_slicing(ni, n, t, 256, 0);
            check_pair_slicing(n, n, t, 1, 0);
            check_pair_slicing(n, n, t, 7, 0);
        }
    }
}

static void sizes() {
    // the formulas against the layouts they describe
    for (int64_t n : {int64_t(1), int64_t(10), int64_t(1000), int64_t(65536)}) {
        for (int64_t T : {int64_t(1), int64_t(7), int64_t(13), int64_t(1000)}) {
            for (int64_t K : {int64_t(1), int64_t(4), int64_t(13), int64_t(100)}) {
                const int64_t nc = cdiv(T, K);
                const int64_t layout = nc * 6 * n + nc * 8 + nc * 3 * n + 3 * n;
                EXPECT(tape_doubles(n, T, K) == layout);
                const int64_t ws = vjp_workspace_doubles(n, K);
                EXPECT(ws == (K == 1 ? 16 * n : 16 * n + 2 * (3 * n * (K + 1) + 3 * n * K)));
                if (K > 1) {   // the second segment buffer ends where the workspace does
                    EXPECT(vjp_segment_offset(n, K, 1) + vjp_segment_accel_offset(n, K) +
                               3 * n * K == ws);
                    EXPECT(vjp_segment_offset(n, K, 0) + vjp_segment_accel_offset(n, K) +
                               3 * n * K == vjp_segment_offset(n, K, 1));
                }
            }
            for (int64_t b : {int64_t(1), int64_t(64), int64_t(DNB_BATCH_MAX)})
                EXPECT(batch_tape_doubles(b, n, T) == (6 * T + 3 * (T + 1)) * b * n);
        }
    }
    EXPECT(tape_doubles(10, 0, 3) == 0 && batch_tape_doubles(2, 10, 0) == 0);
    // invalid arguments
    EXPECT(tape_doubles(0, 5, 1) == -1 && tape_doubles(10, -1, 1) == -1 &&
           tape_doubles(10, 5, 0) == -1 && tape_doubles(MAX_N + 1, 5, 1) == -1);
    EXPECT(vjp_workspace_doubles(0, 1) == -1 && vjp_workspace_doubles(10, 0) == -1);
    EXPECT(vjp_reversed_workspace_doubles(10) == 170 && vjp_reversed_workspace_doubles(0) == -1);
    EXPECT(vjp_reversed_workspace_doubles(MAX_N + 1) == -1);
    EXPECT(batch_tape_doubles(0, 10, 5) == -1 && batch_tape_doubles(DNB_BATCH_MAX + 1, 10, 5) == -1);
    // sizes whose products leave int64 are refused rather than wrapped
    const int64_t big = int64_t(1) << 62;
    EXPECT(tape_doubles(MAX_N, big, 1) == -1);
    EXPECT(tape_doubles(MAX_N, INT64_MAX, 1) == -1);
    EXPECT(tape_doubles(MAX_N, INT64_MAX, INT64_MAX) == 9 * MAX_N + 8 + 3 * MAX_N);
    EXPECT(vjp_workspace_doubles(MAX_N, INT64_MAX) == -1);
    EXPECT(vjp_workspace_doubles(MAX_N, big) == -1);
    EXPECT(batch_tape_doubles(DNB_BATCH_MAX, MAX_N, big) == -1);
    EXPECT(batch_tape_doubles(DNB_BATCH_MAX, MAX_N, INT64_MAX) == -1);
    EXPECT(batch_tape_doubles(DNB_BATCH_MAX, MAX_N, 1000) == 9003 * MAX_N * DNB_BATCH_MAX);
    // the largest accepted lengths still have byte counts inside int64
    for (int64_t T = 1; T < (int64_t(1) << 40); T = T * 3 + 1) {
        const int64_t l = tape_doubles(MAX_N, T, 1);
        EXPECT(l == -1 || (l > 0 && l <= MAX_DOUBLES));
        const int64_t lb = batch_tape_doubles(DNB_BATCH_MAX, MAX_N, T);
        EXPECT(lb == -1 || (lb > 0 && lb <= MAX_DOUBLES));
    }
}

static void potential() {
    const dnb_pot ok = {4.3009e-6, 1e-3, 1e12, 16.0, 6.5e10, 3.0, 0.28};
    EXPECT(pot_error(ok) == nullptr);
    dnb_pot p = ok;
    p.eps = 0.0;
    EXPECT(pot_error(p) == nullptr);
    p = ok; p.eps = -1e-3;
    EXPECT(pot_error(p) != nullptr);
    p = ok; p.rs_nfw = 0.0;
    EXPECT(pot_error(p) != nullptr);
    p = ok; p.m_nfw = 0.0; p.rs_nfw = 0.0;   // no halo: its scale radius is unused
    EXPECT(pot_error(p) == nullptr);
    p = ok; p.a_mn = -1.0;
    EXPECT(pot_error(p) != nullptr);
    p = ok; p.a_mn = 0.0; p.b_mn = 0.0;
    EXPECT(pot_error(p) != nullptr);
    p = ok; p.a_mn = 0.0;                     // a = 0: a Plummer sphere of scale b
    EXPECT(pot_error(p) == nullptr);
    double dnb_pot::*fields[] = {&dnb_pot::G, &dnb_pot::eps, &dnb_pot::m_nfw, &dnb_pot::rs_nfw,
                                 &dnb_pot::m_mn, &dnb_pot::a_mn, &dnb_pot::b_mn};
    const double bad[] = {NAN, INFINITY, -INFINITY};
    for (auto f : fields)
        for (double b : bad) {
            p = ok;
            p.*f = b;
            EXPECT(pot_error(p) != nullptr);
        }
}

static void ring() {
    std::vector<double> mem(1 << 16);
    double* base = mem.data();
    TapeRing r;
    EXPECT(r.find(base) == nullptr);
    const double* pos = base + 60000;
    auto desc = [&](int64_t off, const double* p, int64_t n, int64_t T, int64_t K) {
        return TapeDesc{base + off, p, nullptr, n, T, K, 0.1, {}, 0, 0, nullptr};
    };
    // 20 tapes into a ring of 16: the oldest 4 drop out
    for (int k = 0; k < 20; ++k) r.remember(desc(1000 * k, base + 50000 + k, 10, 5, 1));
    EXPECT(r.count == TapeRing::SIZE);
    for (int k = 0; k < 4; ++k) EXPECT(r.find(base + 1000 * k) == nullptr);
    for (int k = 4; k < 20; ++k) EXPECT(r.find(base + 1000 * k) != nullptr);
    // a run that moves the positions of tape 7 makes it stale
    r.forget(base + 50000 + 7, nullptr, 0);
    EXPECT(r.find(base + 7000) == nullptr && r.find(base + 8000) != nullptr);
    // a tape written over part of tape 9 (its 10 x 5 steps: 5 * (98) + 30 = 520 doubles)
    const int64_t l9 = tape_doubles(10, 5, 1);
    EXPECT(l9 == 520);
    r.forget(pos, base + 9000 + l9 - 1, 10);
    EXPECT(r.find(base + 9000) == nullptr && r.find(base + 10000) != nullptr);
    r.forget(pos, base + 11000 + l9, 10);   // just past tape 11: no overlap
    EXPECT(r.find(base + 11000) != nullptr);
    r.forget(pos, base + 12000 - 10, 10);   // just before tape 12: no overlap
    EXPECT(r.find(base + 12000) != nullptr);
    // the batched pair blocks' remapped index: a bijection for every shape, and
    // the blocks 256 apart share member and slice
    {
        const int64_t shapes[][3] = {{16, 8, 512}, {4, 32, 1}, {4, 8, 1000}, {1, 64, 3},
                                     {16, 8, 64},  {4, 8, 4096}, {2, 8, 33}, {256, 32, 1},
                                     {3, 17, 19}, {4, 8, 31}, {1, 8, 1}};
        for (const auto& sh : shapes) {
            const int64_t nb = sh[0], S = sh[1], B = sh[2], tot = nb * S * B;
            std::vector<char> seen((size_t)tot, 0);
            for (int64_t L = 0; L < tot; ++L) {
                const BatchBlockIdx t = batch_block_index(L, nb, S, B);
                EXPECT(t.x >= 0 && t.x < nb && t.y >= 0 && t.y < S && t.b >= 0 && t.b < B);
                const int64_t k = (t.b * S + t.y) * nb + t.x;
                EXPECT(!seen[(size_t)k]);
                seen[(size_t)k] = 1;
            }
        }
        for (int64_t k = 1; k < 8; ++k) {
            const BatchBlockIdx a = batch_block_index(37, 16, 8, 512);
            const BatchBlockIdx b = batch_block_index(37 + 256 * k, 16, 8, 512);
            EXPECT(a.y == b.y && a.b == b.b && b.x == a.x + k);
        }
    }
    // a run that moves a tape's final velocities drops them from its record only
    {
        TapeRing rv;
        const double* vel = base + 40000;
        rv.remember(TapeDesc{base, pos, nullptr, 10, 5, 1, 0.1, {}, 0, 0, vel});
        rv.forget(base + 30000, nullptr, 0, vel);
        EXPECT(rv.find(base) != nullptr && rv.find(base)->vel == nullptr);
    }
    // a batched descriptor measures its length with the batched formula
    TapeRing rb;
    rb.remember(TapeDesc{base, pos, nullptr, 10, 3, 1, 0.0, {}, 4, 77, nullptr});
    const int64_t lb = batch_tape_doubles(4, 10, 3);
    EXPECT(lb == (6 * 3 + 3 * 4) * 4 * 10);
    rb.forget(nullptr, base + lb - 1, 1);
    EXPECT(rb.find(base) == nullptr);
    // table hash: deterministic and sensitive to every byte
    double t1[2][8] = {{1, 2, 3, 4, 5, 6, 7, 8}, {9, 10, 11, 12, 13, 14, 15, 16}};
    double t2[2][8];
    memcpy(t2, t1, sizeof t1);
    EXPECT(table_hash(&t1[0][0], 2) == table_hash(&t2[0][0], 2));
    for (int b = 0; b < 2 * 8 * 8; ++b) {
        unsigned char* c = (unsigned char*)&t2[0][0];
        c[b] ^= 1;
        EXPECT(table_hash(&t1[0][0], 2) != table_hash(&t2[0][0], 2));
        c[b] ^= 1;
    }
    EXPECT(table_hash(&t1[0][0], 1) != table_hash(&t1[0][0], 2));
}

int main() {
    geometry();
    sizes();
    potential();
    ring();
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("host logic ok\n");
    return 0;
}
