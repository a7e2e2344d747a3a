// Host-side logic of libdnb that needs no GPU: launch geometry, buffer sizes,
// argument validation of the host-galaxy parameters, and the ring of tape
// descriptors the reverse sweeps check their arguments against.  Plain C++17
// without HIP, so that it also builds with a host compiler under AddressSanitizer
// and UndefinedBehaviorSanitizer (tests/c/host_logic_test.cpp).
#pragma once

#include <stdint.h>
#include <string.h>

#include <cmath>

#include "../../include/dnb.h"

namespace dnb {

// ---------------------------------------------------------------- geometry --
constexpr int BS = 256;              // threads per block of every particle kernel
constexpr int TILE = 256;            // sources staged in LDS per tile
constexpr int SUBTILE = 128;         // sources summed in plain FP32 before a TwoSum
constexpr int TARGET_BLOCKS = 16384; // pair-kernel blocks wanted per launch (64 per CU)
constexpr int S_MAX = 64;            // maximum number of source slices
constexpr int SLICE_GRAIN = 32;      // pair-kernel source slices are multiples of this
constexpr int REC = 8;               // doubles per block record of the O(N) kernels
constexpr int RT = 64;               // targets per block of the FP32C slice reductions (a wave)
constexpr int RG = BS / RT;          // slice groups per block of those reductions
constexpr int64_t MAX_N = int64_t(1) << 26;   // largest context (particles)

// Target block x, source slice y and member b of the block with linear index L
// of a batched pair launch over (nblk target blocks, S slices, B members).  The
// dispatcher deals consecutive blocks out to the XCDs and their compute units in
// turn, so the blocks one compute unit holds at a time lie about 256 apart in L.
// Read as L = r + 256 q, with x = q mod nblk and (member, slice) index
// r + 256 (q / nblk), those blocks share member and slice and differ in the
// target block, so their sources stay in the unit's scalar cache; this covers
// the largest multiple of 256 (member, slice) pairs, and the pairs left over take
// the plain order.  A bijection of [0, nblk S B) onto the blocks (constexpr, so
// device code calls it too).
struct BatchBlockIdx {
    int64_t x, y, b;
};
constexpr BatchBlockIdx batch_block_index(int64_t L, int64_t nblk, int64_t S, int64_t B) {
    const int64_t G = 256;
    const int64_t Q = (S * B) / G;
    const int64_t head = nblk * G * Q;
    int64_t x = 0, c = 0;
    if (L < head) {
        const int64_t q = L / G;
        x = q % nblk;
        c = L % G + G * (q / nblk);
    } else {
        x = (L - head) % nblk;
        c = G * Q + (L - head) / nblk;
    }
    return BatchBlockIdx{x, c % S, c / S};
}

// ceil(a / b) for a >= 0, b > 0 (without forming a + b, which could overflow).
inline int64_t cdiv(int64_t a, int64_t b) { return a / b + (a % b != 0 ? 1 : 0); }

// Length of the staged source arrays: n rounded up to whole sub-tiles; the
// entries past n are far-away zero-mass particles.
inline int64_t pad_sources(int64_t n) { return cdiv(n, SUBTILE) * SUBTILE; }

// Source slicing of the O(N^2) kernels: the grid is (target blocks) x S, each
// block owns tpb targets (one per lane) and sums one contiguous slice of
// sources.  Small N gets more slices so that the launch still fills the 256
// compute units with about `target` blocks.  slicing_for serves the MMD and
// energy kernels (slices of whole LDS tiles); pair_slicing below the pair
// kernels.
struct Slicing {
    int S;          // number of slices
    int jslice;     // sources per slice (a multiple of TILE, SLICE_GRAIN for the pair kernels)
    int nblk;       // target blocks
    int64_t npad;   // row stride of the partial buffers (n rounded up to tpb)
};

inline Slicing slicing_for(int64_t n, int tpb, int target) {
    Slicing s;
    s.nblk = (int)cdiv(n, tpb);
    s.npad = (int64_t)s.nblk * tpb;
    int64_t want = target / s.nblk;
    int64_t max_by_tiles = cdiv(n, TILE);   // at least one tile per slice
    if (want > max_by_tiles) want = max_by_tiles;
    if (want > S_MAX) want = S_MAX;
    if (want < 1) want = 1;
    s.jslice = (int)(cdiv(cdiv(n, want), TILE) * TILE);
    s.S = (int)cdiv(n, s.jslice);
    return s;
}

// Source slicing of the pair kernels: ni targets (blocks of BS) against n
// sources in slices of a multiple of SLICE_GRAIN sources (a slice shorter than a
// sub-tile is summed as one short sub-tile), S <= smax.  A small system gets
// short slices so that its launch still spreads over many compute units.
inline Slicing pair_slicing(int64_t ni, int64_t n, int target, int smax) {
    Slicing s;
    s.nblk = (int)cdiv(ni, BS);
    s.npad = (int64_t)s.nblk * BS;
    int64_t want = target / s.nblk;
    const int64_t max_by_grain = cdiv(n, SLICE_GRAIN);
    if (want > max_by_grain) want = max_by_grain;
    if (want > smax) want = smax;
    if (want < 1) want = 1;
    s.jslice = (int)(cdiv(cdiv(n, want), SLICE_GRAIN) * SLICE_GRAIN);
    s.S = (int)cdiv(n, s.jslice);
    return s;
}

// Upper bound of S * npad over all n <= max_n for blocks of at most tpb targets:
// S <= want = clamp(target / nblk, 1, S_MAX), so S * npad <= want * nblk * tpb
// <= max(target * tpb, npad(max_n)).
inline int64_t max_slice_rows(int64_t max_n, int tpb, int target) {
    const int64_t np = cdiv(max_n, tpb) * tpb;
    const int64_t small = (int64_t)target * tpb;
    return np > small ? np : small;
}

// ------------------------------------------------------------ buffer sizes --
// Largest buffer length (doubles) any size query returns: its byte count then
// fits an int64 and a size_t with room to spare.
constexpr int64_t MAX_DOUBLES = int64_t(1) << 58;

// a * b, or -1 when a, b >= 0 and the product exceeds MAX_DOUBLES.
inline int64_t mul_capped(int64_t a, int64_t b) {
    if (a == 0 || b == 0) return 0;
    if (a > MAX_DOUBLES / b) return -1;
    return a * b;
}

// Doubles of the tape of dnb_simulate: per checkpoint the state (6n), two
// staging centres (8) and the internal acceleration (3n), then the internal
// acceleration at the final positions (3n).  -1 for invalid or oversized input.
inline int64_t tape_doubles(int64_t n, int64_t T, int64_t K) {
    if (n < 1 || n > MAX_N || T < 0 || K < 1) return -1;
    if (T == 0) return 0;
    const int64_t per = mul_capped(cdiv(T, K), 9 * n + 8);
    if (per < 0 || per > MAX_DOUBLES - 3 * n) return -1;
    return per + 3 * n;
}

// Doubles of the workspace of dnb_simulate_vjp: 16n of per-sweep rows and, with
// checkpoints K > 1 steps apart, two buffers of a recomputed segment (one
// recomputed while the sweep reads the other), each the segment's positions
// (3n (K + 1)) and accelerations (3n K).
inline int64_t vjp_workspace_doubles(int64_t n, int64_t K) {
    if (n < 1 || n > MAX_N || K < 1) return -1;
    if (K == 1) return 16 * n;
    const int64_t seg = mul_capped(12 * n, K);
    if (seg < 0 || seg > MAX_DOUBLES - 22 * n) return -1;
    return seg + 22 * n;
}

// Doubles of the workspace of dnb_simulate_vjp_reversed: the velocity being
// stepped back (3n), the per-particle parameter sums (8n) and two buffers of
// rebuilt positions (6n), whatever the checkpoint spacing.
inline int64_t vjp_reversed_workspace_doubles(int64_t n) {
    if (n < 1 || n > MAX_N) return -1;
    return 17 * n;
}

// Offset (doubles) of segment buffer b (0 or 1) in that workspace, and its
// accelerations' offset within the buffer.
inline int64_t vjp_segment_offset(int64_t n, int64_t K, int b) {
    return 16 * n + (int64_t)b * (6 * n * K + 3 * n);
}
inline int64_t vjp_segment_accel_offset(int64_t n, int64_t K) { return 3 * n * (K + 1); }

// Doubles of the tape of dnb_simulate_batch: every step's state (6 n per member)
// and the internal accelerations at the n_steps + 1 positions (3 n per member).
inline int64_t batch_tape_doubles(int64_t batch, int64_t n, int64_t T) {
    if (batch < 1 || batch > DNB_BATCH_MAX || n < 1 || n > MAX_N || T < 0) return -1;
    if (T == 0) return 0;
    const int64_t t9 = mul_capped(T, 9);
    if (t9 < 0 || t9 > MAX_DOUBLES - 3) return -1;
    const int64_t per_member = mul_capped(t9 + 3, n);
    if (per_member < 0) return -1;
    return mul_capped(per_member, batch);
}

// ---------------------------------------------------------- potential check --
// Why a host-galaxy parameter set cannot be used, or nullptr when it can.
inline const char* pot_error(const dnb_pot& p) {
    const double v[7] = {p.G, p.eps, p.m_nfw, p.rs_nfw, p.m_mn, p.a_mn, p.b_mn};
    for (double x : v)
        if (!std::isfinite(x)) return "non-finite potential parameter";
    if (p.eps < 0) return "eps must be >= 0";
    if (p.m_nfw != 0 && !(p.rs_nfw > 0)) return "rs_nfw must be > 0";
    if (p.m_mn != 0 && (p.a_mn < 0 || p.b_mn < 0)) return "a_mn and b_mn must be >= 0";
    if (p.m_mn != 0 && p.a_mn == 0 && p.b_mn == 0)
        return "a_mn = b_mn = 0 makes the disk a point mass; use b_mn > 0";
    return nullptr;
}

// ------------------------------------------------------- tape descriptors ---
// What dnb_simulate (batch = 0) or dnb_simulate_batch wrote a tape for.
struct TapeDesc {
    const double* tape;
    const double* pos;   // the in-place position array: the final positions
    const double* mass;
    int64_t n, n_steps, ckpt_every;
    double dt;
    double pot[7];       // G, eps, m_nfw, rs_nfw, m_mn, a_mn, b_mn
    int64_t batch;       // 0: dnb_simulate; else the members of dnb_simulate_batch
    uint64_t table;      // hash of the batch's host parameter table (0 for a single system)
    const double* vel;   // the in-place velocity array: the final velocities (single system)

    int64_t length() const {
        return batch ? batch_tape_doubles(batch, n, n_steps) : tape_doubles(n, n_steps, ckpt_every);
    }
};

// The descriptors of the most recent tapes (a ring, newest at head - 1).
struct TapeRing {
    static constexpr int SIZE = 16;
    TapeDesc d[SIZE];
    int count = 0;   // valid entries (<= SIZE)
    int head = 0;    // next slot to write

    void remember(const TapeDesc& t) {
        d[head] = t;
        head = (head + 1) % SIZE;
        if (count < SIZE) ++count;
    }

    // A run that moves the positions pos in place makes every tape whose final
    // positions are pos stale; a tape written over [tape, tape + len) replaces
    // every tape it overlaps.  A run that moves the velocities vel in place only
    // drops them from the tapes whose final velocities they were: the sweep that
    // steps backward from them refuses such a tape, the one that recomputes
    // forward does not read them.
    void forget(const double* pos, const double* tape, int64_t len,
                const double* vel = nullptr) {
        for (int k = 0; k < count; ++k) {
            TapeDesc& t = d[k];
            if (!t.tape) continue;
            const int64_t tl = t.length();
            const bool overlap = tape && len > 0 && tl > 0 && tape < t.tape + tl &&
                                 t.tape < tape + len;
            if (t.pos == pos || overlap) t.tape = nullptr;
            else if (vel && t.vel == vel) t.vel = nullptr;
        }
    }

    // The live descriptor of a tape at this address, or nullptr.
    const TapeDesc* find(const double* tape) const {
        for (int k = 0; k < count; ++k)
            if (d[k].tape && d[k].tape == tape) return &d[k];
        return nullptr;
    }
};

// FNV-1a over the bytes of a batch's host parameter table [batch][8].
inline uint64_t table_hash(const double* params, int64_t batch) {
    const unsigned char* b = (const unsigned char*)params;
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < sizeof(double) * 8 * (size_t)batch; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace dnb
