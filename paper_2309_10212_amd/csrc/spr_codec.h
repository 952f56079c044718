// spr_codec.h — block decoder of the fixed-rate codec (format version 1).
//
// A record of 64*R bits holds one 4^3 block (Sec. 3.1 compresses blocks at a
// fixed rate): bit 0 = nonzero flag, bits 1..8 = biased block exponent, then
// bit planes k = 29 .. 0 of the 64 transform coefficients in embedded order:
// per plane, one refinement bit for every coefficient that was significant
// before the plane (ascending coefficient index), then group tests over the
// insignificant coefficients at or after a cursor: a 0 ends the plane; a 1 is
// followed by one bit per candidate up to the first 1 (that candidate becomes
// significant) and its sign bit, and the cursor moves past it.  Decoding stops
// where the record ends.  The inverse two-level integer S-transform then runs
// along z, y and x.
#pragma once

#include <cstdint>

namespace spr {

// ------------------------------------------------- codec: coefficient order --
// Embedded coding visits coefficient positions sorted by the sum of their
// per-axis transform levels (L:0, H:1, h0:2, h1:2), ties by raster index.
struct OrderTable {
    uint8_t ord[64];
};

static constexpr OrderTable make_order() {
    OrderTable t{};
    int lev[4] = {0, 1, 2, 2};
    int n = 0;
    for (int s = 0; s <= 6; ++s)
        for (int i = 0; i < 64; ++i)
            if (lev[i & 3] + lev[(i >> 2) & 3] + lev[(i >> 4) & 3] == s) t.ord[n++] = (uint8_t)i;
    return t;
}

static constexpr OrderTable kOrder = make_order();

// 32-bit two's complement lifting (the codec's integer arithmetic): sums
// wrap modulo 2^32 (done in unsigned arithmetic), halving is an arithmetic
// shift (rounds toward minus infinity).
__device__ __forceinline__ int32_t half32(int32_t x) { return x >> 1; }
__device__ __forceinline__ int32_t add32(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
__device__ __forceinline__ int32_t sub32(int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); }

__device__ __forceinline__ void inv4(int32_t &p0, int32_t &p1, int32_t &p2, int32_t &p3) {
    int32_t L = p0, H = p1, h0 = p2, h1 = p3;
    int32_t l1 = sub32(L, half32(H));
    int32_t l0 = add32(l1, H);
    int32_t a1 = sub32(l0, half32(h0));
    int32_t a0 = add32(a1, h0);
    int32_t a3 = sub32(l1, half32(h1));
    int32_t a2 = add32(a3, h1);
    p0 = a0; p1 = a1; p2 = a2; p3 = a3;
}

// --------------------------------------------------- codec: thread decode --
// One thread decodes one block; the lanes of a wave decode 64 blocks side by
// side, so every loop below runs until its slowest lane is done.  Instead of
// one iteration per bit, the decoder takes two passes over the record:
//
//  1. Significance pass: one iteration per group test.  A test that hits is
//     resolved in the same iteration: the candidate scan is the run of zeros
//     before the next 1 in a 64-bit window of the record, the target is the
//     candidate of that rank (a popcount binary search), and the sign bit
//     follows it.  At a plane end the plane's refinement bits are skipped
//     (there are as many as significant coefficients) and the pass records
//     where they start.  Newly significant coefficients are listed in stream
//     order.  The body has no branch: list and record writes always go to the
//     next free slot and count only when they hold an entry.
//  2. Plane pass: for the first significant plane and then each recorded
//     plane, the plane's bit word over the 64 coefficients is built (the
//     refinement bits - a window of the record at the recorded start -
//     deposited in ascending order into the coefficients significant before
//     the plane, plus the coefficients that became significant in it) and
//     OR-ed into the magnitudes, which are registers with compile-time
//     indices.
//
// Record words past the record read as 0 from LDS, so windows never need a
// bound check and refinement bits past the end deposit nothing, which is
// what a decoder that stops at the end produces.

// Per-wave LDS of the thread decoder, lane-interleaved ([slot * 64 + lane]):
// rec holds record words 0 .. RWMAX+1 (2*rate real ones, then zeros); per
// plane with refinement bits (at most 29 plus a spare slot) run holds the
// position of its first refinement bit (bits 0..9: it lies inside the record,
// at most 1024 bits) and, in bits 10..15, the number of coefficients listed
// before it modulo 64 (1 .. 64 there, so 0 stands for 64); ev lists the newly
// significant coefficients in stream order (at most 64 plus a spare slot).  The planes
// with refinement bits are consecutive: entry r is plane k_top - 1 - r, k_top
// the first significant plane.
// dep4 is the 4-bit deposit table: byte 16*mask + src holds the low
// popcount(mask) bits of src placed, in ascending order, at the set bits of
// mask.  It is filled once per workgroup by fill_dep4.
template <int RWMAX>
struct DecodeLds {
    uint32_t rec[(RWMAX + 2) * 64];
    uint32_t dep4[64];
    uint16_t run[30 * 64];
    uint8_t ev[65 * 64];
};

// Lane l writes table bytes 4l .. 4l+3 (mask l/4, sources 4(l%4) .. +3).
// The caller synchronises the workgroup before the first decode.
template <int RWMAX>
__device__ __forceinline__ void fill_dep4(DecodeLds<RWMAX> &L, uint32_t lane) {
    const uint32_t mask = lane >> 2;
    uint32_t word = 0;
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
        const uint32_t src = 4u * (lane & 3u) + c;
        uint32_t out = 0, r = 0;
#pragma unroll
        for (uint32_t b = 0; b < 4; ++b) {
            if ((mask >> b) & 1u) { out |= ((src >> r) & 1u) << b; ++r; }
        }
        word |= out << (8u * c);
    }
    L.dep4[lane] = word;
}

// 64 bits of the record from bit position pos (pos < 32 * RWMAX).
__device__ __forceinline__ uint64_t rec_window(const uint32_t *rec, uint32_t lane, uint32_t pos) {
    const uint32_t w = pos >> 5, s = pos & 31u;
    const uint64_t a0 = rec[w * 64 + lane], a1 = rec[(w + 1) * 64 + lane], a2 = rec[(w + 2) * 64 + lane];
    const uint32_t lo = (uint32_t)(((a1 << 32) | a0) >> s);
    const uint32_t hi = (uint32_t)(((a2 << 32) | a1) >> s);
    return ((uint64_t)hi << 32) | lo;
}

// Coefficients listed before a recorded plane, from its run entry.
__device__ __forceinline__ uint32_t run_count(uint16_t v) {
    const uint32_t n = (uint32_t)v >> 10;
    return n != 0u ? n : 64u;
}

// Index of the r-th set bit (from 0, ascending) of x; any value in 0..63 when
// x has r or fewer set bits.
__device__ __forceinline__ uint32_t select_bit(uint64_t x, uint32_t r) {
    const uint32_t lo = (uint32_t)x;
    uint32_t n = (uint32_t)__builtin_popcount(lo);
    bool up = r >= n;
    uint32_t w = up ? (uint32_t)(x >> 32) : lo;
    r = up ? r - n : r;
    uint32_t b = up ? 32u : 0u;
#pragma unroll
    for (uint32_t s = 16; s >= 1; s >>= 1) {
        n = (uint32_t)__builtin_popcount(w & ((1u << s) - 1u));
        up = r >= n;
        r = up ? r - n : r;
        w = up ? w >> s : w;
        b = up ? b + s : b;
    }
    return b;
}

// m[j] |= bit j of D at plane k, for the 64 coefficients.  A group of 16
// coefficients whose bits are zero on every lane of the wave (the high
// coefficients of early planes) is skipped: OR-ing zeros changes nothing.
__device__ __forceinline__ void or_plane(uint32_t (&m)[64], uint64_t D, uint32_t k) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const uint32_t d = (uint32_t)(D >> (16 * g)) & 0xFFFFu;
        if (__ballot(d != 0u) != 0ull) {
#pragma unroll
            for (int j = 0; j < 16; ++j) m[16 * g + j] |= ((d >> j) & 1u) << k;
        }
    }
}

// Deposit of the low bits of b at the set bits of mask (ascending), 32 bits
// wide, four mask bits at a time through the table.
__device__ __forceinline__ uint32_t deposit32(const uint8_t *dep4, uint32_t mask, uint32_t b) {
    uint32_t D = 0, r = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t mn = (mask >> (4 * i)) & 15u;
        D |= (uint32_t)dep4[mn * 16u + ((b >> r) & 15u)] << (4 * i);   // r <= 28 here
        r += (uint32_t)__builtin_popcount(mn);
    }
    return D;
}

// Decodes the record into q[64] (raster order) and the block exponent.
// Returns false for an all-zero block (q untouched).  L: this wave's LDS;
// lane: lane id within the wave; rate: 1..16 bits per value (RWMAX >= 2 rate).
template <int RWMAX>
__device__ __forceinline__ bool thread_decode(const uint32_t *__restrict__ rec, int rate, DecodeLds<RWMAX> &L,
                                              uint32_t lane, int32_t (&q)[64], int &e_out) {
    const uint32_t rw = 2u * (uint32_t)rate;
    // the record lives in global memory: global (not flat) loads, all issued
    // before the LDS stores, so the words arrive in one round trip
    typedef const __attribute__((address_space(1))) uint32_t *grec_t;
    const grec_t g = (grec_t)rec;
    const uint32_t w0 = g[0];
    if (!(w0 & 1u)) return false;
    uint32_t words[RWMAX + 1];
#pragma unroll
    for (int j = 1; j < RWMAX + 2; ++j) words[j - 1] = (uint32_t)j < rw ? g[j] : 0u;
    L.rec[lane] = w0;
#pragma unroll
    for (int j = 1; j < RWMAX + 2; ++j) L.rec[j * 64 + lane] = words[j - 1];
    e_out = (int)((w0 >> 1) & 0xFFu) - 127;
    const uint32_t B = 64u * (uint32_t)rate;

    // 1. significance pass.  Invariant at the top: pos < B.
    uint64_t S = 0, NEG = 0;
    uint32_t pos = 9, c = 0, nev = 0, nrun = 0, k_top = 0;
    int k = 29;
    bool scanning = false;   // a scan continues (its group-test bit was read already)
    // Planes above the first significant coefficient have no refinement bits
    // and end at their first group test, a 0: skip the run of them at once
    // (at most all 30 planes; 9 + 30 bits always lie inside the record).
    {
        const uint32_t z0 = (uint32_t)__builtin_ctzll(rec_window(L.rec, lane, pos) | (1ull << 30));
        pos += z0;
        k -= (int)z0;
    }
    bool live = k >= 0;
    while (live) {
        const uint64_t win = rec_window(L.rec, lane, pos);
        const uint64_t cand = c >= 64u ? 0ull : (~S & (~0ull << c));
        const uint32_t ncand = (uint32_t)__builtin_popcountll(cand);
        const uint32_t off = scanning ? 0u : 1u;
        const bool hit = cand != 0ull && (scanning || (win & 1ull) != 0ull);
        const uint64_t sw = win >> off;                 // scan bits (>= 63 valid)
        const uint32_t lim = ncand < 62u ? ncand : 62u; // scan bits examined; the sign needs one more
        const uint32_t z = (uint32_t)__builtin_ctzll(sw | (1ull << lim));
        const bool found = hit && z < lim;
        const bool more = hit && !found && ncand > lim; // 62 zeros and candidates left: the scan goes on
        const uint32_t t = select_bit(cand, found ? z : 61u);
        const uint32_t past_sign = pos + off + z + 2u;
        const bool apply = found && past_sign <= B;     // the sign bit lies inside the record
        const uint64_t tb = apply ? 1ull << t : 0ull;
        S |= tb;
        NEG |= ((sw >> (z + 1u)) & 1ull) != 0ull ? tb : 0ull;
        L.ev[nev * 64 + lane] = (uint8_t)t;
        k_top = (apply && nev == 0u) ? (uint32_t)k : k_top;
        nev += apply ? 1u : 0u;
        c = (apply || more) ? t + 1u : c;
        scanning = more;
        uint32_t npos = found ? past_sign : (more ? pos + off + 62u : pos + (cand != 0ull ? 1u : 0u));
        // plane end (no hit): the next plane's refinement bits start at npos
        const bool pe = !hit;
        const int kn = pe ? k - 1 : k;
        const bool next_plane = pe && kn >= 0;
        L.run[nrun * 64 + lane] = (uint16_t)((npos & 1023u) | (nev << 10));   // read back only when recorded
        nrun += (next_plane && S != 0ull && npos < B) ? 1u : 0u;
        npos += next_plane ? (uint32_t)__builtin_popcountll(S) : 0u;
        c = pe ? 0u : c;
        k = kn;
        pos = npos;
        live = !(hit && !found && !more) && kn >= 0 && pos < B;   // a scan without a 1 ends the record
    }

    // 2. plane pass: m[j] = magnitude of coefficient j (order space)
    uint32_t m[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) m[j] = 0u;
    uint64_t Sr = 0;
    uint32_t e = 0;
    {
        // the first significant plane has no refinement bits
        const uint32_t ne = nrun > 0u ? run_count(L.run[lane]) : nev;
        for (; e < ne; ++e) Sr |= 1ull << L.ev[e * 64 + lane];
        or_plane(m, Sr, k_top);
    }
    for (uint32_t r = 0; r < nrun; ++r) {
        const uint32_t ne = r + 1u < nrun ? run_count(L.run[(r + 1u) * 64 + lane]) : nev;
        const uint64_t bits = rec_window(L.rec, lane, (uint32_t)L.run[r * 64 + lane] & 1023u);
        // deposit, in 32-bit halves: the refinement bits of coefficients 32..63
        // follow those of 0..31 (as many as the low half has significant ones)
        const uint8_t *dep4 = reinterpret_cast<const uint8_t *>(L.dep4);
        const uint32_t slo = (uint32_t)Sr, shi = (uint32_t)(Sr >> 32);
        const uint32_t Dlo = deposit32(dep4, slo, (uint32_t)bits);
        uint32_t Dhi = 0;
        if (__ballot(shi != 0u) != 0ull) Dhi = deposit32(dep4, shi, (uint32_t)(bits >> __builtin_popcount(slo)));
        uint64_t Sn = Sr;
        for (; e < ne; ++e) Sn |= 1ull << L.ev[e * 64 + lane];
        or_plane(m, ((uint64_t)Dhi << 32 | Dlo) | (Sn & ~Sr), k_top - 1u - r);
        Sr = Sn;
    }

#pragma unroll
    for (int j = 0; j < 64; ++j) {
        int32_t v = (int32_t)m[j];   // magnitudes < 2^30
        if ((NEG >> j) & 1ull) v = -v;
        q[kOrder.ord[j]] = v;
    }
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int x = 0; x < 4; ++x) inv4(q[x + 4 * y], q[x + 4 * y + 16], q[x + 4 * y + 32], q[x + 4 * y + 48]);
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
        for (int x = 0; x < 4; ++x) inv4(q[x + 16 * z], q[x + 16 * z + 4], q[x + 16 * z + 8], q[x + 16 * z + 12]);
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
        for (int y = 0; y < 4; ++y) inv4(q[4 * y + 16 * z], q[4 * y + 16 * z + 1], q[4 * y + 16 * z + 2], q[4 * y + 16 * z + 3]);
    return true;
}

}  // namespace spr
