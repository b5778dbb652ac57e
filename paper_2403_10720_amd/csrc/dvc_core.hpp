// dvc_core.hpp -- device primitives of the gfx950 Da Vinci Code engine:
// Philox4x32-10, the uniform pick, k-th set bit, the packed state and one
// guess of a random playout, all on 24-bit tile masks held in registers.
//
// Rules: Sec. II-A of Zhang et al. (arXiv 2403.10720); random playouts:
// Sec. II-B.  Tile id t = 2*value + colour, so a player's ascending row is
// simply the set bits of its mask, lowest first.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dvc {

constexpr uint32_t kAll = 0xFFFFFFu;        // the 24 tiles
constexpr uint32_t kBlack = 0x555555u;      // even ids
constexpr uint32_t kWhite = 0xAAAAAAu;      // odd ids
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

struct Words { uint32_t w0, w1, w2, w3; };

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplies; the key advances by the Weyl constants between rounds.
__device__ __forceinline__ void philox_round(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                             uint32_t &x3, uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)x0 * kPhiloxM0;
    const uint64_t p1 = (uint64_t)x2 * kPhiloxM1;
    // three-input xor in one instruction (truth table 0x96)
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x1, k0, 0x96);
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x3, k1, 0x96);
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
}

__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        philox_round(c0, c1, c2, c3, k0, k1);
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return Words{c0, c1, c2, c3};
}

// Rounds 2..10 only, for callers that have done round 1 themselves.
__device__ __forceinline__ Words philox_rounds_2_to_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                       uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
        philox_round(c0, c1, c2, c3, k0, k1);
    }
    return Words{c0, c1, c2, c3};
}

// uniform pick among k options: floor(w * k / 2^32)
__device__ __forceinline__ uint32_t pick(uint32_t w, uint32_t k)
{
    return __umulhi(w, k);
}

// index of the k-th lowest set bit of m (k < popcount(m)); branch-free
// binary search on bit counts of the low half at every level.
__device__ __forceinline__ uint32_t kth_bit(uint32_t m, uint32_t k)
{
    uint32_t pos = 0, c;
    c = __popc(m & 0xFFFFu); if (k >= c) { k -= c; m >>= 16; pos += 16; }
    c = __popc(m & 0xFFu);   if (k >= c) { k -= c; m >>= 8;  pos += 8; }
    c = __popc(m & 0xFu);    if (k >= c) { k -= c; m >>= 4;  pos += 4; }
    c = __popc(m & 0x3u);    if (k >= c) { k -= c; m >>= 2;  pos += 2; }
    c = m & 1u;              if (k >= c) { pos += 1; }
    return pos;
}

// uniform random member of a non-empty mask
__device__ __forceinline__ uint32_t pick_bit(uint32_t m, uint32_t w)
{
    return kth_bit(m, pick(w, (uint32_t)__popc(m)));
}

// k-th set bit through a 2 KB LDS table: tab[8*b + i] is the position of the
// i-th set bit of byte b.  Two bit counts choose the byte that holds the
// k-th bit of the 24-bit mask, one LDS byte read finishes the search.
constexpr uint32_t kKthTableBytes = 256u * 8u;

__device__ __forceinline__ void fill_kth_table(uint8_t *tab)
{
    for (uint32_t i = threadIdx.x; i < kKthTableBytes; i += blockDim.x) {
        const uint32_t b = i >> 3, k = i & 7u;
        uint32_t pos = 0u, cnt = 0u;
        for (uint32_t bit = 0; bit < 8u; ++bit)
            if ((b >> bit) & 1u) {
                if (cnt == k) pos = bit;
                ++cnt;
            }
        tab[i] = (uint8_t)pos;
    }
}

__device__ __forceinline__ uint32_t kth_bit_tab(uint32_t m, uint32_t k, const uint8_t *tab)
{
    const uint32_t c0 = (uint32_t)__popc(m & 0xFFu);
    const uint32_t c01 = (uint32_t)__popc(m & 0xFFFFu);
    const bool b2 = k >= c01, b1 = k >= c0;
    const uint32_t sh = b2 ? 16u : (b1 ? 8u : 0u);
    const uint32_t base = b2 ? c01 : (b1 ? c0 : 0u);
    const uint32_t byte = (m >> sh) & 0xFFu;
    return sh + tab[(byte << 3) | ((k - base) & 7u)];
}

__device__ __forceinline__ uint32_t pick_bit_tab(uint32_t m, uint32_t w, const uint8_t *tab)
{
    return kth_bit_tab(m, pick(w, (uint32_t)__popc(m)), tab);
}

// Game state in registers: one tile mask per seat (seats >= P are empty).
struct State {
    uint32_t h0, h1, h2, h3;  // rows
    uint32_t rev;             // revealed tiles
    uint32_t m;               // seat to move
    uint32_t P;               // players
    uint32_t phase;           // 0 turn start, 1 mover has had its draw
    int32_t drawn;            // tile drawn this turn, -1 none
};

// row of seat q, as two levels of selects (no branches)
__device__ __forceinline__ uint32_t hand_of(const State &s, uint32_t q)
{
    const uint32_t lo = (q & 1u) ? s.h1 : s.h0;
    const uint32_t hi = (q & 1u) ? s.h3 : s.h2;
    return (q & 2u) ? hi : lo;
}

__device__ __forceinline__ void add_to_hand(State &s, uint32_t q, uint32_t bit)
{
    s.h0 |= q == 0u ? bit : 0u;
    s.h1 |= q == 1u ? bit : 0u;
    s.h2 |= q == 2u ? bit : 0u;
    s.h3 |= q == 3u ? bit : 0u;
}

// Decode the packed 16-byte format; returns false for a malformed state.
__device__ __forceinline__ bool decode(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                       State &s)
{
    const uint32_t b0 = w0 & kAll, b1 = w1 & kAll, b2 = w2 & kAll;
    s.h0 = b0 & ~b1 & ~b2;
    s.h1 = ~b0 & b1 & ~b2 & kAll;
    s.h2 = b0 & b1 & ~b2;
    s.h3 = ~b0 & ~b1 & b2 & kAll;
    s.rev = w3 & kAll;
    s.m = (w0 >> 24) & 3u;
    s.P = ((w0 >> 26) & 3u) + 1u;
    s.phase = (w0 >> 28) & 1u;
    const uint32_t dvalid = (w0 >> 29) & 1u;
    const uint32_t dtile = (w1 >> 24) & 31u;
    s.drawn = dvalid ? (int32_t)dtile : -1;
    const uint32_t owned = s.h0 | s.h1 | s.h2 | s.h3;
    const uint32_t bad_code = b2 & (b0 | b1);                  // codes 5..7
    const uint32_t seats_mask = s.P == 2 ? (s.h2 | s.h3) : s.P == 3 ? s.h3 : 0u;
    const uint32_t hm = hand_of(s, s.m);
    bool ok = (w0 >> 30) == 0u && (w1 >> 29) == 0u && (w2 >> 24) == 0u && (w3 >> 24) == 0u;
    ok = ok && (dvalid || dtile == 0u);
    ok = ok && s.P >= 2u && bad_code == 0u && seats_mask == 0u;
    ok = ok && (s.rev & ~owned) == 0u;
    ok = ok && s.m < s.P && (hm & ~s.rev) != 0u;
    ok = ok && !(s.phase == 0u && dvalid);
    ok = ok && (!dvalid || (dtile < 24u && ((hm & ~s.rev) >> dtile) & 1u));
    return ok;
}

__device__ __forceinline__ void encode(const State &s, uint32_t &w0, uint32_t &w1, uint32_t &w2,
                                       uint32_t &w3)
{
    // owner codes: seat0=1 (001), seat1=2 (010), seat2=3 (011), seat3=4 (100)
    w0 = (s.h0 | s.h2) | (s.m << 24) | ((s.P - 1u) << 26) | (s.phase << 28) |
         (s.drawn >= 0 ? (1u << 29) : 0u);
    w1 = (s.h1 | s.h2) | (s.drawn >= 0 ? ((uint32_t)s.drawn << 24) : 0u);
    w2 = s.h3;
    w3 = s.rev;
}

// seats that still hold a hidden tile
__device__ __forceinline__ uint32_t alive_mask(const State &s)
{
    const uint32_t r = ~s.rev;
    return ((s.h0 & r) ? 1u : 0u) | ((s.h1 & r) ? 2u : 0u) | ((s.h2 & r) ? 4u : 0u) |
           ((s.h3 & r) ? 8u : 0u);
}

// next seat after m (cyclic over P seats) that is in the alive mask
__device__ __forceinline__ uint32_t next_alive(uint32_t alive, uint32_t m, uint32_t P)
{
    // rotate the seat mask so that seat m+1 is bit 0
    const uint32_t full = alive | (alive << P);
    const uint32_t rot = (full >> (m + 1u)) & ((1u << P) - 1u);
    const uint32_t k = (uint32_t)__builtin_ctz(rot | (1u << P));   // rot != 0 when called
    const uint32_t q = m + 1u + k;
    return q >= P ? q - P : q;
}

// Candidate tile ids for target tile t of row `ho`, as seen by a mover with
// row `hm`: the target's colour, strictly between the nearest revealed tiles
// of the target row around t, neither in the mover's row nor revealed.
__device__ __forceinline__ uint32_t candidates(uint32_t t, uint32_t ho, uint32_t hm, uint32_t rev)
{
    const uint32_t tb = 1u << t;
    const uint32_t ro = ho & rev;
    const uint32_t below = ro & (tb - 1u);
    const uint32_t above = ro & ~(tb | (tb - 1u));
    // bits strictly above the highest revealed tile below t
    const uint32_t lo_ok = below ? ~((2u << (31u - (uint32_t)__builtin_clz(below))) - 1u) : 0xFFFFFFFFu;
    // bits strictly below the lowest revealed tile above t
    const uint32_t hi_ok = above ? ((1u << (uint32_t)__builtin_ctz(above)) - 1u) : 0xFFFFFFFFu;
    const uint32_t col = (t & 1u) ? kWhite : kBlack;
    return ~(hm | rev) & col & lo_ok & hi_ok & kAll;
}

}  // namespace dvc
