// gen.hip -- synthetic game states on the GPU.
//
// The deal of Sec. II-A (every player takes tiles from the shuffled pool and
// keeps them in ascending order) extended to mid-game positions: a pool size
// is drawn, the tiles drawn since the deal are handed out round-robin from
// seat 0, a random subset of every row is revealed (one tile always stays
// hidden), and optionally the seat to move draws.  The words of state s come
// one after another from Philox blocks (n>>2, 0xFFFFFFFF, 0xFFFFFFFF, s).
//
// One wavefront per state.  Every word a state can use lies in its first 14
// blocks, so lane b computes block b at once, and four shuffles then put word
// w in lane w: a word is one read from its lane when its turn comes.  The 23
// swap targets of the tile shuffle are picked in parallel, one per lane.  The
// shuffles are followed from the tiles' side:
// lane t (t < 24) keeps the position of tile t through the swaps of the
// Fisher-Yates shuffle, so a row, a set of revealed tiles or the pool is one
// ballot -- no per-state array and no serial chain through memory.
#include "dvc_core.hpp"
#include "dvc_internal.hpp"

namespace dvc {

// States per 256-thread workgroup: one per wavefront.
constexpr uint32_t kGenBlock = 256;
constexpr uint32_t kGenStatesPerBlock = kGenBlock / 64u;

__global__ void __launch_bounds__(kGenBlock) init_states_kernel(uint4 *out, uint32_t n, DealArgs d,
                                                                uint32_t k0, uint32_t k1,
                                                                uint32_t base)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t i = __builtin_amdgcn_readfirstlane(blockIdx.x * kGenStatesPerBlock +
                                                      (threadIdx.x >> 6));
    if (i >= n) return;   // the whole wavefront
    // words: at most 2 (players, pool) + 23 (shuffle) + 4 + 22 (reveals: at
    // most 24 - P of them) + 2 (draw coin, draw) = 53, i.e. blocks 0..13
    const Words blk = philox(lane, 0xFFFFFFFFu, 0xFFFFFFFFu, base + i, k0, k1);
    // lane w holds word w (component w % 4 of block w / 4)
    const int src = (int)(lane >> 2);
    const uint32_t c0 = (uint32_t)__shfl((int)blk.w0, src, 64);
    const uint32_t c1 = (uint32_t)__shfl((int)blk.w1, src, 64);
    const uint32_t c2 = (uint32_t)__shfl((int)blk.w2, src, 64);
    const uint32_t c3 = (uint32_t)__shfl((int)blk.w3, src, 64);
    const uint32_t cl = lane & 3u;
    const uint32_t words = cl == 0u ? c0 : cl == 1u ? c1 : cl == 2u ? c2 : c3;
    uint32_t nw = 0u;
    auto word = [&]() -> uint32_t {
        const uint32_t w = __builtin_amdgcn_readlane(words, nw);
        ++nw;
        return w;
    };
    const bool tile_lane = lane < 24u;

    uint32_t P = (uint32_t)d.p_min;
    if (d.p_max > d.p_min) P += pick(word(), (uint32_t)(d.p_max - d.p_min + 1));
    const uint32_t h0 = (uint32_t)d.hand[P];
    const uint32_t cap = 24u - P * h0;
    uint32_t pile;
    if (d.fresh) {
        pile = cap;
    } else {
        uint32_t lo = min<uint32_t>((uint32_t)d.pile_min, cap);
        uint32_t hi = min<uint32_t>((uint32_t)d.pile_max, cap);
        hi = max(hi, lo);
        pile = lo + pick(word(), hi - lo + 1u);
    }
    // Fisher-Yates over positions 23..1: the tiles at positions k and j swap.
    // Step t (k = 23 - t) uses word nw + t; lane t picks its j.
    const uint32_t fw = (uint32_t)__shfl((int)words, (int)((nw + lane) & 63u), 64);
    const uint32_t jv = lane < 23u ? pick(fw, 24u - lane) : 0u;
    nw += 23u;
    uint32_t pos = lane;
#pragma unroll
    for (uint32_t t = 0; t < 23u; ++t) {
        const uint32_t k = 23u - t;
        const uint32_t j = __builtin_amdgcn_readlane(jv, t);
        pos = pos == k ? j : (pos == j ? k : pos);
    }
    // rows: seat q takes the next h_q positions of the shuffled array
    const uint32_t drawn_since = 24u - P * h0 - pile;
    uint32_t hand[4] = {0u, 0u, 0u, 0u};
    uint32_t start = 0u;
#pragma unroll
    for (uint32_t q = 0; q < 4u; ++q) {
        if (q >= P) break;
        const uint32_t h = h0 + drawn_since / P + (q < drawn_since % P ? 1u : 0u);
        hand[q] = (uint32_t)__ballot(tile_lane && pos >= start && pos < start + h);
        start += h;
    }
    // reveal a random subset of every row: a partial Fisher-Yates over the
    // row's slots, whose first nrev slots at the end are revealed
    uint32_t rev = 0u;
#pragma unroll
    for (uint32_t q = 0; q < 4u; ++q) {
        if (q >= P) break;
        const uint32_t hq = hand[q];
        const uint32_t h = (uint32_t)__popc(hq);
        const uint32_t rmax = min<uint32_t>((uint32_t)d.revealed_max, h - 1u);
        const uint32_t nrev = d.fresh ? 0u : pick(word(), rmax + 1u);
        const bool mine = tile_lane && ((hq >> (lane & 31u)) & 1u);
        uint32_t slot = tile_lane ? (uint32_t)__popc(hq & ((1u << lane) - 1u)) : 0u;
        // step k uses word nw + k; lane k picks its swap target
        const uint32_t rw = (uint32_t)__shfl((int)words, (int)((nw + lane) & 63u), 64);
        const uint32_t jr = lane < h ? lane + pick(rw, h - lane) : 0u;
        nw += nrev;
        for (uint32_t k = 0; k < nrev; ++k) {
            const uint32_t j = __builtin_amdgcn_readlane(jr, k);
            slot = slot == k ? j : (slot == j ? k : slot);
        }
        rev |= (uint32_t)__ballot(mine && slot < nrev);
    }
    State s;
    s.h0 = hand[0]; s.h1 = hand[1]; s.h2 = hand[2]; s.h3 = hand[3];
    s.rev = rev;
    s.P = P;
    s.m = drawn_since % P;
    s.phase = 0u;
    s.drawn = -1;
    bool do_draw = d.root_draw != 0;
    if (!do_draw && d.phase_mix) do_draw = word() < 0x80000000u;
    const uint32_t pool = ~(hand[0] | hand[1] | hand[2] | hand[3]) & kAll;
    if (do_draw && pool != 0u) {
        const uint32_t t = pick_bit(pool, word());
        add_to_hand(s, s.m, 1u << t);
        s.drawn = (int32_t)t;
        s.phase = 1u;
    }
    if (lane == 0) {
        uint4 o;
        encode(s, o.x, o.y, o.z, o.w);
        out[i] = o;
    }
}

hipError_t launch_init_states(uint4 *out, uint32_t n, const DealArgs &d, uint32_t k0, uint32_t k1,
                              uint32_t index_base, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(init_states_kernel, dim3((n + kGenStatesPerBlock - 1u) / kGenStatesPerBlock),
                       dim3(kGenBlock), 0, st, out, n, d, k0, k1, index_base);
    return hipGetLastError();
}

}  // namespace dvc
