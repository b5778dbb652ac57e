// gen.hip -- synthetic game states on the GPU.
//
// The deal of Sec. II-A (every player takes tiles from the shuffled pool and
// keeps them in ascending order) extended to mid-game positions: a pool size
// is drawn, the tiles drawn since the deal are handed out round-robin from
// seat 0, a random subset of every row is revealed (one tile always stays
// hidden), and optionally the seat to move draws.  One thread per state; the
// words of state s come one after another from Philox blocks
// (n>>2, 0xFFFFFFFF, 0xFFFFFFFF, s).
#include "dvc_core.hpp"
#include "dvc_internal.hpp"

namespace dvc {

struct WordStream {
    uint32_t k0, k1, c3, n;
    Words blk;
    __device__ uint32_t next()
    {
        const uint32_t slot = n & 3u;
        if (slot == 0u) blk = philox(n >> 2, 0xFFFFFFFFu, 0xFFFFFFFFu, c3, k0, k1);
        ++n;
        return slot == 0u ? blk.w0 : slot == 1u ? blk.w1 : slot == 2u ? blk.w2 : blk.w3;
    }
};

// One wavefront per workgroup: the per-state work is a serial chain of word
// draws, so small workgroups spread a batch over as many compute units as
// possible.
constexpr uint32_t kGenBlock = 64;

__global__ void __launch_bounds__(kGenBlock) init_states_kernel(uint4 *out, uint32_t n, DealArgs d,
                                                                uint32_t k0, uint32_t k1,
                                                                uint32_t base)
{
    __shared__ uint8_t scratch_rows[kGenBlock][24];
    const uint32_t i = blockIdx.x * kGenBlock + threadIdx.x;
    if (i >= n) return;
    uint8_t *perm = scratch_rows[threadIdx.x];
    WordStream ws{k0, k1, base + i, 0u, Words{0u, 0u, 0u, 0u}};

    uint32_t P = (uint32_t)d.p_min;
    if (d.p_max > d.p_min) P += pick(ws.next(), (uint32_t)(d.p_max - d.p_min + 1));
    const uint32_t h0 = (uint32_t)d.hand[P];
    const uint32_t cap = 24u - P * h0;
    uint32_t pile;
    if (d.fresh) {
        pile = cap;
    } else {
        uint32_t lo = min<uint32_t>((uint32_t)d.pile_min, cap);
        uint32_t hi = min<uint32_t>((uint32_t)d.pile_max, cap);
        hi = max(hi, lo);
        pile = lo + pick(ws.next(), hi - lo + 1u);
    }
    // Fisher-Yates shuffle of the 24 tile ids
    for (uint32_t k = 0; k < 24u; ++k) perm[k] = (uint8_t)k;
    for (uint32_t k = 23u; k >= 1u; --k) {
        const uint32_t j = pick(ws.next(), k + 1u);
        const uint8_t tmp = perm[k];
        perm[k] = perm[j];
        perm[j] = tmp;
    }
    const uint32_t drawn_since = 24u - P * h0 - pile;
    uint32_t hand[4] = {0u, 0u, 0u, 0u};
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4u; ++q) {
        if (q >= P) break;
        const uint32_t h = h0 + drawn_since / P + (q < drawn_since % P ? 1u : 0u);
        for (uint32_t k = 0; k < h; ++k) hand[q] |= 1u << perm[pos++];
    }
    // reveal a random subset of every row (partial Fisher-Yates over slots)
    uint32_t rev = 0u;
#pragma unroll
    for (uint32_t q = 0; q < 4u; ++q) {
        if (q >= P) break;
        const uint32_t h = (uint32_t)__popc(hand[q]);
        uint32_t rmax = min<uint32_t>((uint32_t)d.revealed_max, h - 1u);
        const uint32_t nrev = d.fresh ? 0u : pick(ws.next(), rmax + 1u);
        for (uint32_t k = 0; k < h; ++k) perm[k] = (uint8_t)k;
        for (uint32_t k = 0; k < nrev; ++k) {
            const uint32_t j = k + pick(ws.next(), h - k);
            const uint8_t tmp = perm[k];
            perm[k] = perm[j];
            perm[j] = tmp;
            rev |= 1u << kth_bit(hand[q], perm[k]);
        }
    }
    State s;
    s.h0 = hand[0]; s.h1 = hand[1]; s.h2 = hand[2]; s.h3 = hand[3];
    s.rev = rev;
    s.P = P;
    s.m = drawn_since % P;
    s.phase = 0u;
    s.drawn = -1;
    bool do_draw = d.root_draw != 0;
    if (!do_draw && d.phase_mix) do_draw = ws.next() < 0x80000000u;
    const uint32_t pool = ~(hand[0] | hand[1] | hand[2] | hand[3]) & kAll;
    if (do_draw && pool != 0u) {
        const uint32_t t = pick_bit(pool, ws.next());
        add_to_hand(s, s.m, 1u << t);
        s.drawn = (int32_t)t;
        s.phase = 1u;
    }
    uint4 o;
    encode(s, o.x, o.y, o.z, o.w);
    out[i] = o;
}

hipError_t launch_init_states(uint4 *out, uint32_t n, const DealArgs &d, uint32_t k0, uint32_t k1,
                              uint32_t index_base, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(init_states_kernel, dim3((n + kGenBlock - 1u) / kGenBlock), dim3(kGenBlock), 0,
                       st, out, n, d, k0, k1, index_base);
    return hipGetLastError();
}

}  // namespace dvc
