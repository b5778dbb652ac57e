// search.hip -- Monte Carlo Tree Search for the Da Vinci Code game on gfx950.
//
// Sec. II-B of Zhang et al. (arXiv 2403.10720): selection, expansion,
// simulation (random playouts) and back-propagation; Sec. III-A: a node is a
// guess (tile position, guessed number), guessing stops after a right guess
// inside the tree, and nodes at a fixed depth threshold are not expanded.
// The opponents' tiles are a black box, so each iteration first samples a
// plausible set of numbers for them.
//
// One wavefront owns one tree for the whole search (a persistent loop over
// the iterations; trees are independent, so no grid-wide synchronisation):
//   * the sampler runs 64 attempts at once, one per lane, and the lowest
//     successful attempt wins;
//   * at every tree level the lanes compute the legal value mask of 64 of
//     the 72 (target, slot) pairs at once, find the lowest untried action
//     with a ballot, or score 64 children per pass with FP32 UCT and reduce
//     with a wavefront arg-max (ties to the earliest child);
//   * the leaf's playouts run one per lane, seat wins are summed by ballots;
//   * back-propagation updates the path nodes from their own lanes.
// Per-tree statistics are left in the first words of the tree's workspace:
// nodes, child blocks, root visits, leaves scored by the network, leaves
// played out in value mode, iterations that used the sampler's fallback.
// Tree storage lives in the caller's workspace: per node a record (last
// child block, child count, bitmaps of the keys that already have a child)
// followed by its first block of 64 child entries {key | chooser << 16, N,
// W, node id}; nodes with more than 64 children chain overflow blocks.  A
// node's record and first 64 children arrive in one round of loads, and its
// children are scored 64 at a time.
//
// Each of the paper's three simplifications can be switched off:
//   * continue choice: after a right guess the same player chooses between
//     stopping (key 864) and another guess (key 865 + action), so records
//     carry a second bitmap and a stop flag;
//   * no depth threshold (max_depth 0);
//   * vanilla: the root's children are world nodes, one per distinct sampled
//     set of opponent numbers; their entries hold the 48-bit world key in
//     the key and W words, and the guesses hang below them.
#include "dvc_core.hpp"
#include "dvc_internal.hpp"

namespace dvc {

// record: pad, last block, child count, stop flag, 36 bitmap words of plain
// guesses (72 (target, slot) pairs x 16 bits), with the continue choice 36
// more for the guesses after a right guess, padded to 16 bytes
constexpr uint32_t kNodeWordsPlain = 40;
constexpr uint32_t kNodeWordsCont = 80;
constexpr uint32_t kBlockEntries = 64;
constexpr uint32_t kEntryWords = 4;
constexpr uint32_t kBlockWords = kBlockEntries * kEntryWords;
constexpr uint32_t kStopKey = kMaxActions;   // 864; a guess after a right guess is 865 + action
// tree header: nodes, overflow blocks, root visits, network leaves, played
// leaves, sampler fallbacks, failed flag, deepest leaf (tree levels below the
// root, world nodes not counted); from word 8, four 64-bit sums of
// shader clock cycles spent sampling worlds, descending, evaluating leaves
// and back-propagating
constexpr uint32_t kHdrFailed = 6;
constexpr uint32_t kHdrCycles = 8;
constexpr uint32_t kTreeHeaderWords = 16;
constexpr uint32_t kNoBlock = 0xFFFFFFFFu;
constexpr uint32_t kDetAttempts = 64;
constexpr uint32_t kDfsMaxCalls = 1u << 22;
// path entries of one iteration: a game has at most 23 guesses (each reveals
// a tile and the winner keeps one), stops only follow right guesses, and a
// world node adds one: at most 47
constexpr uint32_t kMaxPath = 64;

MctsShape mcts_shape(uint32_t iters, uint32_t cont, uint32_t vanilla)
{
    MctsShape sh;
    sh.node_words = cont ? kNodeWordsCont : kNodeWordsPlain;
    sh.node_stride = sh.node_words + kBlockWords;
    // one node per iteration, two with world nodes
    sh.nodes_cap = (vanilla ? 2u * iters : iters) + 1u;
    sh.ovf_cap = sh.nodes_cap / kBlockEntries + 2u;
    uint64_t words = kTreeHeaderWords + (uint64_t)sh.nodes_cap * sh.node_stride +
                     (uint64_t)sh.ovf_cap * kBlockWords + sh.nodes_cap + sh.ovf_cap;
    words = (words + 3u) & ~(uint64_t)3u;
    sh.agg_off = words;                     // vanilla: per-action (N, W) over the worlds
    if (vanilla) words += 2u * kMaxActions;
    sh.tree_words = (words + 3u) & ~(uint64_t)3u;   // keep every tree 16-byte aligned
    return sh;
}

__device__ __forceinline__ void set_hand(State &s, uint32_t q, uint32_t v)
{
    s.h0 = q == 0u ? v : s.h0;
    s.h1 = q == 1u ? v : s.h1;
    s.h2 = q == 2u ? v : s.h2;
    s.h3 = q == 3u ? v : s.h3;
}

// bits strictly above `lo` (lo may be -1)
__device__ __forceinline__ uint32_t above_bits(int32_t lo)
{
    return lo < 0 ? 0xFFFFFFFFu : ~((2u << (uint32_t)lo) - 1u);
}

// bits strictly below `hi` (hi <= 24)
__device__ __forceinline__ uint32_t below_bits(uint32_t hi) { return (1u << hi) - 1u; }

__device__ __forceinline__ uint32_t colour_mask(uint32_t t) { return (t & 1u) ? kWhite : kBlack; }

// Sequential word stream: word n of block (n>>2, c1, c2, c3).
struct SeqWords {
    uint32_t k0, k1, c1, c2, c3, n;
    Words blk;
    __device__ uint32_t next()
    {
        const uint32_t slot = n & 3u;
        if (slot == 0u) blk = philox(n >> 2, c1, c2, c3, k0, k1);
        ++n;
        return slot == 0u ? blk.w0 : slot == 1u ? blk.w1 : slot == 2u ? blk.w2 : blk.w3;
    }
};

// ---------------------------------------------------------------------------
// Sampling a world the searching player cannot tell from the real one.
// Per opponent (seat order from the mover's left), per run of hidden slots
// between revealed tiles (lo, hi): right to left the largest value each slot
// may take (largest available tile of its colour below the next bound), then
// left to right a uniform value in (previous, bound].  Available: not in the
// mover's row, not revealed, not yet used.  Returns false if a run cannot be
// filled.
// ---------------------------------------------------------------------------
__device__ bool det_attempt(const State &R, uint32_t attempt, uint32_t iter, uint32_t tr,
                            uint32_t k0, uint32_t k1, State &out, const uint8_t *tab)
{
    SeqWords ws{k0, k1, 0x80000000u + attempt, iter, tr, 0u, Words{0u, 0u, 0u, 0u}};
    uint32_t avail = ~(hand_of(R, R.m) | R.rev) & kAll;
    out = R;
    for (uint32_t k = 1; k < 4u; ++k) {
        if (k >= R.P) break;
        const uint32_t o = R.m + k >= R.P ? R.m + k - R.P : R.m + k;
        const uint32_t row = hand_of(R, o);
        const uint32_t revrow = row & R.rev;
        uint32_t rem = row & ~R.rev;
        uint32_t newrow = revrow;
        while (rem) {
            const uint32_t t0 = (uint32_t)__builtin_ctz(rem);
            const uint32_t below = revrow & ((1u << t0) - 1u);
            const uint32_t above = revrow & ~((2u << t0) - 1u);
            const int32_t lo = below ? 31 - __builtin_clz(below) : -1;
            const uint32_t hi = above ? (uint32_t)__builtin_ctz(above) : 24u;
            const uint32_t seg = rem & above_bits(lo) & below_bits(hi);
            rem &= ~seg;
            // right to left: bounds
            uint32_t bounds = 0u, cur = hi, x = seg;
            while (x) {
                const uint32_t tj = 31u - (uint32_t)__builtin_clz(x);
                x &= ~(1u << tj);
                const uint32_t cand = avail & colour_mask(tj) & below_bits(cur);
                if (!cand) return false;
                cur = 31u - (uint32_t)__builtin_clz(cand);
                bounds |= 1u << cur;
            }
            if ((int32_t)cur <= lo) return false;
            // left to right: values
            int32_t prev = lo;
            x = seg;
            uint32_t bb = bounds;
            while (x) {
                const uint32_t tj = (uint32_t)__builtin_ctz(x);
                x &= x - 1u;
                const uint32_t uj = (uint32_t)__builtin_ctz(bb);
                bb &= bb - 1u;
                const uint32_t cand = avail & colour_mask(tj) & above_bits(prev) & below_bits(uj + 1u);
                const uint32_t v = kth_bit_tab(cand, pick(ws.next(), (uint32_t)__popc(cand)), tab);
                avail &= ~(1u << v);
                newrow |= 1u << v;
                prev = (int32_t)v;
            }
        }
        set_hand(out, o, newrow);
    }
    return true;
}

// Deterministic fallback: the lexicographically smallest consistent world
// (slots ordered by opponent from the mover's left, then left to right),
// by depth-first search trying the lowest tile first.  Gives up (false)
// after kDfsMaxCalls search calls.  Runs in one lane; its per-slot arrays
// live in LDS (`sl`), so the kernel needs no scratch memory.
struct DfsSlots {
    uint8_t o[24], col[24], hi[24], seg[24];
    int8_t lo[24], assign[24], tried[24];
};

__device__ bool det_fallback(const State &R, State &out, DfsSlots &sl)
{
    uint32_t ns = 0;
    for (uint32_t k = 1; k < 4u; ++k) {
        if (k >= R.P) break;
        const uint32_t o = R.m + k >= R.P ? R.m + k - R.P : R.m + k;
        const uint32_t row = hand_of(R, o);
        const uint32_t revrow = row & R.rev;
        uint32_t rem = row & ~R.rev;
        bool first = true;
        int32_t last_lo = -2;
        while (rem) {
            const uint32_t t0 = (uint32_t)__builtin_ctz(rem);
            rem &= rem - 1u;
            const uint32_t below = revrow & ((1u << t0) - 1u);
            const uint32_t above = revrow & ~((2u << t0) - 1u);
            const int32_t lo = below ? 31 - __builtin_clz(below) : -1;
            sl.o[ns] = (uint8_t)o;
            sl.col[ns] = (uint8_t)(t0 & 1u);
            sl.lo[ns] = (int8_t)lo;
            sl.hi[ns] = (uint8_t)(above ? (uint32_t)__builtin_ctz(above) : 24u);
            sl.seg[ns] = (uint8_t)(first || lo != last_lo);
            first = false;
            last_lo = lo;
            ++ns;
        }
    }
    uint32_t avail = ~(hand_of(R, R.m) | R.rev) & kAll;
    int32_t k = 0;
    uint32_t calls = 1;
    if (ns > 0) sl.tried[0] = -1;
    while (k < (int32_t)ns) {
        const int32_t prev = sl.seg[k] ? sl.lo[k] : sl.assign[k - 1];
        const int32_t from = sl.tried[k] < 0 ? prev + 1 : sl.tried[k] + 1;
        const uint32_t cand = avail & (sl.col[k] ? kWhite : kBlack) & below_bits(sl.hi[k]) &
                              ~((1u << (uint32_t)from) - 1u);
        if (cand) {
            const uint32_t x = (uint32_t)__builtin_ctz(cand);
            sl.tried[k] = (int8_t)x;
            sl.assign[k] = (int8_t)x;
            avail &= ~(1u << x);
            ++k;
            if (++calls > kDfsMaxCalls) return false;
            if (k < (int32_t)ns) sl.tried[k] = -1;
        } else {
            sl.tried[k] = -1;
            --k;
            if (k < 0) return false;
            avail |= 1u << (uint32_t)sl.assign[k];
        }
    }
    out = R;
    out.h0 &= R.rev;
    out.h1 &= R.rev;
    out.h2 &= R.rev;
    out.h3 &= R.rev;
    add_to_hand(out, R.m, hand_of(R, R.m));
    for (uint32_t j = 0; j < ns; ++j) add_to_hand(out, sl.o[j], 1u << (uint32_t)sl.assign[j]);
    return true;
}

// Legal guessed values (12-bit mask over v) of pair k = (r-1)*24 + s for the
// mover of S: target seat (m + r) mod P still in, slot s exists and is
// hidden, value 2v + colour is a consistent candidate.
// Straight-line code: every lane computes the candidate mask (the k-th-bit
// lookup stays inside the table for any slot) and the conditions select it.
__device__ __forceinline__ uint32_t legal_values(const State &S, uint32_t k, const uint8_t *tab)
{
    const uint32_t r = k / 24u + 1u, slot = k - (k / 24u) * 24u;
    const uint32_t q = S.m + r >= S.P ? S.m + r - S.P : S.m + r;
    const uint32_t row = hand_of(S, q);
    const uint32_t t = kth_bit_tab(row, slot, tab);
    const bool ok = (r < S.P) & ((row & ~S.rev) != 0u) & (slot < (uint32_t)__popc(row)) &
                    !((S.rev >> t) & 1u);
    uint32_t x = candidates(t, row, hand_of(S, S.m), S.rev) >> (t & 1u);
    x &= 0x555555u;
    x = (x | (x >> 1)) & 0x333333u;
    x = (x | (x >> 2)) & 0x0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return ok ? x & 0xFFFu : 0u;
}

// The k-th lowest set bit of a 24-bit mask m (k < popcount(m)), with m and
// k the same in every lane of the wavefront and every lane active: lane j <
// 24 holds bit j and counts the set bits below it, one ballot finds the
// lane.  The descent's state is the same in every lane, so its moves use
// this instead of the per-lane table.  0 when m has no k-th bit.
__device__ __forceinline__ uint32_t kth_bit_wave(uint32_t m, uint32_t k)
{
    // lanes 32-63 repeat lanes 0-31 and only the low half of the ballot is
    // read; bitwise, not short-circuit, conditions keep it branch-free
    const uint32_t l = threadIdx.x & 31u;
    const bool hit = (((m >> l) & 1u) != 0u) & (__builtin_amdgcn_mbcnt_lo(m, 0u) == k);
    const uint32_t b = (uint32_t)__ballot(hit);
    return b ? (uint32_t)__builtin_ctz(b) : 0u;
}

// a uniformly drawn set bit of m (word w), as kth_bit_wave
__device__ __forceinline__ uint32_t pick_bit_wave(uint32_t m, uint32_t w)
{
    return kth_bit_wave(m, pick(w, (uint32_t)__popc(m)));
}

// The turn passes: the next seat with hidden tiles becomes the mover and
// draws with word w1 (if the pool is not empty).  Wave-uniform state.
__device__ __forceinline__ void end_turn(State &S, uint32_t alive, uint32_t w1)
{
    S.m = next_alive(alive, S.m, S.P);
    S.phase = 1u;
    S.drawn = -1;
    const uint32_t pool = ~(S.h0 | S.h1 | S.h2 | S.h3) & kAll;
    if (pool) {
        const uint32_t d = pick_bit_wave(pool, w1);
        add_to_hand(S, S.m, 1u << d);
        S.drawn = (int32_t)d;
    }
}

// The chance words of the in-tree guesses of one iteration: lane d holds
// block (d, 0xC0000000, iter, tree), the words of the guess at depth d
// (a descent is at most 64 levels deep); chance_at reads depth d's block.
__device__ __forceinline__ Words chance_at(const Words &cw, uint32_t depth)
{
    Words w;
    w.w0 = __builtin_amdgcn_readlane(cw.w0, depth);
    w.w1 = __builtin_amdgcn_readlane(cw.w1, depth);
    w.w2 = 0u;
    w.w3 = __builtin_amdgcn_readlane(cw.w3, depth);
    return w;
}

// Play tree key `key` -- a guess, the stop (kStopKey), or a guess after a
// right guess (kStopKey + 1 + action) -- with the chance words w of block
// (depth, 0xC0000000, iter, tree): w0 picks the mover's own tile to reveal
// after a wrong guess with nothing drawn, w1 the next player's draw.  A right
// guess ends the turn unless cont_mode is set; then `cont` is set and the
// mover, still holding the drawn tile hidden, decides again.  Returns true
// if the game ended.
__device__ __forceinline__ bool apply_action(State &S, uint32_t key, bool cont_mode, const Words &w,
                                             uint32_t &winner, bool &cont)
{
    cont = false;
    if (key == kStopKey) {
        end_turn(S, alive_mask(S), w.w1);
        return false;
    }
    const uint32_t action = key > kStopKey ? key - kStopKey - 1u : key;
    const uint32_t r = action / 288u + 1u;
    const uint32_t slot = (action / 12u) % 24u;
    const uint32_t v = action % 12u;
    const uint32_t q = S.m + r >= S.P ? S.m + r - S.P : S.m + r;
    const uint32_t row = hand_of(S, q);
    const uint32_t t = kth_bit_wave(row, slot);
    const bool right = 2u * v + (t & 1u) == t;
    const uint32_t hm = hand_of(S, S.m);
    const uint32_t own = pick_bit_wave(hm & ~S.rev, w.w0);
    const uint32_t wrong_bit = 1u << (S.drawn >= 0 ? (uint32_t)S.drawn : own);
    S.rev |= right ? (1u << t) : wrong_bit;
    const uint32_t alive = alive_mask(S);
    if (__popc(alive) == 1) {
        S.phase = 1u;
        S.drawn = -1;
        winner = (uint32_t)__builtin_ctz(alive);
        return true;
    }
    if (right && cont_mode) {
        cont = true;
        return false;
    }
    end_turn(S, alive, w.w1);
    return false;
}

// A leaf reached right after a right guess (continue choice): the random
// policy's continue coin, w3 of that guess's chance block w, decides once for
// all the leaf's playouts -- below 2^31 the mover goes on guessing, else the
// turn passes (w1 draws).
__device__ __forceinline__ void leaf_continue_coin(State &S, const Words &w)
{
    if (w.w3 >= 0x80000000u) end_turn(S, alive_mask(S), w.w1);
}

// The sampled world as a 48-bit key (lo: tiles 0-15, hi: tiles 16-23), 2 bits
// per tile: the seat relative to the root mover m of the opponent holding the
// tile hidden, else 0.
__device__ __forceinline__ void world_key(const State &S, uint32_t m, uint32_t &lo, uint32_t &hi)
{
    uint64_t key = 0u;
    for (uint32_t k = 1; k < 4u; ++k) {
        if (k >= S.P) break;
        const uint32_t o = m + k >= S.P ? m + k - S.P : m + k;
        uint32_t x = hand_of(S, o) & ~S.rev;
        while (x) {
            const uint32_t t = (uint32_t)__builtin_ctz(x);
            x &= x - 1u;
            key |= (uint64_t)k << (2u * t);
        }
    }
    lo = (uint32_t)key;
    hi = (uint32_t)(key >> 32);
}

// v itself, in a vector register: the compiler keeps values computed from it
// there as well, out of the scarce scalar registers
__device__ __forceinline__ uint32_t in_vgpr(uint32_t v)
{
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// greater of two scores (no NaN arises: every visited child has N >= 1)
__device__ __forceinline__ float score_max(float a, float b) { return a > b ? a : b; }

template <int CTRL>
__device__ __forceinline__ float dpp_f(float s)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s), CTRL, 0xF, 0xF, false));
}

// Wavefront arg-max of scores whose index is base + lane: the greatest score
// (every lane gets it) and the lowest lane holding it, which is the lowest
// index on ties; lane -1 when every score is -inf (nothing playable).  The
// maximum is reduced within each 16-lane row by lane exchanges (lane ^ 1,
// lane ^ 2, then the mirror images within 8 and within 16 lanes), then over
// the four rows' maxima; the lane is the lowest set bit of the ballot of
// lanes equal to it.  All 64 lanes must be active.
__device__ __forceinline__ int wave_argmax_lane(float s, float &best)
{
    float m = s;
    m = score_max(m, dpp_f<0xB1>(m));    // quad_perm [1, 0, 3, 2]
    m = score_max(m, dpp_f<0x4E>(m));    // quad_perm [2, 3, 0, 1]
    m = score_max(m, dpp_f<0x141>(m));   // row_half_mirror
    m = score_max(m, dpp_f<0x140>(m));   // row_mirror
    const float r0 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(m), 0));
    const float r1 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(m), 16));
    const float r2 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(m), 32));
    const float r3 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(m), 48));
    best = score_max(score_max(r0, r1), score_max(r2, r3));
    const uint64_t hit = __ballot(s == best);
    return best == -__builtin_inff() ? -1 : (int)__builtin_ctzll(hit);
}

__device__ __forceinline__ void wave_argmax_u(uint32_t &n, uint32_t &idx)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t on = __shfl_xor(n, off, 64);
        const uint32_t oi = __shfl_xor(idx, off, 64);
        const bool take = on > n || (on == n && oi < idx);
        n = take ? on : n;
        idx = take ? oi : idx;
    }
}

struct MctsArgs {
    const uint4 *roots;
    uint32_t n_trees, trees_per_root, iters, ppl, dmax;   // tree t searches root t / trees_per_root
    float c_uct;
    uint32_t k0, k1, tree_base;
    const float *ln;
    uint32_t *ws;
    MctsShape sh;
    uint32_t cont_mode, vanilla;   // simplifications 2 and 1 switched off
    uint32_t lpp;                  // leaves per pass
    uint32_t pipe;                 // pipelined passes: wins credited one pass late
    int32_t *best;    // [n_trees] or null
    uint32_t *kids;   // [n_trees][864][3] or null
    // value mode: leaves are scored by the network; a leaf whose value for
    // the root player is within `band` of 1/2 is played out instead
    uint32_t leaf_eval, fb_ppl;
    float band;
    const void *net;
};

__device__ __forceinline__ void write_no_children(const MctsArgs &a, uint32_t t, uint32_t lane)
{
    if (!a.kids) return;
    uint32_t *k = a.kids + (size_t)t * kMaxActions * 3u;
    for (uint32_t c = lane; c < kMaxActions; c += 64u) {
        k[c * 3u + 0u] = 0xFFFFu;
        k[c * 3u + 1u] = 0u;
        k[c * 3u + 2u] = 0u;
    }
}

// Orders one tree's memory accesses between its lanes.  A tree is one
// wavefront; in the value-mode kernel four trees share a workgroup (and its
// LDS copy of the second-layer weights) but never wait for each other, so
// their orderings are fences plus a wavefront barrier, not workgroup barriers.
template <bool SHARED_GROUP>
__device__ __forceinline__ void tree_sync()
{
    if (SHARED_GROUP) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Trees per workgroup: value mode stages the 256 x 256 second-layer weights
// in LDS once per workgroup for its four trees; playout mode runs one tree per
// workgroup.  Pipelined passes (PIPE): one tree per workgroup of two
// wavefronts, one descending pass k + 1 while the other evaluates pass k,
// with two pass buffers used in turn.
template <bool VALUE, bool PIPE> struct TreeGroup {
    static constexpr uint32_t kTrees = PIPE ? 1u : (VALUE ? 4u : 1u);
    static constexpr uint32_t kWaves = PIPE ? 2u : kTrees;
    // leaves evaluated together: value mode puts their perspectives into the
    // 16 rows of one matrix tile, four per leaf
    static constexpr uint32_t kPass = VALUE ? 4u : 16u;
    static constexpr uint32_t kBufs = PIPE ? 2u : 1u;
};

// VALUE: value mode (network leaves) -- one wavefront per SIMD, so that the
// evaluation can keep many weight loads in flight; otherwise playout leaves
// only.  PIPE: pipelined passes, wavefront 0 of the workgroup samples,
// descends and backs up, wavefront 1 evaluates.
template <bool VALUE, bool PIPE>
__global__ void __launch_bounds__((64 * TreeGroup<VALUE, PIPE>::kWaves))
__attribute__((amdgpu_waves_per_eu(VALUE ? (PIPE ? 2 : 1) : 4, VALUE ? (PIPE ? 2 : 1) : 8)))
mcts_tree_kernel(MctsArgs a)
{
    constexpr uint32_t TG = TreeGroup<VALUE, PIPE>::kTrees;
    constexpr uint32_t NBUF = TreeGroup<VALUE, PIPE>::kBufs;
    // a tree's wavefront orders its own memory accesses with wavefront
    // barriers when it shares the workgroup with other wavefronts
    constexpr bool WS = VALUE || PIPE;
    // pipelined passes with network leaves: the evaluating wavefront, which
    // has time to spare, also samples the worlds (with playout leaves it has
    // none)
    constexpr bool ESAMPLE = PIPE && VALUE;
    __shared__ uint8_t tab[kKthTableBytes];
    __shared__ uint32_t legal_all[TG][73];
    __shared__ uint32_t legal_root_all[TG][73];   // the root's, the same in every world
    __shared__ uint4 rcache_all[TG][2 * kBlockEntries];   // the root's first two child blocks
    constexpr uint32_t BM = TreeGroup<VALUE, PIPE>::kPass;
    __shared__ uint32_t path_all[TG][NBUF][BM][kMaxPath];
    __shared__ uint4 leaf_all[TG][NBUF][BM];
    __shared__ uint32_t np_all[TG][NBUF][BM];
    __shared__ uint32_t meta_all[TG][NBUF][2];   // a pass's decided leaves, their winners
    __shared__ uint32_t wins_all[TG][4u * BM];
    __shared__ float vals_all[TG][NBUF][BM][4];
    __shared__ DfsSlots dfs_all[TG];
    __shared__ uint4 fb_rows[TG];   // rows of the sampler's fallback world
    __shared__ uint8_t fslot_all[TG][64];   // the sampler's iterations left in a round
    __shared__ uint4 wres_all[TG][64];      // and their worlds found in the round
    // worlds of a pass sampled by the evaluating wavefront (rows; flag 1:
    // the sampler gave up)
    __shared__ uint4 wrows_all[ESAMPLE ? 2 : 1][ESAMPLE ? BM : 1];
    __shared__ uint32_t wflag_all[ESAMPLE ? 2 : 1][ESAMPLE ? BM : 1];
    __shared__ __attribute__((aligned(16))) uint16_t w2_lds[(VALUE && !PIPE) ? kVnH * kVnH : 8];
    __shared__ __attribute__((aligned(16))) uint16_t hs_pipe[(VALUE && PIPE) ? 16 : 1][kVnH + 8];
    __shared__ VnSmall vn_small[1];
    // pipelined passes: [0] the step + 1 at which the descending wavefront
    // gave up (0: it did not); [1..7] the evaluating wavefront's statistics:
    // network / played-out leaves, evaluation cycles, sampler fallbacks,
    // sampling cycles
    __shared__ uint32_t pipe_x[8];
    fill_kth_table(tab);
    if (VALUE) {
        vn_stage_small(vn_ptrs(const_cast<void *>(a.net)), vn_small[0]);
        // second-layer weights (bf16) as A operands of the transposed product
        if (!PIPE) vn_stage_w2t(vn_ptrs(const_cast<void *>(a.net)), w2_lds);
    }
    if (threadIdx.x == 0) pipe_x[0] = 0u;
    __syncthreads();   // the only workgroup barrier outside pipelined passes
    const uint32_t wv = TG == 1u ? 0u : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // pipelined passes: 0 samples, descends and backs up, 1 evaluates
    const uint32_t role = PIPE ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0u;
    const uint32_t t = blockIdx.x * TG + wv;
    if (t >= a.n_trees) return;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t *legal_s = legal_all[wv];
    DfsSlots &dfs_slots = dfs_all[wv];
    const uint32_t tr = a.tree_base + t;
    uint32_t *W = a.ws + (uint64_t)t * a.sh.tree_words;
    const uint32_t nodes_cap = a.sh.nodes_cap, node_words = a.sh.node_words;
    const uint32_t node_stride = a.sh.node_stride;
    const uint32_t ovf_base = kTreeHeaderWords + nodes_cap * node_stride;
    uint32_t *bnext = W + ovf_base + a.sh.ovf_cap * kBlockWords;
    // word offset (from W) of child block b: blocks below nodes_cap are the
    // nodes' inline blocks, the rest overflow blocks
    auto block_off = [&](uint32_t b) __attribute__((always_inline)) -> uint32_t {
        return b < nodes_cap ? kTreeHeaderWords + b * node_stride + node_words
                             : ovf_base + (b - nodes_cap) * kBlockWords;
    };
    auto rec_off = [&](uint32_t nd) __attribute__((always_inline)) -> uint32_t { return kTreeHeaderWords + nd * node_stride; };

    const uint4 rs = a.roots[t / a.trees_per_root];
    State R;
    const bool ok = decode(rs.x, rs.y, rs.z, rs.w, R);
    const uint32_t pool0 = ~(R.h0 | R.h1 | R.h2 | R.h3) & kAll;
    if (!ok || __popc(alive_mask(R)) < 2 || (R.phase == 0u && pool0 != 0u)) {
        if (role != 0u) return;   // both wavefronts of a pipelined tree leave here
        if (lane == 0) {
            atomicOr(&g_error_word, kErrState);
            if (a.best) a.best[t] = -1;
        }
        if (lane < kTreeHeaderWords) W[lane] = lane == kHdrFailed ? 1u : 0u;
        write_no_children(a, t, lane);
        return;
    }
    if (role == 0u) {
        for (uint32_t k = lane; k < node_words; k += 64u) W[rec_off(0u) + k] = 0u;
        if (lane == 0) bnext[0] = kNoBlock;
    }
    uint32_t n_nodes = 1u, n_ovf = 0u, n_root = 0u;
    uint32_t n_net = 0u, n_played = 0u, n_sampler_fallback = 0u, deepest = 0u;   // statistics
    bool failed = false, have_fallback = false;
    uint64_t cyc[4] = {0u, 0u, 0u, 0u};   // shader clock per phase (statistics)
    // with network leaves the statistics stay in vector registers, out of
    // the scalar ones, which the network's evaluation also needs (measured
    // faster); the playout kernels keep them scalar (in vector registers they
    // pushed the sequential kernel past 128 registers, into scratch)
    auto cyc_add = [&](uint32_t k, uint64_t d) __attribute__((always_inline)) {
        const uint64_t v = cyc[k] + d;
        cyc[k] = VALUE ? (uint64_t)in_vgpr((uint32_t)v) | ((uint64_t)in_vgpr((uint32_t)(v >> 32)) << 32)
                       : v;
    };
    // Worlds of iterations ib .. ib + 63, sampled together (lane l: iteration
    // ib + l) at every 64th iteration: the world's rows as owner bit-planes,
    // and the lanes whose iteration has a world (the others take the
    // fallback world).
    uint32_t wpl0 = 0u, wpl1 = 0u, wpl2 = 0u;
    uint64_t wok = 0u;
    // The root's first two child blocks (in LDS), its guess bitmap words
    // (laid out as the descent loads them), child count and next two block
    // ids (in registers), kept on chip: the wavefront that owns the tree
    // makes every change to them, to memory and here at the same points, so
    // the root level of a descent issues no global loads.  Not for vanilla
    // trees, whose root children are worlds.
    const bool rc_on = !a.vanilla;
    // The root's legal guesses, the same in every sampled world: a guess
    // names an opponent's row slot and a value; which slots are hidden, their
    // colours, the revealed tiles around them and the mover's own tiles are
    // what the searching player sees, and the sampler keeps them all.
    // Kept in LDS (registers are scarce across the playouts).
    uint32_t *legal_root = legal_root_all[wv];
    if (role == 0u) {   // the wavefront that descends
        legal_root[lane] = legal_values(R, lane, tab);
        uint32_t l1 = 0u;
        if (__builtin_amdgcn_readfirstlane(
                (uint32_t)(R.P == 4u && __popc(hand_of(R, (R.m + 3u) & 3u)) > 16)) != 0u &&
            lane < 8u)
            l1 = legal_values(R, 64u + lane, tab);
        if (lane < 9u) legal_root[64u + lane] = l1;   // [72]: no stop at the root
    }
    // (the 128 entries in LDS, the rest in registers)
    uint4 *rc_ent = rcache_all[wv];
    if (role == 0u) {
        rc_ent[lane] = make_uint4(0u, 0u, 0u, 0u);
        rc_ent[kBlockEntries + lane] = make_uint4(0u, 0u, 0u, 0u);
    }
    uint32_t rc_cb0 = 0u, rc_cb1 = 0u, rc_nc = 0u, rc_nx0 = kNoBlock, rc_nx1 = kNoBlock;
    // root child slot (0 .. 127, else not cached) of the entry at word offset e
    auto rc_slot = [&](uint32_t e) __attribute__((always_inline)) -> uint32_t {
        const uint32_t b0 = block_off(0u);
        if (e - b0 < kBlockWords) return (e - b0) / kEntryWords;
        if (rc_nx0 != kNoBlock && e - block_off(rc_nx0) < kBlockWords)
            return kBlockEntries + (e - block_off(rc_nx0)) / kEntryWords;
        return 0xFFFFFFFFu;
    };
    // visits dn for cached slot `slot`; its W word set to wbits when set_w
    auto rc_update = [&](uint32_t slot, uint32_t dn, bool set_w, uint32_t wbits) __attribute__((always_inline)) {
        if (slot < 2u * kBlockEntries && lane == 0u) {
            uint4 &en = rc_ent[slot];
            en.y += dn;
            if (set_w) en.z = wbits;
        }
    };
    tree_sync<WS>();

    // Iterations run in passes of B = leaves_per_pass: each descent of a pass
    // adds its visit counts along its path at once (the next descent sees
    // them, with no wins yet); then the pass's leaves are evaluated together
    // -- their playouts packed into the same 64 lanes, or their perspectives
    // into the rows of one matrix tile -- and each path gets its wins, in
    // iteration order.  B = 1 is the plain sequential search.
    const uint32_t nplay = VALUE ? a.fb_ppl : a.ppl;   // visits of every leaf
    // ---- 1. sample the world of iteration `it`: its lowest successful
    // attempt, else the fallback world.  The worlds of iterations ib .. ib +
    // 63 are sampled together at every 64th iteration: attempt 0 of each in
    // its own lane, then rounds in which the iterations still without a world
    // try attempts a0 .. a0 + K - 1 side by side, 64 / K iterations per pass,
    // for K = 4, 8, 16, 32 and the last 3 (attempts 1 .. 63 in five rounds).
    // Every iteration keeps its lowest successful attempt.  Returns false
    // when the fallback search gives up.
    auto sample_world = [&](uint32_t it, State &S) __attribute__((always_inline)) -> bool {
        if ((it & 63u) == 0u) {
            State Sw;
            const bool valid = it + lane < a.iters;
            const bool got0 = det_attempt(R, 0u, it + lane, tr, a.k0, a.k1, Sw, tab);
            wok = __ballot(got0 || !valid);   // lanes past the last iteration count as done
            wpl0 = Sw.h0 | Sw.h2;
            wpl1 = Sw.h1 | Sw.h2;
            wpl2 = Sw.h3;
            // round K: attempts K - 3 .. K - 3 + Kr - 1 (Kr = K, or 3 for the last)
            uint8_t *fslot = fslot_all[wv];   // slot n: the lane of the n-th iteration left
            uint4 *wres = wres_all[wv];       // lane l's world from this round (w = 1: found)
            for (uint32_t K = 4u; K <= 64u; K *= 2u) {
                const uint64_t left = ~wok;
                if (left == 0ull) break;
                const uint32_t Kr = K == 64u ? 3u : K;
                tree_sync<WS>();   // the previous round has read its slots and worlds
                if ((left >> lane) & 1ull)
                    fslot[__builtin_amdgcn_mbcnt_hi((uint32_t)(left >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)left, 0u))] =
                        (uint8_t)lane;
                wres[lane].w = 0u;
                tree_sync<WS>();
                const uint32_t nl = (uint32_t)__popcll(left), G = 64u / Kr;
                const uint32_t g = lane / Kr, r = lane - g * Kr;
                for (uint32_t p0 = 0; p0 < nl; p0 += G) {
                    const bool act = g < G && p0 + g < nl;
                    const uint32_t fl = act ? fslot[p0 + g] : 0u;
                    State Sa;
                    const bool got = act && det_attempt(R, K - 3u + r, it + fl, tr, a.k0, a.k1, Sa,
                                                        tab);
                    const uint64_t gotm = __ballot(got);
                    // the group's lowest successful attempt hands its world to the iteration
                    const uint64_t below = (gotm >> (act ? g * Kr : 0u)) & ((1ull << r) - 1ull);
                    if (got && below == 0ull)
                        wres[fl] = make_uint4(Sa.h0 | Sa.h2, Sa.h1 | Sa.h2, Sa.h3, 1u);
                }
                tree_sync<WS>();
                const uint4 wr = wres[lane];
                if (wr.w != 0u) {
                    wpl0 = wr.x;
                    wpl1 = wr.y;
                    wpl2 = wr.z;
                }
                wok |= __ballot(wr.w != 0u);
            }
        }
        const uint32_t wl = it & 63u;
        if ((wok >> wl) & 1u) {
            S = R;
            const uint32_t p0 = __builtin_amdgcn_readlane(wpl0, wl);
            const uint32_t p1 = __builtin_amdgcn_readlane(wpl1, wl);
            const uint32_t p2 = __builtin_amdgcn_readlane(wpl2, wl);
            S.h0 = p0 & ~p1 & ~p2;
            S.h1 = ~p0 & p1 & ~p2 & kAll;
            S.h2 = p0 & p1 & ~p2;
            S.h3 = p2;
            return true;
        }
        // the fallback world depends on the root only: search it once (it
        // differs from the root in its rows only; they are kept in LDS)
        if (!have_fallback) {
            State F = R;
            bool fok = false;
            if (lane == 0) fok = det_fallback(R, F, dfs_slots);
            fok = __builtin_amdgcn_readfirstlane((uint32_t)fok) != 0u;
            if (!fok) {
                if (lane == 0) atomicOr(&g_error_word, kErrLimit);
                return false;
            }
            if (lane == 0) fb_rows[wv] = make_uint4(F.h0, F.h1, F.h2, F.h3);
            have_fallback = true;
            tree_sync<WS>();
        }
        const uint4 fr = fb_rows[wv];
        S = R;
        S.h0 = __builtin_amdgcn_readfirstlane(fr.x);
        S.h1 = __builtin_amdgcn_readfirstlane(fr.y);
        S.h2 = __builtin_amdgcn_readfirstlane(fr.z);
        S.h3 = __builtin_amdgcn_readfirstlane(fr.w);
        ++n_sampler_fallback;
        return true;
    };
    // ---- 3. evaluate a pass's leaves (pass buffer buf, iterations i0 ..
    // i0 + nb - 1): playouts packed into the 64 lanes, or network rows; the
    // decided leaves get their winner's share.  Results in vals_all[wv][buf].
    auto eval_pass = [&](uint32_t buf, uint32_t i0, uint32_t nb, uint32_t term_mask,
                     uint32_t winners) __attribute__((always_inline)) {
        uint32_t play_mask = ((1u << nb) - 1u) & ~term_mask;   // leaves to play out
        if (VALUE && play_mask) {
            // rows 4b + q: leaf b, seat perspective q < P
            const uint32_t r = lane & 15u, lb = r >> 2, q = r & 3u;
            RowFeat rf = no_row();
            if (lb < nb && ((play_mask >> lb) & 1u)) {
                const uint4 ps = leaf_all[wv][buf][lb];
                if (q < ((ps.x >> 26) & 3u) + 1u) rf = row_features(ps, q);
            }
            // the value of row 4b + k: lane 4b + k of vrow (transposed
            // products), or v4[k] of lane group b (the wavefront's own tile)
            float vrow = 0.0f, v4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (PIPE)
                vn_eval16_wave(vn_ptrs(const_cast<void *>(a.net)), rf, hs_pipe, vn_small[0], v4);
            else
                vrow = vn_eval_tree_t(vn_ptrs(const_cast<void *>(a.net)), rf, w2_lds, vn_small[0]);
#pragma unroll
            for (uint32_t b = 0; b < BM; ++b) {
                if (!((play_mask >> b) & 1u)) continue;
                float v[4];
#pragma unroll
                for (uint32_t k = 0; k < 4u; ++k)
                    v[k] = __uint_as_float(__builtin_amdgcn_readlane(
                        __float_as_uint(PIPE ? v4[k] : vrow), PIPE ? 16u * b : 4u * b + k));
                const float vm = R.m == 0u ? v[0] : R.m == 1u ? v[1] : R.m == 2u ? v[2] : v[3];
                const float dv = vm - 0.5f;
                if (!((dv < 0.0f ? -dv : dv) < a.band)) {
                    play_mask &= ~(1u << b);
                    ++n_net;
                    if (lane == 0)
#pragma unroll
                        for (uint32_t k = 0; k < 4u; ++k) vals_all[wv][buf][b][k] = (float)a.fb_ppl * v[k];
                }
            }
        }
        // playouts of the leaves in play_mask, packed: playout g of the pass
        // is playout g % nplay of leaf g / nplay
        if (play_mask) {
            if (lane < 4u * BM) wins_all[wv][lane] = 0u;
            tree_sync<WS>();
            const uint32_t trk1 = tr ^ a.k1;
            for (uint32_t pb = 0; pb < nb * nplay; pb += 64u) {
                const uint32_t gp = pb + lane;
                const uint32_t lb = gp / nplay;
                const bool act = lb < nb && ((play_mask >> lb) & 1u);
                const uint32_t b_lo = pb / nplay;
                const uint32_t b_hi = (pb + 63u) / nplay < nb - 1u ? (pb + 63u) / nplay : nb - 1u;
                if (!((play_mask >> b_lo) & ((2u << (b_hi - b_lo)) - 1u))) continue;
                uint32_t w = 4u;
                if (act) {
                    const uint4 ps = leaf_all[wv][buf][lb];
                    State s;
                    decode(ps.x, ps.y, ps.z, ps.w, s);
                    const uint32_t p = gp - lb * nplay;
                    const uint64_t pl = (uint64_t)(i0 + lb) * kPhiloxM1;
                    PlayoutKey pk;
                    pk.a = (uint32_t)(pl >> 32) ^ p ^ a.k0;
                    pk.b = (uint32_t)pl;
                    pk.gm_lo = 0u;
                    pk.gm_hi = 0u;
                    bool over = false;
                    uint32_t len = 0u;
                    // the words of step g+1 do not depend on the game, so
                    // they are computed while step g runs (one wavefront per
                    // tree has no other wavefront to hide latencies behind)
                    Words wd = step_words(pk, trk1, a.k0, a.k1);
                    next_step(pk);
                    while (!over) {
                        const Words wn = step_words(pk, trk1, a.k0, a.k1);
                        next_step(pk);
                        over = guess_step(s, wd, w, tab);
                        wd = wn;
                        if (++len >= kMaxGuesses && !over) {
                            atomicOr(&g_error_word, kErrLimit);
                            over = true;
                            w = 4u;
                        }
                    }
                }
                // seat wins of every leaf in this chunk
                for (uint32_t b = b_lo; b <= b_hi; ++b) {
                    const bool mine = act && lb == b;
                    const uint32_t c0 = (uint32_t)__popcll(__ballot(mine && w == 0u));
                    const uint32_t c1 = (uint32_t)__popcll(__ballot(mine && w == 1u));
                    const uint32_t c2 = (uint32_t)__popcll(__ballot(mine && w == 2u));
                    const uint32_t c3 = (uint32_t)__popcll(__ballot(mine && w == 3u));
                    if (lane == 0) {
                        wins_all[wv][4u * b + 0u] += c0;
                        wins_all[wv][4u * b + 1u] += c1;
                        wins_all[wv][4u * b + 2u] += c2;
                        wins_all[wv][4u * b + 3u] += c3;
                    }
                }
            }
            tree_sync<WS>();
            for (uint32_t b = 0; b < nb; ++b) {
                if (!((play_mask >> b) & 1u)) continue;
                if (a.leaf_eval) ++n_played;
                if (lane == 0)
#pragma unroll
                    for (uint32_t k = 0; k < 4u; ++k) vals_all[wv][buf][b][k] = (float)wins_all[wv][4u * b + k];
            }
        }
        for (uint32_t b = 0; b < nb; ++b) {
            if (!((term_mask >> b) & 1u)) continue;
            const uint32_t wn = (winners >> (2u * b)) & 3u;
            if (lane == 0)
#pragma unroll
                for (uint32_t k = 0; k < 4u; ++k) vals_all[wv][buf][b][k] = k == wn ? (float)nplay : 0.0f;
        }
        tree_sync<WS>();

    };
    // ---- 4. back-propagation of a pass: each path gets its leaf's wins, in order
    auto backprop_pass = [&](uint32_t buf, uint32_t nb) __attribute__((always_inline)) {
        for (uint32_t b = 0; b < nb; ++b) {
            const uint32_t npb = np_all[wv][buf][b];
            uint32_t e = 0u, nw = 0u;
            if (lane < npb && !(a.vanilla && lane == 0u)) {   // a world node's W word holds its key
                e = path_all[wv][buf][b][lane];
                // the chooser's value by a computed index: a chain of selects
                // over the four LDS entries was compiled into branches that
                // left seat 3's lanes reading seat 2's entry
                const uint4 en = *reinterpret_cast<const uint4 *>(W + e);
                const uint32_t chooser = (en.x >> 16) & 3u;
                const float wc = vals_all[wv][buf][b][chooser];
                nw = __float_as_uint(__uint_as_float(en.z) + wc);
                W[e + 2u] = nw;
            }
            if (rc_on && npb > 0u)   // lane 0 holds the root child's entry
                rc_update(rc_slot(__builtin_amdgcn_readlane(e, 0)), 0u, true,
                          __builtin_amdgcn_readlane(nw, 0));
            tree_sync<WS>();
        }

    };

    // Pipelined passes, the evaluating wavefront: step k evaluates pass
    // k - 1 (and, with network leaves, samples the worlds of pass k + 1)
    // while the other wavefront descends pass k; both then meet at the
    // step's workgroup barrier (after one more barrier before the first
    // step), and the descending wavefront backs up pass k - 1 while this one
    // goes on with step k + 1.  The two run the same number of steps (or
    // both stop at the step where the descending wavefront gave up).
    const uint32_t n_pass = (a.iters + a.lpp - 1u) / a.lpp;
    if (PIPE && role == 1u) {
        // the worlds of pass kp into world buffer kp & 1 (in iteration
        // order); after a world the sampler gave up on, none
        bool gave_up = false;
        auto sample_pass = [&](uint32_t kp) __attribute__((always_inline)) {
            if (!ESAMPLE || kp >= n_pass || gave_up) return;
            const uint32_t ip = kp * a.lpp, nbp = a.iters - ip < a.lpp ? a.iters - ip : a.lpp;
            const uint64_t t0 = clock64();
            for (uint32_t b = 0; b < nbp; ++b) {
                State Sw;
                const bool ok = sample_world(ip + b, Sw);
                if (lane == 0) {
                    wrows_all[kp & 1u][b] = make_uint4(Sw.h0, Sw.h1, Sw.h2, Sw.h3);
                    wflag_all[kp & 1u][b] = ok ? 0u : 1u;
                }
                if (!ok) {
                    gave_up = true;
                    break;
                }
            }
            cyc_add(0u, clock64() - t0);
        };
        sample_pass(0u);
        __syncthreads();   // the first pass's worlds
        for (uint32_t k = 0; k <= n_pass; ++k) {
            if (k >= 1u) {
                const uint32_t ip = (k - 1u) * a.lpp, buf = (k - 1u) & 1u;
                const uint64_t t2 = clock64();
                eval_pass(buf, ip, a.iters - ip < a.lpp ? a.iters - ip : a.lpp,
                          meta_all[wv][buf][0], meta_all[wv][buf][1]);
                cyc_add(2u, clock64() - t2);
            }
            sample_pass(k + 1u);
            __syncthreads();
            if (pipe_x[0] == k + 1u) break;
        }
        if (lane == 0) {
            pipe_x[1] = n_net;
            pipe_x[2] = n_played;
            pipe_x[3] = (uint32_t)cyc[2];
            pipe_x[4] = (uint32_t)(cyc[2] >> 32);
            pipe_x[5] = n_sampler_fallback;
            pipe_x[6] = (uint32_t)cyc[0];
            pipe_x[7] = (uint32_t)(cyc[0] >> 32);
        }
        __syncthreads();
        return;
    }
    if (PIPE) __syncthreads();   // the first pass's worlds
    for (uint32_t k = 0; k < n_pass + (PIPE ? 1u : 0u); ++k) {
        const uint32_t buf = PIPE ? (k & 1u) : 0u;
        const uint32_t i0 = k * a.lpp;
        // pipelined passes end with a step that only backs up the last pass
        const uint32_t nb = k < n_pass ? (a.iters - i0 < a.lpp ? a.iters - i0 : a.lpp) : 0u;
        uint32_t term_mask = 0u, winners = 0u;   // per leaf of the pass: decided, winner (2 bits)
        for (uint32_t b = 0; b < nb; ++b) {
            const uint32_t it = i0 + b;
            uint32_t *path_e = path_all[wv][buf][b];
            const uint64_t t0 = clock64();
            // ---- 1. the iteration's world: sampled here, or (pipelined
            // passes with network leaves) by the other wavefront one step ahead
            State S;
            if (ESAMPLE) {
                const uint4 wr = wrows_all[buf][b];
                if (wflag_all[buf][b] != 0u) {
                    failed = true;
                    break;
                }
                // the same in every lane: scalar registers, scalar branches
                S = R;
                S.h0 = __builtin_amdgcn_readfirstlane(wr.x);
                S.h1 = __builtin_amdgcn_readfirstlane(wr.y);
                S.h2 = __builtin_amdgcn_readfirstlane(wr.z);
                S.h3 = __builtin_amdgcn_readfirstlane(wr.w);
            } else if (!sample_world(it, S)) {
                failed = true;
                break;
            }
            if (!PIPE) {
                // the descent's state in vector registers: held in scalar
                // ones it pushes other scalars out to spill slots (measured
                // slower); the pipelined kernels run faster without this
                S.h0 = in_vgpr(S.h0);
                S.h1 = in_vgpr(S.h1);
                S.h2 = in_vgpr(S.h2);
                S.h3 = in_vgpr(S.h3);
                S.rev = in_vgpr(S.rev);
                S.m = in_vgpr(S.m);
                S.P = in_vgpr(S.P);
                S.phase = in_vgpr(S.phase);
                S.drawn = in_vgpr(S.drawn);
            }
            const uint64_t t1 = clock64();
            cyc_add(0u, t1 - t0);
            // ---- 2. descend ----------------------------------------------------
            const Words cw = philox(lane, 0xC0000000u, it, tr, a.k0, a.k1);
            // Append a child {ex | ..., 0, ez, id} to `parent` (child count nc);
            // returns its id and its entry's word offset.
            auto append_child = [&](uint32_t parent, uint32_t nc, uint32_t ex, uint32_t ez,
                                    uint32_t &e_out) __attribute__((always_inline)) -> uint32_t {
                const uint32_t rec = rec_off(parent);
                const uint32_t c = n_nodes++;
                uint32_t blk = parent;
                if (nc >= kBlockEntries) {
                    blk = W[rec + 1u];
                    if ((nc & (kBlockEntries - 1u)) == 0u) {
                        const uint32_t ob = nodes_cap + n_ovf++;
                        if (lane == 0) {
                            bnext[ob] = kNoBlock;
                            bnext[blk] = ob;
                            W[rec + 1u] = ob;
                        }
                        blk = ob;
                    }
                }
                const uint32_t e = block_off(blk) + (nc & (kBlockEntries - 1u)) * kEntryWords;
                if (lane == 0) {
                    W[e + 0u] = ex;
                    W[e + 1u] = 0u;
                    W[e + 2u] = ez;
                    W[e + 3u] = c;
                    W[rec + 2u] = nc + 1u;
                    bnext[c] = kNoBlock;
                }
                for (uint32_t k = lane; k < node_words; k += 64u) W[rec_off(c) + k] = k == 1u ? c : 0u;
                e_out = e;
                return c;
            };
            uint32_t node = 0u, node_n = n_root, depth = 0u, np = 0u, winner = 0u, last_block = 0u;
            bool term = false, cont = false;
            if (a.vanilla) {
                // the world node of this sample among the root's children, by key
                uint32_t klo, khi;
                world_key(S, R.m, klo, khi);
                const uint32_t nr = W[rec_off(0u) + 2u];
                uint32_t blk = 0u, found_e = 0u;
                bool found = false;
                for (uint32_t base = 0; base < nr; base += kBlockEntries) {
                    const uint32_t eo = block_off(blk) + lane * kEntryWords;
                    const uint4 ent = *reinterpret_cast<const uint4 *>(W + eo);
                    const uint64_t hit = __ballot(base + lane < nr && ent.x == klo && ent.z == khi);
                    if (hit) {
                        const uint32_t l = (uint32_t)__builtin_ctzll(hit);
                        node = __builtin_amdgcn_readlane(ent.w, l);
                        node_n = __builtin_amdgcn_readlane(ent.y, l);
                        found_e = block_off(blk) + l * kEntryWords;
                        found = true;
                        break;
                    }
                    if (base + kBlockEntries < nr) blk = bnext[blk];
                }
                if (!found) {
                    node = append_child(0u, nr, klo, khi, found_e);
                    node_n = 0u;
                }
                path_e[np++] = found_e;
                tree_sync<WS>();
            }
            for (;;) {
                if (term || depth >= a.dmax || np >= kMaxPath - 1u) break;
                // one round of loads: bitmaps, child count, first 64 children, LN
                const uint32_t rec = rec_off(node);
                const uint32_t half = cont ? 36u : 0u;
                // the root (a turn start: no continue choice there) from registers
                const bool at_root = rc_on && node == 0u;
                uint32_t cbw0, cbw1, nchild_v, next0_v;
                uint4 ent0;
                if (at_root) {
                    cbw0 = rc_cb0;
                    cbw1 = rc_cb1;
                    nchild_v = rc_nc;
                    ent0 = rc_ent[lane];
                    next0_v = rc_nx0;
                } else {
                    cbw0 = W[rec + 4u + half + (lane >> 1)];
                    cbw1 = lane < 8u ? W[rec + 36u + half + (lane >> 1)] : lane == 8u ? W[rec + 3u] : 0u;
                    nchild_v = W[rec + 2u];
                    ent0 = *reinterpret_cast<const uint4 *>(W + rec + node_words + lane * kEntryWords);
                    next0_v = bnext[node];   // the second child block, if any
                }
                const float lp = a.ln[node_n];
                uint32_t l0, l1;
                if (at_root) {
                    l0 = legal_root[lane];
                    l1 = lane < 9u ? legal_root[64u + lane] : 0u;
                } else {
                    l0 = legal_values(S, lane, tab);
                    // pairs 64-71 are slots 16-23 of the third opponent: only
                    // a four-player game with a row of 17 tiles or more has them
                    l1 = (lane == 8u && cont) ? 1u : 0u;
                    const bool wide = S.P == 4u && __popc(hand_of(S, (S.m + 3u) & 3u)) > 16;
                    if (__builtin_amdgcn_readfirstlane((uint32_t)wide) != 0u && lane < 8u)
                        l1 = legal_values(S, 64u + lane, tab);
                }
                // the legal table the scoring reads: the root's as it is
                const uint32_t *legal_t = at_root ? legal_root : legal_s;
                if (!at_root) {
                    legal_s[lane] = l0;
                    if (lane < 9u) legal_s[64u + lane] = l1;
                }
                const uint32_t cb0 = (cbw0 >> ((lane & 1u) * 16u)) & 0xFFFu;
                const uint32_t cb1 = lane == 8u ? (cbw1 & 1u) : (cbw1 >> ((lane & 1u) * 16u)) & 0xFFFu;
                const uint32_t u0 = l0 & ~cb0, u1 = l1 & ~cb1;
                const uint64_t b0 = __ballot(u0 != 0u), b1 = __ballot(u1 != 0u);
                tree_sync<WS>();
                // uniform values every lane loaded, read once after the loads
                // have landed, so that the loops over blocks stay scalar
                const uint32_t nchild = __builtin_amdgcn_readfirstlane(nchild_v);
                const uint32_t next0 = __builtin_amdgcn_readfirstlane(next0_v);
                if (b0 | b1) {
                    // expansion: the lowest playable key that has no child yet --
                    // the stop before the guesses after a right guess
                    // the record word that gets the new key's bit, as this
                    // level loaded it: word 3 is lane 8's cbw1, a guess bitmap
                    // word that of the pair's lane (cbw0, or cbw1 past pair 63)
                    uint32_t key, word, bit, old;
                    if ((b1 >> 8) & 1u) {
                        key = kStopKey;
                        word = 3u;
                        bit = 1u;
                        old = __builtin_amdgcn_readlane(cbw1, 8);
                    } else {
                        uint32_t pair, vbits;
                        if (b0) {
                            pair = (uint32_t)__builtin_ctzll(b0);
                            vbits = __builtin_amdgcn_readlane(u0, pair);
                        } else {
                            const uint32_t l = (uint32_t)__builtin_ctzll(b1);
                            vbits = __builtin_amdgcn_readlane(u1, l);
                            pair = 64u + l;
                        }
                        const uint32_t v = (uint32_t)__builtin_ctz(vbits);
                        key = pair * 12u + v + (cont ? kStopKey + 1u : 0u);
                        word = 4u + half + (pair >> 1);
                        bit = 1u << (v + (pair & 1u) * 16u);
                        old = pair < 64u ? __builtin_amdgcn_readlane(cbw0, pair)
                                         : __builtin_amdgcn_readlane(cbw1, pair - 64u);
                    }
                    uint32_t e;
                    const uint32_t c = append_child(node, nchild, key | (S.m << 16), 0u, e);
                    if (lane == 0) W[rec + word] = old | bit;
                    if (at_root) {
                        const uint4 ne = make_uint4(key | (S.m << 16), 0u, 0u, c);
                        if (nchild < 2u * kBlockEntries && lane == 0u) rc_ent[nchild] = ne;
                        // a new overflow block starts at child 64 and at child 128
                        if (nchild == kBlockEntries) rc_nx0 = nodes_cap + n_ovf - 1u;
                        if (nchild == 2u * kBlockEntries) rc_nx1 = nodes_cap + n_ovf - 1u;
                        rc_nc = nchild + 1u;
                        if (4u + (lane >> 1) == word) rc_cb0 |= bit;
                        if ((lane < 8u ? 36u + (lane >> 1) : lane == 8u ? 3u : 0u) == word) rc_cb1 |= bit;
                    }
                    path_e[np++] = e;
                    last_block = depth;
                    term = apply_action(S, key, a.cont_mode != 0u, chance_at(cw, depth), winner,
                                        cont);
                    tree_sync<WS>();
                    break;
                }
                // selection: UCT over the playable children, 64 per pass
                float best_s = -__builtin_inff();
                uint32_t best_i = 0xFFFFFFFFu, best_e = 0u, best_act = 0u, best_node = 0u, best_n = 0u;
                // block blk's entries are scored while the next block's (and
                // the block id after it) are being loaded
                uint32_t blk = node, nxt = next0;
                uint4 ent = ent0;
                for (uint32_t base = 0; base < nchild; base += kBlockEntries) {
                    const bool more = base + kBlockEntries < nchild;
                    uint4 ent_n = ent;
                    uint32_t nxt_n = kNoBlock;
                    if (more) {
                        if (at_root && base == 0u) {
                            ent_n = rc_ent[kBlockEntries + lane];
                            nxt_n = rc_nx1;
                        } else {
                            ent_n = *reinterpret_cast<const uint4 *>(W + block_off(nxt) + lane * kEntryWords);
                            if (base + 2u * kBlockEntries < nchild)
                                nxt_n = __builtin_amdgcn_readfirstlane(bnext[nxt]);
                        }
                    }
                    // straight-line scoring: every lane computes a score (a
                    // lane past the children reads some entry: its pair index
                    // is clamped into the legal table) and the playable ones
                    // keep it
                    const uint32_t ci = base + lane;
                    const uint32_t key = ent.x & 0xFFFFu;
                    const bool after_right = key > kStopKey;
                    const uint32_t act = after_right ? key - kStopKey - 1u : key;
                    const uint32_t pr = act / 12u < 72u ? act / 12u : 72u;
                    const bool legal = (legal_t[pr] >> ((act - pr * 12u) & 31u)) & 1u;
                    const bool playable =
                        (ci < nchild) & (key == kStopKey ? cont : (after_right == cont) & legal);
                    const float n = (float)ent.y;
                    const float q = __uint_as_float(ent.z) / n;
                    const float ex = lp / n;
                    const float u = a.c_uct * sqrtf(ex);
                    const float sc = playable ? q + u : -__builtin_inff();
                    float bs;
                    const int bl = wave_argmax_lane(sc, bs);
                    if (bl >= 0 && (best_i == 0xFFFFFFFFu || bs > best_s)) {
                        const uint32_t wl = (uint32_t)bl;
                        best_s = bs;
                        best_i = base + wl;
                        best_e = block_off(blk) + wl * kEntryWords;
                        best_act = __builtin_amdgcn_readlane(ent.x, wl) & 0xFFFFu;
                        best_n = __builtin_amdgcn_readlane(ent.y, wl);
                        best_node = __builtin_amdgcn_readlane(ent.w, wl);
                    }
                    if (more) {
                        blk = nxt;
                        ent = ent_n;
                        nxt = nxt_n;
                    }
                }
                node = best_node;
                node_n = best_n;
                path_e[np++] = best_e;
                last_block = depth;
                term = apply_action(S, best_act, a.cont_mode != 0u, chance_at(cw, depth), winner,
                                    cont);
                ++depth;
                tree_sync<WS>();
            }
            if (!term && cont) leaf_continue_coin(S, chance_at(cw, last_block));
            deepest = np - a.vanilla > deepest ? np - a.vanilla : deepest;
            cyc_add(1u, clock64() - t1);
            if (!PIPE && a.lpp == 1u) {
                // the sequential search: the leaf is evaluated and backed up
                // before the next descent
                const uint64_t t2 = clock64();
                // ---- 3. evaluate the leaf: playouts, or the value network ---------
                uint32_t wins0 = 0u, wins1 = 0u, wins2 = 0u, wins3 = 0u;
                float vals[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                bool use_vals = false;
                if (VALUE && !term) {
                    // one row per seat perspective q = lane % 16 < P
                    uint4 ps;
                    encode(S, ps.x, ps.y, ps.z, ps.w);
                    const uint32_t q = lane & 15u;
                    RowFeat rf = q < S.P ? row_features(ps, q) : no_row();
                    const float vrow = vn_eval_tree_t(vn_ptrs(const_cast<void *>(a.net)), rf,
                                                      w2_lds, vn_small[0]);
                    float v[4];
        #pragma unroll
                    for (uint32_t k = 0; k < 4u; ++k)
                        v[k] = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(vrow), k));
                    const float vm = R.m == 0u ? v[0] : R.m == 1u ? v[1] : R.m == 2u ? v[2] : v[3];
                    const float dv = vm - 0.5f;
                    if (!((dv < 0.0f ? -dv : dv) < a.band)) {
                        use_vals = true;
                        ++n_net;
        #pragma unroll
                        for (uint32_t k = 0; k < 4u; ++k) vals[k] = (float)a.fb_ppl * v[k];
                    }
                }
                if (term) {
                    wins0 = winner == 0u ? nplay : 0u;
                    wins1 = winner == 1u ? nplay : 0u;
                    wins2 = winner == 2u ? nplay : 0u;
                    wins3 = winner == 3u ? nplay : 0u;
                } else if (!use_vals) {
                    const uint64_t pl = (uint64_t)it * kPhiloxM1;
                    const uint32_t trk1 = tr ^ a.k1;
                    for (uint32_t pb = 0; pb < nplay; pb += 64u) {
                        const uint32_t p = pb + lane;
                        const bool act = p < nplay;
                        uint32_t w = 4u;
                        if (act) {
                            State s = S;
                            PlayoutKey pk;
                            pk.a = (uint32_t)(pl >> 32) ^ p ^ a.k0;
                            pk.b = (uint32_t)pl;
                            pk.gm_lo = 0u;
                            pk.gm_hi = 0u;
                            bool over = false;
                            uint32_t len = 0u;
                            // the words of step g+1 do not depend on the game, so
                            // they are computed while step g runs (one wavefront per
                            // tree has no other wavefront to hide latencies behind)
                            Words wd = step_words(pk, trk1, a.k0, a.k1);
                            next_step(pk);
                            while (!over) {
                                const Words wn = step_words(pk, trk1, a.k0, a.k1);
                                next_step(pk);
                                over = guess_step(s, wd, w, tab);
                                wd = wn;
                                if (++len >= kMaxGuesses && !over) {
                                    atomicOr(&g_error_word, kErrLimit);
                                    over = true;
                                    w = 4u;
                                }
                            }
                        }
                        wins0 += (uint32_t)__popcll(__ballot(act && w == 0u));
                        wins1 += (uint32_t)__popcll(__ballot(act && w == 1u));
                        wins2 += (uint32_t)__popcll(__ballot(act && w == 2u));
                        wins3 += (uint32_t)__popcll(__ballot(act && w == 3u));
                    }
                }

                if (!term && !use_vals && a.leaf_eval) ++n_played;
                if (!use_vals) {
                    vals[0] = (float)wins0;
                    vals[1] = (float)wins1;
                    vals[2] = (float)wins2;
                    vals[3] = (float)wins3;
                }

                const uint64_t t3 = clock64();
                cyc_add(2u, t3 - t2);
                // ---- 4. back-propagation --------------------------------------------
                n_root += nplay;
                uint32_t e = 0u, nw = 0u;
                if (lane < np) {
                    // the entry {key | chooser << 16, N, W, id} in one load
                    e = path_e[lane];
                    const uint4 en = *reinterpret_cast<const uint4 *>(W + e);
                    W[e + 1u] = en.y + nplay;
                    if (!(a.vanilla && lane == 0u)) {   // a world node's W word holds its key
                        const uint32_t chooser = en.x >> 16;
                        const float wc = chooser == 0u ? vals[0] : chooser == 1u ? vals[1] : chooser == 2u ? vals[2] : vals[3];
                        nw = __float_as_uint(__uint_as_float(en.z) + wc);
                        W[e + 2u] = nw;
                    }
                }
                if (rc_on && np > 0u)   // lane 0 holds the root child's entry
                    rc_update(rc_slot(__builtin_amdgcn_readlane(e, 0)), nplay, true,
                              __builtin_amdgcn_readlane(nw, 0));
                tree_sync<WS>();
                cyc_add(3u, clock64() - t3);
                continue;
            }
            // the leaf and its path, for the evaluation and the wins
            if (lane == 0) {
                uint4 ps;
                encode(S, ps.x, ps.y, ps.z, ps.w);
                leaf_all[wv][buf][b] = ps;
                np_all[wv][buf][b] = np;
            }
            term_mask |= term ? 1u << b : 0u;
            winners |= (term ? winner : 0u) << (2u * b);
            // visit counts at once
            n_root += nplay;
            if (lane < np) W[path_e[lane] + 1u] += nplay;
            if (rc_on && np > 0u) rc_update(rc_slot(path_e[0]), nplay, false, 0u);
            tree_sync<WS>();
        }
        if (PIPE) {
            // pass k descended, pass k - 1 evaluated: back up pass k - 1.  A
            // search that gave up still meets the step's barrier, and tells
            // the other wavefront which step it stopped at (it may read the
            // word only after this wavefront has gone on to the next step)
            if (lane == 0) {
                meta_all[wv][buf][0] = term_mask;
                meta_all[wv][buf][1] = winners;
                if (failed) pipe_x[0] = k + 1u;
            }
            __syncthreads();
            if (failed) break;
            if (k >= 1u) {
                const uint32_t ip = (k - 1u) * a.lpp;
                const uint64_t t3 = clock64();
                backprop_pass(buf ^ 1u, a.iters - ip < a.lpp ? a.iters - ip : a.lpp);
                cyc_add(3u, clock64() - t3);
            }
            continue;
        }
        if (failed) break;
        if (a.lpp == 1u) continue;
        const uint64_t t2 = clock64();
        eval_pass(0u, i0, nb, term_mask, winners);
        const uint64_t t3 = clock64();
        cyc_add(2u, t3 - t2);
        backprop_pass(0u, nb);
        cyc_add(3u, clock64() - t3);
    }
    if (PIPE) {
        __syncthreads();   // the evaluating wavefront's statistics
        n_net = pipe_x[1];
        n_played = pipe_x[2];
        cyc[2] = (uint64_t)pipe_x[3] | ((uint64_t)pipe_x[4] << 32);
        n_sampler_fallback += pipe_x[5];   // counted by whichever wavefront samples
        cyc[0] += (uint64_t)pipe_x[6] | ((uint64_t)pipe_x[7] << 32);
    }

    // ---- decision and root statistics ----------------------------------------
    if (lane == 0) {
        W[0] = n_nodes;
        W[1] = n_ovf;
        W[2] = n_root;
        W[3] = n_net;
        W[4] = n_played;
        W[5] = n_sampler_fallback;
        W[kHdrFailed] = failed ? 1u : 0u;
        W[kHdrFailed + 1u] = deepest;
        for (uint32_t q = 0; q < 4u; ++q) {
            W[kHdrCycles + 2u * q] = (uint32_t)cyc[q];
            W[kHdrCycles + 2u * q + 1u] = (uint32_t)(cyc[q] >> 32);
        }
    }
    if (failed) {
        if (lane == 0 && a.best) a.best[t] = -1;
        write_no_children(a, t, lane);
        return;
    }
    uint32_t *kid = a.kids ? a.kids + (size_t)t * kMaxActions * 3u : nullptr;
    if (a.vanilla) {
        // a guess is judged over all worlds: its (N, W) summed over the world
        // nodes in creation order; most visits wins, the lowest action id on
        // ties; the statistics come back indexed by action id
        uint32_t *agg = W + a.sh.agg_off;
        for (uint32_t c = lane; c < 2u * kMaxActions; c += 64u) agg[c] = 0u;
        tree_sync<WS>();
        const uint32_t nw = W[rec_off(0u) + 2u];
        uint32_t wblk = 0u;
        for (uint32_t wi = 0; wi < nw; ++wi) {
            if (wi > 0u && (wi & (kBlockEntries - 1u)) == 0u) wblk = bnext[wblk];
            const uint32_t wnode = W[block_off(wblk) + (wi & (kBlockEntries - 1u)) * kEntryWords + 3u];
            const uint32_t nc = W[rec_off(wnode) + 2u];
            uint32_t blk = wnode;
            for (uint32_t base = 0; base < nc; base += kBlockEntries) {
                if (base + lane < nc) {
                    // one child per action below a world node: no two lanes collide
                    const uint4 ent = *reinterpret_cast<const uint4 *>(W + block_off(blk) + lane * kEntryWords);
                    const uint32_t act = ent.x & 0xFFFFu;
                    agg[2u * act] += ent.y;
                    agg[2u * act + 1u] = __float_as_uint(__uint_as_float(agg[2u * act + 1u]) +
                                                         __uint_as_float(ent.z));
                }
                if (base + kBlockEntries < nc) blk = bnext[blk];
            }
            tree_sync<WS>();
        }
        uint64_t key = 0ull;   // N << 32 | (863 - action): most visits, lowest id on ties
        for (uint32_t c = lane; c < kMaxActions; c += 64u) {
            const uint32_t n = agg[2u * c];
            const uint64_t kc = n ? ((uint64_t)n << 32) | (kMaxActions - 1u - c) : 0ull;
            key = kc > key ? kc : key;
            if (kid) {
                kid[c * 3u + 0u] = n ? c : 0xFFFFu;
                kid[c * 3u + 1u] = n;
                kid[c * 3u + 2u] = agg[2u * c + 1u];
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor(key, off, 64);
            key = o > key ? o : key;
        }
        if (lane == 0 && a.best)
            a.best[t] = key == 0ull ? -1 : (int32_t)(kMaxActions - 1u - (uint32_t)(key & 0xFFFFFFFFull));
        return;
    }
    const uint32_t nchild = W[rec_off(0u) + 2u];
    uint32_t blk = 0u;
    uint32_t best_n = 0u, best_i = 0xFFFFFFFFu, best_act = 0xFFFFu;
    for (uint32_t base = 0; base < kMaxActions; base += kBlockEntries) {
        const uint32_t ci = base + lane;
        uint32_t act = 0xFFFFu, n = 0u, wbits = 0u;
        if (base < nchild && ci < nchild) {
            const uint32_t e = block_off(blk) + lane * kEntryWords;
            act = W[e] & 0xFFFFu;
            n = W[e + 1u];
            wbits = W[e + 2u];
        }
        if (kid && ci < kMaxActions) {
            kid[ci * 3u + 0u] = act;
            kid[ci * 3u + 1u] = n;
            kid[ci * 3u + 2u] = wbits;
        }
        uint32_t bn = ci < nchild ? n : 0u;
        uint32_t bi = ci < nchild ? ci : 0xFFFFFFFFu;
        wave_argmax_u(bn, bi);
        if (bi != 0xFFFFFFFFu && (best_i == 0xFFFFFFFFu || bn > best_n)) {
            best_n = bn;
            best_i = bi;
            best_act = __builtin_amdgcn_readlane(act, bi - base);
        }
        if (base + kBlockEntries < nchild) blk = bnext[blk];
    }
    if (lane == 0 && a.best) a.best[t] = best_i == 0xFFFFFFFFu ? -1 : (int32_t)best_act;
}

// Root-parallel search (Sec. III-B): the K trees of one root are amalgamated
// into one root by summing each action's (N, W) over the trees in tree order;
// the decision is the most visited action, the lowest action id on ties.  One
// 256-thread workgroup per root; a root with a failed tree gets no decision.
constexpr uint32_t kMergeThreads = 256;

__global__ void __launch_bounds__(kMergeThreads)
mcts_merge_kernel(const uint32_t *ws, MctsShape sh, uint32_t K, int32_t *best, uint32_t *merged)
{
    const uint64_t tree_words = sh.tree_words;
    const uint32_t nodes_cap = sh.nodes_cap, ovf_cap = sh.ovf_cap, node_stride = sh.node_stride;
    __shared__ uint32_t sn[kMaxActions];
    __shared__ float sw[kMaxActions];
    __shared__ uint32_t s_failed;
    __shared__ uint64_t s_best[kMergeThreads / 64u];
    const uint32_t r = blockIdx.x, tid = threadIdx.x;
    for (uint32_t c = tid; c < kMaxActions; c += kMergeThreads) {
        sn[c] = 0u;
        sw[c] = 0.0f;
    }
    if (tid == 0) s_failed = 0u;
    __syncthreads();
    const uint32_t ovf_base = kTreeHeaderWords + nodes_cap * node_stride;
    for (uint32_t k = 0; k < K; ++k) {
        const uint32_t *W = ws + ((uint64_t)r * K + k) * tree_words;
        const uint32_t *bnext = W + ovf_base + ovf_cap * kBlockWords;
        if (W[kHdrFailed] != 0u) {
            if (tid == 0) s_failed = 1u;
            continue;   // uniform across the workgroup
        }
        const uint32_t nchild = W[kTreeHeaderWords + 2u];
        for (uint32_t ci = tid; ci < nchild; ci += kMergeThreads) {
            uint32_t blk = 0u;
            for (uint32_t j = 0; j < (ci >> 6); ++j) blk = bnext[blk];
            const uint32_t off = blk < nodes_cap ? kTreeHeaderWords + blk * node_stride + sh.node_words
                                                 : ovf_base + (blk - nodes_cap) * kBlockWords;
            const uint32_t *e = W + off + (ci & (kBlockEntries - 1u)) * kEntryWords;
            const uint32_t act = e[0] & 0xFFFFu;
            // one tree has at most one child per action: no two threads collide
            sn[act] += e[1];
            sw[act] += __uint_as_float(e[2]);
        }
        __syncthreads();
    }
    // most visited action, lowest id on ties: key = N << 32 | (864 - 1 - action)
    uint64_t key = 0ull;
    for (uint32_t c = tid; c < kMaxActions; c += kMergeThreads) {
        const uint64_t kc = sn[c] ? ((uint64_t)sn[c] << 32) | (kMaxActions - 1u - c) : 0ull;
        key = kc > key ? kc : key;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(key, off, 64);
        key = o > key ? o : key;
    }
    if ((tid & 63u) == 0u) s_best[tid >> 6] = key;
    __syncthreads();
    const bool failed = s_failed != 0u;
    if (tid == 0) {
        uint64_t b = 0ull;
        for (uint32_t i = 0; i < kMergeThreads / 64u; ++i) b = s_best[i] > b ? s_best[i] : b;
        best[r] = failed || b == 0ull ? -1 : (int32_t)(kMaxActions - 1u - (uint32_t)(b & 0xFFFFFFFFull));
    }
    if (merged) {
        uint32_t *m = merged + (size_t)r * kMaxActions * 3u;
        for (uint32_t c = tid; c < kMaxActions; c += kMergeThreads) {
            const bool live = !failed && sn[c] != 0u;
            m[c * 3u + 0u] = live ? c : 0xFFFFu;
            m[c * 3u + 1u] = live ? sn[c] : 0u;
            m[c * 3u + 2u] = live ? __float_as_uint(sw[c]) : 0u;
        }
    }
}

hipError_t launch_mcts(const uint4 *roots, uint32_t n_trees, uint32_t trees_per_root,
                       uint32_t iters, uint32_t ppl,
                       uint32_t dmax, float c_uct, uint32_t k0, uint32_t k1, uint32_t tree_base,
                       const float *ln, uint32_t *ws, int32_t *best, uint32_t *kids,
                       uint32_t leaf_eval, float band, uint32_t fb_ppl, const void *net,
                       uint32_t cont, uint32_t vanilla, uint32_t lpp, uint32_t pipe,
                       hipStream_t st)
{
    if (n_trees == 0) return hipSuccess;
    MctsArgs a;
    a.roots = roots;
    a.n_trees = n_trees;
    a.trees_per_root = trees_per_root;
    a.iters = iters;
    a.ppl = ppl;
    a.dmax = dmax == 0u ? 0xFFFFFFFFu : dmax;   // 0: no depth threshold
    a.c_uct = c_uct;
    a.k0 = k0;
    a.k1 = k1;
    a.tree_base = tree_base;
    a.ln = ln;
    a.ws = ws;
    a.sh = mcts_shape(iters, cont, vanilla);
    a.cont_mode = cont;
    a.vanilla = vanilla;
    a.lpp = lpp;
    a.pipe = pipe;
    a.best = best;
    a.kids = kids;
    a.leaf_eval = leaf_eval;
    a.band = band;
    a.fb_ppl = fb_ppl;
    a.net = net;
    if (pipe) {
        // one tree per workgroup: a descending and an evaluating wavefront
        if (leaf_eval)
            hipLaunchKernelGGL((mcts_tree_kernel<true, true>), dim3(n_trees), dim3(128), 0, st, a);
        else
            hipLaunchKernelGGL((mcts_tree_kernel<false, true>), dim3(n_trees), dim3(128), 0, st, a);
    } else if (leaf_eval) {
        hipLaunchKernelGGL((mcts_tree_kernel<true, false>), dim3((n_trees + 3u) / 4u), dim3(256), 0,
                           st, a);
    } else {
        hipLaunchKernelGGL((mcts_tree_kernel<false, false>), dim3(n_trees), dim3(64), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_mcts_merge(const uint32_t *ws, uint32_t n_roots, uint32_t trees_per_root,
                             uint32_t iters, uint32_t cont, int32_t *best, uint32_t *merged,
                             hipStream_t st)
{
    if (n_roots == 0) return hipSuccess;
    hipLaunchKernelGGL(mcts_merge_kernel, dim3(n_roots), dim3(kMergeThreads), 0, st, ws,
                       mcts_shape(iters, cont, 0u), trees_per_root, best, merged);
    return hipGetLastError();
}

}  // namespace dvc
