// rollout.hip -- random playouts of the Da Vinci Code game on gfx950.
//
// Sec. II-B of Zhang et al. (arXiv 2403.10720): in every simulation the game
// is played to the end by taking each decision at random.  The paper
// attributes the GPU's poor scaling to branch divergence (turns of different
// length; finished threads wait for the longest game, Sec. IV-B).  Here the
// guess step is straight-line predicated code on 24-bit masks, and the
// persistent kernel refills a lane as soon as its game ends, so a wavefront
// keeps its 64 lanes busy until the work queue runs dry.
#include "dvc_core.hpp"
#include "dvc_internal.hpp"

namespace dvc {

// ---------------------------------------------------------------------------
// One guess.  w0 draw, w1 target, w2 value, w3 continue coin / own reveal.
// Returns true when the game is decided; `winner` is then the last seat with
// a hidden tile.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool guess_step(State &s, const Words &w, uint32_t &winner,
                                           const uint8_t *tab)
{
    const uint32_t owned = s.h0 | s.h1 | s.h2 | s.h3;
    const uint32_t pool = ~owned & kAll;
    const bool turn_start = s.phase == 0u;
    const bool draw = turn_start && pool != 0u;
    // The target is a hidden tile of another player, so it never is the tile
    // the mover draws: its pick does not wait for the draw's (two of the
    // step's three table lookups run side by side).
    const uint32_t hm0 = hand_of(s, s.m);
    const uint32_t targets = owned & ~hm0 & ~s.rev;
    const uint32_t t = pick_bit_tab(targets, w.w1, tab);
    const uint32_t d = pick_bit_tab(pool, w.w0, tab);
    const uint32_t dbit = draw ? (1u << d) : 0u;
    add_to_hand(s, s.m, dbit);
    s.drawn = turn_start ? (draw ? (int32_t)d : -1) : s.drawn;
    s.phase = 1u;

    const uint32_t hm = hm0 | dbit;
    const uint32_t tb = 1u << t;
    const uint32_t o = (s.h0 & tb) ? 0u : (s.h1 & tb) ? 1u : (s.h2 & tb) ? 2u : 3u;
    const uint32_t cand = candidates(t, hand_of(s, o), hm, s.rev);
    const uint32_t v = pick_bit_tab(cand, w.w2, tab);
    const bool right = v == t;

    // a wrong guess reveals the drawn tile; only with nothing drawn (empty
    // pool) is a random own hidden tile needed, so that search is skipped
    // by the whole wave in the common case
    uint32_t wrong_tile = (uint32_t)s.drawn;
    if (s.drawn < 0) wrong_tile = pick_bit_tab(hm & ~s.rev, w.w3, tab);
    s.rev |= right ? tb : (1u << (wrong_tile & 31u));

    const uint32_t alive = alive_mask(s);
    const bool over = __popc(alive) == 1;
    winner = (uint32_t)__builtin_ctz(alive | 16u);
    const bool go_on = right && w.w3 < 0x80000000u;
    const bool pass = !over && !go_on;
    s.m = pass ? next_alive(alive, s.m, s.P) : s.m;
    s.phase = pass ? 0u : s.phase;
    s.drawn = pass ? -1 : s.drawn;
    return over;
}

// Philox round 1 for counter (g, p, l, tr) only multiplies g and l: the l
// product is fixed for a playout and g*M0 grows by M0 per step.
struct PlayoutKey {
    uint32_t a, b;          // round-1 words 0 and 1 (from p, l)
    uint32_t gm_lo, gm_hi;  // g * M0
};

__device__ __forceinline__ PlayoutKey playout_key(uint32_t p, uint32_t l, uint32_t k0)
{
    const uint64_t pl = (uint64_t)l * kPhiloxM1;
    PlayoutKey pk;
    pk.a = (uint32_t)(pl >> 32) ^ p ^ k0;
    pk.b = (uint32_t)pl;
    pk.gm_lo = 0u;
    pk.gm_hi = 0u;
    return pk;
}

__device__ __forceinline__ Words step_words(const PlayoutKey &pk, uint32_t trk1, uint32_t k0,
                                            uint32_t k1)
{
    return philox_rounds_2_to_10(pk.a, pk.b, pk.gm_hi ^ trk1, pk.gm_lo, k0, k1);
}

__device__ __forceinline__ void next_step(PlayoutKey &pk)
{
    const uint64_t g = ((uint64_t)pk.gm_hi << 32 | pk.gm_lo) + kPhiloxM0;
    pk.gm_lo = (uint32_t)g;
    pk.gm_hi = (uint32_t)(g >> 32);
}

// The leaf array is read-only for a whole launch, so a wave-uniform leaf
// state is read with scalar loads through the constant address space (the
// wait for it then does not also wait for the lanes' outstanding stores).
typedef const __attribute__((address_space(4))) uint32_t *const_u32_ptr;

__device__ __forceinline__ void load_uniform_state(const uint4 *base, uint32_t idx, uint32_t &w0,
                                                   uint32_t &w1, uint32_t &w2, uint32_t &w3)
{
    const_u32_ptr p = (const_u32_ptr)((uintptr_t)base) + 4u * idx;
    w0 = p[0];
    w1 = p[1];
    w2 = p[2];
    w3 = p[3];
}

__device__ __forceinline__ void record_win(uint32_t *seat_wins, uint32_t leaf, uint32_t winner)
{
    if (seat_wins && winner < 4u) atomicAdd(&seat_wins[(size_t)leaf * 4u + winner], 1u);
}

// Every guess reveals one more of the 24 tiles and the winner keeps a hidden
// one, so a game from a valid state ends within 23 guesses; reaching the cap
// means the state was not valid after all.
constexpr uint32_t kMaxGuesses = 23u;

// ---------------------------------------------------------------------------
// Variant 1: one lane per playout; lanes whose game ended wait for the rest.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) rollout_lane_per_playout(RolloutArgs a)
{
    __shared__ uint8_t tab[kKthTableBytes];
    fill_kth_table(tab);
    __syncthreads();
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.total) return;
    const uint32_t leaf = j / a.ppl;
    const uint32_t p = j - leaf * a.ppl;
    const uint4 st = a.leaves[leaf];
    State s;
    if (!decode(st.x, st.y, st.z, st.w, s)) {
        atomicOr(&g_error_word, kErrState);
        if (a.winner) a.winner[j] = -1;
        if (a.length) a.length[j] = -1;
        return;
    }
    PlayoutKey pk = playout_key(p, a.leaf_base + leaf, a.k0);
    const uint32_t trk1 = a.tree ^ a.k1;
    uint32_t alive = alive_mask(s);
    bool over = __popc(alive) == 1;
    uint32_t winner = (uint32_t)__builtin_ctz(alive | 16u);
    uint32_t len = 0;
    while (!over) {
        const Words w = step_words(pk, trk1, a.k0, a.k1);
        over = guess_step(s, w, winner, tab);
        next_step(pk);
        ++len;
        if (!over && len >= kMaxGuesses) {
            atomicOr(&g_error_word, kErrLimit);
            over = true;
            winner = 4u;
        }
    }
    if (a.winner) a.winner[j] = (int8_t)(winner < 4u ? (int)winner : -1);
    if (a.length) a.length[j] = (int16_t)len;
    record_win(a.seat_wins, leaf, winner);
}

// ---------------------------------------------------------------------------
// Variant 2: persistent waves with lane refill and work stealing.
//
// Every wave steals chunks of `chunk` consecutive playout ids (playout id =
// leaf * ppl + p) from a global counter and stages the chunk's leaf states in
// its own LDS slot.  After each guess step the lanes whose game ended write
// their outcome, their seat wins are summed per leaf across the wave with
// ballots, and they take the next playout ids of the chunk (ballot + mbcnt
// prefix), so no lane idles while the wave still has work.  Outputs depend
// only on the playout id, never on which lane or wave ran it.
// ---------------------------------------------------------------------------
template <int WAVES>
__global__ void __launch_bounds__(WAVES * 64) rollout_persistent(RolloutArgs a)
{
    __shared__ uint4 stage[WAVES][kStageLeaves];
    __shared__ uint8_t tab[kKthTableBytes];
    fill_kth_table(tab);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    uint4 *my = stage[threadIdx.x >> 6];
    uint32_t *queue = &g_queue[a.queue_slot][0];

    uint32_t rcur = 0, rend = 0, leaf0 = 0;   // wave-uniform: current chunk
    bool drained = false;                     // wave-uniform: queue empty
    bool active = false;
    State s;
    s.h0 = s.h1 = s.h2 = s.h3 = s.rev = 0u;
    s.m = 0u; s.P = 2u; s.phase = 1u; s.drawn = -1;
    PlayoutKey pk = {0u, 0u, 0u, 0u};
    uint32_t j = 0, leaf = 0, len = 0, winner = 0;
    const uint32_t trk1 = a.tree ^ a.k1;
    uint64_t steps = 0;

    for (;;) {
        // ---- refill idle lanes ------------------------------------------
        uint64_t idle = __ballot(!active);
        while (idle != 0ull) {
            if (rcur == rend) {
                if (drained) break;
                uint32_t c = 0;
                if (lane == 0) c = atomicAdd(&queue[0], 1u);
                c = __builtin_amdgcn_readfirstlane(c);
                const uint64_t start = (uint64_t)c * a.chunk;
                if (start >= a.total) { drained = true; break; }
                rcur = (uint32_t)start;
                rend = (uint32_t)min<uint64_t>(start + a.chunk, a.total);
                leaf0 = rcur / a.ppl;
                const uint32_t nl = (rend - 1u) / a.ppl - leaf0 + 1u;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                for (uint32_t k = lane; k < nl; k += 64u) my[k] = a.leaves[leaf0 + k];
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            const uint32_t take = min<uint32_t>((uint32_t)__popcll(idle), rend - rcur);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
            const bool mine = ((idle >> lane) & 1ull) && rank < take;
            if (mine) {
                j = rcur + rank;
                leaf = j / a.ppl;
                const uint32_t p = j - leaf * a.ppl;
                const uint4 st = my[leaf - leaf0];
                const bool ok = decode(st.x, st.y, st.z, st.w, s);
                pk = playout_key(p, a.leaf_base + leaf, a.k0);
                len = 0;
                const uint32_t alive = alive_mask(s);
                winner = (uint32_t)__builtin_ctz(alive | 16u);
                if (!ok) {
                    atomicOr(&g_error_word, kErrState);
                    if (a.winner) a.winner[j] = -1;
                    if (a.length) a.length[j] = -1;
                } else if (__popc(alive) == 1) {
                    if (a.winner) a.winner[j] = (int8_t)(winner < 4u ? (int)winner : -1);
                    if (a.length) a.length[j] = 0;
                    record_win(a.seat_wins, leaf, winner);
                } else {
                    active = true;
                }
            }
            rcur += take;
            idle &= ~__ballot(mine);
        }
        const uint64_t act = __ballot(active);
        if (act == 0ull) {
            if (drained) break;
            continue;
        }
        ++steps;

        // ---- one guess for every active lane ----------------------------
        bool over = false;
        if (active) {
            const Words w = step_words(pk, trk1, a.k0, a.k1);
            over = guess_step(s, w, winner, tab);
            next_step(pk);
            ++len;
            if (!over && len >= kMaxGuesses) {
                atomicOr(&g_error_word, kErrLimit);
                over = true;
                winner = 4u;
            }
        }

        // ---- finished games: outputs and per-leaf seat wins -------------
        const bool fin = active && over;
        if (fin) {
            if (a.winner) a.winner[j] = (int8_t)(winner < 4u ? (int)winner : -1);
            if (a.length) a.length[j] = (int16_t)len;
        }
        if (a.seat_wins) {
            uint64_t fmask = __ballot(fin);
            while (fmask != 0ull) {
                const uint32_t first = (uint32_t)__builtin_ctzll(fmask);
                const uint32_t L = __builtin_amdgcn_readlane(leaf, first);
                const uint64_t same = __ballot(fin && leaf == L);
                const uint32_t c0 = (uint32_t)__popcll(__ballot(fin && leaf == L && winner == 0u));
                const uint32_t c1 = (uint32_t)__popcll(__ballot(fin && leaf == L && winner == 1u));
                const uint32_t c2 = (uint32_t)__popcll(__ballot(fin && leaf == L && winner == 2u));
                const uint32_t c3 = (uint32_t)__popcll(__ballot(fin && leaf == L && winner == 3u));
                if (lane < 4u) {
                    const uint32_t c = lane == 0u ? c0 : lane == 1u ? c1 : lane == 2u ? c2 : c3;
                    if (c) atomicAdd(&a.seat_wins[(size_t)L * 4u + lane], c);
                }
                fmask &= ~same;
            }
        }
        active = active && !over;
    }

    if (a.stats && lane == 0) atomicAdd(&a.stats[0], (unsigned long long)steps);
    // the last workgroup out leaves the queue slot at zero for the next call
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&queue[1], 1u);
        if (done == gridDim.x - 1u) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// Variant 3: persistent waves over single-leaf work items.
//
// An item is up to `item_chunk` consecutive playouts of ONE leaf: item c
// covers leaf c / parts, playouts (c % parts) * item_chunk onwards.  Waves
// steal batches of `batch` items from a global counter and prefetch the next
// batch id one batch ahead, so the atomic's round trip is hidden behind a
// batch of guesses.  The item's leaf state is wave-uniform: it is loaded,
// decoded and validated once in scalar registers and copied into every lane
// the item refills (ballot + mbcnt prefix over the idle lanes).  A decided or
// malformed leaf finishes its whole item at once.
// ---------------------------------------------------------------------------
template <int WAVES>
__global__ void __launch_bounds__(WAVES * 64) rollout_items(RolloutArgs a)
{
    __shared__ uint8_t tab[kKthTableBytes];
    fill_kth_table(tab);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t *queue = &g_queue[a.queue_slot][0];
    const uint32_t trk1 = a.tree ^ a.k1;

    uint32_t item = 0, item_end = 0;         // wave-uniform: items of the current batch
    uint32_t pending = 0;                    // lane 0: prefetched batch id
    if (lane == 0) pending = atomicAdd(&queue[0], 1u);
    bool drained = false;
    uint32_t it_leaf = 0, it_p = 0, it_pend = 0, it_pa = 0, it_pb = 0;   // current item
    State it_s;
    it_s.h0 = it_s.h1 = it_s.h2 = it_s.h3 = it_s.rev = 0u;
    it_s.m = 0u; it_s.P = 2u; it_s.phase = 1u; it_s.drawn = -1;

    bool active = false;
    State s = it_s;
    PlayoutKey pk = {0u, 0u, 0u, 0u};
    uint32_t j = 0, leaf = 0, len = 0, winner = 0;
    uint64_t steps = 0;

    for (;;) {
        // ---- refill idle lanes from the current item --------------------
        uint64_t idle = __ballot(!active);
        while (idle != 0ull && !drained) {
            if (it_p == it_pend) {
                if (item == item_end) {
                    const uint32_t b = __builtin_amdgcn_readfirstlane(pending);
                    if ((uint64_t)b * a.batch >= a.n_items) { drained = true; break; }
                    item = b * a.batch;
                    item_end = min(item + a.batch, a.n_items);
                    if (lane == 0) pending = atomicAdd(&queue[0], 1u);
                }
                const uint32_t c = item++;
                it_leaf = c / a.parts;
                it_p = (c - it_leaf * a.parts) * a.item_chunk;
                it_pend = min(it_p + a.item_chunk, a.ppl);
                uint32_t w0, w1, w2, w3;
                load_uniform_state(a.leaves, it_leaf, w0, w1, w2, w3);
                const bool ok = decode(w0, w1, w2, w3, it_s);
                const uint32_t alive = alive_mask(it_s);
                if (!ok || __popc(alive) == 1) {
                    const int8_t wv = ok ? (int8_t)__builtin_ctz(alive) : (int8_t)-1;
                    const int16_t lv = ok ? (int16_t)0 : (int16_t)-1;
                    for (uint32_t p = it_p + lane; p < it_pend; p += 64u) {
                        const uint32_t jj = it_leaf * a.ppl + p;
                        if (a.winner) a.winner[jj] = wv;
                        if (a.length) a.length[jj] = lv;
                    }
                    if (lane == 0) {
                        if (!ok)
                            atomicOr(&g_error_word, kErrState);
                        else if (a.seat_wins)
                            atomicAdd(&a.seat_wins[(size_t)it_leaf * 4u + (uint32_t)wv],
                                      it_pend - it_p);
                    }
                    it_p = it_pend;
                    continue;
                }
                const uint64_t pl = (uint64_t)(a.leaf_base + it_leaf) * kPhiloxM1;
                it_pa = (uint32_t)(pl >> 32) ^ a.k0;
                it_pb = (uint32_t)pl;
            }
            const uint32_t take = min<uint32_t>((uint32_t)__popcll(idle), it_pend - it_p);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
            const bool mine = ((idle >> lane) & 1ull) && rank < take;
            if (mine) {
                const uint32_t p = it_p + rank;
                s = it_s;
                pk.a = it_pa ^ p;
                pk.b = it_pb;
                pk.gm_lo = 0u;
                pk.gm_hi = 0u;
                j = it_leaf * a.ppl + p;
                leaf = it_leaf;
                len = 0;
                active = true;
            }
            it_p += take;
            idle &= ~__ballot(mine);
        }
        if (__ballot(active) == 0ull) {
            if (drained) break;
            continue;
        }
        ++steps;

        // ---- one guess for every active lane ----------------------------
        bool over = false;
        if (active) {
            const Words w = step_words(pk, trk1, a.k0, a.k1);
            over = guess_step(s, w, winner, tab);
            next_step(pk);
            ++len;
            if (!over && len >= kMaxGuesses) {
                atomicOr(&g_error_word, kErrLimit);
                over = true;
                winner = 4u;
            }
        }

        // ---- finished games: outputs and per-leaf seat wins -------------
        const bool fin = active && over;
        if (fin) {
            if (a.winner) a.winner[j] = (int8_t)(winner < 4u ? (int)winner : -1);
            if (a.length) a.length[j] = (int16_t)len;
        }
        if (a.seat_wins) {
            uint64_t fmask = __ballot(fin);
            while (fmask != 0ull) {
                const uint32_t first = (uint32_t)__builtin_ctzll(fmask);
                const uint32_t L = __builtin_amdgcn_readlane(leaf, first);
                const bool mineL = fin && leaf == L;
                const uint64_t same = __ballot(mineL);
                const uint32_t c0 = (uint32_t)__popcll(__ballot(mineL && winner == 0u));
                const uint32_t c1 = (uint32_t)__popcll(__ballot(mineL && winner == 1u));
                const uint32_t c2 = (uint32_t)__popcll(__ballot(mineL && winner == 2u));
                const uint32_t c3 = (uint32_t)__popcll(__ballot(mineL && winner == 3u));
                if (lane < 4u) {
                    const uint32_t c = lane == 0u ? c0 : lane == 1u ? c1 : lane == 2u ? c2 : c3;
                    if (c) atomicAdd(&a.seat_wins[(size_t)L * 4u + lane], c);
                }
                fmask &= ~same;
            }
        }
        active = active && !over;
    }

    if (a.stats && lane == 0) atomicAdd(&a.stats[0], (unsigned long long)steps);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&queue[1], 1u);
        if (done == gridDim.x - 1u) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// Variant 4: K playouts per lane, back to back.
//
// Lane g runs playout ids g, g + S, ..., g + (K-1)S (S = lanes in the grid).
// When its game ends it starts the next one at once instead of waiting for
// the rest of the wave; the next leaf state is loaded while the current game
// runs, and outcomes stay packed in a register (7 bits per game) until the
// lane's last game, so the loop issues no stores and its only memory waits
// are for loads issued a game earlier.  Seat wins are summed across the wave
// with ballots at the end.  Meant for launches with a few playouts per lane
// at full occupancy; outputs equal every other variant's.
// ---------------------------------------------------------------------------
constexpr uint32_t kOutError = 0x7Fu;     // packed outcome of a malformed leaf

// Outputs of playout jj (packed outcome `code`: winner | length << 2, or
// kOutError), and the wave's seat wins summed per leaf with ballots, one
// atomic per (leaf, seat) present: to the table, or with `lsum` to the
// workgroup's LDS sums of leaves leaf0, leaf0 + 1, ...  Every lane of the
// wavefront takes part.
__device__ __forceinline__ void emit_outcome(const RolloutArgs &a, uint32_t jj, uint32_t code,
                                             uint32_t lane, uint32_t *lsum = nullptr,
                                             uint32_t leaf0 = 0u)
{
    const bool has = jj < a.total;
    const bool err = code == kOutError;
    const uint32_t w = code & 3u;
    if (has) {
        if (a.winner) a.winner[jj] = err ? (int8_t)-1 : (int8_t)w;
        if (a.length) a.length[jj] = err ? (int16_t)-1 : (int16_t)(code >> 2);
    }
    if (a.seat_wins) {
        const uint32_t lf = has ? jj / a.ppl : 0u;
        const bool fin = has && !err;
        uint64_t fmask = __ballot(fin);
        while (fmask != 0ull) {
            const uint32_t first = (uint32_t)__builtin_ctzll(fmask);
            const uint32_t L = __builtin_amdgcn_readlane(lf, first);
            const bool mineL = fin && lf == L;
            const uint64_t same = __ballot(mineL);
            const uint32_t c0 = (uint32_t)__popcll(__ballot(mineL && w == 0u));
            const uint32_t c1 = (uint32_t)__popcll(__ballot(mineL && w == 1u));
            const uint32_t c2 = (uint32_t)__popcll(__ballot(mineL && w == 2u));
            const uint32_t c3 = (uint32_t)__popcll(__ballot(mineL && w == 3u));
            if (lane < 4u) {
                const uint32_t c = lane == 0u ? c0 : lane == 1u ? c1 : lane == 2u ? c2 : c3;
                if (c) {
                    if (lsum) atomicAdd(&lsum[(L - leaf0) * 4u + lane], c);
                    else atomicAdd(&a.seat_wins[(size_t)L * 4u + lane], c);
                }
            }
            fmask &= ~same;
        }
    }
}

template <int K, bool PIPE>
__global__ void __launch_bounds__(256) rollout_static(RolloutArgs a)
{
    __shared__ uint8_t tab[kKthTableBytes];
    fill_kth_table(tab);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t S = gridDim.x * blockDim.x;
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t trk1 = a.tree ^ a.k1;

    uint32_t k = 0, j = g, leaf = 0, len = 0, winner = 0, packed = 0u;
    bool over = true, valid = false;
    State s;
    s.h0 = s.h1 = s.h2 = s.h3 = s.rev = 0u;
    s.m = 0u; s.P = 2u; s.phase = 1u; s.drawn = -1;
    PlayoutKey pk = {0u, 0u, 0u, 0u};
    Words wcur = {0u, 0u, 0u, 0u};
    uint4 next_st = make_uint4(0u, 0u, 0u, 0u);
    if (j < a.total) next_st = a.leaves[j / a.ppl];
    bool need_start = j < a.total;

    for (;;) {
        // start the lane's next game from the prefetched state
        if (need_start) {
            leaf = j / a.ppl;
            const uint32_t p = j - leaf * a.ppl;
            valid = decode(next_st.x, next_st.y, next_st.z, next_st.w, s);
            pk = playout_key(p, a.leaf_base + leaf, a.k0);
            if (PIPE) {
                wcur = step_words(pk, trk1, a.k0, a.k1);
                next_step(pk);
            }
            len = 0u;
            const uint32_t alive = alive_mask(s);
            winner = (uint32_t)__builtin_ctz(alive | 16u);
            over = !valid || __popc(alive) == 1;
            if (!valid) atomicOr(&g_error_word, kErrState);
            const uint32_t jn = j + S;
            if (k + 1u < (uint32_t)K && jn < a.total) next_st = a.leaves[jn / a.ppl];
            need_start = false;
        }
        const bool live = k < (uint32_t)K && j < a.total;
        if (__ballot(live) == 0ull) break;
        if (live && !over) {
            if (PIPE) {
                // the next step's words do not depend on the game: computing
                // them now overlaps their latency with this step's
                const Words wn = step_words(pk, trk1, a.k0, a.k1);
                next_step(pk);
                over = guess_step(s, wcur, winner, tab);
                wcur = wn;
            } else {
                const Words w = step_words(pk, trk1, a.k0, a.k1);
                over = guess_step(s, w, winner, tab);
                next_step(pk);
            }
            ++len;
            if (!over && len >= kMaxGuesses) {
                atomicOr(&g_error_word, kErrLimit);
                over = true;
                winner = 4u;
            }
        }
        if (live && over) {
            const uint32_t code = (!valid || winner > 3u) ? kOutError : (winner | (len << 2));
            packed |= code << (7u * k);
            ++k;
            j += S;
            need_start = k < (uint32_t)K && j < a.total;
        }
    }

    // outputs, and seat wins summed per leaf across the wave
#pragma unroll
    for (uint32_t kk = 0; kk < (uint32_t)K; ++kk)
        emit_outcome(a, g + kk * S, (packed >> (7u * kk)) & 0x7Fu, lane);
}

// ---------------------------------------------------------------------------
// Variant 7: one playout per lane, compacted at a few fixed step counts.
//
// Games end at different steps, and a wavefront runs until its longest game
// has ended (the divergence the paper blames for the GPU's scaling, Sec.
// IV-B).  At each checkpoint step the workgroup packs its unfinished games
// into its first lanes, in lane order, through LDS: a wavefront left with no
// game skips the rest of the loop, so later steps are issued for about as
// many wavefronts as there are games.  Every unfinished game has played
// exactly the checkpoint's number of steps, so the step counter (and the
// Philox counter word it feeds) stays uniform.  A game's packed outcome is
// recorded in LDS under its original slot; after the last step the outputs
// and seat wins are written per original slot exactly as variant 4 writes
// them, so every output equals the other variants'.
// ---------------------------------------------------------------------------
constexpr uint32_t kCompactSched[2][5] = {{6u, 9u, 12u, 0u, 0u}, {5u, 8u, 11u, 14u, 17u}};
constexpr int kCompactCount[2] = {3, 5};

// the packed format of a state already checked by decode()
__device__ __forceinline__ void unpack_valid(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                             State &s)
{
    const uint32_t b0 = w0 & kAll, b1 = w1 & kAll, b2 = w2 & kAll;
    s.h0 = b0 & ~b1 & ~b2;
    s.h1 = ~b0 & b1 & ~b2 & kAll;
    s.h2 = b0 & b1 & ~b2;
    s.h3 = b2;
    s.rev = w3 & kAll;
    s.m = (w0 >> 24) & 3u;
    s.P = ((w0 >> 26) & 3u) + 1u;
    s.phase = (w0 >> 28) & 1u;
    s.drawn = ((w0 >> 29) & 1u) ? (int32_t)((w1 >> 24) & 31u) : -1;
}

template <int SCHED>
__global__ void __launch_bounds__(256) rollout_compact(RolloutArgs a)
{
    constexpr int NCP = kCompactCount[SCHED];
    __shared__ uint8_t tab[kKthTableBytes];
    __shared__ uint32_t mig[7][256];       // packed state, playout id, round-1 key words
    __shared__ uint8_t outc[256];          // packed outcome per original slot
    __shared__ uint32_t wcnt[4];
    __shared__ uint32_t lsum[256 * 4];     // store_wins: seat wins of the workgroup's leaves
    fill_kth_table(tab);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t base = blockIdx.x * 256u;
    const uint32_t trk1 = a.tree ^ a.k1;

    uint32_t j = base + tid, winner = 0u;
    bool live = false;
    State s;
    s.h0 = s.h1 = s.h2 = s.h3 = s.rev = 0u;
    s.m = 0u; s.P = 2u; s.phase = 1u; s.drawn = -1;
    PlayoutKey pk = {0u, 0u, 0u, 0u};
    outc[tid] = (uint8_t)kOutError;
    if (a.store_wins) {
#pragma unroll
        for (uint32_t q = 0; q < 4u; ++q) lsum[4u * tid + q] = 0u;
    }
    if (j < a.total) {
        const uint32_t leaf = j / a.ppl;
        const uint4 st = a.leaves[leaf];
        if (!decode(st.x, st.y, st.z, st.w, s)) {
            atomicOr(&g_error_word, kErrState);
        } else {
            const uint32_t alive = alive_mask(s);
            winner = (uint32_t)__builtin_ctz(alive | 16u);
            if (__popc(alive) == 1) {
                outc[tid] = (uint8_t)winner;          // decided before any guess
            } else {
                live = true;
                pk = playout_key(j - leaf * a.ppl, a.leaf_base + leaf, a.k0);
            }
        }
    }
    __syncthreads();   // k-th-bit table ready

#pragma unroll
    for (int seg = 0; seg <= NCP; ++seg) {
        const uint32_t first = seg == 0 ? 0u : kCompactSched[SCHED][seg - 1];
        const uint32_t limit = seg < NCP ? kCompactSched[SCHED][seg] : kMaxGuesses;
        for (uint32_t step = first; step < limit; ++step) {
            if (__ballot(live) == 0ull) break;
            if (live) {
                const Words w = step_words(pk, trk1, a.k0, a.k1);
                const bool over = guess_step(s, w, winner, tab);
                next_step(pk);
                if (over) {
                    outc[j - base] = (uint8_t)(winner | ((step + 1u) << 2));
                    live = false;
                }
            }
        }
        if (seg == NCP) {
            // still undecided after the most guesses a valid game can take
            if (live) atomicOr(&g_error_word, kErrLimit);
            break;
        }
        // pack the unfinished games into the first lanes of the workgroup
        const uint64_t lm = __ballot(live);
        if (lane == 0u) wcnt[wv] = (uint32_t)__popcll(lm);
        __syncthreads();
        uint32_t before = 0u, n_live = 0u;
#pragma unroll
        for (uint32_t w = 0; w < 4u; ++w) {
            const uint32_t c = wcnt[w];
            before += w < wv ? c : 0u;
            n_live += c;
        }
        if (live) {
            const uint32_t dst = before + __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(lm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)lm, 0u));
            uint32_t e0, e1, e2, e3;
            encode(s, e0, e1, e2, e3);
            mig[0][dst] = e0;
            mig[1][dst] = e1;
            mig[2][dst] = e2;
            mig[3][dst] = e3;
            mig[4][dst] = j;
            mig[5][dst] = pk.a;
            mig[6][dst] = pk.b;
        }
        __syncthreads();
        live = tid < n_live;
        if (live) {
            unpack_valid(mig[0][tid], mig[1][tid], mig[2][tid], mig[3][tid], s);
            j = mig[4][tid];
            pk.a = mig[5][tid];
            pk.b = mig[6][tid];
            const uint64_t gm = (uint64_t)limit * kPhiloxM0;   // the step counter times M0
            pk.gm_lo = (uint32_t)gm;
            pk.gm_hi = (uint32_t)(gm >> 32);
        }
    }
    __syncthreads();   // every game's outcome is in outc
    if (!a.store_wins) {
        emit_outcome(a, base + tid, outc[tid], lane);
        return;
    }
    // the workgroup holds whole leaves (ppl divides 256): sum them in LDS and
    // store each leaf's four counts once, over whatever the table held
    const uint32_t leaf0 = base / a.ppl;
    emit_outcome(a, base + tid, outc[tid], lane, lsum, leaf0);
    __syncthreads();
    const uint32_t last = (base + 255u < a.total ? base + 255u : a.total - 1u) / a.ppl;
    const uint32_t nw4 = 4u * (last - leaf0 + 1u);
    if (a.seat_wins)
        for (uint32_t e = tid; e < nw4; e += 256u) a.seat_wins[(size_t)leaf0 * 4u + e] = lsum[e];
}

// ---------------------------------------------------------------------------
// Variant 8: variant 7 with two games per lane, advanced together.
//
// A guess step is one long chain of dependent operations (the Philox rounds,
// then the table lookups of the guess); a lane that carries two games issues
// two independent chains side by side, so a wavefront has work to issue while
// either chain waits.  A workgroup of 256 lanes holds 512 games: game slot k
// lives in lane k / 2 (k even: first game, odd: second).  Both games of a
// lane run every step; a finished game's step is computed and discarded (its
// outcome was recorded when it ended), so the step needs no branch.  At
// steps 5, 8, 11, 14, 17 the workgroup packs its unfinished games into its first
// slots, in slot order, exactly as variant 7 does with one game per lane, so
// a wavefront whose 128 slots are empty stops issuing.  Outputs per original
// slot, identical to every other variant's.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) rollout_compact2(RolloutArgs a)
{
    constexpr int NCP = kCompactCount[1];
    __shared__ uint8_t tab[kKthTableBytes];
    __shared__ uint32_t mig[7][512];       // packed state, playout id, round-1 key words
    __shared__ uint8_t outc[512];          // packed outcome per original slot
    __shared__ uint32_t wcnt[4];
    __shared__ uint32_t lsum[512 * 4];     // store_wins: seat wins of the workgroup's leaves
    fill_kth_table(tab);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t base = blockIdx.x * 512u;
    const uint32_t trk1 = a.tree ^ a.k1;

    // game g of the lane (g = 0, 1): slot 2 tid + g
    uint32_t j[2], winner[2] = {0u, 0u};
    bool live[2] = {false, false};
    State s[2];
    PlayoutKey pk[2];
#pragma unroll
    for (uint32_t g = 0; g < 2u; ++g) {
        j[g] = base + 2u * tid + g;
        s[g].h0 = s[g].h1 = s[g].h2 = s[g].h3 = s[g].rev = 0u;
        s[g].m = 0u; s[g].P = 2u; s[g].phase = 1u; s[g].drawn = -1;
        pk[g] = PlayoutKey{0u, 0u, 0u, 0u};
        outc[2u * tid + g] = (uint8_t)kOutError;
    }
    if (a.store_wins) {
#pragma unroll
        for (uint32_t q = 0; q < 8u; ++q) lsum[8u * tid + q] = 0u;
    }
#pragma unroll
    for (uint32_t g = 0; g < 2u; ++g) {
        if (j[g] < a.total) {
            const uint32_t leaf = j[g] / a.ppl;
            const uint4 st = a.leaves[leaf];
            if (!decode(st.x, st.y, st.z, st.w, s[g])) {
                atomicOr(&g_error_word, kErrState);
            } else {
                const uint32_t alive = alive_mask(s[g]);
                winner[g] = (uint32_t)__builtin_ctz(alive | 16u);
                if (__popc(alive) == 1) {
                    outc[j[g] - base] = (uint8_t)winner[g];   // decided before any guess
                } else {
                    live[g] = true;
                    pk[g] = playout_key(j[g] - leaf * a.ppl, a.leaf_base + leaf, a.k0);
                }
            }
        }
    }
    __syncthreads();   // k-th-bit table ready

#pragma unroll
    for (int seg = 0; seg <= NCP; ++seg) {
        const uint32_t first = seg == 0 ? 0u : kCompactSched[1][seg - 1];
        const uint32_t limit = seg < NCP ? kCompactSched[1][seg] : kMaxGuesses;
        for (uint32_t step = first; step < limit; ++step) {
            if (__ballot(live[0] | live[1]) == 0ull) break;
            const Words w0 = step_words(pk[0], trk1, a.k0, a.k1);
            const Words w1 = step_words(pk[1], trk1, a.k0, a.k1);
            uint32_t wn0 = winner[0], wn1 = winner[1];
            const bool over0 = guess_step(s[0], w0, wn0, tab);
            const bool over1 = guess_step(s[1], w1, wn1, tab);
            next_step(pk[0]);
            next_step(pk[1]);
            if (live[0] && over0) {
                outc[j[0] - base] = (uint8_t)(wn0 | ((step + 1u) << 2));
                live[0] = false;
            }
            if (live[1] && over1) {
                outc[j[1] - base] = (uint8_t)(wn1 | ((step + 1u) << 2));
                live[1] = false;
            }
        }
        if (seg == NCP) {
            // still undecided after the most guesses a valid game can take
            if (live[0] | live[1]) atomicOr(&g_error_word, kErrLimit);
            break;
        }
        // pack the unfinished games into the first slots of the workgroup,
        // in slot order (lane order, first game before second)
        const uint64_t l0 = __ballot(live[0]), l1 = __ballot(live[1]);
        if (lane == 0u) wcnt[wv] = (uint32_t)(__popcll(l0) + __popcll(l1));
        __syncthreads();
        uint32_t before = 0u, n_live = 0u;
#pragma unroll
        for (uint32_t w = 0; w < 4u; ++w) {
            const uint32_t c = wcnt[w];
            before += w < wv ? c : 0u;
            n_live += c;
        }
        const uint32_t below =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(l0 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)l0, 0u)) +
            __builtin_amdgcn_mbcnt_hi((uint32_t)(l1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)l1, 0u));
#pragma unroll
        for (uint32_t g = 0; g < 2u; ++g) {
            if (live[g]) {
                const uint32_t dst = before + below + (g == 1u && live[0] ? 1u : 0u);
                uint32_t e0, e1, e2, e3;
                encode(s[g], e0, e1, e2, e3);
                mig[0][dst] = e0;
                mig[1][dst] = e1;
                mig[2][dst] = e2;
                mig[3][dst] = e3;
                mig[4][dst] = j[g];
                mig[5][dst] = pk[g].a;
                mig[6][dst] = pk[g].b;
            }
        }
        __syncthreads();
        const uint64_t gm = (uint64_t)limit * kPhiloxM0;   // the step counter times M0
#pragma unroll
        for (uint32_t g = 0; g < 2u; ++g) {
            const uint32_t k = 2u * tid + g;
            live[g] = k < n_live;
            if (live[g]) {
                unpack_valid(mig[0][k], mig[1][k], mig[2][k], mig[3][k], s[g]);
                j[g] = mig[4][k];
                pk[g].a = mig[5][k];
                pk[g].b = mig[6][k];
                pk[g].gm_lo = (uint32_t)gm;
                pk[g].gm_hi = (uint32_t)(gm >> 32);
            }
        }
    }
    __syncthreads();   // every game's outcome is in outc
    if (!a.store_wins) {
        emit_outcome(a, base + tid, outc[tid], lane);
        emit_outcome(a, base + 256u + tid, outc[256u + tid], lane);
        return;
    }
    // the workgroup holds whole leaves (ppl divides 512): sum them in LDS and
    // store each leaf's four counts once, over whatever the table held
    const uint32_t leaf0 = base / a.ppl;
    emit_outcome(a, base + tid, outc[tid], lane, lsum, leaf0);
    emit_outcome(a, base + 256u + tid, outc[256u + tid], lane, lsum, leaf0);
    __syncthreads();
    const uint32_t last = (base + 511u < a.total ? base + 511u : a.total - 1u) / a.ppl;
    const uint32_t nw4 = 4u * (last - leaf0 + 1u);
    if (a.seat_wins)
        for (uint32_t e = tid; e < nw4; e += 256u) a.seat_wins[(size_t)leaf0 * 4u + e] = lsum[e];
}

// ---------------------------------------------------------------------------
// Variant 9: variant 7's compaction, with the lanes it frees refilled.
//
// Compaction alone retires a wavefront once its workgroup's games fit in
// fewer lanes, and a new workgroup starts only when a whole workgroup's
// wavefront slots are free: at 1M playouts the SIMDs held 4.4 wavefronts on
// average against the 8 their registers allow.  Here a workgroup owns `span`
// consecutive playouts (256 K): its lanes start on the first 256, and every
// kRefillCheck steps the unfinished games are packed into the first lanes
// (in lane order, through LDS) and the lanes behind them start the range's
// next playouts, so the wavefronts stay full until the range runs out and
// the whole grid can be resident at once.  Each game carries its own number
// of guesses, which sets its Philox step counter and its length.  Outcomes
// are kept per playout of the range in LDS and written out as variant 7
// writes them, so every output equals the other variants'.
// ---------------------------------------------------------------------------
constexpr uint32_t kRefillCheck = 4u;        // guesses between checkpoints
constexpr uint32_t kRefillMaxSpan = 512u;    // playouts per workgroup
constexpr uint32_t kRefillLeafCache = 16u;   // leaf states of the range kept in LDS

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
rollout_compact_refill(RolloutArgs a, uint32_t span)
{
    __shared__ uint8_t tab[kKthTableBytes];
    __shared__ uint32_t mig[8][256];   // packed state, playout id, round-1 key words, guesses
    __shared__ uint8_t outc[kRefillMaxSpan];
    __shared__ uint4 leafst[kRefillLeafCache];
    __shared__ uint32_t lsum[kRefillLeafCache * 4u];   // store_wins: seat wins per leaf
    __shared__ uint32_t wcnt[4];
    fill_kth_table(tab);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t base = blockIdx.x * span;          // < total: the grid covers it exactly
    const uint32_t end = a.total - base < span ? a.total : base + span;
    const uint32_t leaf0 = base / a.ppl, nleaf = (end - 1u) / a.ppl - leaf0 + 1u;
    const bool cached = nleaf <= kRefillLeafCache;    // else leaf states from memory
    if (cached && tid < nleaf) leafst[tid] = a.leaves[leaf0 + tid];
    for (uint32_t i = tid; i < span; i += 256u) outc[i] = (uint8_t)kOutError;
    if (tid < 4u * kRefillLeafCache) lsum[tid] = 0u;
    const uint32_t trk1 = a.tree ^ a.k1;
    __syncthreads();   // table, leaf states, outcomes

    uint32_t j = 0u, winner = 0u, len = 0u;
    bool live = false;
    State s;
    s.h0 = s.h1 = s.h2 = s.h3 = s.rev = 0u;
    s.m = 0u; s.P = 2u; s.phase = 1u; s.drawn = -1;
    PlayoutKey pk = {0u, 0u, 0u, 0u};
    // playout jj of the range starts in this lane (a game decided before any
    // guess is recorded at once; a malformed leaf keeps the error outcome)
    auto start = [&](uint32_t jj) __attribute__((always_inline)) {
        j = jj;
        len = 0u;
        const uint32_t leaf = jj / a.ppl;
        const uint4 st = cached ? leafst[leaf - leaf0] : a.leaves[leaf];
        if (!decode(st.x, st.y, st.z, st.w, s)) {
            atomicOr(&g_error_word, kErrState);
            return;
        }
        const uint32_t alive = alive_mask(s);
        winner = (uint32_t)__builtin_ctz(alive | 16u);
        if (__popc(alive) == 1) {
            outc[jj - base] = (uint8_t)winner;
            return;
        }
        live = true;
        pk = playout_key(jj - leaf * a.ppl, a.leaf_base + leaf, a.k0);
    };
    if (base + tid < end) start(base + tid);
    uint32_t next = base + 256u;   // the range's next playout to start
    for (;;) {
        for (uint32_t c = 0; c < kRefillCheck; ++c) {
            if (__ballot(live) == 0ull) break;
            if (live) {
                const Words w = step_words(pk, trk1, a.k0, a.k1);
                const bool over = guess_step(s, w, winner, tab);
                next_step(pk);
                ++len;
                if (over) {
                    outc[j - base] = (uint8_t)(winner | (len << 2));
                    live = false;
                } else if (len >= kMaxGuesses) {
                    // still undecided after the most guesses a valid game can take
                    atomicOr(&g_error_word, kErrLimit);
                    live = false;
                }
            }
        }
        // pack the unfinished games into the first lanes, refill the rest
        const uint64_t lm = __ballot(live);
        if (lane == 0u) wcnt[wv] = (uint32_t)__popcll(lm);
        __syncthreads();
        uint32_t before = 0u, n_live = 0u;
#pragma unroll
        for (uint32_t w = 0; w < 4u; ++w) {
            const uint32_t c = wcnt[w];
            before += w < wv ? c : 0u;
            n_live += c;
        }
        if (n_live == 0u && next >= end) break;   // the same in every lane
        if (live) {
            const uint32_t dst = before + __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(lm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)lm, 0u));
            uint32_t e0, e1, e2, e3;
            encode(s, e0, e1, e2, e3);
            mig[0][dst] = e0;
            mig[1][dst] = e1;
            mig[2][dst] = e2;
            mig[3][dst] = e3;
            mig[4][dst] = j;
            mig[5][dst] = pk.a;
            mig[6][dst] = pk.b;
            mig[7][dst] = len;
        }
        __syncthreads();
        live = tid < n_live;
        if (live) {
            unpack_valid(mig[0][tid], mig[1][tid], mig[2][tid], mig[3][tid], s);
            j = mig[4][tid];
            pk.a = mig[5][tid];
            pk.b = mig[6][tid];
            len = mig[7][tid];
            const uint64_t gm = (uint64_t)len * kPhiloxM0;   // the step counter times M0
            pk.gm_lo = (uint32_t)gm;
            pk.gm_hi = (uint32_t)(gm >> 32);
        } else if (next + (tid - n_live) < end) {
            start(next + (tid - n_live));
        }
        next += 256u - n_live;
    }
    __syncthreads();   // every game's outcome is in outc
    const bool store = a.store_wins != 0u && cached;
    for (uint32_t i = tid; i < span; i += 256u)
        emit_outcome(a, base + i, outc[i], lane, store ? lsum : nullptr, leaf0);
    if (!store) return;
    // the workgroup holds whole leaves: store each leaf's four counts once,
    // over whatever the table held
    __syncthreads();
    if (a.seat_wins && tid < 4u * nleaf) a.seat_wins[(size_t)leaf0 * 4u + tid] = lsum[tid];
}

// ---------------------------------------------------------------------------
// Variant 5: one wavefront per single-leaf item of up to 64*K playouts.  A
// lane whose game ended takes the item's next playout at once (ballot +
// mbcnt prefix over the lanes that finished); the leaf's start state stays
// in registers, so a restart is a handful of register moves and no memory
// access.  Lanes idle only while the item's last games finish.  Seat wins
// are counted per lane in two registers of 16-bit fields and summed across
// the wave once at the end.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) rollout_refill(RolloutArgs a)
{
    __shared__ uint8_t tab[kKthTableBytes];
    fill_kth_table(tab);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t item = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (item >= a.n_items) return;                       // whole wavefront
    const uint32_t leaf = item / a.parts;
    const uint32_t p0 = (item - leaf * a.parts) * a.item_chunk;
    const uint32_t p1 = min(p0 + a.item_chunk, a.ppl);
    uint32_t w0, w1, w2, w3;
    load_uniform_state(a.leaves, leaf, w0, w1, w2, w3);
    State s0;
    const bool ok = decode(w0, w1, w2, w3, s0);
    const uint32_t alive0 = alive_mask(s0);
    if (!ok || __popc(alive0) == 1) {
        // a decided or malformed leaf finishes the whole item at once
        const int8_t wv = ok ? (int8_t)__builtin_ctz(alive0) : (int8_t)-1;
        const int16_t lv = ok ? (int16_t)0 : (int16_t)-1;
        for (uint32_t p = p0 + lane; p < p1; p += 64u) {
            const uint32_t j = leaf * a.ppl + p;
            if (a.winner) a.winner[j] = wv;
            if (a.length) a.length[j] = lv;
        }
        if (lane == 0) {
            if (!ok)
                atomicOr(&g_error_word, kErrState);
            else if (a.seat_wins)
                atomicAdd(&a.seat_wins[(size_t)leaf * 4u + (uint32_t)wv], p1 - p0);
        }
        return;
    }
    const uint32_t trk1 = a.tree ^ a.k1;
    const uint64_t pl = (uint64_t)(a.leaf_base + leaf) * kPhiloxM1;
    const uint32_t ka = (uint32_t)(pl >> 32) ^ a.k0, kb = (uint32_t)pl;
    uint32_t p = p0 + lane;
    bool active = p < p1;
    uint32_t next = p0 + 64u;                             // wave-uniform
    State s = s0;
    PlayoutKey pk = {ka ^ p, kb, 0u, 0u};
    uint32_t len = 0u, winner = 0u;
    uint32_t wins01 = 0u, wins23 = 0u;                    // 16-bit counters
    while (__ballot(active) != 0ull) {
        bool over = false;
        if (active) {
            const Words w = step_words(pk, trk1, a.k0, a.k1);
            over = guess_step(s, w, winner, tab);
            next_step(pk);
            ++len;
            if (!over && len >= kMaxGuesses) {
                atomicOr(&g_error_word, kErrLimit);
                over = true;
                winner = 4u;
            }
        }
        const uint64_t fin = __ballot(over);
        if (fin != 0ull) {
            if (over) {
                const uint32_t j = leaf * a.ppl + p;
                if (a.winner) a.winner[j] = winner < 4u ? (int8_t)winner : (int8_t)-1;
                if (a.length) a.length[j] = (int16_t)len;
                const uint32_t inc = winner < 4u ? 1u << ((winner & 1u) * 16u) : 0u;
                if (winner < 2u) wins01 += inc; else wins23 += inc;
            }
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(fin >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fin, 0u));
            const uint32_t np = next + rank;
            next += (uint32_t)__popcll(fin);
            if (over) {
                p = np;
                active = np < p1;
                s = s0;
                pk.a = ka ^ np;
                pk.b = kb;
                pk.gm_lo = 0u;
                pk.gm_hi = 0u;
                len = 0u;
            }
        }
    }
    if (a.seat_wins) {
        for (int off = 32; off > 0; off >>= 1) {
            wins01 += __shfl_xor(wins01, off, 64);
            wins23 += __shfl_xor(wins23, off, 64);
        }
        if (lane < 4u) {
            const uint32_t c = lane == 0u ? wins01 & 0xFFFFu : lane == 1u ? wins01 >> 16
                             : lane == 2u ? wins23 & 0xFFFFu : wins23 >> 16;
            if (c) atomicAdd(&a.seat_wins[(size_t)leaf * 4u + lane], c);
        }
    }
}

__global__ void fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_rollout(const RolloutArgs &a, int variant, int block, int grid, hipStream_t st)
{
    if (a.total == 0) return hipSuccess;
    if (variant == 1) {
        const uint32_t blocks = (a.total + 255u) / 256u;
        hipLaunchKernelGGL(rollout_lane_per_playout, dim3(blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    if (variant == 6) {
        // variant 4 with one playout per lane and the next step's random
        // words computed during the current step
        const uint32_t blocks = (a.total + 255u) / 256u;
        hipLaunchKernelGGL((rollout_static<1, true>), dim3(blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    if (variant == 4) {
        // playouts per lane (1, 2 or 4); automatic = 1: more playouts per
        // lane only lengthened the launch at every size measured (1M to 67M
        // playouts), the hardware refilling finished waves being cheaper
        int kk = grid > 0 ? grid : 1;
        kk = kk < 1 ? 1 : (kk > 4 ? 4 : kk);
        if (kk == 3) kk = 4;
        const uint32_t per_block = 256u * (uint32_t)kk;
        const uint32_t blocks = (uint32_t)((a.total + per_block - 1u) / per_block);
        switch (kk) {
        case 1: hipLaunchKernelGGL((rollout_static<1, false>), dim3(blocks), dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((rollout_static<2, false>), dim3(blocks), dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((rollout_static<4, false>), dim3(blocks), dim3(256), 0, st, a); break;
        }
        return hipGetLastError();
    }
    if (variant == 7) {
        // one playout per lane, compacted at steps 6, 9, 12 (grid 0 or 1) or
        // 5, 8, 11, 14, 17 (grid 2)
        const uint32_t blocks = (a.total + 255u) / 256u;
        if (grid == 2)
            hipLaunchKernelGGL(rollout_compact<1>, dim3(blocks), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL(rollout_compact<0>, dim3(blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    if (variant == 8) {
        // two games per lane, compacted at steps 5, 8, 11, 14, 17
        const uint32_t blocks = (a.total + 511u) / 512u;
        hipLaunchKernelGGL(rollout_compact2, dim3(blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    if (variant == 9) {
        // K = grid (1 or 2, default 2) batches of 256 playouts per workgroup,
        // compacted and refilled every four guesses
        const uint32_t span = 256u * (grid == 1 ? 1u : 2u);
        const uint32_t blocks = (uint32_t)((a.total + span - 1u) / span);
        hipLaunchKernelGGL(rollout_compact_refill, dim3(blocks), dim3(256), 0, st, a, span);
        return hipGetLastError();
    }
    if (variant == 5) {
        // one wavefront per item, four per workgroup
        const uint32_t blocks = (a.n_items + 3u) / 4u;
        hipLaunchKernelGGL(rollout_refill, dim3(blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    int waves = block > 0 ? block / 64 : 4;
    if (grid <= 0) grid = default_rollout_grid(waves);
    if (variant == 3) {
        switch (waves) {
        case 1: hipLaunchKernelGGL(rollout_items<1>, dim3(grid), dim3(64), 0, st, a); break;
        case 2: hipLaunchKernelGGL(rollout_items<2>, dim3(grid), dim3(128), 0, st, a); break;
        case 4: hipLaunchKernelGGL(rollout_items<4>, dim3(grid), dim3(256), 0, st, a); break;
        case 8: hipLaunchKernelGGL(rollout_items<8>, dim3(grid), dim3(512), 0, st, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (waves) {
    case 1: hipLaunchKernelGGL(rollout_persistent<1>, dim3(grid), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL(rollout_persistent<2>, dim3(grid), dim3(128), 0, st, a); break;
    case 4: hipLaunchKernelGGL(rollout_persistent<4>, dim3(grid), dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL(rollout_persistent<8>, dim3(grid), dim3(512), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dvc
