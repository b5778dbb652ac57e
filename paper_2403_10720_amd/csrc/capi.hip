// capi.hip -- the extern "C" entry points declared in include/dvc.h:
// argument checks, launch-shape choice and kernel launches on the caller's
// stream.  Nothing here allocates per call.
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "dvc.h"
#include "dvc_internal.hpp"

namespace dvc {

static std::atomic<uint32_t> g_next_slot{0};

// the network blob and the workspaces are read as 16-byte fragments
static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0u; }

uint32_t next_queue_slot()
{
    return g_next_slot.fetch_add(1u, std::memory_order_relaxed) % (uint32_t)kQueueSlots;
}

static int device_cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

int default_rollout_grid(int waves_per_block)
{
    // two waves per SIMD: four SIMDs per compute unit
    const int waves = device_cu_count() * 4 * 2;
    return (waves + waves_per_block - 1) / waves_per_block;
}

static int status_of(hipError_t e) { return e == hipSuccess ? DVC_OK : DVC_EHIP; }

// LN[k] = float(log(double(k))): the natural-log table of the UCT score, built
// on the host once and kept on every device that runs a search.  Tables that
// are outgrown stay allocated (a search still running may read them).
static std::mutex g_ln_mutex;
static std::vector<float> g_ln_host;
static float *g_ln_dev[64] = {nullptr};
static uint64_t g_ln_size[64] = {0};

static const float *ln_table(uint64_t need, int *status)
{
    std::lock_guard<std::mutex> lock(g_ln_mutex);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        *status = DVC_EHIP;
        return nullptr;
    }
    if (g_ln_size[dev] >= need) return g_ln_dev[dev];
    uint64_t cap = 1ull << 20;
    while (cap < need) cap <<= 1;
    if (g_ln_host.size() < cap) {
        const uint64_t old = g_ln_host.size();
        g_ln_host.resize(cap);
        for (uint64_t k = old; k < cap; ++k)
            g_ln_host[k] = k == 0 ? 0.0f : (float)std::log((double)k);
    }
    float *p = nullptr;
    if (hipMalloc(&p, cap * sizeof(float)) != hipSuccess) {
        *status = DVC_ENOMEM;
        return nullptr;
    }
    if (hipMemcpy(p, g_ln_host.data(), cap * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p);   // never handed out; the copy failure is what gets reported
        *status = DVC_EHIP;
        return nullptr;
    }
    g_ln_dev[dev] = p;
    g_ln_size[dev] = cap;
    return p;
}

// Philox4x32-10 on the host (Salmon et al., SC'11), for the few words the
// host itself draws: ten rounds of two 32x32->64 multiplies, the key advanced
// by the Weyl constants between rounds.
static void philox_host(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)x0 * 0xD2511F53u, p1 = (uint64_t)x2 * 0xCD9E8D57u;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0, y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

// playouts per leaf x leaves per pass candidates of the search autotuner:
// every pass holds at most 64 playouts (the tree's wavefront), plus one leaf
// per pass with 64 and 128 playouts; each shape is tried with and without
// pipelined passes
struct SearchShape {
    int32_t ppl, lpp, pipe;
};
static const SearchShape kSearchCandidates[] = {
    {4, 1, 0}, {4, 2, 0}, {4, 4, 0}, {4, 8, 0}, {4, 16, 0}, {8, 1, 0}, {8, 2, 0}, {8, 4, 0},
    {8, 8, 0}, {16, 1, 0}, {16, 2, 0}, {16, 4, 0}, {32, 1, 0}, {32, 2, 0}, {64, 1, 0},
    {128, 1, 0}, {4, 1, 1}, {4, 2, 1}, {4, 4, 1}, {4, 8, 1}, {4, 16, 1}, {8, 1, 1}, {8, 2, 1},
    {8, 4, 1}, {8, 8, 1}, {16, 1, 1}, {16, 2, 1}, {16, 4, 1}, {32, 1, 1}, {32, 2, 1},
    {64, 1, 1}, {128, 1, 1}};
constexpr int32_t kAutoMaxPpl = 128;

static bool is_auto(const dvc_mcts_params *p)
{
    return p->leaf_eval == 0 && p->playouts_per_leaf == 0 && p->leaves_per_pass == 0 &&
           p->pipeline == 0;
}

static bool mcts_params_ok(const dvc_mcts_params *p)
{
    if (p == nullptr) return false;
    const bool aut = is_auto(p);
    if (p->iterations < 1 || (p->playouts_per_leaf < 1 && !aut) || p->max_depth < 0 ||
        p->max_depth > 64)
        return false;
    if ((p->continue_choice != 0 && p->continue_choice != 1) || (p->vanilla != 0 && p->vanilla != 1))
        return false;
    // pipelined passes keep no world nodes
    if ((p->pipeline != 0 && p->pipeline != 1) || (p->pipeline && p->vanilla)) return false;
    // leaves evaluated together: value mode fits four leaves' perspectives in
    // one matrix tile, playout mode packs up to 16 leaves' playouts
    if (!aut && (p->leaves_per_pass < 1 || p->leaves_per_pass > (p->leaf_eval ? 4 : 16)))
        return false;
    if (!(p->c_uct >= 0.0f) || std::isinf(p->c_uct)) return false;
    if (p->leaf_eval != 0 && p->leaf_eval != 1) return false;
    if (p->leaf_eval == 1 && (p->valuenet == nullptr || !aligned16(p->valuenet) ||
                              p->fallback_playouts < 1 || !(p->fallback_band >= 0.0f)))
        return false;
    // visit counts stay exact in float (an automatic shape may take up to
    // kAutoMaxPpl playouts per leaf)
    const uint64_t w_leaf = (uint64_t)(p->leaf_eval ? p->fallback_playouts
                                       : aut ? kAutoMaxPpl : p->playouts_per_leaf);
    if ((uint64_t)p->iterations * w_leaf >= (1ull << 24)) return false;
    return true;
}

// the autotuner's choices: (device, log2 trees, log2 iterations, max depth,
// continue choice, vanilla) -> (playouts per leaf, leaves per pass,
// pipelined passes)
static std::mutex g_search_tune_mutex;
static std::map<std::tuple<int, int, int, int, int, int>, SearchShape> g_search_tuned;

static int floor_log2(uint64_t x)
{
    int lg = 0;
    while ((2ull << lg) <= x) ++lg;
    return lg;
}

static std::tuple<int, int, int, int, int, int> search_key(int64_t n_trees,
                                                           const dvc_mcts_params *p)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    return std::make_tuple(dev, floor_log2((uint64_t)(n_trees > 0 ? n_trees : 1)),
                           floor_log2((uint64_t)p->iterations), p->max_depth, p->continue_choice,
                           p->vanilla);
}

// The parameters a search runs with: an automatic shape (playout leaves,
// playouts per leaf, leaves per pass and pipeline all 0) becomes the
// autotuner's choice for this size class, else 32 playouts with two leaves
// per pass, not pipelined (the fastest shape within two points of the
// sequential 32-playout search's self-agreement on 2048 mixed mid-game
// roots x 1024 iterations, measured on gfx950 before pipelined passes).
static dvc_mcts_params resolved(const dvc_mcts_params *p, int64_t n_trees)
{
    dvc_mcts_params r = *p;
    if (!is_auto(p)) return r;
    SearchShape sh{32, 2, 0};
    {
        std::lock_guard<std::mutex> lock(g_search_tune_mutex);
        auto it = g_search_tuned.find(search_key(n_trees, p));
        if (it != g_search_tuned.end()) sh = it->second;
    }
    r.playouts_per_leaf = sh.ppl;
    r.leaves_per_pass = sh.lpp;
    r.pipeline = sh.pipe;
    return r;
}

}  // namespace dvc

using namespace dvc;

extern "C" {

const char *dvc_version(void) { return "dvc-gfx950 0.1"; }

const char *dvc_status_str(int status)
{
    switch (status) {
    case DVC_OK: return "ok";
    case DVC_EINVAL: return "invalid argument";
    case DVC_ESTATE: return "malformed game state";
    case DVC_EHIP: return "HIP runtime error";
    case DVC_ENOMEM: return "workspace too small or allocation failed";
    case DVC_ELIMIT: return "internal bound reached";
    case DVC_ETOOBIG: return "request exceeds the static scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

int dvc_check(void *stream)
{
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return DVC_EHIP;
    uint32_t w = 0u, zero = 0u;
    if (hipMemcpyFromSymbol(&w, HIP_SYMBOL(g_error_word), sizeof(w), 0, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return DVC_EHIP;
    if (w != 0u &&
        hipMemcpyToSymbol(HIP_SYMBOL(g_error_word), &zero, sizeof(zero), 0, hipMemcpyHostToDevice) !=
            hipSuccess)
        return DVC_EHIP;
    if (w & kErrState) return DVC_ESTATE;
    if (w & kErrLimit) return DVC_ELIMIT;
    return DVC_OK;
}

int dvc_init_states(dvc_state_t *out, int64_t n, const dvc_deal_params *p, uint64_t seed,
                    uint32_t index_base, void *stream)
{
    if (n < 0 || n >= (1ll << 32) || p == nullptr || (n > 0 && out == nullptr)) return DVC_EINVAL;
    if (p->p_min < 2 || p->p_max > 4 || p->p_min > p->p_max) return DVC_EINVAL;
    for (int P = p->p_min; P <= p->p_max; ++P)
        if (p->hand[P] < 1 || P * p->hand[P] > 24) return DVC_EINVAL;
    if (p->pile_min < 0 || p->pile_max < 0 || p->revealed_max < 0) return DVC_EINVAL;
    DealArgs d;
    d.p_min = p->p_min;
    d.p_max = p->p_max;
    for (int k = 0; k < 5; ++k) d.hand[k] = p->hand[k];
    d.pile_min = p->pile_min;
    d.pile_max = p->pile_max;
    d.revealed_max = p->revealed_max;
    d.fresh = p->fresh;
    d.root_draw = p->root_draw;
    d.phase_mix = p->phase_mix;
    return status_of(launch_init_states(reinterpret_cast<uint4 *>(out), (uint32_t)n, d,
                                        (uint32_t)seed, (uint32_t)(seed >> 32), index_base,
                                        (hipStream_t)stream));
}

// ---------------------------------------------------------------------------
// rollout launch shapes: an explicit variant, else the autotuner's choice for
// the batch's size class on this device, else a rule from measurements
// ---------------------------------------------------------------------------
struct Shape {
    int variant, block, grid;
};

static std::mutex g_tune_mutex;
static std::map<std::tuple<int, int, int>, Shape> g_tuned;   // (device, log2 total, ppl class)

static std::tuple<int, int, int> tune_key(uint64_t total, int32_t ppl)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    int lg = 0;
    while ((2ull << lg) <= total) ++lg;
    return std::make_tuple(dev, lg, ppl >= 256 ? 2 : ppl >= 64 ? 1 : 0);
}

static Shape automatic_shape(uint64_t total, int32_t ppl)
{
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        auto it = g_tuned.find(tune_key(total, ppl));
        if (it != g_tuned.end()) return it->second;
    }
    // measured on gfx950 (two-player mid-game leaves): up to 2M playouts one
    // playout per lane with the workgroup's unfinished games packed at steps
    // 5, 8, 11, 14, 17 (variant 7; 0.107 ms at 1M in the bench step, the same as
    // variant 9 with 256 playouts per workgroup, 0.122 ms for variant 4); up
    // to 4M the games packed every four guesses and the freed lanes refilled,
    // 512 playouts per workgroup (variant 9; 0.339 vs 0.357 ms for variant 7);
    // beyond that in-wave refill over 256-playout items when leaves have at
    // least 256 playouts (variant 5; 1.18 ms vs 1.21 ms for variant 9 and
    // 1.29 ms for variant 7 at 16M), else variant 9 with 512 playouts per
    // workgroup (1.24 ms vs 1.38 ms for variant 7 and 1.63 ms for variant 5
    // at 262,144 leaves x 64)
    if (total <= (2ull << 20)) return Shape{7, 0, 2};
    if (total <= (4ull << 20)) return Shape{9, 0, 2};
    return ppl >= 256 ? Shape{5, 0, 4} : Shape{9, 0, 2};
}

static int rollout_impl(const dvc_state_t *leaves, int64_t n_leaves, int32_t ppl, uint64_t seed,
                        uint32_t tree_id, uint32_t leaf_id_base, int8_t *winner, int16_t *length,
                        uint32_t *seat_wins, Shape sh, int32_t flags, hipStream_t st)
{
    const int v = sh.variant, block = sh.block, grid = sh.grid;
    RolloutArgs a;
    a.leaves = reinterpret_cast<const uint4 *>(leaves);
    a.n_leaves = (uint32_t)n_leaves;
    a.ppl = (uint32_t)ppl;
    a.total = (uint32_t)((uint64_t)n_leaves * (uint64_t)ppl);
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.tree = tree_id;
    a.leaf_base = leaf_id_base;
    // variant 2: a chunk never spans more than kStageLeaves leaves
    const uint64_t max_chunk = (uint64_t)(kStageLeaves - 1u) * (uint64_t)ppl;
    a.chunk = (uint32_t)(max_chunk < 256u ? max_chunk : 256u);
    // single-leaf items: variant 3 one playout per lane, variant 5 up to
    // 64*K playouts (K = grid, default 4)
    const int k5 = grid > 0 ? grid : 4;
    if (v == 5 && k5 != 1 && k5 != 2 && k5 != 4 && k5 != 8) return DVC_EINVAL;
    const uint32_t per_item = v == 5 ? 64u * (uint32_t)k5 : 64u;
    a.item_chunk = (uint32_t)ppl < per_item ? (uint32_t)ppl : per_item;
    a.parts = ((uint32_t)ppl + a.item_chunk - 1u) / a.item_chunk;
    const uint64_t n_items = (uint64_t)n_leaves * a.parts;
    if (n_items >= (1ull << 32)) return DVC_EINVAL;
    a.n_items = (uint32_t)n_items;
    a.batch = 128u / a.item_chunk > 0u ? 128u / a.item_chunk : 1u;
    a.queue_slot = next_queue_slot();
    a.winner = winner;
    a.length = length;
    a.seat_wins = seat_wins;
    a.stats = nullptr;
    // variants 7, 8 and 9 with whole leaves per workgroup (256, 512 and
    // 256 K playouts; variant 9 at most 16 leaves) store each leaf's sums
    // themselves: no zeroing launch
    const uint32_t per_group = v == 8 ? 512u : v == 9 ? 256u * (grid == 1 ? 1u : 2u) : 256u;
    a.store_wins = (seat_wins && !(flags & DVC_ROLLOUT_ACCUMULATE) && (v == 7 || v == 8 || v == 9) &&
                    (uint32_t)ppl <= per_group && per_group % (uint32_t)ppl == 0u &&
                    (v != 9 || per_group / (uint32_t)ppl <= 16u)) ? 1u : 0u;
    if (a.total == 0) return DVC_OK;
    if (seat_wins && !(flags & DVC_ROLLOUT_ACCUMULATE) && !a.store_wins) {
        hipError_t e = launch_fill_u32(seat_wins, (uint64_t)n_leaves * 4u, 0u, st);
        if (e != hipSuccess) return DVC_EHIP;
    }
    return status_of(launch_rollout(a, v, block, grid, st));
}

static int rollout_args_ok(const dvc_state_t *leaves, int64_t n_leaves, int32_t ppl)
{
    if (n_leaves < 0 || ppl < 1 || (n_leaves > 0 && leaves == nullptr)) return DVC_EINVAL;
    if ((uint64_t)n_leaves * (uint64_t)ppl >= (1ull << 32)) return DVC_EINVAL;
    return DVC_OK;
}

int dvc_rollout_ex(const dvc_state_t *leaves, int64_t n_leaves, int32_t ppl, uint64_t seed,
                   uint32_t tree_id, uint32_t leaf_id_base, int8_t *winner, int16_t *length,
                   uint32_t *seat_wins, int32_t variant, int32_t block, int32_t grid, int32_t flags,
                   void *stream)
{
    if ((flags & ~DVC_ROLLOUT_ACCUMULATE) != 0) return DVC_EINVAL;
    const int ok = rollout_args_ok(leaves, n_leaves, ppl);
    if (ok != DVC_OK) return ok;
    if (variant < 0 || variant > 9) return DVC_EINVAL;
    if (block != 0 && block != 64 && block != 128 && block != 256 && block != 512) return DVC_EINVAL;
    if (grid < 0 || (variant == 9 && grid > 2)) return DVC_EINVAL;
    const Shape sh = variant != 0 ? Shape{variant, block, grid}
                                  : automatic_shape((uint64_t)n_leaves * (uint64_t)ppl, ppl);
    return rollout_impl(leaves, n_leaves, ppl, seed, tree_id, leaf_id_base, winner, length,
                        seat_wins, sh, flags, (hipStream_t)stream);
}

int dvc_rollout_autotune(const dvc_state_t *leaves, int64_t n_leaves, int32_t ppl, uint64_t seed,
                         uint32_t tree_id, uint32_t leaf_id_base, int8_t *winner, int16_t *length,
                         uint32_t *seat_wins, int32_t *chosen, void *stream)
{
    const int ok = rollout_args_ok(leaves, n_leaves, ppl);
    if (ok != DVC_OK) return ok;
    const uint64_t total = (uint64_t)n_leaves * (uint64_t)ppl;
    if (total == 0) return DVC_EINVAL;
    static const Shape kCandidates[] = {{7, 0, 2}, {9, 0, 2}, {9, 0, 1}, {8, 0, 0}, {4, 0, 1},
                                        {1, 0, 0}, {4, 0, 2}, {5, 0, 2}, {5, 0, 4}, {5, 0, 8}};
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);   // cleanup: the failure is already reported
        return DVC_EHIP;
    }
    int status = DVC_OK;
    Shape best = kCandidates[0];
    float best_ms = 0.0f;
    bool have = false;
    for (const Shape &c : kCandidates) {
        // the first launch warms up, the second is timed
        for (int rep = 0; rep < 2 && status == DVC_OK; ++rep) {
            if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) status = DVC_EHIP;
            if (status == DVC_OK)
                status = rollout_impl(leaves, n_leaves, ppl, seed, tree_id, leaf_id_base, winner,
                                      length, seat_wins, c, 0, st);
            if (status == DVC_OK && rep == 1 && hipEventRecord(e1, st) != hipSuccess)
                status = DVC_EHIP;
        }
        float ms = 0.0f;
        if (status == DVC_OK &&
            (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            status = DVC_EHIP;
        if (status != DVC_OK) break;
        if (!have || ms < best_ms) {
            best = c;
            best_ms = ms;
            have = true;
        }
    }
    (void)hipEventDestroy(e0);   // the timing is done; a failure here changes nothing
    (void)hipEventDestroy(e1);
    if (status != DVC_OK) return status;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        g_tuned[tune_key(total, ppl)] = best;
    }
    if (chosen) {
        chosen[0] = best.variant;
        chosen[1] = best.block;
        chosen[2] = best.grid;
    }
    return DVC_OK;
}

int dvc_rollout(const dvc_state_t *leaves, int64_t n_leaves, int32_t ppl, uint64_t seed,
                uint32_t tree_id, uint32_t leaf_id_base, int8_t *winner, int16_t *length,
                uint32_t *seat_wins, void *stream)
{
    return dvc_rollout_ex(leaves, n_leaves, ppl, seed, tree_id, leaf_id_base, winner, length,
                          seat_wins, 0, 0, 0, 0, stream);
}

size_t dvc_mcts_workspace_bytes(int64_t n_trees, const dvc_mcts_params *params)
{
    if (n_trees < 0 || !mcts_params_ok(params)) return 0;
    const MctsShape sh = mcts_shape((uint32_t)params->iterations, (uint32_t)params->continue_choice,
                                    (uint32_t)params->vanilla);
    return (size_t)n_trees * sh.tree_words * sizeof(uint32_t);
}

// merge = false: one tree per root, statistics in creation order;
// merge = true: trees_per_root trees per root amalgamated by action id.
// static_ln: a natural-log table of static_ln_entries entries to use instead
// of the library-allocated one (the allocation-free entry point's).
static int run_search(const dvc_state_t *roots, int64_t n_roots, int64_t trees_per_root, bool merge,
                      const dvc_mcts_params *user_params, uint64_t seed, uint32_t tree_id_base,
                      void *workspace, size_t workspace_bytes, int32_t *best_action,
                      dvc_child_stat *children, void *stream, const float *static_ln = nullptr,
                      uint64_t static_ln_entries = 0)
{
    if (n_roots < 0 || trees_per_root < 1 || trees_per_root > 65536 ||
        !mcts_params_ok(user_params))
        return DVC_EINVAL;
    const dvc_mcts_params rp = resolved(user_params, n_roots * trees_per_root);
    const dvc_mcts_params *params = &rp;
    if (merge && params->vanilla) return DVC_EINVAL;   // world nodes are not merged
    const int64_t n_trees = n_roots * trees_per_root;
    if (n_trees >= (1ll << 31)) return DVC_EINVAL;
    if (n_roots == 0) return DVC_OK;
    if (roots == nullptr || best_action == nullptr || workspace == nullptr) return DVC_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 16u != 0u) return DVC_EINVAL;
    if (workspace_bytes < dvc_mcts_workspace_bytes(n_trees, params)) return DVC_ENOMEM;
    int status = DVC_OK;
    const uint64_t w_leaf =
        (uint64_t)(params->leaf_eval ? params->fallback_playouts : params->playouts_per_leaf);
    const uint64_t need = (uint64_t)params->iterations * w_leaf + 1u;
    if (static_ln != nullptr && need > static_ln_entries) return DVC_ETOOBIG;
    const float *ln = static_ln != nullptr ? static_ln : ln_table(need, &status);
    if (ln == nullptr) return status;
    hipError_t e = launch_mcts(reinterpret_cast<const uint4 *>(roots), (uint32_t)n_trees,
                               (uint32_t)trees_per_root, (uint32_t)params->iterations,
                               (uint32_t)params->playouts_per_leaf, (uint32_t)params->max_depth,
                               params->c_uct, (uint32_t)seed, (uint32_t)(seed >> 32), tree_id_base,
                               ln, reinterpret_cast<uint32_t *>(workspace),
                               merge ? nullptr : best_action,
                               merge ? nullptr : reinterpret_cast<uint32_t *>(children),
                               (uint32_t)params->leaf_eval, params->fallback_band,
                               (uint32_t)params->fallback_playouts, params->valuenet,
                               (uint32_t)params->continue_choice, (uint32_t)params->vanilla,
                               (uint32_t)params->leaves_per_pass, (uint32_t)params->pipeline,
                               (hipStream_t)stream);
    if (e != hipSuccess || !merge) return status_of(e);
    return status_of(launch_mcts_merge(reinterpret_cast<const uint32_t *>(workspace),
                                       (uint32_t)n_roots, (uint32_t)trees_per_root,
                                       (uint32_t)params->iterations,
                                       (uint32_t)params->continue_choice, best_action,
                                       reinterpret_cast<uint32_t *>(children),
                                       (hipStream_t)stream));
}

int mcts_search(const dvc_state_t *roots, int64_t n_trees, const dvc_mcts_params *params,
                uint64_t seed, uint32_t tree_id_base, void *workspace, size_t workspace_bytes,
                int32_t *best_action, dvc_child_stat *root_children, void *stream)
{
    return run_search(roots, n_trees, 1, false, params, seed, tree_id_base, workspace, workspace_bytes,
                      best_action, root_children, stream);
}

// ---------------------------------------------------------------------------
// Allocation-free search.  The trees and the natural-log table live in
// `scratch`, a file-scope device array: every device the library runs on
// holds its own copy, at its own address, until the process ends.  Its first
// kScratchLnEntries floats are the table LN[k] = float(log(double k)),
// written once per device at set-up; the rest holds the trees of the call
// in flight.  Host code never passes the array's name to a kernel or a copy
// (on the host it is a stand-in, not a device address): it uses the address
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr uint64_t kScratchLnEntries = 1ull << 20;
constexpr uint64_t kScratchLnBytes = kScratchLnEntries * sizeof(float);
constexpr uint64_t kScratchBytes = kScratchLnBytes + ((uint64_t)DVC_NOALLOC_TREE_BYTES);
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static std::mutex g_scratch_mutex;
static uint8_t *g_scratch_dev[64] = {nullptr};

// Set-up on the current device, once: the array's device address, then the
// log table written into its first bytes (synchronous copies from a stack
// buffer, no allocation).  Returns the address, or null with *status set.
static uint8_t *scratch_on_device(int *status)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        *status = DVC_EHIP;
        return nullptr;
    }
    if (g_scratch_dev[dev] != nullptr) return g_scratch_dev[dev];
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
        *status = DVC_EHIP;
        return nullptr;
    }
    constexpr uint64_t kChunk = 4096;
    float buf[kChunk];
    for (uint64_t base = 0; base < kScratchLnEntries; base += kChunk) {
        for (uint64_t k = 0; k < kChunk; ++k) {
            const uint64_t i = base + k;
            buf[k] = i == 0 ? 0.0f : (float)std::log((double)i);
        }
        if (hipMemcpy(static_cast<uint8_t *>(ptr) + base * sizeof(float), buf, sizeof(buf),
                      hipMemcpyHostToDevice) != hipSuccess) {
            *status = DVC_EHIP;
            return nullptr;
        }
    }
    g_scratch_dev[dev] = static_cast<uint8_t *>(ptr);
    return g_scratch_dev[dev];
}

int mcts_search_noalloc(const dvc_state_t *roots, int64_t n_trees, const dvc_mcts_params *params,
                        uint64_t seed, uint32_t tree_id_base, int32_t *best_action,
                        dvc_child_stat *root_children, void *stream)
{
    if (n_trees < 0 || !mcts_params_ok(params)) return DVC_EINVAL;
    const dvc_mcts_params rp = resolved(params, n_trees);
    const size_t need = dvc_mcts_workspace_bytes(n_trees, &rp);
    if (n_trees > 0 && need == 0) return DVC_EINVAL;
    if (need > (size_t)DVC_NOALLOC_TREE_BYTES) return DVC_ETOOBIG;
    int status = DVC_OK;
    uint8_t *base = scratch_on_device(&status);
    if (base == nullptr) return status;
    return run_search(roots, n_trees, 1, false, &rp, seed, tree_id_base, base + kScratchLnBytes,
                      (size_t)DVC_NOALLOC_TREE_BYTES, best_action, root_children, stream,
                      reinterpret_cast<const float *>(base), kScratchLnEntries);
}

int dvc_mcts_autotune(const dvc_state_t *roots, int64_t n_trees, const dvc_mcts_params *params,
                      uint64_t seed, uint32_t tree_id_base, void *workspace, size_t workspace_bytes,
                      float tolerance, int32_t *best_action, dvc_mcts_tuning *result,
                      void *stream)
{
    if (params == nullptr || params->leaf_eval != 0 || params->playouts_per_leaf < 1 ||
        params->leaves_per_pass != 1 || params->pipeline != 0 || n_trees < 1 ||
        !(tolerance >= 0.0f) || best_action == nullptr)
        return DVC_EINVAL;
    dvc_mcts_params cand = *params;
    cand.playouts_per_leaf = kAutoMaxPpl;   // every candidate's visit counts stay exact
    if (!mcts_params_ok(params) || !mcts_params_ok(&cand)) return DVC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const size_t n = (size_t)n_trees;
    std::vector<int32_t> ref(n), ref2(n), got(n), chosen_dec(n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);   // cleanup: the failure is already reported
        return DVC_EHIP;
    }
    // one search with its decisions copied to `out` and its time in *ms
    auto run = [&](const dvc_mcts_params &mp, uint64_t sd, std::vector<int32_t> &out,
                   float *ms) -> int {
        if (hipEventRecord(e0, st) != hipSuccess) return DVC_EHIP;
        int rc = run_search(roots, n_trees, 1, false, &mp, sd, tree_id_base, workspace,
                            workspace_bytes, best_action, nullptr, stream);
        if (rc != DVC_OK) return rc;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return DVC_EHIP;
        if (ms && hipEventElapsedTime(ms, e0, e1) != hipSuccess) return DVC_EHIP;
        if (hipMemcpy(out.data(), best_action, n * sizeof(int32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return DVC_EHIP;
        return DVC_OK;
    };
    auto agreement = [&](const std::vector<int32_t> &a, const std::vector<int32_t> &b) {
        size_t k = 0;
        for (size_t i = 0; i < n; ++i) k += a[i] == b[i];
        return (float)k / (float)n;
    };
    // the reference: the sequential search with the caller's playouts per
    // leaf, under the caller's seed and under a second seed
    int status = run(*params, seed, ref, nullptr);
    if (status == DVC_OK) status = run(*params, seed ^ 0x9E3779B97F4A7C15ull, ref2, nullptr);
    const float ceiling = status == DVC_OK ? agreement(ref, ref2) : 0.0f;
    SearchShape best{params->playouts_per_leaf, 1, 0};
    float best_ms = 0.0f, best_agree = 0.0f;
    bool have = false;
    for (const SearchShape &c : kSearchCandidates) {
        if (status != DVC_OK) break;
        if (c.pipe && params->vanilla) continue;   // pipelined passes keep no world nodes
        cand.playouts_per_leaf = c.ppl;
        cand.leaves_per_pass = c.lpp;
        cand.pipeline = c.pipe;
        float ms = 0.0f;
        // candidates run under a third seed, so that the caller's own shape is
        // judged like the others (its agreement is then the seed-to-seed one)
        status = run(cand, seed + 1u, got, &ms);
        if (status != DVC_OK) break;
        const float agree = agreement(got, ref);
        if (agree + tolerance >= ceiling && (!have || ms < best_ms)) {
            best = c;
            best_ms = ms;
            best_agree = agree;
            chosen_dec = got;
            have = true;
        }
    }
    (void)hipEventDestroy(e0);   // the timing is done; a failure here changes nothing
    (void)hipEventDestroy(e1);
    if (status != DVC_OK) return status;
    if (!have) {   // no candidate within the tolerance: the caller's own shape
        chosen_dec = ref;
        best_agree = 1.0f;
    }
    if (hipMemcpy(best_action, chosen_dec.data(), n * sizeof(int32_t), hipMemcpyHostToDevice) !=
        hipSuccess)
        return DVC_EHIP;
    {
        std::lock_guard<std::mutex> lock(g_search_tune_mutex);
        g_search_tuned[search_key(n_trees, params)] = best;
    }
    if (result) {
        result->playouts_per_leaf = best.ppl;
        result->leaves_per_pass = best.lpp;
        result->pipeline = best.pipe;
        result->decisions_per_s = have ? (float)((double)n_trees / (best_ms * 1e-3)) : 0.0f;
        result->agreement = best_agree;
        result->self_agreement = ceiling;
    }
    return DVC_OK;
}

int mcts_search_root_parallel(const dvc_state_t *roots, int64_t n_roots, int32_t trees_per_root,
                              const dvc_mcts_params *params, uint64_t seed, uint32_t tree_id_base,
                              void *workspace, size_t workspace_bytes, int32_t *best_action,
                              dvc_child_stat *merged_children, void *stream)
{
    return run_search(roots, n_roots, trees_per_root, true, params, seed, tree_id_base, workspace,
                      workspace_bytes, best_action, merged_children, stream);
}

size_t dvc_valuenet_bytes(void) { return vn_bytes(); }

int dvc_valuenet_init(void *net, uint64_t seed, void *stream)
{
    if (net == nullptr || !aligned16(net)) return DVC_EINVAL;
    return status_of(launch_vn_init(net, (uint32_t)seed, (uint32_t)(seed >> 32), (hipStream_t)stream));
}

int dvc_valuenet_set_params(void *net, const float *params, void *stream)
{
    if (net == nullptr || params == nullptr || !aligned16(net)) return DVC_EINVAL;
    return status_of(launch_vn_set_params(net, params, (hipStream_t)stream));
}

int dvc_valuenet_get_params(const void *net, float *params, void *stream)
{
    if (net == nullptr || params == nullptr || !aligned16(net)) return DVC_EINVAL;
    return status_of(launch_vn_get_params(net, params, (hipStream_t)stream));
}

int dvc_valuenet_get_moments(const void *net, float *m, float *v, void *stream)
{
    if (net == nullptr || m == nullptr || v == nullptr || !aligned16(net)) return DVC_EINVAL;
    return status_of(launch_vn_get_moments(net, m, v, (hipStream_t)stream));
}

int dvc_valuenet_infer(const void *net, const dvc_state_t *states, const uint8_t *persp, int64_t n,
                       float *v_out, void *stream)
{
    if (n < 0 || n >= (1ll << 31)) return DVC_EINVAL;
    if (n == 0) return DVC_OK;
    if (net == nullptr || states == nullptr || persp == nullptr || v_out == nullptr ||
        !aligned16(net))
        return DVC_EINVAL;
    return status_of(launch_vn_infer(net, reinterpret_cast<const uint4 *>(states), persp,
                                     (uint32_t)n, v_out, (hipStream_t)stream));
}

int dvc_valuenet_epoch_order(uint64_t seed, int64_t epoch, int64_t n_data, uint32_t *perm_a,
                             uint32_t *perm_b)
{
    if (epoch < 0 || epoch > 0xFFFFFFFFll || n_data < 1 || n_data > (1ll << 32) ||
        (n_data & (n_data - 1)) != 0 || perm_a == nullptr || perm_b == nullptr)
        return DVC_EINVAL;
    const uint32_t ctr[4] = {(uint32_t)epoch, 0xFFFFFFFDu, 0u, 0u};
    uint32_t w[4];
    philox_host(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), w);
    const uint64_t mask = (uint64_t)n_data - 1u;
    *perm_a = n_data == 1 ? 1u : (uint32_t)((uint64_t)(w[0] | 1u) & mask);
    *perm_b = (uint32_t)((uint64_t)w[1] & mask);
    return DVC_OK;
}

size_t dvc_valuenet_train_workspace_bytes(int64_t batch)
{
    if (batch < 32 || batch > 65536 || batch % 32 != 0) return 0;
    return vn_train_ws_bytes((uint32_t)batch);
}

int dvc_valuenet_train_step(void *net, const dvc_state_t *states, const uint8_t *persp,
                            const float *labels, int64_t n_data, uint32_t perm_a, uint32_t perm_b,
                            uint32_t row_base, int32_t batch, int64_t step, float lr, void *ws,
                            size_t ws_bytes, float *loss_out, float *grad_out, void *stream)
{
    if (net == nullptr || states == nullptr || persp == nullptr || labels == nullptr || ws == nullptr ||
        !aligned16(net) || !aligned16(ws))
        return DVC_EINVAL;
    if (batch < 32 || batch > 65536 || batch % 32 != 0 || n_data < 1 || n_data >= (1ll << 32) ||
        step < 1 || !(lr > 0.0f))
        return DVC_EINVAL;
    if (ws_bytes < vn_train_ws_bytes((uint32_t)batch)) return DVC_ENOMEM;
    const double c1 = 1.0 - std::pow(0.9, (double)step), c2 = 1.0 - std::pow(0.999, (double)step);
    return status_of(launch_vn_train_step(net, reinterpret_cast<const uint4 *>(states), persp, labels,
                                          (uint32_t)n_data, perm_a, perm_b, row_base,
                                          (uint32_t)batch, lr, (float)c1, (float)c2, ws, loss_out,
                                          grad_out, (hipStream_t)stream));
}

int dvc_valuenet_labels(const dvc_state_t *states, int64_t n, int32_t playouts, uint64_t seed,
                        uint32_t tree_id, uint32_t index_base, uint8_t *persp_out,
                        float *labels_out, uint32_t *seat_wins_ws, void *stream)
{
    if (n < 0 || playouts < 1) return DVC_EINVAL;
    if (n == 0) return DVC_OK;
    if (states == nullptr || persp_out == nullptr || labels_out == nullptr || seat_wins_ws == nullptr)
        return DVC_EINVAL;
    int rc = dvc_rollout(states, n, playouts, seed, tree_id, index_base, nullptr, nullptr,
                         seat_wins_ws, stream);
    if (rc != DVC_OK) return rc;
    return status_of(launch_vn_labels(reinterpret_cast<const uint4 *>(states), (uint32_t)n,
                                      (uint32_t)playouts, (uint32_t)seed, (uint32_t)(seed >> 32),
                                      index_base, seat_wins_ws, persp_out, labels_out,
                                      (hipStream_t)stream));
}

}  // extern "C"
