// dvc_internal.hpp -- shared declarations of the library's translation unit
// (kernel argument blocks, device-global error word and work queues,
// launchers).  The library is built as one translation unit (dvc_lib.hip),
// so the device globals below are defined exactly once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dvc {

constexpr uint32_t kErrState = 1u;   // a malformed state was read
constexpr uint32_t kErrLimit = 2u;   // a kernel reached an internal bound
constexpr int kQueueSlots = 1024;    // independent work-queue counter pairs
constexpr uint32_t kStageLeaves = 64;  // leaf states staged per wave
constexpr uint32_t kMaxActions = 864;  // ((P-1)*24 slots) * 12 values, P <= 4

// Sticky error word of the device, or-ed by kernels, read and cleared by
// dvc_check().
__device__ uint32_t g_error_word = 0u;
// Work-stealing counters: [slot][0] next chunk, [slot][1] finished
// workgroups.  A persistent kernel's last workgroup returns its slot to zero,
// so every call starts from zeros without a memset.
__device__ uint32_t g_queue[kQueueSlots][2];

struct RolloutArgs {
    const uint4 *leaves;
    uint32_t n_leaves, ppl, total;   // total = n_leaves * ppl < 2^32
    uint32_t k0, k1, tree, leaf_base;
    uint32_t chunk;                  // variant 2: playout ids per stolen chunk
    uint32_t item_chunk;             // variant 3: playouts per single-leaf item
    uint32_t parts;                  // variant 3: items per leaf
    uint32_t n_items;                // variant 3: n_leaves * parts
    uint32_t batch;                  // variant 3: items per stolen batch
    uint32_t queue_slot;
    int8_t *winner;
    int16_t *length;
    uint32_t *seat_wins;
    uint32_t store_wins;             // variant 7, ppl dividing 256: store each leaf's sums
                                     // (the table is not zeroed beforehand)
    unsigned long long *stats;       // optional: [0] += wave steps
};

struct DealArgs {
    int32_t p_min, p_max;
    int32_t hand[5];
    int32_t pile_min, pile_max, revealed_max, fresh, root_draw, phase_mix;
};

int default_rollout_grid(int waves_per_block);
hipError_t launch_rollout(const RolloutArgs &a, int variant, int block, int grid, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st);
// one tree's workspace: node records with their first child blocks,
// overflow blocks, the block chain, and (vanilla) per-action sums
struct MctsShape {
    uint32_t node_words, node_stride, nodes_cap, ovf_cap;
    uint64_t agg_off, tree_words;
};
MctsShape mcts_shape(uint32_t iters, uint32_t cont, uint32_t vanilla);
hipError_t launch_mcts(const uint4 *roots, uint32_t n_trees, uint32_t trees_per_root,
                       uint32_t iters, uint32_t ppl, uint32_t dmax, float c_uct, uint32_t k0, uint32_t k1, uint32_t tree_base,
                       const float *ln, uint32_t *ws, int32_t *best, uint32_t *kids,
                       uint32_t leaf_eval, float band, uint32_t fb_ppl, const void *net,
                       uint32_t cont, uint32_t vanilla, uint32_t lpp, uint32_t pipe,
                       hipStream_t st);
hipError_t launch_mcts_merge(const uint32_t *ws, uint32_t n_roots, uint32_t trees_per_root,
                             uint32_t iters, uint32_t cont, int32_t *best, uint32_t *merged,
                             hipStream_t st);
size_t vn_bytes();
size_t vn_train_ws_bytes(uint32_t batch);
hipError_t launch_vn_init(void *net, uint32_t k0, uint32_t k1, hipStream_t st);
hipError_t launch_vn_shadow(void *net, hipStream_t st);
hipError_t launch_vn_infer(const void *net, const uint4 *states, const uint8_t *persp, uint32_t n,
                           float *v_out, hipStream_t st);
hipError_t launch_vn_train_step(void *net, const uint4 *states, const uint8_t *persp,
                                const float *labels, uint32_t n_data, uint32_t perm_a,
                                uint32_t perm_b, uint32_t row_base, uint32_t batch, float lr,
                                float c1, float c2, void *ws, float *loss_out, float *grad_out,
                                hipStream_t st);
hipError_t launch_vn_set_params(void *net, const float *params, hipStream_t st);
hipError_t launch_vn_get_params(const void *net, float *params, hipStream_t st);
hipError_t launch_vn_get_moments(const void *net, float *m, float *v, hipStream_t st);
hipError_t launch_vn_labels(const uint4 *states, uint32_t n, uint32_t playouts, uint32_t k0,
                            uint32_t k1, uint32_t index_base, const uint32_t *seat_wins,
                            uint8_t *persp, float *labels, hipStream_t st);
hipError_t launch_init_states(uint4 *out, uint32_t n, const DealArgs &d, uint32_t k0, uint32_t k1,
                              uint32_t index_base, hipStream_t st);

}  // namespace dvc
