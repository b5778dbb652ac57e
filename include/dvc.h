/*
 * dvc.h -- C ABI of the MI355X (gfx950) Da Vinci Code Monte Carlo Tree
 * Search engine: synthetic states, massively parallel random playouts and
 * the tree search that feeds them leaves.
 *
 * Method: Zhang et al., "Development and Application of a Monte Carlo Tree
 * Search Algorithm for Simulating Da Vinci Code Game Strategies",
 * arXiv 2403.10720.  Game rules: Sec. II-A; MCTS and random playouts:
 * Sec. II-B; simplified search (node = tile position + guessed number, no
 * further guess after a right guess inside the tree, fixed expansion depth):
 * Sec. III-A; per-thread simulations merged into one tree: Sec. III-B..D.
 *
 * Conventions for every entry point
 *   - Buffers are device memory owned by the caller (for example torch
 *     tensors), unless a comment says "host".  The library never frees them.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Calls enqueue work on it and return without waiting.
 *   - Return value: DVC_OK (0) or a negative dvc_status.  Argument errors are
 *     detected on the host and returned at once, with nothing enqueued.
 *     Errors found by a kernel (a malformed state) set a sticky per-device
 *     error word that dvc_check() returns (and clears) after synchronising.
 *   - Outputs are a pure function of the inputs, the seed and the id bases:
 *     they do not depend on the launch shape, on the batch a leaf or tree is
 *     part of, or on the stream.
 *   - The library prints nothing and never aborts.
 *   - Device memory the library allocates itself: the natural-log table of
 *     the tree search, once per device on the first search that needs it
 *     (grown, never freed, when a later search needs more entries; the
 *     growing call copies it synchronously, so make one search before
 *     capturing a graph), and the static scratch of mcts_search_noalloc
 *     (part of the library's code object, one per device).  Everything else
 *     lives in caller buffers.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 * (seed & 0xFFFFFFFF, seed >> 32).  A pick among k options from a word w is
 * floor(w * k / 2^32).  Counter layouts (c0, c1, c2, c3):
 *   guess step g of playout p of leaf l of tree tr      (g, p, l, tr)
 *     word 0 draw, word 1 target tile, word 2 guessed value,
 *     word 3 continue coin (go on iff w3 < 2^31) or own tile to reveal;
 *     a word whose choice does not arise is skipped, never shifted.
 *   determinization attempt a of iteration i, word n   (n>>2, 0x80000000+a, i, tr)
 *   in-tree guess at depth d of iteration i             (d, 0xC0000000, i, tr)
 *     word 0 own tile to reveal, word 1 next player's draw, word 3 the
 *     continue coin of a leaf reached right after a right guess (continue
 *     choice on, see dvc_mcts_params)
 *   synthetic state s, word n                           (n>>2, 0xFFFFFFFF, 0xFFFFFFFF, s)
 *   value network: initial weight k (k>>2, 0xFFFFFFFE, 0, 0), training pair
 *   perspective (0, 0xFFFFFFFC, 0, i), batch order of an epoch (e, 0xFFFFFFFD, 0, 0)
 */
#ifndef DVC_H
#define DVC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------------------
 * Packed game state, 16 bytes (Sec. II-A: 24 numbered tiles, values 0..11 in
 * black and white; every player keeps an ascending row; colours are public).
 *
 * Tile id t = 2*value + colour (0 black, 1 white), so ids sort by value and
 * black sorts before white on equal values.  A row is the set of tile ids a
 * player owns; its order is implied by the ids.
 *   w[0..2] bits 0-23 : bit-plane k of the 3-bit owner code of tile t
 *                       (0 = draw pool, 1..4 = seat 0..3)
 *   w[3]    bits 0-23 : revealed tiles
 *   w[0]    bits 24-25: seat to move; 26-27: players - 1 (2..4 players);
 *           bit 28: phase (0 = turn start, 1 = the mover has had its draw);
 *           bit 29: a drawn tile is recorded
 *   w[1]    bits 24-28: the drawn tile id (zero when none is recorded)
 *   all other bits are zero.
 * Valid state: owner codes <= players; pool tiles are not revealed; the mover
 * has a hidden tile; phase 0 records no drawn tile; a recorded drawn tile is
 * a hidden tile of the mover.  A state where only one player has hidden tiles
 * is valid and already decided.
 * ------------------------------------------------------------------------- */
typedef struct { uint32_t w[4]; } dvc_state_t;

enum dvc_status {
    DVC_OK = 0,
    DVC_EINVAL = -1,  /* bad argument (size, pointer, parameter)            */
    DVC_ESTATE = -2,  /* a malformed packed state was found                 */
    DVC_EHIP = -3,    /* a HIP runtime call failed                          */
    DVC_ENOMEM = -4,  /* workspace too small / library allocation failed    */
    DVC_ELIMIT = -5,  /* a kernel hit an internal bound                     */
    DVC_ETOOBIG = -6  /* beyond the static scratch of mcts_search_noalloc   */
};

/* Parameters of the synthetic state generator.
 * A deal gives every player hand[P] tiles (Sec. II-A: four tiles); beyond the
 * deal, a pool size is drawn, the tiles drawn since the deal are handed out
 * round-robin from seat 0, and a random number of every row's tiles is
 * revealed, always leaving one hidden.                                      */
typedef struct {
    int32_t p_min, p_max;       /* players, uniform in [p_min, p_max], 2..4         */
    int32_t hand[5];            /* tiles dealt per player, indexed by player count  */
    int32_t pile_min, pile_max; /* pool size, uniform, capped at 24 - P*hand[P]     */
    int32_t revealed_max;       /* revealed tiles per row, uniform in 0..min(this, h-1) */
    int32_t fresh;              /* 1: fresh deal (full pool, nothing revealed)      */
    int32_t root_draw;          /* 1: the seat to move draws (phase 1)              */
    int32_t phase_mix;          /* 1: it draws with probability 1/2                 */
} dvc_deal_params;

/* dvc_init_states -- write n synthetic states out[0..n) for state indices
 * index_base .. index_base+n-1 (word stream of state s above).  Sec. II-A
 * deal, extended to mid-game positions.  `out` is device memory of n*16 B.
 * Returns DVC_EINVAL for n < 0, a NULL out with n > 0, or parameters outside
 * the ranges above.                                                          */
int dvc_init_states(dvc_state_t *out, int64_t n, const dvc_deal_params *params /* host */,
                    uint64_t seed, uint32_t index_base, void *stream);

/* dvc_rollout -- random playouts (Sec. II-B: the game is played out by taking
 * every decision at random) from n_leaves leaf states, playouts_per_leaf each.
 * Playout p of leaf i uses leaf id l = leaf_id_base + i and tree id tree_id.
 * One guess step:
 *   at turn start the mover draws a uniformly random pool tile (if any);
 *   the target is uniform over the hidden tiles of all other players, pooled,
 *   in ascending id order; the guessed value is uniform over the tile ids of
 *   the target's colour strictly between the nearest revealed tiles around it
 *   in its row that are neither in the mover's row nor revealed;
 *   a right guess reveals the target and the mover goes on with probability
 *   1/2; a wrong guess reveals the mover's drawn tile, or a uniformly random
 *   hidden tile of its own when it drew nothing, and ends the turn; a player
 *   without hidden tiles is out; the next player in seat order still in moves.
 * Outputs (each may be NULL):
 *   winner[i*ppl + p]  int8   absolute seat of the last player standing
 *   length[i*ppl + p]  int16  number of guesses (= tiles revealed)
 *   seat_wins[i*4 + s] uint32 playouts of leaf i won by seat s
 * A malformed leaf yields winner -1, length -1, no wins, and DVC_ESTATE in the
 * error word.  Returns DVC_EINVAL for n_leaves < 0, playouts_per_leaf < 1,
 * n_leaves*playouts_per_leaf >= 2^32 or leaves == NULL with n_leaves > 0.  */
int dvc_rollout(const dvc_state_t *leaves, int64_t n_leaves, int32_t playouts_per_leaf,
                uint64_t seed, uint32_t tree_id, uint32_t leaf_id_base,
                int8_t *winner, int16_t *length, uint32_t *seat_wins, void *stream);

/* dvc_rollout with a choice of kernel, for measurement.  variant: 0 =
 * automatic (the shape dvc_rollout_autotune chose for this size class, else
 * up to 2M playouts variant 7 with steps 5, 8, 11, 14, 17, up to 4M variant 9
 * with 512 playouts per workgroup; above, variant 5 if playouts_per_leaf >=
 * 256, else variant 9 with 512), 1 = one lane per playout,
 * 2 = lane refill + work stealing over LDS-staged leaf chunks, 3 = lane
 * refill + work stealing over single-leaf items, 4 = several playouts per
 * lane back to back (`grid` then gives the playouts per lane, 1/2/4),
 * 5 = one wavefront per item of up to 64*K playouts of one leaf, lanes
 * refilled from the item as their games end (`grid` gives K, 1/2/4/8,
 * default 4), 6 = variant 4 with one playout per lane and each step's
 * random words computed during the step before, 7 = one playout per lane
 * with the workgroup's unfinished games packed into its first lanes at
 * fixed step counts (Sec. IV-B's divergence: wavefronts left without a game
 * stop issuing; `grid` 0/1 = steps 6, 9, 12, 2 = steps 5, 8, 11, 14, 17),
 * 8 = variant 7 (steps 5, 8, 11, 14, 17) with two games per lane advanced
 * together, 512 playouts per workgroup, 9 = variant 7's packing every four
 * guesses, the lanes it frees starting the workgroup's next playouts
 * (`grid` gives the workgroup's 256-playout batches, 1 or 2, default 2).
 * block/grid 0 = automatic.  Same outputs for every variant and shape.
 * flags: DVC_ROLLOUT_ACCUMULATE adds the wins to seat_wins instead of
 * overwriting it (the caller zeroes it once; several calls then tally into
 * one table).  Errors as dvc_rollout, plus DVC_EINVAL for an unknown
 * variant, block size or flag.                                             */
#define DVC_ROLLOUT_ACCUMULATE 1
int dvc_rollout_ex(const dvc_state_t *leaves, int64_t n_leaves, int32_t playouts_per_leaf,
                   uint64_t seed, uint32_t tree_id, uint32_t leaf_id_base,
                   int8_t *winner, int16_t *length, uint32_t *seat_wins,
                   int32_t variant, int32_t block, int32_t grid, int32_t flags, void *stream);

/* dvc_rollout_autotune -- runs this batch with every rollout kernel shape in
 * a fixed candidate list (variant 7 with steps 5, 8, 11, 14, 17, variant 9
 * with 512 and 256 playouts per workgroup, variant 8, variant 4 with 1 or 2
 * playouts per lane, variant 1, variant 5 with 128/256/512-playout items),
 * each launched twice with the
 * second launch timed by HIP events on `stream`, and remembers the fastest
 * for batches of the same size class (device, floor(log2(n_leaves *
 * playouts_per_leaf)), playouts_per_leaf >= 256 / >= 64 / smaller): later
 * calls with variant 0 in that class use it (a library-owned table, guarded
 * by a lock, kept until the process ends).  The outputs are this batch's
 * playouts, exactly as dvc_rollout writes them (every shape computes the same
 * outputs).  chosen (host, may be NULL) receives {variant, block, grid}.
 * Synchronizes the stream.  Errors as dvc_rollout; DVC_EINVAL for an empty
 * batch; DVC_EHIP if an event call fails.                                  */
int dvc_rollout_autotune(const dvc_state_t *leaves, int64_t n_leaves, int32_t playouts_per_leaf,
                         uint64_t seed, uint32_t tree_id, uint32_t leaf_id_base,
                         int8_t *winner, int16_t *length, uint32_t *seat_wins,
                         int32_t *chosen /* host [3] */, void *stream);

/* ---------------------------------------------------------------------------
 * Tree search (Sec. II-B, Sec. III-A).
 * An action is a guess (r, s, v): target seat (mover + r) mod P, r = 1..P-1;
 * slot s of the target's row (0 = lowest) at guess time; value v (the colour
 * is the slot's).  action_id = ((r-1)*24 + s)*12 + v < 864.  It is legal when
 * the target still has hidden tiles, slot s exists and is hidden, and 2v+colour
 * is a consistent value for the mover (see dvc_rollout).
 * Iteration i of tree tr:
 *   1. sample a world consistent with what the root mover sees (the opponent
 *      tiles are a black box, Sec. III-A): per opponent from the mover's left,
 *      per run of hidden slots between revealed tiles, bounds right to left
 *      (largest available tile of the slot's colour below the next bound),
 *      then values left to right, uniform in (previous, bound]; up to 64
 *      attempts, then the smallest consistent world in slot order;
 *   2. descend from the root: a decided state is the leaf; at depth
 *      max_depth the node is the leaf; else the lowest legal action id that
 *      is not yet a child is expanded and its child is the leaf; else the
 *      legal child with the greatest UCT score, in FP32 with one rounding per
 *      operation: n=N; q=W/n; e=LN[N_parent]/n; u=c_uct*sqrt(e); score=q+u,
 *      LN[k]=float(log(double k)), first child in creation order on ties.
 *      Playing a guess in the tree ends the turn (a right guess reveals the
 *      target, a wrong one the drawn or a random own hidden tile); the next
 *      player draws;
 *   3. playouts_per_leaf playouts from the leaf with leaf id i (a decided
 *      leaf counts all of them as won by its winner);
 *   4. every node on the path: N += playouts; every non-root node:
 *      W += wins of the seat that chose its action.
 * Value mode (leaf_eval = 1): step 3 evaluates the leaf with the value
 * network for every seat's perspective; if the root player's value v_M has
 * |v_M - 1/2| < fallback_band the leaf is played out with fallback_playouts
 * playouts instead.  Every leaf then weighs w = fallback_playouts: N += w and
 * W += wins of the chooser (playouts) or w * v_chooser (network).
 * Decision: the root child with the most visits, earliest created on ties.
 *
 * Leaf batching (leaves_per_pass = B > 1): the iterations run in passes of
 * B.  Each descent of a pass adds its visit counts along its path as soon as
 * its leaf is found (the pass's later descents see them, with no wins yet);
 * then the pass's leaves are evaluated together -- their playouts share the
 * 64 lanes of the tree's wavefront, their network rows one matrix tile --
 * and each path gets its leaf's wins, in iteration order.  Every leaf keeps
 * its iteration index for its world, chance words and playouts.  B = 1 is
 * the sequential search above.
 *
 * Pipelined passes (pipeline = 1): the wins of pass k are credited after the
 * descents of pass k + 1 (before its leaves are evaluated), the last pass's
 * at the end, so a descent of pass k sees the wins of passes up to k - 2.
 * Each tree then runs as two wavefronts, one descending pass k + 1 while the
 * other evaluates pass k (Sec. III-B: simulations of several workers side by
 * side).  With B = 1 too.  Not with vanilla.
 *
 * The paper's three simplifications (Sec. III-A) can each be switched off:
 *   max_depth 0 -- no depth threshold: nodes expand until the game ends;
 *   continue_choice 1 -- a right guess no longer ends the turn: the same
 *      player then chooses between stopping (tree key 864: the turn passes
 *      and the next player draws, word 1) and another guess (key 865 +
 *      action id), so a player's further guesses are nodes of their own.
 *      Expansion takes the lowest key, so the stop comes first.  A leaf
 *      reached right after a right guess draws the random policy's continue
 *      coin once for all its playouts: word 3 of that guess's chance block,
 *      below 2^31 the mover keeps guessing, else the turn passes (word 1);
 *   vanilla 1 -- each sampled world is a node of its own (Sec. III-A): the
 *      root's children are world nodes, one per distinct set of hidden
 *      opponent tiles in the order first sampled, and every iteration
 *      descends below the node of its world (UCT there uses that node's
 *      visit count).  A guess's root statistics are its (N, W) summed over
 *      the world nodes in creation order; the decision is the most visited
 *      guess, the lowest action id on ties, and root_children is indexed by
 *      action id (action 0xFFFF where no world has the guess).  Not
 *      available to mcts_search_root_parallel.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t iterations;         /* per tree, >= 1                                   */
    int32_t playouts_per_leaf;  /* >= 1                                             */
    int32_t max_depth;          /* expansion depth threshold, 1..64; 0: none        */
    float c_uct;                /* exploration constant (sqrt 2 rounded to float)   */
    int32_t leaf_eval;          /* 0: playouts; 1: value network with fallback      */
    float fallback_band;        /* value mode: playouts when |v - 0.5| < band       */
    int32_t fallback_playouts;  /* value mode: playouts of a fallback leaf          */
    const void *valuenet;       /* value mode: dvc_valuenet blob (device, 16-aligned) */
    int32_t continue_choice;    /* 1: stop-or-guess choice after a right guess      */
    int32_t vanilla;            /* 1: sampled worlds are the root's children        */
    int32_t leaves_per_pass;    /* B: leaves evaluated together, 1..16 (value mode
                                   1..4); 1 = the sequential search              */
    int32_t pipeline;           /* 1: pipelined passes (see above); not with vanilla */
} dvc_mcts_params;
/* Automatic shape: with playout leaves, playouts_per_leaf = 0 together with
 * leaves_per_pass = 0 and pipeline = 0 asks for the shape (playouts per
 * leaf, leaves per pass, pipelined or not) dvc_mcts_autotune chose for this
 * size class (device, floor(log2 n_trees), floor(log2 iterations), max_depth,
 * continue_choice, vanilla), else 32 playouts per leaf with two leaves per
 * pass, not pipelined (the fastest such shape within two points of the
 * sequential 32-playout search's seed-to-seed agreement, measured on 2048
 * mixed mid-game roots x 1024 iterations).  Such searches need
 * iterations * 128 < 2^24.                                                 */

/* one root child, in creation order (vanilla: indexed by action id); action
 * 0xFFFF marks unused entries */
typedef struct { uint16_t action; uint16_t pad; uint32_t n; float w; } dvc_child_stat;

#define DVC_MAX_ACTIONS 864

/* Device workspace needed by mcts_search for n_trees trees. */
size_t dvc_mcts_workspace_bytes(int64_t n_trees, const dvc_mcts_params *params /* host */);

/* mcts_search -- one decision for each of n_trees roots (tree ids
 * tree_id_base + t).  Roots must be valid and undecided, in phase 1 (or
 * phase 0 with an empty pool).  best_action[t] receives the chosen action id;
 * root_children (may be NULL) receives [n_trees][864] child statistics.
 * workspace: device memory of at least dvc_mcts_workspace_bytes(), 16-byte
 * aligned; it holds the trees after the call (and their per-tree counters).
 * Returns DVC_EINVAL on bad sizes/params or a misaligned workspace,
 * DVC_ENOMEM if the workspace is too small; malformed roots set DVC_ESTATE in
 * the error word and get best_action -1 and no children.                    */
int mcts_search(const dvc_state_t *roots, int64_t n_trees, const dvc_mcts_params *params /* host */,
                uint64_t seed, uint32_t tree_id_base, void *workspace, size_t workspace_bytes,
                int32_t *best_action, dvc_child_stat *root_children, void *stream);

/* mcts_search_noalloc -- mcts_search for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): no workspace argument and no allocation
 * in the call.  The trees and the natural-log table live in a library-owned
 * static device array, one per device, kept until the process ends:
 * DVC_NOALLOC_TREE_BYTES of trees (dvc_mcts_workspace_bytes(n_trees, params)
 * must not exceed it) and a table of 2^20 entries (iterations times the
 * playouts per leaf -- fallback playouts in value mode -- below 2^20).  The
 * first call on a device sets the array up (its address, then the table,
 * copied synchronously); later calls only enqueue the search.  Same results
 * as mcts_search with the same arguments.  Every call on one device shares
 * that device's array: calls that overlap on one GPU (other streams, other
 * host threads) race, so serialise them.  The array keeps the last call's
 * trees; a call does not depend on them.  Returns DVC_ETOOBIG beyond either
 * limit; other errors as mcts_search.                                    */
#define DVC_NOALLOC_TREE_BYTES (64ull << 20)
int mcts_search_noalloc(const dvc_state_t *roots, int64_t n_trees,
                        const dvc_mcts_params *params /* host */, uint64_t seed,
                        uint32_t tree_id_base, int32_t *best_action,
                        dvc_child_stat *root_children, void *stream);

/* dvc_mcts_autotune -- picks playouts per leaf and leaves per pass for
 * searches like this one (Sec. IV-B: the paper sweeps threads and warps for
 * the simulations; here the leaf's playouts and the leaves evaluated together
 * share the tree's 64 lanes).  params: playout leaves, playouts_per_leaf =
 * the reference P_ref >= 1, leaves_per_pass = 1, pipeline = 0.  Runs the
 * reference (the sequential search with P_ref playouts per leaf) under `seed`
 * and under a second seed (seed ^ 0x9E3779B97F4A7C15); their root-move
 * agreement is the ceiling A0.  Then every candidate (4 playouts x 1/2/4/8/16
 * leaves per pass, 8 x 1/2/4/8, 16 x 1/2/4, 32 x 1/2, 64 x 1, 128 x 1, each
 * without and with pipelined passes; vanilla searches without only) runs once
 * under seed + 1, timed by HIP events on `stream`, and is admitted when its
 * agreement with the
 * reference is at least A0 - tolerance.  The fastest admitted candidate (the
 * reference shape when none is) is remembered for the size class (see the
 * automatic shape above; a library-owned table guarded by a lock, kept until
 * the process ends) and described in *result (host, may be NULL).
 * best_action (device, n_trees) receives the chosen candidate's decisions.
 * workspace as for mcts_search with iterations and variants of params.
 * Synchronizes the stream; 34 searches of this size (18 for vanilla).
 * DVC_EINVAL for value leaves, leaves_per_pass != 1, pipeline != 0,
 * n_trees < 1, a negative tolerance, or iterations * 128 >= 2^24; other
 * errors as mcts_search.                                                   */
typedef struct {
    int32_t playouts_per_leaf, leaves_per_pass;   /* the choice                  */
    float decisions_per_s;                        /* its measured rate           */
    float agreement;                              /* its agreement with the reference */
    float self_agreement;                         /* A0                           */
    int32_t pipeline;                             /* the choice: pipelined passes */
} dvc_mcts_tuning;
int dvc_mcts_autotune(const dvc_state_t *roots, int64_t n_trees, const dvc_mcts_params *params /* host */,
                      uint64_t seed, uint32_t tree_id_base, void *workspace, size_t workspace_bytes,
                      float tolerance, int32_t *best_action, dvc_mcts_tuning *result /* host */,
                      void *stream);

/* mcts_search_root_parallel -- the paper's decomposition (Sec. III-B): each
 * root is searched by trees_per_root (K, 1..65536) independent trees, tree
 * id tree_id_base + r*K + k, each exactly as in mcts_search, and the K trees
 * are amalgamated into one root: a root action's merged N and W are the sums
 * of that action's N and W over the K trees, added in k order (W in float).
 * best_action[r] = the action with the largest merged N, the lowest action id
 * on ties.  merged_children (may be NULL) receives [n_roots][864] statistics
 * indexed by action id (entry a describes action a; action 0xFFFF and zeros
 * where no tree created it).  workspace: dvc_mcts_workspace_bytes(n_roots*K).
 * A root with a malformed state, or any of whose trees gives up, gets
 * best_action -1 and no merged children.  Errors as for mcts_search.       */
int mcts_search_root_parallel(const dvc_state_t *roots, int64_t n_roots, int32_t trees_per_root,
                              const dvc_mcts_params *params /* host */, uint64_t seed,
                              uint32_t tree_id_base, void *workspace, size_t workspace_bytes,
                              int32_t *best_action, dvc_child_stat *merged_children, void *stream);

/* ---------------------------------------------------------------------------
 * Learned leaf evaluator (value network).  The paper weights tree nodes by the
 * results of random playouts (Sec. II-B); this network learns the playout win
 * rate of a perspective seat from (state, win rate) pairs the playout kernel
 * generates, so that most leaves need no playouts.
 * Features (160, zero padded from 148): per tile t (24), the owner relative to
 * the perspective q as a one-hot of 4 ((owner - q) mod P, nothing for pool
 * tiles), revealed, in pool; then (mover - q) mod P as a one-hot of 4.
 * h1 = bf16(relu(W1 x + b1)) (256), h2 = bf16(relu(W2 h1 + b2)) (256),
 * v = sigmoid(w3 . h2 + b3).  Products in bfloat16 on the matrix cores with
 * float32 accumulation; float32 master weights; Adam (beta 0.9 / 0.999,
 * eps 1e-8, bias-corrected) on the mean squared error.
 * Flat parameter order (107265 floats): W1[256][160] (row = output), b1[256],
 * W2[256][256], b2[256], w3[256], b3.
 * ------------------------------------------------------------------------- */
#define DVC_VALUENET_PARAMS 107265

/* bytes of a network blob: weights, Adam moments and bf16 copies (device).
 * Every call taking a blob (and dvc_valuenet_train_step's workspace) needs
 * it 16-byte aligned and returns DVC_EINVAL otherwise.                      */
size_t dvc_valuenet_bytes(void);

/* Initialize a blob: weight k of the flat order takes word k of the Philox
 * stream (k>>2, 0xFFFFFFFE, 0, 0), u = (w >> 8) * 2^-24, U(-b, b) with
 * b = sqrt(6/148) (W1), sqrt(6/256) (W2), 1/16 (w3); biases and moments 0. */
int dvc_valuenet_init(void *net, uint64_t seed, void *stream);

/* Load float32 parameters (device, flat order), reset the Adam moments. */
int dvc_valuenet_set_params(void *net, const float *params, void *stream);

/* Copy the float32 parameters out (device, flat order). */
int dvc_valuenet_get_params(const void *net, float *params, void *stream);

/* Copy the Adam moments out (device, flat order, 107265 floats each): m, the
 * decayed mean of the gradients, and v, the decayed mean of their squares,
 * after the last dvc_valuenet_train_step (Kingma and Ba, 2015; zero after
 * dvc_valuenet_init or dvc_valuenet_set_params).                          */
int dvc_valuenet_get_moments(const void *net, float *m, float *v, void *stream);

/* v_out[i] = value of states[i] for perspective seat persp[i] (< players).
 * A malformed state or perspective sets DVC_ESTATE in the error word.     */
int dvc_valuenet_infer(const void *net, const dvc_state_t *states, const uint8_t *persp,
                       int64_t n, float *v_out, void *stream);

size_t dvc_valuenet_train_workspace_bytes(int64_t batch);

/* One Adam step (number `step` >= 1, learning rate lr) on the mean squared
 * error over `batch` rows; row i is data[(perm_a*(row_base+i) + perm_b) %
 * n_data] of (states, persp, labels).  batch: multiple of 32, <= 65536.
 * loss_out (device float, may be NULL) receives the batch loss before the
 * step; grad_out (device, 107265 floats, may be NULL) the gradient.       */
int dvc_valuenet_train_step(void *net, const dvc_state_t *states, const uint8_t *persp,
                            const float *labels, int64_t n_data, uint32_t perm_a, uint32_t perm_b,
                            uint32_t row_base, int32_t batch, int64_t step, float lr, void *ws,
                            size_t ws_bytes, float *loss_out, float *grad_out, void *stream);

/* Batch order of training epoch `epoch` over n_data pairs (a power of two,
 * 1..2^32): with w0, w1 words 0 and 1 of the Philox block (epoch,
 * 0xFFFFFFFD, 0, 0) under `seed`, perm_a = (w0 | 1) mod n_data (odd, so
 * i -> (perm_a*i + perm_b) mod n_data is a bijection; 1 when n_data is 1)
 * and perm_b = w1 mod n_data, the values dvc_valuenet_train_step takes.
 * Host outputs; no device work.  DVC_EINVAL for an epoch outside
 * 0..2^32-1, an n_data that is not a power of two, or NULL outputs.       */
int dvc_valuenet_epoch_order(uint64_t seed, int64_t epoch, int64_t n_data,
                             uint32_t *perm_a /* host */, uint32_t *perm_b /* host */);

/* Training pairs: for state i (index index_base + i) a perspective seat q =
 * floor(w * P / 2^32) with w word 0 of block (0, 0xFFFFFFFC, 0, index_base+i),
 * and label = (playouts of the state won by q) / playouts, from `playouts`
 * random playouts (tree id tree_id, leaf id index_base + i).  seat_wins_ws:
 * device scratch of n*4 uint32.                                           */
int dvc_valuenet_labels(const dvc_state_t *states, int64_t n, int32_t playouts, uint64_t seed,
                        uint32_t tree_id, uint32_t index_base, uint8_t *persp_out,
                        float *labels_out, uint32_t *seat_wins_ws, void *stream);

/* ---------------------------------------------------------------------------
 * Status
 * ------------------------------------------------------------------------- */
const char *dvc_status_str(int status);

/* Synchronise `stream`, then return and clear the device error word of the
 * current device (DVC_OK when no kernel reported an error).                */
int dvc_check(void *stream);

/* Library version string. */
const char *dvc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DVC_H */
