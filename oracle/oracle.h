/*
 * oracle.h -- plain, slow, single-threaded CPU oracle of the Da Vinci Code
 * Monte Carlo Tree Search hot path (Zhang et al., "Development and Application
 * of a Monte Carlo Tree Search Algorithm for Simulating Da Vinci Code Game
 * Strategies", arXiv 2403.10720).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this code: only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no source with the HIP library; the packed
 * state format and the parameter structs below are re-declared here from the
 * interface description, not included from the library's header.
 *
 * Representation: every player row is an explicit ascending array of tile ids
 * with a per-slot revealed flag, and the draw pile is an explicit ascending
 * array, so that the ordering rule of the game (Sec. II-A: rows are kept in
 * ascending order) is a property the tests can check rather than an artefact
 * of a bit encoding.
 *
 * Functions whose result is pinned by tests: Philox (library routine), the
 * uniform pick (closed form), the rules (invariants, closed form, exact
 * enumeration), the legal guesses and one guess played in the tree (a
 * reference written from the rules), the UCT tree at depth 1 (textbook UCB1)
 * and whole searched trees, playout and value leaves, plain, batched and
 * pipelined passes (a reference loop written from Sec. II-B / III-A), the
 * value network's forward pass, gradient and Adam step (closed forms and an
 * independent numpy forward).  The determinization sampler is pinned against
 * its own exact law, enumerated in the tests from its stated procedure; the
 * paper fixes no distribution, so that law is itself a reading of it.
 */
#ifndef DVC_ORACLE_H
#define DVC_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- packed 16-byte state (interface format) ---------------------------
 * w[0..2] bits 0-23: bit-plane k of the 3-bit owner code of tile t
 *                    (0 = draw pile, 1..4 = seat 0..3).
 * w[3]    bits 0-23: revealed mask.
 * w[0]    bits 24-25 mover, 26-27 players-1, bit 28 phase, bit 29 drawn valid.
 * w[1]    bits 24-28 drawn tile id.
 * all other high bits are zero.
 * Tile id t = 2*value + colour (colour 0 black, 1 white): ids sort by value,
 * black before white on equal value.                                        */
typedef struct { uint32_t w[4]; } orc_packed;

typedef struct {
    int32_t p_min, p_max;
    int32_t hand[5];
    int32_t pile_min, pile_max;
    int32_t revealed_max;
    int32_t fresh;
    int32_t root_draw;
    int32_t phase_mix;
} orc_deal_params;

typedef struct {
    int32_t iterations, playouts_per_leaf, max_depth;
    float c_uct;
    int32_t leaf_eval;
    float fallback_band;
    int32_t fallback_playouts;
    const void *valuenet;
    int32_t continue_choice; /* 1: after a right guess the mover may stop or guess again */
    int32_t vanilla;         /* 1: the root's children are the sampled worlds            */
    int32_t leaves_per_pass; /* B >= 1 descents before their leaves are evaluated        */
    int32_t pipeline;        /* 1: a pass's wins are backed up after the next pass's descents */
} orc_mcts_params;

typedef struct { uint16_t action; uint16_t pad; uint32_t n; float w; } orc_child_stat;

/* explicit game state: ascending rows with per-slot revealed flags */
typedef struct {
    int32_t P;
    int32_t n[4];
    int32_t tile[4][24];
    int32_t rev[4][24];
    int32_t pile_n;
    int32_t pile[24];
    int32_t mover, phase, drawn;
} orc_rows;

#define ORC_MAX_CHILD 864
/* tree keys: guesses 0..863, stop 864, a guess after a right guess 865 + a */
#define ORC_STOP_KEY 864
#define ORC_KEYS (2 * ORC_MAX_CHILD + 1)
/* most leaves evaluated together (leaves_per_pass) */
#define ORC_MAX_PASS 16

/* Philox4x32-10 block (Salmon, Moraes, Dror, Shaw, SC'11). */
void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t oracle_mulshift(uint32_t w, uint32_t k);

/* state codec and validity; returns 0 when valid, else a positive reason code */
int oracle_validate(const orc_packed *s);

/* one playout (random policy) of playout p, leaf l, tree tr; returns winner.
 * If trace is not NULL it receives the explicit state after every guess
 * (at most 23 entries) and *n_trace their number.                           */
int oracle_playout(const orc_packed *s, uint64_t seed, uint32_t p, uint32_t l, uint32_t tr,
                   int *length, orc_rows *trace, int *n_trace);

/* explicit-row codec used by the tests */
int oracle_unpack(const orc_packed *s, orc_rows *r);
void oracle_pack(const orc_rows *r, orc_packed *s);

/* all playouts of n leaves; winner/length/seat_wins may be NULL.
 * returns 0, or -2 when a leaf state is invalid.                            */
int oracle_rollout(const orc_packed *leaves, int64_t n, int32_t ppl, uint64_t seed,
                   uint32_t tree_id, uint32_t leaf_id_base,
                   int8_t *winner, int16_t *length, uint32_t *seat_wins);

/* Same as oracle_rollout but splits leaves over n_threads POSIX threads
 * (identical outputs: every playout has its own counter).                   */
int oracle_rollout_mt(const orc_packed *leaves, int64_t n, int32_t ppl, uint64_t seed,
                      uint32_t tree_id, uint32_t leaf_id_base,
                      int8_t *winner, int16_t *length, uint32_t *seat_wins, int n_threads);

int oracle_init_states(orc_packed *out, int64_t n, const orc_deal_params *p, uint64_t seed,
                       uint32_t index_base);

/* determinized world of iteration i for the root mover; returns the attempt
 * that succeeded (0..63) or 64 for the deterministic fallback, -2 if invalid */
int oracle_determinize(const orc_packed *root, uint64_t seed, uint32_t tree, uint32_t iter,
                       orc_packed *world);

/* legal actions at a state for its mover: writes a 0/1 flag per action id */
int oracle_legal_actions(const orc_packed *s, uint8_t legal[ORC_MAX_CHILD]);

/* apply action at depth d of iteration i (in-tree chance block) */
int oracle_apply_action(const orc_packed *s, int action, uint64_t seed, uint32_t tree,
                        uint32_t iter, uint32_t depth, orc_packed *out, int *terminal,
                        int *winner);

float oracle_ln_entry(uint32_t k);

int oracle_mcts_search(const orc_packed *roots, int64_t n_trees, const orc_mcts_params *mp,
                       uint64_t seed, uint32_t tree_id_base, int32_t *best_action,
                       orc_child_stat *root_children);

/* one node of a searched tree (oracle_mcts_tree_dump) */
typedef struct {
    int32_t parent, key, chooser, depth;
    uint32_t n;
    float w;
    uint64_t world;
} orc_tree_node;

int oracle_mcts_tree_dump(const orc_packed *root, const orc_mcts_params *mp, uint64_t seed,
                          uint32_t tree_id, int32_t *best_action, orc_tree_node *out, int64_t cap);

/* root-parallel search: K trees per root, root statistics summed by action id */
int oracle_mcts_search_merged(const orc_packed *roots, int64_t n_roots, int32_t trees_per_root,
                              const orc_mcts_params *mp, uint64_t seed, uint32_t tree_id_base,
                              int32_t *best_action, orc_child_stat *merged);

/* ---- value network (valuenet.c) ---------------------------------------- */
int oracle_vn_nparams(void);
float oracle_bf16(float x);
int oracle_vn_encode(const orc_packed *s, int32_t q, float feat[160]);
int oracle_vn_forward(const float *params, const orc_packed *states, const int32_t *persp,
                      int64_t n, int bf16, double *v_out);
int oracle_vn_loss_grad(const float *params, const orc_packed *states, const int32_t *persp,
                        const float *labels, int64_t n, int bf16, double *loss, double *grad,
                        double *grad_abs);
void oracle_vn_adam(double *w, double *m, double *v, const double *g, int64_t n, int64_t t,
                    double lr, double b1, double b2, double eps);
void oracle_vn_init(float *params, uint64_t seed);

#ifdef __cplusplus
}
#endif
#endif
