/*
 * mcts.c -- CPU oracle of the simplified Monte Carlo Tree Search for the
 * Da Vinci Code game (Sec. II-B and Sec. III-A of the paper).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The four MCTS steps (selection, expansion, simulation, backpropagation)
 * with the paper's three simplifications (Sec. III-A), each of which can be
 * switched off:
 *   1. a node is only (tile position, guessed number); the sampled set of
 *      plausible opponent numbers is not part of the node.  Off (`vanilla`):
 *      the root's children are the sampled worlds, one node per distinct set
 *      of opponent numbers, and the guesses hang below them;
 *   2. guessing stops after a right guess inside the tree.  Off
 *      (`continue_choice`): after a right guess the same player chooses
 *      between stopping (key 864) and another guess (key 865 + action), so
 *      a player's further guesses are nodes of their own;
 *   3. nodes at a fixed depth threshold are not expanded further: they only
 *      simulate and back up.  Off: max_depth 0.
 * The opponent tiles are a black box to the searching player, so every
 * iteration first samples a plausible set of numbers for them (Sec. III-A);
 * the tree is open loop over those samples.
 *
 * Leaf batching (leaves_per_pass = B): the iterations run in passes of B.
 * Each descent of a pass adds its visit counts along its path as soon as its
 * leaf is found (so the next descent of the pass sees them, with no wins
 * yet); then the pass's leaves are evaluated and each path gets its wins, in
 * iteration order.  B = 1 is the plain sequential search.
 *
 * Pipelined passes (pipeline = 1): the wins of pass k are backed up only
 * after the descents of pass k + 1 (in iteration order, before that pass's
 * leaves are evaluated), and the last pass's after the loop; a descent of
 * pass k thus sees the visits of every earlier descent but the wins of passes
 * up to k - 2.  This is the order in which one worker can descend pass k + 1
 * while another evaluates pass k.
 *
 * Selection uses UCT (Kocsis & Szepesvari 2006) evaluated in single precision
 * with one IEEE rounding per operation, in this order:
 *     n = float(N_c); q = W_c / n; e = LN[N_parent] / n; u = c * sqrt(e);
 *     score = q + u
 * where LN[k] = float(log(double(k))); the first child in creation order
 * with the strictly greatest score wins.  Build with -ffp-contract=off.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int oracle_unpack(const orc_packed *s, orc_rows *r);
void oracle_pack(const orc_rows *r, orc_packed *s);

/* local copies of the small row helpers (rules.c keeps its own static ones) */
static int hidden_count(const orc_rows *s, int q)
{
    int c = 0;
    for (int j = 0; j < s->n[q]; ++j) c += !s->rev[q][j];
    return c;
}

static int alive_count(const orc_rows *s)
{
    int c = 0;
    for (int q = 0; q < s->P; ++q) c += hidden_count(s, q) > 0;
    return c;
}

static int first_alive(const orc_rows *s)
{
    for (int q = 0; q < s->P; ++q)
        if (hidden_count(s, q) > 0) return q;
    return -1;
}

static int next_alive_after(const orc_rows *s, int m)
{
    for (int k = 1; k <= s->P; ++k) {
        int q = (m + k) % s->P;
        if (hidden_count(s, q) > 0) return q;
    }
    return -1;
}

static int owner_of(const orc_rows *s, int t, int *slot)
{
    for (int q = 0; q < s->P; ++q)
        for (int j = 0; j < s->n[q]; ++j)
            if (s->tile[q][j] == t) {
                if (slot) *slot = j;
                return q;
            }
    return -1;
}

static void row_insert(orc_rows *s, int q, int t)
{
    int j = s->n[q];
    while (j > 0 && s->tile[q][j - 1] > t) {
        s->tile[q][j] = s->tile[q][j - 1];
        s->rev[q][j] = s->rev[q][j - 1];
        --j;
    }
    s->tile[q][j] = t;
    s->rev[q][j] = 0;
    s->n[q]++;
}

static void philox_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {c0, c1, c2, c3};
    oracle_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* determinization                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    uint32_t c1, c2, c3;
    uint32_t n;
} dstream;

static uint32_t ds_next(dstream *d)
{
    uint32_t b[4];
    philox_block(d->seed, d->n >> 2, d->c1, d->c2, d->c3, b);
    uint32_t w = b[d->n & 3];
    d->n++;
    return w;
}

/* One attempt of the sampler.  For every opponent (seat order from the
 * mover's left) and every maximal run of hidden slots between two revealed
 * tiles (lo, hi) of its row:
 *   right to left, U_j = largest available tile of the slot's colour below
 *   U_{j+1} (U_{k+1} = hi) -- the largest value the slot can take while the
 *   slots to its right can still be filled;
 *   left to right, t_j is uniform among the available tiles of its colour in
 *   (t_{j-1}, U_j], t_0 = lo.
 * "Available" means: not in the mover's row, not revealed, not yet used.
 * Returns 0 on success, 1 when some opponent's run cannot be filled.        */
static int det_attempt(const orc_rows *root, dstream *ds, orc_rows *world)
{
    *world = *root;
    int M = root->mover;
    int avail[24];
    for (int t = 0; t < 24; ++t) avail[t] = 1;
    for (int q = 0; q < root->P; ++q)
        for (int j = 0; j < root->n[q]; ++j)
            if (q == M || root->rev[q][j]) avail[root->tile[q][j]] = 0;
    for (int k = 1; k < root->P; ++k) {
        int o = (M + k) % root->P;
        int j = 0;
        while (j < root->n[o]) {
            if (root->rev[o][j]) { ++j; continue; }
            int a = j;
            while (j < root->n[o] && !root->rev[o][j]) ++j;
            int b = j;
            int lo = a > 0 ? root->tile[o][a - 1] : -1;
            int hi = b < root->n[o] ? root->tile[o][b] : 24;
            int len = b - a;
            int U[25];
            U[len] = hi;
            for (int i = len - 1; i >= 0; --i) {
                int c = root->tile[o][a + i] & 1;
                int best = -1;
                for (int x = 0; x < U[i + 1]; ++x)
                    if (avail[x] && (x & 1) == c) best = x;
                if (best < 0) return 1;
                U[i] = best;
            }
            if (U[0] <= lo) return 1;
            int prev = lo;
            for (int i = 0; i < len; ++i) {
                int c = root->tile[o][a + i] & 1;
                int cand[24], nc = 0;
                for (int x = prev + 1; x <= U[i]; ++x)
                    if (avail[x] && (x & 1) == c) cand[nc++] = x;
                int x = cand[oracle_mulshift(ds_next(ds), (uint32_t)nc)];
                world->tile[o][a + i] = x;
                avail[x] = 0;
                prev = x;
            }
        }
    }
    world->pile_n = 0;
    for (int t = 0; t < 24; ++t)
        if (avail[t]) world->pile[world->pile_n++] = t;
    return 0;
}

/* Deterministic fallback: the lexicographically smallest consistent
 * assignment of all hidden opponent slots (opponents in seat order from the
 * mover's left, slots left to right), found by depth-first search that tries
 * the lowest tile first.  The true deal is consistent, so it always exists. */
typedef struct {
    int o, j, colour, lo, hi, seg_start;
} dslot;

/* the search gives up (error) after this many calls */
#define ORC_DFS_MAX_CALLS (1L << 22)

static int dfs(dslot *sl, int ns, int k, int *avail, int *assign, long *calls)
{
    if (++*calls > ORC_DFS_MAX_CALLS) return -1;
    if (k == ns) return 1;
    int prev = sl[k].seg_start ? sl[k].lo : assign[k - 1];
    for (int x = prev + 1; x < sl[k].hi; ++x) {
        if (!avail[x] || (x & 1) != sl[k].colour) continue;
        avail[x] = 0;
        assign[k] = x;
        int r = dfs(sl, ns, k + 1, avail, assign, calls);
        if (r != 0) return r;
        avail[x] = 1;
    }
    return 0;
}

static int det_fallback(const orc_rows *root, orc_rows *world)
{
    *world = *root;
    int M = root->mover;
    int avail[24];
    for (int t = 0; t < 24; ++t) avail[t] = 1;
    for (int q = 0; q < root->P; ++q)
        for (int j = 0; j < root->n[q]; ++j)
            if (q == M || root->rev[q][j]) avail[root->tile[q][j]] = 0;
    dslot sl[24];
    int ns = 0;
    for (int k = 1; k < root->P; ++k) {
        int o = (M + k) % root->P;
        for (int j = 0; j < root->n[o]; ++j) {
            if (root->rev[o][j]) continue;
            int lo = -1, hi = 24;
            for (int a = j - 1; a >= 0; --a)
                if (root->rev[o][a]) { lo = root->tile[o][a]; break; }
            for (int a = j + 1; a < root->n[o]; ++a)
                if (root->rev[o][a]) { hi = root->tile[o][a]; break; }
            sl[ns].o = o;
            sl[ns].j = j;
            sl[ns].colour = root->tile[o][j] & 1;
            sl[ns].lo = lo;
            sl[ns].hi = hi;
            sl[ns].seg_start = (j == 0 || root->rev[o][j - 1]);
            ++ns;
        }
    }
    int assign[24];
    long calls = 0;
    if (dfs(sl, ns, 0, avail, assign, &calls) != 1) return 1;
    for (int k = 0; k < ns; ++k) world->tile[sl[k].o][sl[k].j] = assign[k];
    world->pile_n = 0;
    for (int t = 0; t < 24; ++t)
        if (avail[t]) world->pile[world->pile_n++] = t;
    return 0;
}

/* attempts of the random sampler before the deterministic fallback */
#define ORC_DET_ATTEMPTS 64

static int determinize_rows(const orc_rows *root, uint64_t seed, uint32_t tree, uint32_t iter,
                            orc_rows *world)
{
    for (uint32_t a = 0; a < ORC_DET_ATTEMPTS; ++a) {
        dstream ds = {seed, 0x80000000u + a, iter, tree, 0};
        if (det_attempt(root, &ds, world) == 0) return (int)a;
    }
    if (det_fallback(root, world) == 0) return ORC_DET_ATTEMPTS;
    return -3;
}

int oracle_determinize(const orc_packed *root, uint64_t seed, uint32_t tree, uint32_t iter,
                       orc_packed *world)
{
    if (oracle_validate(root)) return -2;
    orc_rows r, w;
    oracle_unpack(root, &r);
    int a = determinize_rows(&r, seed, tree, iter, &w);
    if (a >= 0) oracle_pack(&w, world);
    return a;
}

/* ------------------------------------------------------------------------ */
/* actions                                                                    */
/* ------------------------------------------------------------------------ */
/* action id = ((r-1)*24 + s)*12 + v: target seat (mover + r) mod P, slot s of
 * the target row at guess time, guessed value v (the colour is the slot's). */
static void legal_rows(const orc_rows *s, uint8_t *legal)
{
    memset(legal, 0, ORC_MAX_CHILD);
    int m = s->mover;
    int mine[24] = {0}, revd[24] = {0};
    for (int j = 0; j < s->n[m]; ++j) mine[s->tile[m][j]] = 1;
    for (int q = 0; q < s->P; ++q)
        for (int j = 0; j < s->n[q]; ++j)
            if (s->rev[q][j]) revd[s->tile[q][j]] = 1;
    for (int r = 1; r < s->P; ++r) {
        int q = (m + r) % s->P;
        if (hidden_count(s, q) == 0) continue;
        for (int j = 0; j < s->n[q]; ++j) {
            if (s->rev[q][j]) continue;
            int c = s->tile[q][j] & 1;
            int lo = -1, hi = 24;
            for (int a = j - 1; a >= 0; --a)
                if (s->rev[q][a]) { lo = s->tile[q][a]; break; }
            for (int a = j + 1; a < s->n[q]; ++a)
                if (s->rev[q][a]) { hi = s->tile[q][a]; break; }
            for (int v = 0; v < 12; ++v) {
                int x = 2 * v + c;
                if (x <= lo || x >= hi || mine[x] || revd[x]) continue;
                legal[((r - 1) * 24 + j) * 12 + v] = 1;
            }
        }
    }
}

int oracle_legal_actions(const orc_packed *ps, uint8_t legal[ORC_MAX_CHILD])
{
    if (oracle_validate(ps)) return -2;
    orc_rows s;
    oracle_unpack(ps, &s);
    legal_rows(&s, legal);
    return 0;
}

/* The turn passes: the next seat with hidden tiles draws (word w1). */
static void end_turn(orc_rows *s, int m, uint32_t w1)
{
    int nm = next_alive_after(s, m);
    s->mover = nm;
    s->phase = 1;
    s->drawn = -1;
    if (s->pile_n > 0) {
        int k = (int)oracle_mulshift(w1, (uint32_t)s->pile_n);
        int d = s->pile[k];
        for (int j = k; j + 1 < s->pile_n; ++j) s->pile[j] = s->pile[j + 1];
        s->pile_n--;
        row_insert(s, nm, d);
        s->drawn = d;
    }
}

/* Play tree key `key` (a guess, the stop 864, or a further guess 865 + a).
 * Chance comes from block (depth, 0xC0000000, iter, tree): word 0 picks the
 * mover's own tile to reveal after a wrong guess when nothing was drawn,
 * word 1 is the next player's draw.  A right guess ends the turn unless
 * cont_mode is set; then *cont = 1 and the mover, still in phase 1 with the
 * drawn tile hidden, decides again.  Returns 1 if the game ended.          */
static int apply_rows(orc_rows *s, int key, int cont_mode, uint64_t seed, uint32_t tree,
                      uint32_t iter, uint32_t depth, int *winner, int *cont)
{
    uint32_t w[4];
    philox_block(seed, depth, 0xC0000000u, iter, tree, w);
    int m = s->mover;
    *winner = -1;
    *cont = 0;
    if (key == ORC_STOP_KEY) {
        end_turn(s, m, w[1]);
        return 0;
    }
    int action = key > ORC_STOP_KEY ? key - ORC_STOP_KEY - 1 : key;
    int r = action / 288 + 1, slot = (action / 12) % 24, v = action % 12;
    int q = (m + r) % s->P;
    int t = s->tile[q][slot];
    int guess = 2 * v + (t & 1);
    int right = guess == t;
    if (right) {
        s->rev[q][slot] = 1;
    } else if (s->drawn >= 0) {
        int j = 0, o = owner_of(s, s->drawn, &j);
        s->rev[o][j] = 1;
    } else {
        int nH = 0, Hj[24];
        for (int j = 0; j < s->n[m]; ++j)
            if (!s->rev[m][j]) Hj[nH++] = j;
        s->rev[m][Hj[oracle_mulshift(w[0], (uint32_t)nH)]] = 1;
    }
    if (alive_count(s) == 1) {
        *winner = first_alive(s);
        s->phase = 1;
        s->drawn = -1;
        return 1;
    }
    if (right && cont_mode) {
        *cont = 1;
        return 0;
    }
    end_turn(s, m, w[1]);
    return 0;
}

/* A leaf reached right after a right guess (continue choice on): the random
 * policy's continue coin, word 3 of the chance block of that guess, decides
 * once for all the leaf's playouts -- below 2^31 the mover goes on guessing
 * in the playouts, otherwise the turn passes (word 1 draws).               */
static void leaf_continue_coin(orc_rows *s, uint64_t seed, uint32_t tree, uint32_t iter,
                               uint32_t depth)
{
    uint32_t w[4];
    philox_block(seed, depth, 0xC0000000u, iter, tree, w);
    if (w[3] >= 0x80000000u) end_turn(s, s->mover, w[1]);
}

int oracle_apply_action(const orc_packed *ps, int action, uint64_t seed, uint32_t tree,
                        uint32_t iter, uint32_t depth, orc_packed *out, int *terminal,
                        int *winner)
{
    if (oracle_validate(ps)) return -2;
    if (action < 0 || action >= ORC_MAX_CHILD) return -1;
    orc_rows s;
    oracle_unpack(ps, &s);
    uint8_t legal[ORC_MAX_CHILD];
    legal_rows(&s, legal);
    if (!legal[action]) return -1;
    int cont = 0;
    *terminal = apply_rows(&s, action, 0, seed, tree, iter, depth, winner, &cont);
    oracle_pack(&s, out);
    return 0;
}

float oracle_ln_entry(uint32_t k)
{
    return (float)log((double)k);
}

/* ------------------------------------------------------------------------ */
/* search                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int action, chooser; /* a world node has action -1 and chooser -1 */
    uint64_t world;      /* world node: its key (world_key)            */
    uint32_t N;
    float W;
    int nchild, cap;
    int *child;
    uint8_t *has; /* per tree key: 1 if a child with that key exists */
} onode;

typedef struct {
    onode *v;
    int n, cap;
} otree;

static int tree_new_node(otree *t, int action, int chooser)
{
    if (t->n == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 64;
        t->v = (onode *)realloc(t->v, (size_t)t->cap * sizeof(onode));
    }
    onode *x = &t->v[t->n];
    memset(x, 0, sizeof(*x));
    x->action = action;
    x->chooser = chooser;
    return t->n++;
}

static void node_add_child(otree *t, int parent, int child)
{
    onode *p = &t->v[parent];
    if (!p->has) p->has = (uint8_t *)calloc(ORC_KEYS, 1);
    if (p->nchild == p->cap) {
        p->cap = p->cap ? 2 * p->cap : 8;
        p->child = (int *)realloc(p->child, (size_t)p->cap * sizeof(int));
    }
    p->child[p->nchild++] = child;
    if (t->v[child].action >= 0) p->has[t->v[child].action] = 1;
}

static void tree_free(otree *t)
{
    for (int i = 0; i < t->n; ++i) {
        free(t->v[i].child);
        free(t->v[i].has);
    }
    free(t->v);
}

/* The sampled set of opponent numbers as a 48-bit key: 2 bits per tile, the
 * holder's seat relative to the root mover (1..3) when an opponent holds the
 * tile hidden, else 0.  Two worlds of one root are equal iff their keys are. */
static uint64_t world_key(const orc_rows *w, int M)
{
    uint64_t key = 0;
    for (int q = 0; q < w->P; ++q) {
        if (q == M) continue;
        uint64_t r = (uint64_t)((q - M + w->P) % w->P);
        for (int j = 0; j < w->n[q]; ++j)
            if (!w->rev[q][j]) key |= r << (2 * w->tile[q][j]);
    }
    return key;
}

/* A tree key is playable at a state: guesses only when the mover has not
 * just guessed right, the stop and further guesses only when it has. */
static int key_legal(int key, int cont, const uint8_t *legal)
{
    if (key == ORC_STOP_KEY) return cont;
    if (key > ORC_STOP_KEY) return cont && legal[key - ORC_STOP_KEY - 1];
    return !cont && legal[key];
}

int rollout_rows_wins(const orc_rows *leaf, int32_t ppl, uint64_t seed, uint32_t leaf_id,
                      uint32_t tree_id, uint32_t wins[4]);

/* Leaf evaluation in value mode: the network's win probability of every
 * seat (bf16-mirroring forward); when the root player's value lies within
 * `band` of 1/2 the leaf is played out instead.  Either way the leaf weighs
 * `fallback_playouts`: W gains playout wins, or fallback_playouts * v.    */
static void value_leaf(const orc_rows *S, int root_mover, const orc_mcts_params *mp, uint64_t seed,
                       uint32_t leaf_id, uint32_t tr, float vals[4])
{
    orc_packed ps;
    oracle_pack(S, &ps);
    double v[4] = {0, 0, 0, 0};
    for (int q = 0; q < S->P; ++q) {
        int32_t qq = q;
        oracle_vn_forward((const float *)mp->valuenet, &ps, &qq, 1, 1, &v[q]);
    }
    float vm = (float)v[root_mover];
    float d = vm - 0.5f;
    if (d < 0.0f) d = -d;
    if (d < mp->fallback_band) {
        uint32_t wins[4];
        rollout_rows_wins(S, mp->fallback_playouts, seed, leaf_id, tr, wins);
        for (int k = 0; k < 4; ++k) vals[k] = (float)wins[k];
    } else {
        for (int k = 0; k < 4; ++k) vals[k] = (float)mp->fallback_playouts * (float)v[k];
    }
}

/* One tree's search.  If keep is not NULL the tree is handed to the caller
 * (who frees it) instead of being freed. */
static int search_one(const orc_rows *root, const orc_mcts_params *mp, uint64_t seed,
                      uint32_t tr, const float *LN, int32_t *best_action,
                      orc_child_stat *children_out, otree *keep)
{
    otree T = {0};
    tree_new_node(&T, -1, -1);
    int ppl = mp->leaf_eval ? mp->fallback_playouts : mp->playouts_per_leaf;
    int B = mp->leaves_per_pass;
    int path[ORC_MAX_PASS][128], np[ORC_MAX_PASS], terminal[ORC_MAX_PASS], winner[ORC_MAX_PASS];
    orc_rows leafS[ORC_MAX_PASS];
    uint8_t legal[ORC_MAX_CHILD];
    /* pipelined passes: the previous pass's paths and leaf values, not yet
       backed up */
    int pend_path[ORC_MAX_PASS][128], pend_np[ORC_MAX_PASS], pend_n = 0;
    float pend_vals[ORC_MAX_PASS][4];
    for (int i0 = 0; i0 < mp->iterations; i0 += B) {
        int nb = mp->iterations - i0 < B ? mp->iterations - i0 : B;
        for (int b = 0; b < nb; ++b) {
            int i = i0 + b;
            orc_rows S;
            if (determinize_rows(root, seed, tr, (uint32_t)i, &S) < 0) {
                tree_free(&T);
                return -3;
            }
            int node = 0, depth = 0, cont = 0, last_block = -1;
            int *pth = path[b];
            np[b] = 0;
            terminal[b] = 0;
            winner[b] = -1;
            pth[np[b]++] = 0;
            if (mp->vanilla) {
                /* the world node of this sample: found among the root's
                   children by its key, or appended */
                uint64_t key = world_key(&S, root->mover);
                int found = -1;
                for (int k = 0; k < T.v[0].nchild; ++k)
                    if (T.v[T.v[0].child[k]].world == key) { found = T.v[0].child[k]; break; }
                if (found < 0) {
                    found = tree_new_node(&T, -1, -1);
                    T.v[found].world = key;
                    node_add_child(&T, 0, found);
                }
                node = found;
                pth[np[b]++] = node;
            }
            for (;;) {
                if (terminal[b]) break;
                if (mp->max_depth > 0 && depth >= mp->max_depth) break;
                legal_rows(&S, legal);
                onode *X = &T.v[node];
                /* expansion: the lowest playable key without a child */
                int expand = -1;
                for (int k = 0; k < ORC_KEYS; ++k)
                    if (key_legal(k, cont, legal) && !(X->has && X->has[k])) { expand = k; break; }
                if (expand >= 0) {
                    int c = tree_new_node(&T, expand, S.mover);
                    node_add_child(&T, node, c);
                    terminal[b] = apply_rows(&S, expand, mp->continue_choice, seed, tr, (uint32_t)i,
                                             (uint32_t)depth, &winner[b], &cont);
                    last_block = depth;
                    pth[np[b]++] = c;
                    break;
                }
                /* selection: strictly greater score wins, so ties keep the
                   earliest-created child */
                X = &T.v[node];
                float Lp = LN[X->N];
                int best = -1;
                float best_s = 0.0f;
                for (int k = 0; k < X->nchild; ++k) {
                    onode *c = &T.v[X->child[k]];
                    if (!key_legal(c->action, cont, legal)) continue;
                    float n = (float)c->N;
                    float q = c->W / n;
                    float e = Lp / n;
                    float u = mp->c_uct * sqrtf(e);
                    float s = q + u;
                    if (best < 0 || s > best_s) { best = X->child[k]; best_s = s; }
                }
                terminal[b] = apply_rows(&S, T.v[best].action, mp->continue_choice, seed, tr,
                                         (uint32_t)i, (uint32_t)depth, &winner[b], &cont);
                last_block = depth;
                node = best;
                pth[np[b]++] = best;
                ++depth;
            }
            if (!terminal[b] && cont)
                leaf_continue_coin(&S, seed, tr, (uint32_t)i, (uint32_t)last_block);
            leafS[b] = S;
            /* the visit counts go in at once */
            for (int k = 0; k < np[b]; ++k) T.v[pth[k]].N += (uint32_t)ppl;
        }
        /* pipelined: the previous pass's wins go in now, after this pass's
           descents */
        for (int b = 0; b < pend_n; ++b)
            for (int k = 1; k < pend_np[b]; ++k) {
                onode *x = &T.v[pend_path[b][k]];
                if (x->chooser >= 0) x->W += pend_vals[b][x->chooser];
            }
        pend_n = 0;
        for (int b = 0; b < nb; ++b) {
            int i = i0 + b;
            float vals[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (terminal[b]) {
                vals[winner[b]] = (float)ppl;
            } else if (mp->leaf_eval) {
                value_leaf(&leafS[b], root->mover, mp, seed, (uint32_t)i, tr, vals);
            } else {
                uint32_t wins[4] = {0, 0, 0, 0};
                rollout_rows_wins(&leafS[b], ppl, seed, (uint32_t)i, tr, wins);
                for (int k = 0; k < 4; ++k) vals[k] = (float)wins[k];
            }
            if (mp->pipeline) {
                for (int k = 0; k < np[b]; ++k) pend_path[b][k] = path[b][k];
                pend_np[b] = np[b];
                for (int k = 0; k < 4; ++k) pend_vals[b][k] = vals[k];
                pend_n = b + 1;
                continue;
            }
            for (int k = 1; k < np[b]; ++k) {
                onode *x = &T.v[path[b][k]];
                if (x->chooser >= 0) x->W += vals[x->chooser];
            }
        }
    }
    for (int b = 0; b < pend_n; ++b)   /* the last pipelined pass */
        for (int k = 1; k < pend_np[b]; ++k) {
            onode *x = &T.v[pend_path[b][k]];
            if (x->chooser >= 0) x->W += pend_vals[b][x->chooser];
        }
    onode *R = &T.v[0];
    if (mp->vanilla) {
        /* a guess is judged over all worlds: its statistics are summed over
           the world nodes in creation order; most visits wins, the lowest
           action id on ties; children_out is indexed by action id */
        uint32_t n[ORC_MAX_CHILD];
        float w[ORC_MAX_CHILD];
        for (int a = 0; a < ORC_MAX_CHILD; ++a) { n[a] = 0; w[a] = 0.0f; }
        for (int k = 0; k < R->nchild; ++k) {
            onode *x = &T.v[R->child[k]];
            for (int j = 0; j < x->nchild; ++j) {
                onode *c = &T.v[x->child[j]];
                n[c->action] += c->N;
                w[c->action] += c->W;
            }
        }
        int best = -1;
        for (int a = 0; a < ORC_MAX_CHILD; ++a)
            if (n[a] > 0 && (best < 0 || n[a] > n[best])) best = a;
        *best_action = best;
        if (children_out)
            for (int a = 0; a < ORC_MAX_CHILD; ++a) {
                children_out[a].action = n[a] > 0 ? (uint16_t)a : 0xFFFF;
                children_out[a].pad = 0;
                children_out[a].n = n[a];
                children_out[a].w = w[a];
            }
        if (keep) *keep = T; else tree_free(&T);
        return 0;
    }
    int best = -1;
    uint32_t bestN = 0;
    for (int k = 0; k < R->nchild; ++k) {
        onode *c = &T.v[R->child[k]];
        if (best < 0 || c->N > bestN) { best = k; bestN = c->N; }
    }
    *best_action = best >= 0 ? T.v[R->child[best]].action : -1;
    if (children_out) {
        for (int k = 0; k < ORC_MAX_CHILD; ++k) {
            children_out[k].action = 0xFFFF;
            children_out[k].pad = 0;
            children_out[k].n = 0;
            children_out[k].w = 0.0f;
        }
        for (int k = 0; k < R->nchild; ++k) {
            onode *c = &T.v[R->child[k]];
            children_out[k].action = (uint16_t)c->action;
            children_out[k].n = c->N;
            children_out[k].w = c->W;
        }
    }
    if (keep) *keep = T; else tree_free(&T);
    return 0;
}

static float *ln_table(const orc_mcts_params *mp)
{
    uint64_t w_leaf = (uint64_t)(mp->leaf_eval ? mp->fallback_playouts : mp->playouts_per_leaf);
    uint64_t nln = (uint64_t)mp->iterations * w_leaf + 1;
    float *LN = (float *)malloc(nln * sizeof(float));
    LN[0] = 0.0f;
    for (uint64_t k = 1; k < nln; ++k) LN[k] = oracle_ln_entry((uint32_t)k);
    return LN;
}

int oracle_mcts_search(const orc_packed *roots, int64_t n_trees, const orc_mcts_params *mp,
                       uint64_t seed, uint32_t tree_id_base, int32_t *best_action,
                       orc_child_stat *root_children)
{
    if (n_trees < 0 || mp->iterations < 1 || mp->playouts_per_leaf < 1 || mp->max_depth < 0 ||
        mp->max_depth > 64 || mp->leaf_eval < 0 || mp->leaf_eval > 1 ||
        (mp->continue_choice != 0 && mp->continue_choice != 1) ||
        (mp->vanilla != 0 && mp->vanilla != 1) || mp->leaves_per_pass < 1 ||
        mp->leaves_per_pass > ORC_MAX_PASS || (mp->pipeline != 0 && mp->pipeline != 1) ||
        (mp->pipeline && mp->vanilla))
        return -1;
    if (mp->leaf_eval && (mp->valuenet == NULL || mp->fallback_playouts < 1)) return -1;
    for (int64_t t = 0; t < n_trees; ++t) {
        if (oracle_validate(&roots[t])) return -2;
        orc_rows r;
        oracle_unpack(&roots[t], &r);
        if (alive_count(&r) < 2) return -2;
        if (r.phase == 0 && r.pile_n > 0) return -2;
    }
    float *LN = ln_table(mp);
    int rc = 0;
    for (int64_t t = 0; t < n_trees && rc == 0; ++t) {
        orc_rows r;
        oracle_unpack(&roots[t], &r);
        rc = search_one(&r, mp, seed, tree_id_base + (uint32_t)t, LN, &best_action[t],
                        root_children ? root_children + t * ORC_MAX_CHILD : NULL, NULL);
    }
    free(LN);
    return rc;
}

/* The whole tree of one search (tree id tree_id), nodes in creation order:
 * parent (-1 for the root), key (-1 for the root and world nodes), chooser,
 * depth in guesses and stops (world nodes share the root's 0), N, W, world
 * key.  Writes at most cap nodes; returns the node count, or a negative
 * error as oracle_mcts_search. */
int oracle_mcts_tree_dump(const orc_packed *root, const orc_mcts_params *mp, uint64_t seed,
                          uint32_t tree_id, int32_t *best_action, orc_tree_node *out, int64_t cap)
{
    int32_t b;
    int rc = oracle_mcts_search(root, 0, mp, seed, tree_id, &b, NULL);   /* parameter checks */
    if (rc) return rc;
    if (oracle_validate(root)) return -2;
    orc_rows r;
    oracle_unpack(root, &r);
    if (alive_count(&r) < 2 || (r.phase == 0 && r.pile_n > 0)) return -2;
    float *LN = ln_table(mp);
    otree T = {0};
    rc = search_one(&r, mp, seed, tree_id, LN, best_action, NULL, &T);
    free(LN);
    if (rc) return rc;
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)T.n);
    int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * (size_t)T.n);
    parent[0] = -1;
    depth[0] = 0;
    /* children are always created after their parent */
    for (int x = 0; x < T.n; ++x)
        for (int k = 0; k < T.v[x].nchild; ++k) {
            int c = T.v[x].child[k];
            parent[c] = x;
            depth[c] = depth[x] + (T.v[c].action >= 0);
        }
    for (int x = 0; x < T.n && x < cap; ++x) {
        out[x].parent = parent[x];
        out[x].key = T.v[x].action;
        out[x].chooser = T.v[x].chooser;
        out[x].depth = depth[x];
        out[x].n = T.v[x].N;
        out[x].w = T.v[x].W;
        out[x].world = T.v[x].world;
    }
    int n = T.n;
    free(parent);
    free(depth);
    tree_free(&T);
    return n;
}

/* Root-parallel search (Sec. III-B): each root is searched by K independent
 * trees, tree id tree_id_base + r*K + k, and the trees are amalgamated into
 * one root: a root action's merged visit count and win sum are the sums of
 * that action's (N, W) over the K trees, added in k order.  The decision is
 * the action with the largest merged N, the lowest action id on ties.
 * merged[r][a] is indexed by action id; actions no tree created have action
 * 0xFFFF and zero statistics. */
int oracle_mcts_search_merged(const orc_packed *roots, int64_t n_roots, int32_t trees_per_root,
                              const orc_mcts_params *mp, uint64_t seed, uint32_t tree_id_base,
                              int32_t *best_action, orc_child_stat *merged)
{
    if (n_roots < 0 || trees_per_root < 1 || mp->vanilla) return -1;
    orc_packed *copies = (orc_packed *)malloc(sizeof(orc_packed) * (size_t)(trees_per_root > 0 ? trees_per_root : 1));
    int32_t *best_k = (int32_t *)malloc(sizeof(int32_t) * (size_t)trees_per_root);
    orc_child_stat *kids = (orc_child_stat *)malloc(sizeof(orc_child_stat) * ORC_MAX_CHILD * (size_t)trees_per_root);
    int rc = 0;
    for (int64_t r = 0; r < n_roots && rc == 0; ++r) {
        for (int32_t k = 0; k < trees_per_root; ++k) copies[k] = roots[r];
        rc = oracle_mcts_search(copies, trees_per_root, mp, seed,
                                tree_id_base + (uint32_t)(r * trees_per_root), best_k, kids);
        if (rc) break;
        uint32_t n[ORC_MAX_CHILD];
        float w[ORC_MAX_CHILD];
        for (int a = 0; a < ORC_MAX_CHILD; ++a) { n[a] = 0; w[a] = 0.0f; }
        for (int32_t k = 0; k < trees_per_root; ++k)
            for (int c = 0; c < ORC_MAX_CHILD; ++c) {
                const orc_child_stat *s = &kids[(size_t)k * ORC_MAX_CHILD + c];
                if (s->action == 0xFFFF) break;
                n[s->action] += s->n;
                w[s->action] += s->w;
            }
        int best = -1;
        for (int a = 0; a < ORC_MAX_CHILD; ++a)
            if (n[a] > 0 && (best < 0 || n[a] > n[best])) best = a;
        best_action[r] = best;
        if (merged) {
            for (int a = 0; a < ORC_MAX_CHILD; ++a) {
                orc_child_stat *m = &merged[(size_t)r * ORC_MAX_CHILD + a];
                m->action = n[a] > 0 ? (uint16_t)a : 0xFFFF;
                m->pad = 0;
                m->n = n[a];
                m->w = w[a];
            }
        }
    }
    free(copies);
    free(best_k);
    free(kids);
    return rc;
}
