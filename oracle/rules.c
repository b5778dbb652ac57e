/*
 * rules.c -- CPU oracle: random numbers, state codec, the rules of one
 * playout, leaf rollouts and the synthetic state generator.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain C, single-threaded except
 * for oracle_rollout_mt, which runs the same per-playout function on several
 * threads for the CPU baseline.
 *
 * Game rules restated from Sec. II-A of the paper:
 *   - 24 numbered tiles, values 0..11 in black and white (jokers excluded);
 *   - every player keeps a row in ascending order, visible only to its owner;
 *     the colour of every tile is public;
 *   - a turn: draw a tile from the pool and insert it in order, then guess the
 *     value of an opponent tile; a right guess reveals that tile and lets the
 *     player guess again or stop; a wrong guess reveals the player's newly
 *     drawn tile and ends the turn;
 *   - a player whose tiles are all revealed is out; the last one standing wins.
 * The random playout picks every decision at random (Sec. II-B).  Readings of
 * points the paper leaves open (which tile is targeted, which values count as
 * consistent, continue probability, wrong guess with an empty pool, turn
 * order, tie order of equal values) are listed with the interface format.
 */
#include "oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: a 10-round Feistel-like bijection on four 32-bit words.   */
/* Each round multiplies words 0 and 2 by fixed odd constants, keeps the     */
/* low halves and xors the high halves with the other two words and the      */
/* round key; the two key words are advanced by Weyl constants between       */
/* rounds (Salmon et al., SC'11, Sec. 3).                                    */
/* ------------------------------------------------------------------------ */
void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform pick of one of k items from a 32-bit word: floor(w * k / 2^32) */
uint32_t oracle_mulshift(uint32_t w, uint32_t k)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)k) >> 32);
}

static void key_of(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

/* sequential word stream: word n lives in block (n>>2, c1, c2, c3), slot n&3 */
typedef struct {
    uint32_t key[2];
    uint32_t c1, c2, c3;
    uint32_t n;
    uint32_t block[4];
    uint32_t block_id;
    int have;
} wstream;

static void ws_init(wstream *ws, uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3)
{
    key_of(seed, ws->key);
    ws->c1 = c1; ws->c2 = c2; ws->c3 = c3;
    ws->n = 0; ws->have = 0;
}

static uint32_t ws_next(wstream *ws)
{
    uint32_t b = ws->n >> 2;
    if (!ws->have || ws->block_id != b) {
        uint32_t ctr[4] = {b, ws->c1, ws->c2, ws->c3};
        oracle_philox(ctr, ws->key, ws->block);
        ws->block_id = b;
        ws->have = 1;
    }
    uint32_t w = ws->block[ws->n & 3];
    ws->n++;
    return w;
}

/* ------------------------------------------------------------------------ */
/* explicit state helpers                                                   */
/* ------------------------------------------------------------------------ */
static int colour_of(int t) { return t & 1; }

/* returns the seat owning tile t and its slot, or -1 when t is in the pile */
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

static int is_revealed(const orc_rows *s, int t)
{
    int j = 0, q = owner_of(s, t, &j);
    return q >= 0 && s->rev[q][j];
}

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

/* insert tile t as a hidden tile into row q, keeping ascending order */
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

static void pile_remove_at(orc_rows *s, int k)
{
    for (int j = k; j + 1 < s->pile_n; ++j) s->pile[j] = s->pile[j + 1];
    s->pile_n--;
}

static void reveal_tile(orc_rows *s, int t)
{
    int j = 0, q = owner_of(s, t, &j);
    if (q >= 0) s->rev[q][j] = 1;
}

/* mover m draws pile[k] into its row */
static int draw_at(orc_rows *s, int m, int k)
{
    int d = s->pile[k];
    pile_remove_at(s, k);
    row_insert(s, m, d);
    return d;
}

/* ------------------------------------------------------------------------ */
/* codec                                                                    */
/* ------------------------------------------------------------------------ */
int oracle_unpack(const orc_packed *ps, orc_rows *r)
{
    memset(r, 0, sizeof(*r));
    const uint32_t *w = ps->w;
    r->mover = (int)((w[0] >> 24) & 3u);
    r->P = (int)((w[0] >> 26) & 3u) + 1;
    r->phase = (int)((w[0] >> 28) & 1u);
    int dvalid = (int)((w[0] >> 29) & 1u);
    r->drawn = dvalid ? (int)((w[1] >> 24) & 31u) : -1;
    if ((w[0] >> 30) != 0u) return 1;
    if ((w[1] >> 29) != 0u) return 1;
    if ((w[2] >> 24) != 0u || (w[3] >> 24) != 0u) return 1;
    if (!dvalid && ((w[1] >> 24) & 31u) != 0u) return 1;
    if (r->P < 2) return 2;
    for (int t = 0; t < 24; ++t) {
        int code = (int)(((w[0] >> t) & 1u) | (((w[1] >> t) & 1u) << 1) | (((w[2] >> t) & 1u) << 2));
        int rv = (int)((w[3] >> t) & 1u);
        if (code == 0) {
            if (rv) return 3;
            r->pile[r->pile_n++] = t;
        } else {
            int q = code - 1;
            if (q >= r->P) return 4;
            r->tile[q][r->n[q]] = t;
            r->rev[q][r->n[q]] = rv;
            r->n[q]++;
        }
    }
    return 0;
}

void oracle_pack(const orc_rows *r, orc_packed *ps)
{
    uint32_t w[4] = {0, 0, 0, 0};
    for (int q = 0; q < r->P; ++q)
        for (int j = 0; j < r->n[q]; ++j) {
            int t = r->tile[q][j];
            uint32_t code = (uint32_t)(q + 1);
            w[0] |= (code & 1u) << t;
            w[1] |= ((code >> 1) & 1u) << t;
            w[2] |= ((code >> 2) & 1u) << t;
            if (r->rev[q][j]) w[3] |= 1u << t;
        }
    w[0] |= ((uint32_t)r->mover & 3u) << 24;
    w[0] |= ((uint32_t)(r->P - 1) & 3u) << 26;
    w[0] |= ((uint32_t)r->phase & 1u) << 28;
    if (r->drawn >= 0) {
        w[0] |= 1u << 29;
        w[1] |= ((uint32_t)r->drawn & 31u) << 24;
    }
    for (int k = 0; k < 4; ++k) ps->w[k] = w[k];
}

int oracle_validate(const orc_packed *ps)
{
    orc_rows r;
    int e = oracle_unpack(ps, &r);
    if (e) return e;
    if (r.mover >= r.P) return 5;
    if (hidden_count(&r, r.mover) == 0) return 6;
    if (r.phase == 0 && r.drawn >= 0) return 7;
    if (r.drawn >= 0) {
        int j = 0, q = owner_of(&r, r.drawn, &j);
        if (q != r.mover || r.rev[q][j]) return 8;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* one random playout                                                        */
/* ------------------------------------------------------------------------ */
/* Candidate values for the hidden tile of row o at slot j, as the mover m
 * sees it: same colour, strictly between the nearest revealed tiles on its
 * left and right in that row, not in m's own row and not revealed anywhere.
 * Writes the candidate tile ids ascending and returns their number.        */
static int candidates(const orc_rows *s, int m, int o, int j, int *out)
{
    int t = s->tile[o][j];
    int lo = -1, hi = 24;
    for (int k = j - 1; k >= 0; --k)
        if (s->rev[o][k]) { lo = s->tile[o][k]; break; }
    for (int k = j + 1; k < s->n[o]; ++k)
        if (s->rev[o][k]) { hi = s->tile[o][k]; break; }
    int c = 0;
    for (int x = 0; x < 24; ++x) {
        if (colour_of(x) != colour_of(t)) continue;
        if (x <= lo || x >= hi) continue;
        int own = 0;
        for (int k = 0; k < s->n[m]; ++k)
            if (s->tile[m][k] == x) own = 1;
        if (own || is_revealed(s, x)) continue;
        out[c++] = x;
    }
    return c;
}

static int playout_rows(orc_rows *s, const uint32_t key[2], uint32_t p, uint32_t l, uint32_t tr,
                        int *length, orc_rows *trace, int *n_trace)
{
    int len = 0;
    if (n_trace) *n_trace = 0;
    if (alive_count(s) == 1) {
        *length = 0;
        return first_alive(s);
    }
    for (uint32_t g = 0;; ++g) {
        uint32_t ctr[4] = {g, p, l, tr}, w[4];
        oracle_philox(ctr, key, w);
        int m = s->mover;
        if (s->phase == 0) {
            if (s->pile_n > 0)
                s->drawn = draw_at(s, m, (int)oracle_mulshift(w[0], (uint32_t)s->pile_n));
            else
                s->drawn = -1;
            s->phase = 1;
        }
        /* target: uniform over the hidden tiles of every other seat, pooled,
           in ascending tile order */
        int T[24], nT = 0;
        for (int t = 0; t < 24; ++t) {
            int j = 0, q = owner_of(s, t, &j);
            if (q >= 0 && q != m && !s->rev[q][j]) T[nT++] = t;
        }
        int t = T[oracle_mulshift(w[1], (uint32_t)nT)];
        int jt = 0, o = owner_of(s, t, &jt);
        int C[24];
        int nC = candidates(s, m, o, jt, C);
        int v = C[oracle_mulshift(w[2], (uint32_t)nC)];
        len++;
        int turn_over;
        if (v == t) {
            s->rev[o][jt] = 1;
            turn_over = !(w[3] < 0x80000000u);
        } else {
            if (s->drawn >= 0) {
                reveal_tile(s, s->drawn);
            } else {
                int H[24], nH = 0;
                for (int k = 0; k < s->n[m]; ++k)
                    if (!s->rev[m][k]) H[nH++] = s->tile[m][k];
                reveal_tile(s, H[oracle_mulshift(w[3], (uint32_t)nH)]);
            }
            turn_over = 1;
        }
        if (trace) trace[(*n_trace)++] = *s;
        if (alive_count(s) == 1) {
            *length = len;
            return first_alive(s);
        }
        if (turn_over) {
            s->mover = next_alive_after(s, m);
            s->phase = 0;
            s->drawn = -1;
        }
    }
}

int oracle_playout(const orc_packed *ps, uint64_t seed, uint32_t p, uint32_t l, uint32_t tr,
                   int *length, orc_rows *trace, int *n_trace)
{
    if (oracle_validate(ps)) return -2;
    orc_rows s;
    oracle_unpack(ps, &s);
    uint32_t key[2];
    key_of(seed, key);
    return playout_rows(&s, key, p, l, tr, length, trace, n_trace);
}

int oracle_rollout(const orc_packed *leaves, int64_t n, int32_t ppl, uint64_t seed,
                   uint32_t tree_id, uint32_t leaf_id_base,
                   int8_t *winner, int16_t *length, uint32_t *seat_wins)
{
    if (n < 0 || ppl < 0) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (oracle_validate(&leaves[i])) return -2;
    uint32_t key[2];
    key_of(seed, key);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t wins[4] = {0, 0, 0, 0};
        orc_rows s0;
        oracle_unpack(&leaves[i], &s0);
        for (int32_t p = 0; p < ppl; ++p) {
            orc_rows s = s0;
            int len = 0;
            int win = playout_rows(&s, key, (uint32_t)p, leaf_id_base + (uint32_t)i, tree_id, &len,
                                   NULL, NULL);
            wins[win]++;
            if (winner) winner[i * ppl + p] = (int8_t)win;
            if (length) length[i * ppl + p] = (int16_t)len;
        }
        if (seat_wins)
            for (int k = 0; k < 4; ++k) seat_wins[i * 4 + k] = wins[k];
    }
    return 0;
}

typedef struct {
    const orc_packed *leaves;
    int64_t lo, hi;
    int32_t ppl;
    uint64_t seed;
    uint32_t tree_id, leaf_id_base;
    int8_t *winner;
    int16_t *length;
    uint32_t *seat_wins;
} rollout_job;

static void *rollout_worker(void *arg)
{
    rollout_job *j = (rollout_job *)arg;
    int64_t n = j->hi - j->lo;
    oracle_rollout(j->leaves + j->lo, n, j->ppl, j->seed, j->tree_id,
                   j->leaf_id_base + (uint32_t)j->lo,
                   j->winner ? j->winner + j->lo * j->ppl : NULL,
                   j->length ? j->length + j->lo * j->ppl : NULL,
                   j->seat_wins ? j->seat_wins + j->lo * 4 : NULL);
    return NULL;
}

int oracle_rollout_mt(const orc_packed *leaves, int64_t n, int32_t ppl, uint64_t seed,
                      uint32_t tree_id, uint32_t leaf_id_base,
                      int8_t *winner, int16_t *length, uint32_t *seat_wins, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    for (int64_t i = 0; i < n; ++i)
        if (oracle_validate(&leaves[i])) return -2;
    pthread_t th[256];
    rollout_job jobs[256];
    for (int k = 0; k < n_threads; ++k) {
        jobs[k].leaves = leaves;
        jobs[k].lo = n * k / n_threads;
        jobs[k].hi = n * (k + 1) / n_threads;
        jobs[k].ppl = ppl;
        jobs[k].seed = seed;
        jobs[k].tree_id = tree_id;
        jobs[k].leaf_id_base = leaf_id_base;
        jobs[k].winner = winner;
        jobs[k].length = length;
        jobs[k].seat_wins = seat_wins;
        pthread_create(&th[k], NULL, rollout_worker, &jobs[k]);
    }
    for (int k = 0; k < n_threads; ++k) pthread_join(th[k], NULL);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* synthetic state generator                                                 */
/* ------------------------------------------------------------------------ */
/* Deal (Sec. II-A: every player takes four tiles, rows ascending) extended
 * to mid-game positions: a pool size is drawn, the tiles drawn since the
 * deal are handed out round-robin from seat 0, and a random number of each
 * row's tiles is revealed (at least one tile of every row stays hidden).
 * The words of state index s come sequentially from blocks
 * (n>>2, 0xFFFFFFFF, 0xFFFFFFFF, s).                                        */
static void gen_one(orc_rows *r, const orc_deal_params *dp, uint64_t seed, uint32_t s)
{
    wstream ws;
    ws_init(&ws, seed, 0xFFFFFFFFu, 0xFFFFFFFFu, s);
    int P = dp->p_min;
    if (dp->p_max > dp->p_min) P = dp->p_min + (int)oracle_mulshift(ws_next(&ws), (uint32_t)(dp->p_max - dp->p_min + 1));
    int h0 = dp->hand[P];
    int cap = 24 - P * h0;
    int pile;
    if (dp->fresh) {
        pile = cap;
    } else {
        int lo = dp->pile_min < cap ? dp->pile_min : cap;
        int hi = dp->pile_max < cap ? dp->pile_max : cap;
        if (hi < lo) hi = lo;
        pile = lo + (int)oracle_mulshift(ws_next(&ws), (uint32_t)(hi - lo + 1));
    }
    /* Fisher-Yates shuffle of the 24 tile ids */
    int perm[24];
    for (int i = 0; i < 24; ++i) perm[i] = i;
    for (int i = 23; i >= 1; --i) {
        int j = (int)oracle_mulshift(ws_next(&ws), (uint32_t)(i + 1));
        int tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    }
    int drawn_since_deal = 24 - P * h0 - pile;
    memset(r, 0, sizeof(*r));
    r->P = P;
    int pos = 0;
    for (int q = 0; q < P; ++q) {
        int h = h0 + drawn_since_deal / P + (q < drawn_since_deal % P ? 1 : 0);
        for (int k = 0; k < h; ++k) row_insert(r, q, perm[pos++]);
    }
    /* the rest is the pool, ascending */
    int inpool[24] = {0};
    for (int k = pos; k < 24; ++k) inpool[perm[k]] = 1;
    for (int t = 0; t < 24; ++t)
        if (inpool[t]) r->pile[r->pile_n++] = t;
    /* revealed tiles: a partial Fisher-Yates over each row's slots */
    for (int q = 0; q < P; ++q) {
        int h = r->n[q];
        int rmax = dp->revealed_max < h - 1 ? dp->revealed_max : h - 1;
        if (rmax < 0) rmax = 0;
        int nrev = dp->fresh ? 0 : (int)oracle_mulshift(ws_next(&ws), (uint32_t)(rmax + 1));
        int idx[24];
        for (int k = 0; k < h; ++k) idx[k] = k;
        for (int i = 0; i < nrev; ++i) {
            int j = i + (int)oracle_mulshift(ws_next(&ws), (uint32_t)(h - i));
            int tmp = idx[i]; idx[i] = idx[j]; idx[j] = tmp;
            r->rev[q][idx[i]] = 1;
        }
    }
    r->mover = drawn_since_deal % P;
    r->phase = 0;
    r->drawn = -1;
    int do_draw = dp->root_draw;
    if (!do_draw && dp->phase_mix) do_draw = ws_next(&ws) < 0x80000000u;
    if (do_draw && r->pile_n > 0) {
        r->drawn = draw_at(r, r->mover, (int)oracle_mulshift(ws_next(&ws), (uint32_t)r->pile_n));
        r->phase = 1;
    }
}

int oracle_init_states(orc_packed *out, int64_t n, const orc_deal_params *dp, uint64_t seed,
                       uint32_t index_base)
{
    if (n < 0) return -1;
    if (dp->p_min < 2 || dp->p_max > 4 || dp->p_min > dp->p_max) return -1;
    for (int P = dp->p_min; P <= dp->p_max; ++P)
        if (dp->hand[P] < 1 || P * dp->hand[P] > 24) return -1;
    if (dp->pile_min < 0 || dp->pile_max < 0 || dp->revealed_max < 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        orc_rows r;
        gen_one(&r, dp, seed, index_base + (uint32_t)i);
        oracle_pack(&r, &out[i]);
    }
    return 0;
}

/* ppl playouts from an explicit state (used by the tree search) */
int rollout_rows_wins(const orc_rows *leaf, int32_t ppl, uint64_t seed, uint32_t leaf_id,
                      uint32_t tree_id, uint32_t wins[4])
{
    uint32_t key[2];
    key_of(seed, key);
    for (int k = 0; k < 4; ++k) wins[k] = 0;
    for (int32_t p = 0; p < ppl; ++p) {
        orc_rows s = *leaf;
        int len = 0;
        int win = playout_rows(&s, key, (uint32_t)p, leaf_id, tree_id, &len, NULL, NULL);
        wins[win]++;
    }
    return 0;
}
