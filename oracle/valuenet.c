/*
 * valuenet.c -- CPU oracle of the learned leaf evaluator: a small value
 * network (multi-layer perceptron) that estimates, from a full game state and
 * a perspective seat q, the probability that q wins a random playout.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper evaluates leaves by random playouts only (Sec. II-B); this network
 * is the learned replacement the engine trains on (state, playout win rate)
 * pairs.  Definitions restated here:
 *   features (160, zero padded from 148): for every tile t, the owner seat
 *     relative to q as a one-hot of 4 ((owner - q) mod P, nothing for pool
 *     tiles), revealed, in pool; then (mover - q) mod P as a one-hot of 4;
 *   h1 = relu(W1 x + b1), 256;  h2 = relu(W2 h1 + b2), 256;
 *   z = w3 . h2 + b3;  v = 1 / (1 + exp(-z));  loss = mean (v - y)^2.
 * Parameters are one flat float array: W1 [256][160] (row = output), b1 [256],
 * W2 [256][256], b2 [256], w3 [256], b3 [1].
 *
 * Two arithmetic modes:
 *   exact (bf16 = 0): every operation in double precision on the float
 *     parameters -- the plain definition, pinned by finite differences;
 *   bf16 mirror (bf16 = 1): the rounding points of the GPU kernels -- weights
 *     W1, W2, w3 rounded to bfloat16 (round to nearest even), h1 and h2
 *     rounded to bfloat16 after the activation, the back-propagated dh2 and
 *     dh1 rounded to bfloat16 before they enter a matrix product -- with
 *     every sum still accumulated in double.
 * Adam (Kingma and Ba, 2015) with bias correction, in double.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define VN_IN 160
#define VN_H 256
#define VN_FEAT 148

enum {
    OFF_W1 = 0,
    OFF_B1 = OFF_W1 + VN_H * VN_IN,
    OFF_W2 = OFF_B1 + VN_H,
    OFF_B2 = OFF_W2 + VN_H * VN_H,
    OFF_W3 = OFF_B2 + VN_H,
    OFF_B3 = OFF_W3 + VN_H,
    VN_NPARAM = OFF_B3 + 1
};

int oracle_unpack(const orc_packed *s, orc_rows *r);

int oracle_vn_nparams(void) { return VN_NPARAM; }

/* round a float to the nearest bfloat16 (ties to even), returned as float */
float oracle_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return x; /* inf / nan unchanged */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    u &= 0xFFFF0000u;
    float y;
    memcpy(&y, &u, 4);
    return y;
}

static double rnd(double x, int bf16) { return bf16 ? (double)oracle_bf16((float)x) : x; }

int oracle_vn_encode(const orc_packed *s, int32_t q, float feat[VN_IN])
{
    orc_rows r;
    if (oracle_unpack(s, &r)) return -2;
    if (q < 0 || q >= r.P) return -1;
    memset(feat, 0, VN_IN * sizeof(float));
    for (int seat = 0; seat < r.P; ++seat)
        for (int j = 0; j < r.n[seat]; ++j) {
            int t = r.tile[seat][j];
            int rel = ((seat - q) % r.P + r.P) % r.P;
            feat[t * 6 + rel] = 1.0f;
            if (r.rev[seat][j]) feat[t * 6 + 4] = 1.0f;
        }
    for (int j = 0; j < r.pile_n; ++j) feat[r.pile[j] * 6 + 5] = 1.0f;
    feat[144 + ((r.mover - q) % r.P + r.P) % r.P] = 1.0f;
    return 0;
}

/* forward pass of one row; stores the intermediate values for backward */
typedef struct {
    double x[VN_IN], a1[VN_H], h1[VN_H], a2[VN_H], h2[VN_H];
    double z, v;
} vn_row;

/* The weights the products read: W1, W2 and w3 rounded to bfloat16 in the
 * mirror mode (each weight is rounded the same way wherever it is read, so
 * rounding them once per call gives the same values as rounding at every
 * use), the float parameters otherwise.  Biases stay float.               */
static double *product_weights(const float *P, int bf16)
{
    double *Q = (double *)malloc(VN_NPARAM * sizeof(double));
    for (int k = 0; k < VN_NPARAM; ++k) {
        const int is_bias = (k >= OFF_B1 && k < OFF_W2) || (k >= OFF_B2 && k < OFF_W3) || k == OFF_B3;
        Q[k] = is_bias ? (double)P[k] : rnd(P[k], bf16);
    }
    return Q;
}

/* Q: product_weights() of the parameters */
static void forward_row(const double *Q, const float *x, int bf16, vn_row *o)
{
    for (int i = 0; i < VN_IN; ++i) o->x[i] = x[i];
    for (int k = 0; k < VN_H; ++k) {
        double acc = 0.0;
        for (int i = 0; i < VN_IN; ++i) acc += Q[OFF_W1 + k * VN_IN + i] * o->x[i];
        o->a1[k] = acc + Q[OFF_B1 + k];
        o->h1[k] = rnd(o->a1[k] > 0.0 ? o->a1[k] : 0.0, bf16);
    }
    for (int k = 0; k < VN_H; ++k) {
        double acc = 0.0;
        for (int i = 0; i < VN_H; ++i) acc += Q[OFF_W2 + k * VN_H + i] * o->h1[i];
        o->a2[k] = acc + Q[OFF_B2 + k];
        o->h2[k] = rnd(o->a2[k] > 0.0 ? o->a2[k] : 0.0, bf16);
    }
    double acc = 0.0;
    for (int i = 0; i < VN_H; ++i) acc += Q[OFF_W3 + i] * o->h2[i];
    o->z = acc + Q[OFF_B3];
    o->v = 1.0 / (1.0 + exp(-o->z));
}

int oracle_vn_forward(const float *params, const orc_packed *states, const int32_t *persp,
                      int64_t n, int bf16, double *v_out)
{
    float x[VN_IN];
    vn_row *o = (vn_row *)malloc(sizeof(vn_row));
    double *Q = product_weights(params, bf16);
    int rc = 0;
    for (int64_t i = 0; i < n && rc == 0; ++i) {
        if (oracle_vn_encode(&states[i], persp[i], x)) {
            rc = -2;
            break;
        }
        forward_row(Q, x, bf16, o);
        v_out[i] = o->v;
    }
    free(Q);
    free(o);
    return rc;
}

/* loss = mean over rows of (v - y)^2 and its gradient w.r.t. every parameter.
 * grad_abs (may be NULL) receives, per parameter, the sum of the absolute
 * values of the per-row terms that make up its gradient: the scale against
 * which a gradient summed in another order, or with an operand rounded the
 * other way, is judged.                                                    */
int oracle_vn_loss_grad(const float *params, const orc_packed *states, const int32_t *persp,
                        const float *labels, int64_t n, int bf16, double *loss, double *grad,
                        double *grad_abs)
{
    float x[VN_IN];
    vn_row *o = (vn_row *)malloc(sizeof(vn_row));
    double *Q = product_weights(params, bf16);
    double dh2[VN_H], dh1[VN_H];
    memset(grad, 0, VN_NPARAM * sizeof(double));
    if (grad_abs) memset(grad_abs, 0, VN_NPARAM * sizeof(double));
    double L = 0.0;
    int rc = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (oracle_vn_encode(&states[r], persp[r], x)) {
            rc = -2;
            break;
        }
        forward_row(Q, x, bf16, o);
        double e = o->v - (double)labels[r];
        L += e * e;
        double dz = 2.0 * e / (double)n * o->v * (1.0 - o->v);
        grad[OFF_B3] += dz;
        for (int i = 0; i < VN_H; ++i) {
            grad[OFF_W3 + i] += dz * o->h2[i];
            double d = dz * Q[OFF_W3 + i];
            dh2[i] = rnd(o->a2[i] > 0.0 ? d : 0.0, bf16);
        }
        for (int k = 0; k < VN_H; ++k) {
            grad[OFF_B2 + k] += dh2[k];
            for (int i = 0; i < VN_H; ++i) grad[OFF_W2 + k * VN_H + i] += dh2[k] * o->h1[i];
        }
        for (int i = 0; i < VN_H; ++i) {
            double acc = 0.0;
            for (int k = 0; k < VN_H; ++k) acc += dh2[k] * Q[OFF_W2 + k * VN_H + i];
            dh1[i] = rnd(o->a1[i] > 0.0 ? acc : 0.0, bf16);
        }
        for (int k = 0; k < VN_H; ++k) {
            grad[OFF_B1 + k] += dh1[k];
            for (int i = 0; i < VN_IN; ++i) grad[OFF_W1 + k * VN_IN + i] += dh1[k] * o->x[i];
        }
        if (grad_abs) {
            grad_abs[OFF_B3] += fabs(dz);
            for (int i = 0; i < VN_H; ++i) grad_abs[OFF_W3 + i] += fabs(dz * o->h2[i]);
            for (int k = 0; k < VN_H; ++k) {
                grad_abs[OFF_B2 + k] += fabs(dh2[k]);
                for (int i = 0; i < VN_H; ++i)
                    grad_abs[OFF_W2 + k * VN_H + i] += fabs(dh2[k] * o->h1[i]);
                grad_abs[OFF_B1 + k] += fabs(dh1[k]);
                for (int i = 0; i < VN_IN; ++i)
                    grad_abs[OFF_W1 + k * VN_IN + i] += fabs(dh1[k] * o->x[i]);
            }
        }
    }
    *loss = L / (double)n;
    free(Q);
    free(o);
    return rc;
}

/* one Adam step on double copies of the parameters and moments (t >= 1) */
void oracle_vn_adam(double *w, double *m, double *v, const double *g, int64_t n, int64_t t,
                    double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Initial parameters: weight k of the flat layout takes word k of the Philox
 * stream (k>>2, 0xFFFFFFFE, 0, 0), u = (w >> 8) * 2^-24 in [0, 1), scaled to
 * U(-b, b): b = sqrt(6/148) for W1, sqrt(6/256) for W2, 1/16 for w3; biases 0.
 */
void oracle_vn_init(float *params, uint64_t seed)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int k = 0; k < VN_NPARAM; ++k) {
        uint32_t ctr[4] = {(uint32_t)k >> 2, 0xFFFFFFFEu, 0u, 0u}, w[4];
        oracle_philox(ctr, key, w);
        float u = (float)(w[k & 3] >> 8) * (1.0f / 16777216.0f);
        float b;
        if (k < OFF_B1) b = sqrtf(6.0f / (float)VN_FEAT);
        else if (k >= OFF_W2 && k < OFF_B2) b = sqrtf(6.0f / (float)VN_H);
        else if (k >= OFF_W3 && k < OFF_B3) b = 1.0f / 16.0f;
        else b = 0.0f;
        params[k] = (2.0f * u - 1.0f) * b;
    }
}
