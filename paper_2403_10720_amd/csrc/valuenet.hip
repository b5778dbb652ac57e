// valuenet.hip -- the learned leaf evaluator on gfx950 matrix cores.
//
// A small value network estimates, from a full game state and a perspective
// seat q, the probability that q wins a random playout (the quantity the
// paper's playouts estimate, Sec. II-B).  Features (160, zero padded from
// 148): per tile the owner seat relative to q (one-hot of 4, nothing for pool
// tiles), revealed, in pool; then (mover - q) mod P one-hot of 4.
//   h1 = bf16(relu(W1 x + b1)), h2 = bf16(relu(W2 h1 + b2)), z = w3.h2 + b3,
//   v = sigmoid(z), loss = mean (v - y)^2, Adam on float32 master weights.
// Products use v_mfma_f32_16x16x32_bf16 with bfloat16 operands and float32
// accumulation.  A wavefront owns 16 rows: it encodes its features straight
// into the A operand, runs both layers, and (training) back-propagates the
// data gradient through layer 2.  A second kernel contracts the stored
// activations over the batch into the weight gradients (and sums the bias
// gradients and the loss); a third takes the Adam step of the weights.
//
// Net blob (device, caller-owned, dvc_valuenet_bytes()):
//   u32 header[64]; float master[NPAD], m[NPAD], v[NPAD];
//   bf16 W1b[256][160], W2b[256][256], W2Tb[256][256] (W2 transposed),
//   W1Tb[160][256] (W1 transposed), w3b[256].
#include "dvc_core.hpp"
#include "dvc_internal.hpp"

namespace dvc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kVnIn = 160, kVnH = 256;
constexpr uint32_t kOffW1 = 0, kOffB1 = 40960, kOffW2 = 41216, kOffB2 = 106752, kOffW3 = 107008,
                   kOffB3 = 107264, kVnParams = 107265;
constexpr uint32_t kVnPad = 107328;                       // params rounded up to 64
constexpr uint32_t kVnHeaderWords = 64;
constexpr uint64_t kVnMasterOff = kVnHeaderWords * 4u;     // byte offsets
constexpr uint64_t kVnMOff = kVnMasterOff + (uint64_t)kVnPad * 4u;
constexpr uint64_t kVnVOff = kVnMOff + (uint64_t)kVnPad * 4u;
constexpr uint64_t kVnW1bOff = kVnVOff + (uint64_t)kVnPad * 4u;
constexpr uint64_t kVnW2bOff = kVnW1bOff + 40960u * 2u;
constexpr uint64_t kVnW2TbOff = kVnW2bOff + 65536u * 2u;
constexpr uint64_t kVnW3bOff = kVnW2TbOff + 65536u * 2u;
constexpr uint64_t kVnBytes = kVnW3bOff + 256u * 2u;

// The bf16 shadows of W1, W2 and W2 transposed are stored as ready-made B
// operands of the 16x16x32 product: fragment q = j * KS + s (output column
// tile j, k block s, KS = 5 for W1 and 8 for W2) holds, for lane l = 16 g +
// r, the 8 values W[16 j + r][32 s + 8 g .. + 7] at (q * 64 + l) * 8, so a
// wavefront reads a fragment as one contiguous kilobyte.
__host__ __device__ constexpr uint32_t vn_frag(uint32_t row, uint32_t col, uint32_t ks)
{
    return ((((row >> 4) * ks + (col >> 5)) * 64u + ((col >> 3) & 3u) * 16u + (row & 15u)) << 3) +
           (col & 7u);
}

struct VnPtrs {
    uint32_t *header;
    float *master, *m, *v;
    uint16_t *w1b, *w2b, *w2tb, *w3b;
};

__host__ __device__ inline VnPtrs vn_ptrs(void *net)
{
    uint8_t *b = (uint8_t *)net;
    VnPtrs p;
    p.header = (uint32_t *)b;
    p.master = (float *)(b + kVnMasterOff);
    p.m = (float *)(b + kVnMOff);
    p.v = (float *)(b + kVnVOff);
    p.w1b = (uint16_t *)(b + kVnW1bOff);
    p.w2b = (uint16_t *)(b + kVnW2bOff);
    p.w2tb = (uint16_t *)(b + kVnW2TbOff);
    p.w3b = (uint16_t *)(b + kVnW3bOff);
    return p;
}

// Inside the kernels the features are kept kind-major: internal feature p =
// 24 * kind + t for tile t and kind 0..3 (owner seat relative to q), 4
// (revealed), 5 (pool); 144 + m for (mover - q) mod P = m; zero above.  The
// canonical (tile-major) index f = 6 t + kind of the master weights maps to p
// = vn_perm(f); the bf16 shadows of W1 and the weight gradient of W1 use p.
// This order makes a block of 32 features one word of the concatenated
// masks, so a lane's 8 features are one byte.
__device__ __forceinline__ uint32_t vn_perm(uint32_t f)
{
    if (f >= 144u) return f;
    const uint32_t t = f / 6u;
    return 24u * (f - 6u * t) + t;
}

// float -> bfloat16 bits, round to nearest even (the gfx950 conversion
// instruction; the values converted here are finite)
__device__ __forceinline__ uint16_t bf16_bits(float x)
{
    const __bf16 b = (__bf16)x;
    uint16_t u;
    __builtin_memcpy(&u, &b, 2);
    return u;
}
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bf16_round(float x) { return bf16_to_f(bf16_bits(x)); }

// ---------------------------------------------------------------------------
// initialization and shadows
// ---------------------------------------------------------------------------
__global__ void vn_init_kernel(void *net, uint32_t k0, uint32_t k1, float bw1, float bw2, float bw3)
{
    VnPtrs p = vn_ptrs(net);
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        for (uint32_t i = 0; i < kVnHeaderWords; ++i) p.header[i] = 0u;
    }
    if (k >= kVnPad) return;
    float w = 0.0f;
    if (k < kVnParams) {
        const Words b = philox(k >> 2, 0xFFFFFFFEu, 0u, 0u, k0, k1);
        const uint32_t word = (k & 3u) == 0u ? b.w0 : (k & 3u) == 1u ? b.w1 : (k & 3u) == 2u ? b.w2 : b.w3;
        const float u = (float)(word >> 8) * (1.0f / 16777216.0f);
        const float bound = k < kOffB1 ? bw1 : (k >= kOffW2 && k < kOffB2) ? bw2
                          : (k >= kOffW3 && k < kOffB3) ? bw3 : 0.0f;
        w = (2.0f * u - 1.0f) * bound;
    }
    p.master[k] = w;
    p.m[k] = 0.0f;
    p.v[k] = 0.0f;
}

// bf16 copies of the weights in the layouts the products read
__global__ void vn_shadow_kernel(void *net)
{
    VnPtrs p = vn_ptrs(net);
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 40960u) {
        const uint32_t n = k / kVnIn, f = vn_perm(k % kVnIn);
        p.w1b[vn_frag(n, f, 5u)] = bf16_bits(p.master[kOffW1 + k]);
    }
    if (k < 65536u) {
        const uint32_t n = k / kVnH, i = k % kVnH;
        const uint16_t b = bf16_bits(p.master[kOffW2 + k]);
        p.w2b[vn_frag(n, i, 8u)] = b;
        p.w2tb[vn_frag(i, n, 8u)] = b;
    }
    if (k < 256u) p.w3b[k] = bf16_bits(p.master[kOffW3 + k]);
}

// ---------------------------------------------------------------------------
// features of one row as bfloat16 bits, 8 consecutive features per call
// ---------------------------------------------------------------------------
struct RowFeat {
    uint32_t rel[4];   // tiles owned by the seat (q + k) mod P
    uint32_t rev, pool, tomove;  // tomove = (mover - q) mod P
    bool ok;
};

__device__ __forceinline__ RowFeat row_features(uint4 st, uint32_t q)
{
    State s;
    RowFeat r;
    r.ok = decode(st.x, st.y, st.z, st.w, s) && q < s.P;
    const uint32_t qq = q < s.P ? q : 0u;
#pragma unroll
    for (uint32_t k = 0; k < 4u; ++k) {
        const uint32_t seat = qq + k >= s.P ? qq + k - s.P : qq + k;
        r.rel[k] = k < s.P ? hand_of(s, seat) : 0u;
    }
    r.rev = s.rev;
    r.pool = ~(s.h0 | s.h1 | s.h2 | s.h3) & kAll;
    r.tomove = s.m >= qq ? s.m - qq : s.m + s.P - qq;
    return r;
}

// word s (bits 32s .. 32s+31) of the internal 160-bit feature vector
__device__ __forceinline__ uint32_t feature_word(const RowFeat &r, uint32_t s)
{
    const uint32_t mv = r.tomove < 4u ? 1u << r.tomove : 0u;
    return s == 0u ? r.rel[0] | (r.rel[1] << 24)
         : s == 1u ? (r.rel[1] >> 8) | (r.rel[2] << 16)
         : s == 2u ? (r.rel[2] >> 16) | (r.rel[3] << 8)
         : s == 3u ? r.rev | (r.pool << 24)
                   : (r.pool >> 8) | (mv << 16);
}

// the eight features 32s + 8g .. 32s + 8g + 7 as bfloat16 1.0 / 0.0
__device__ __forceinline__ bf16x8 feature8(const RowFeat &r, uint32_t s, uint32_t g)
{
    const uint32_t b = feature_word(r, s) >> (8u * g);
    uint4 u;
    u.x = ((b & 1u) ? 0x3F80u : 0u) | ((b & 2u) ? 0x3F800000u : 0u);
    u.y = ((b & 4u) ? 0x3F80u : 0u) | ((b & 8u) ? 0x3F800000u : 0u);
    u.z = ((b & 16u) ? 0x3F80u : 0u) | ((b & 32u) ? 0x3F800000u : 0u);
    u.w = ((b & 64u) ? 0x3F80u : 0u) | ((b & 128u) ? 0x3F800000u : 0u);
    bf16x8 x;
    __builtin_memcpy(&x, &u, 16);
    return x;
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    bf16x8 x;
    __builtin_memcpy(&x, &u, 16);
    return x;
}

__device__ __forceinline__ floatx4 mfma16(bf16x8 a, bf16x8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// forward (and, when training, data backward) for 16 rows per wavefront.
// Operand layouts of the 16x16x32 product (lane l, r = l%16, g = l/16):
//   A[r][8g..8g+7], B[8g..8g+7][r] (8 consecutive k of one column), and
//   D[4g+i][r] for i < 4.
// ---------------------------------------------------------------------------
// Training activations X^T, H1^T, dH1^T and dH2^T (feature f, batch row b;
// batch K a multiple of 32) are stored as ready-made operands of the weight
// gradient products: the 16 x 32 block (features 16T.., rows 32s..) is one
// contiguous kilobyte in lane order, lane 16g + r holding feature 16T + r,
// rows 32s + 8g .. + 7.  An operand load is then one contiguous kilobyte
// rather than 16 rows a batch apart.
__device__ __forceinline__ size_t vn_act_idx(uint32_t f, uint32_t b, uint32_t K)
{
    return ((((size_t)(f >> 4) * (K >> 5) + (b >> 5)) * 64u + ((b >> 3) & 3u) * 16u + (f & 15u))
            << 3) + (b & 7u);
}

struct VnRowsArgs {
    const void *net;
    const uint4 *states;
    const uint8_t *persp;
    const float *labels;
    uint32_t n_rows;          // rows in this launch
    uint32_t n_data, perm_a, perm_b, row_base;   // training: row i is data[(a*(base+i)+b) % n_data]
    uint32_t n_mask;                             // n_data - 1 when n_data is a power of two, else 0
    float *v_out;             // inference output (or null)
    // training outputs (bf16, in the fragment layout of vn_act_idx)
    uint16_t *xt, *h1t, *dh1t, *dh2t;
    float *part;              // per 16-row tile, column-major: part[c * tiles + tile] for the
                              // columns c of [loss, db3, dw3[256], db2[256], db1[256]]
    float inv_batch;
};

// Value of 16 rows (lane l holds the features of row l%16): forward pass on
// the matrix cores.  `hs` is a 16 x 264 bf16 LDS tile; v4[i] receives the
// value of row 4*(l/16)+i.  Shared by batched inference and the tree search.
__device__ __forceinline__ void vn_eval16(const VnPtrs &P, const RowFeat &rf,
                                          uint16_t (*hs)[kVnH + 8], float v4[4])
{
    const uint32_t lane = threadIdx.x & 63u, r = lane & 15u, g = lane >> 4;
    bf16x8 xa[5];
#pragma unroll
    for (uint32_t s = 0; s < 5u; ++s) xa[s] = feature8(rf, s, g);
#pragma unroll 4
    for (uint32_t j = 0; j < 16u; ++j) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (uint32_t s = 0; s < 5u; ++s)
            acc = mfma16(xa[s], load8(P.w1b + ((j * 5u + s) * 64u + lane) * 8u), acc);
        const float b = P.master[kOffB1 + 16u * j + r];
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i) {
            const float h = acc[i] + b;
            hs[4u * g + i][16u * j + r] = bf16_bits(h > 0.0f ? h : 0.0f);
        }
    }
    __syncthreads();
    bf16x8 ha[8];
#pragma unroll
    for (uint32_t s = 0; s < 8u; ++s) ha[s] = load8(&hs[r][32u * s + 8u * g]);
    float zpart[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
    for (uint32_t j = 0; j < 16u; ++j) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s)
            acc = mfma16(ha[s], load8(P.w2b + ((j * 8u + s) * 64u + lane) * 8u), acc);
        const float b = P.master[kOffB2 + 16u * j + r];
        const float w3 = bf16_to_f(P.w3b[16u * j + r]);
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i) {
            const float h = acc[i] + b;
            zpart[i] += bf16_round(h > 0.0f ? h : 0.0f) * w3;
        }
    }
#pragma unroll
    for (uint32_t i = 0; i < 4u; ++i)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) zpart[i] += __shfl_xor(zpart[i], off, 64);
    const float b3 = P.master[kOffB3];
#pragma unroll
    for (uint32_t i = 0; i < 4u; ++i) v4[i] = 1.0f / (1.0f + expf(-(zpart[i] + b3)));
    __syncthreads();   // hs may be reused by the caller
}

// The first layer inside a tree search streams its weight fragments through
// a ring of RING registers: the fragment for product q + RING is requested
// while product q runs, so a wavefront keeps that many loads in flight
// instead of one or two (one wavefront per tree has nothing else to hide the
// L2 latency behind).  Needs the register budget of one wavefront per SIMD.
// The streamed weight fragment is the A operand (16 output units x 32 k)
// and a[s] the B operand (32 k x 16 rows), so out(j, acc) receives D[unit
// 16j + 4g + i][row r].  A weight fragment is the same registers as either
// operand (lane 16g + r holds 8 consecutive k of unit 16j + r).
template <int KS, int RING, typename Epi>
__device__ __forceinline__ void vn_layer_deep_t(const bf16x8 (&a)[KS], const uint16_t *w,
                                                uint32_t lane, Epi out)
{
    constexpr int N = 16 * KS;
    bf16x8 ring[RING];
#pragma unroll
    for (int q = 0; q < RING; ++q) ring[q] = load8(w + ((uint32_t)q * 64u + lane) * 8u);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int q = j * KS + s;
            const bf16x8 b = ring[q % RING];
            if (q + RING < N) ring[q % RING] = load8(w + ((uint32_t)(q + RING) * 64u + lane) * 8u);
            acc = mfma16(b, a[s], acc);
        }
        out((uint32_t)j, acc);
    }
}

// Small per-workgroup LDS copy of the biases and output weights (float):
// b1[256], b2[256], w3[256], b3.
struct VnSmall {
    float b1[kVnH], b2[kVnH], w3[kVnH], b3;
};

__device__ __forceinline__ void vn_stage_small(const VnPtrs &P, VnSmall &sm)
{
    for (uint32_t k = threadIdx.x; k < kVnH; k += blockDim.x) {
        sm.b1[k] = P.master[kOffB1 + k];
        sm.b2[k] = P.master[kOffB2 + k];
        sm.w3[k] = bf16_to_f(P.w3b[k]);
    }
    if (threadIdx.x == 0) sm.b3 = P.master[kOffB3];
}

// 16 bytes at byte offset voff + soff of the buffer `rs` (voff per lane,
// soff the same in every lane): one lane-offset register serves every weight
// fragment request, and requests past the buffer's end read zeros
__device__ __forceinline__ bf16x8 buf_load8(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
    bf16x8 x;
    __builtin_memcpy(&x, &u, 16);
    return x;
}

// raw buffer resource over `bytes` bytes at p (dword 3: 32-bit data format,
// the gfx9 value)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t weight_rsrc(const uint16_t *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

// orders LDS accesses between the lanes of one wavefront
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Value of 16 rows (lane l holds the features of row l % 16) by one
// wavefront that shares its workgroup with another wavefront doing other
// work: the same products as vn_eval16, both layers' weight fragments read
// from L2, biases and output weights from `sm`, the 16 x 264 bf16 tile `hs`
// (this wavefront's own) ordered with wavefront barriers.  v4[i] receives
// the value of row 4 (l / 16) + i.
//
// The wavefront has nothing else to hide the L2 latency behind, so the
// weight fragments of output tile j + 4 (first layer) or j + 3 (second) are
// requested right after tile j is multiplied (requests past the last tile
// repeat it); the scheduling
// barriers keep the compiler from moving the requests back next to their
// uses.
__device__ __forceinline__ void vn_eval16_wave(const VnPtrs &P, const RowFeat &rf,
                                               uint16_t (*hs)[kVnH + 8], const VnSmall &sm,
                                               float v4[4])
{
    const uint32_t lane = threadIdx.x & 63u, r = lane & 15u, g = lane >> 4;
    constexpr uint32_t D1 = 4u, D2 = 3u;
    const __amdgpu_buffer_rsrc_t w1 = weight_rsrc(P.w1b, kVnIn * kVnH * 2u);
    const __amdgpu_buffer_rsrc_t w2 = weight_rsrc(P.w2b, kVnH * kVnH * 2u);
    const uint32_t voff = lane * 16u;   // fragment j of a weight block: byte 1024 j + 16 lane
    bf16x8 xa[5];
#pragma unroll
    for (uint32_t s = 0; s < 5u; ++s) xa[s] = feature8(rf, s, g);
    bf16x8 w1r[D1][5];
#pragma unroll
    for (uint32_t j = 0; j < D1; ++j)
#pragma unroll
        for (uint32_t s = 0; s < 5u; ++s) w1r[j][s] = buf_load8(w1, voff, (j * 5u + s) * 1024u);
#pragma unroll 1
    for (uint32_t j0 = 0; j0 < 16u; j0 += D1) {
#pragma unroll
        for (uint32_t jj = 0; jj < D1; ++jj) {
            const uint32_t j = j0 + jj, jn = j + D1 < 16u ? j + D1 : 15u;
            __builtin_amdgcn_sched_barrier(0);
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (uint32_t s = 0; s < 5u; ++s) acc = mfma16(xa[s], w1r[jj][s], acc);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (uint32_t s = 0; s < 5u; ++s) w1r[jj][s] = buf_load8(w1, voff, (jn * 5u + s) * 1024u);
            __builtin_amdgcn_sched_barrier(0);
            const float b = sm.b1[16u * j + r];
#pragma unroll
            for (uint32_t i = 0; i < 4u; ++i) {
                const float h = acc[i] + b;
                hs[4u * g + i][16u * j + r] = bf16_bits(h > 0.0f ? h : 0.0f);
            }
        }
    }
    // the second layer's first fragments are requested before the tile is read back
    bf16x8 w2r[D2][8];
#pragma unroll
    for (uint32_t j = 0; j < D2; ++j)
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s) w2r[j][s] = buf_load8(w2, voff, (j * 8u + s) * 1024u);
    wave_lds_sync();
    bf16x8 ha[8];
#pragma unroll
    for (uint32_t s = 0; s < 8u; ++s) ha[s] = load8(&hs[r][32u * s + 8u * g]);
    float zpart[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    // output tile j from the ring slot wq, which then requests tile j + D2
    auto layer2_tile = [&](uint32_t j, bf16x8 (&wq)[8]) {
        const uint32_t jn = j + D2 < 16u ? j + D2 : 15u;
        __builtin_amdgcn_sched_barrier(0);
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s) acc = mfma16(ha[s], wq[s], acc);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s) wq[s] = buf_load8(w2, voff, (jn * 8u + s) * 1024u);
        __builtin_amdgcn_sched_barrier(0);
        const float b = sm.b2[16u * j + r], w3 = sm.w3[16u * j + r];
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i) {
            const float h = acc[i] + b;
            zpart[i] += bf16_round(h > 0.0f ? h : 0.0f) * w3;
        }
    };
    // tiles 0 .. 14 three at a time, then tile 15 (ring slot 0)
#pragma unroll 1
    for (uint32_t j0 = 0; j0 < 15u; j0 += D2) {
#pragma unroll
        for (uint32_t jj = 0; jj < D2; ++jj) layer2_tile(j0 + jj, w2r[jj]);
    }
    layer2_tile(15u, w2r[0]);
#pragma unroll
    for (uint32_t i = 0; i < 4u; ++i)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) zpart[i] += __shfl_xor(zpart[i], off, 64);
#pragma unroll
    for (uint32_t i = 0; i < 4u; ++i) v4[i] = 1.0f / (1.0f + expf(-(zpart[i] + sm.b3)));
    wave_lds_sync();   // the tile may be reused
}

// k order of the transposed second product: slot 8g + e of a 32-unit block
// holds unit 4g + e (e < 4) or 16 + 4g + e - 4 (e >= 4) -- the units that
// lane group g holds of the block's two 16-unit output tiles of the first
// product, so those tiles, packed to bfloat16, are the second product's B
// operand as they stand
__host__ __device__ constexpr uint32_t vn_tk(uint32_t slot)
{
    return (slot & 4u) ? 16u + 4u * (slot >> 3) + (slot & 3u) : 4u * (slot >> 3) + (slot & 3u);
}

// Stage the bf16 W2 in LDS as A operands of the transposed second product:
// fragment q = 8j + s, lane 16g + r, element e holds W2[16j + r][32s +
// vn_tk(8g + e)] (the blob's shadow holds W2 as B operands in natural k
// order).  Four consecutive units are one 8-byte copy.
__device__ void vn_stage_w2t(const VnPtrs &P, uint16_t *w2p)
{
    for (uint32_t c = threadIdx.x; c < kVnH * kVnH / 4u; c += blockDim.x) {
        const uint32_t d = 4u * c;
        const uint32_t e = d & 7u, l = (d >> 3) & 63u, q = d >> 9;
        const uint32_t j = q >> 3, s = q & 7u, g = l >> 4, r = l & 15u;
        const uint32_t src = vn_frag(16u * j + r, 32u * s + vn_tk(8u * g + e), 8u);
        *reinterpret_cast<uint2 *>(w2p + d) = *reinterpret_cast<const uint2 *>(P.w2b + src);
    }
}

// Value of 16 rows inside a tree search, computed transposed: H1^T = W1 X^T
// then H2^T = W2 H1^T, so that each layer's output stays in registers (the
// first layer's tiles 2s, 2s + 1, relu'd and packed to bfloat16, are block s
// of the second product's B operand) -- no LDS tile, no barrier.  The
// lane's row is r = lane % 16 (rf; empty rows give some value that callers
// ignore); first-layer weights stream from L2 through a ring of loads,
// second-layer weights come from `w2p` (vn_stage_w2t), biases and output
// weights from `sm`.  Returns the value of row r in lanes r, r + 16, r + 32
// and r + 48 (the same bits in all four).  Same products as vn_eval16, the
// sums in another order.
__device__ __forceinline__ float vn_eval_tree_t(const VnPtrs &P, const RowFeat &rf,
                                                const uint16_t *w2p, const VnSmall &sm)
{
    const uint32_t lane = threadIdx.x & 63u, g = lane >> 4;
    bf16x8 xb[5];
#pragma unroll
    for (uint32_t s = 0; s < 5u; ++s) xb[s] = feature8(rf, s, g);
    uint32_t hw[8][4];
    vn_layer_deep_t<5, 32>(xb, P.w1b, lane, [&](uint32_t j, const floatx4 &acc) {
        uint32_t hq[4];
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i) {
            const float h = acc[i] + sm.b1[16u * j + 4u * g + i];
            hq[i] = bf16_bits(h > 0.0f ? h : 0.0f);
        }
        hw[j >> 1][2u * (j & 1u)] = hq[0] | (hq[1] << 16);
        hw[j >> 1][2u * (j & 1u) + 1u] = hq[2] | (hq[3] << 16);
    });
    bf16x8 hb[8];
#pragma unroll
    for (uint32_t s = 0; s < 8u; ++s) __builtin_memcpy(&hb[s], hw[s], 16);
    float z = 0.0f;
#pragma unroll
    for (uint32_t j = 0; j < 16u; ++j) {
        bf16x8 wb[8];
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s) wb[s] = load8(w2p + ((j * 8u + s) * 64u + lane) * 8u);
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s) acc = mfma16(wb[s], hb[s], acc);
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i) {
            const uint32_t u = 16u * j + 4u * g + i;
            const float h = acc[i] + sm.b2[u];
            z += bf16_round(h > 0.0f ? h : 0.0f) * sm.w3[u];
        }
    }
    z += __shfl_xor(z, 16, 64);
    z += __shfl_xor(z, 32, 64);
    return 1.0f / (1.0f + expf(-(z + sm.b3)));
}

__device__ __forceinline__ RowFeat no_row()
{
    RowFeat rf;
    rf.rel[0] = rf.rel[1] = rf.rel[2] = rf.rel[3] = 0u;
    rf.rev = rf.pool = 0u;
    rf.tomove = 7u;
    rf.ok = false;
    return rf;
}

__global__ void __launch_bounds__(64) vn_infer_kernel(const void *net, const uint4 *states,
                                                       const uint8_t *persp, uint32_t n,
                                                       float *v_out)
{
    __shared__ __attribute__((aligned(16))) uint16_t hs[16][kVnH + 8];
    const VnPtrs P = vn_ptrs(const_cast<void *>(net));
    const uint32_t lane = threadIdx.x, r = lane & 15u, g = lane >> 4;
    const uint32_t row0 = blockIdx.x * 16u, myrow = row0 + r;
    RowFeat rf = no_row();
    if (myrow < n) {
        rf = row_features(states[myrow], persp[myrow]);
        if (!rf.ok) {
            atomicOr(&g_error_word, kErrState);
            rf = no_row();
        }
    }
    float v4[4];
    vn_eval16(P, rf, hs, v4);
    if (r == 0u) {
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i) {
            const uint32_t row = row0 + 4u * g + i;
            if (row < n) v_out[row] = v4[i];
        }
    }
}

constexpr uint32_t kPartWords = 2u + 3u * 256u;   // loss, db3, dw3[256], db2[256], db1[256]
// weight-gradient output tiles of 32 x 32: dW2 (256 x 256) then dW1 (256 x 160)
constexpr uint32_t kVnTilesW2 = 64u, kVnTilesW1 = 40u, kVnGradTiles = kVnTilesW2 + kVnTilesW1;
constexpr uint32_t kVnMaxSlices = 8u;   // batch slices of the weight-gradient products

// data row of batch row `row` of a training step
__device__ __forceinline__ uint32_t vn_train_row(const VnRowsArgs &a, uint32_t row)
{
    const uint64_t x = (uint64_t)a.perm_a * (a.row_base + row) + a.perm_b;
    return a.n_mask ? (uint32_t)x & a.n_mask : (uint32_t)(x % a.n_data);
}

// Training rows (forward, loss, data gradients, bias-gradient partials), MT
// 16-row tiles per workgroup and 4 MT wavefronts: wavefront w computes JJ =
// 4 / MT column tiles of every layer (columns 16 JJ w .., a 4 MT-th of each
// weight matrix) for all MT row tiles, so each weight fragment it loads
// serves MT products and a workgroup streams the 336 KB of weight fragments
// once for 16 MT rows.  The activation and gradient tiles are shared through
// LDS; z sums the wavefronts' partial dot products in wavefront order.
// Every weight fragment, bias and label a wavefront needs is requested a
// stage ahead of its use (the first layer's before the features are built,
// each later layer's while the previous layer's products run), so the
// memory latency is paid a few times per workgroup rather than once per
// column tile.  Workgroups are dealt to the XCDs in turn; with a multiple of
// 8 workgroups, workgroup b takes tile (b % 8) * tiles / 8 + b / 8, so that
// each XCD writes one contiguous eighth of the batch: the slice of the batch
// the weight-gradient kernel later reads on that XCD.  One column of
// partials per workgroup.
// Workgroup barrier that orders LDS accesses only: the global loads and
// stores in flight are not waited for.  The rows kernel's wavefronts share
// data only through LDS (the activations it stores are read by the next
// launch), so its weight prefetches and activation stores run on across
// its barriers.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <uint32_t MT>
__global__ void __launch_bounds__(256 * MT) vn_rows_kernel(VnRowsArgs a)
{
    constexpr uint32_t NW = 4u * MT, JJ = 4u / MT, ROWS = 16u * MT;
    __shared__ __attribute__((aligned(16))) uint16_t hs[ROWS][kVnH + 8];   // h1, then dh2
    __shared__ float zred[NW][ROWS];
    const VnPtrs P = vn_ptrs(const_cast<void *>(a.net));
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6, r = lane & 15u, g = lane >> 4;
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t tb = nb % 8u == 0u ? (b % 8u) * (nb / 8u) + b / 8u : b;
    const uint32_t row0 = tb * ROWS;

    bf16x8 w1f[JJ][5];
#pragma unroll
    for (uint32_t jj = 0; jj < JJ; ++jj)
#pragma unroll
        for (uint32_t s = 0; s < 5u; ++s)
            w1f[jj][s] = load8(P.w1b + (((JJ * wv + jj) * 5u + s) * 64u + lane) * 8u);
    float b1v[JJ], b2v[JJ], w3v[JJ];
#pragma unroll
    for (uint32_t jj = 0; jj < JJ; ++jj) {
        const uint32_t col = 16u * (JJ * wv + jj) + r;
        b1v[jj] = P.master[kOffB1 + col];
        b2v[jj] = P.master[kOffB2 + col];
        w3v[jj] = bf16_to_f(P.w3b[col]);
    }
    const float b3 = P.master[kOffB3];
    // lane r holds row 16m + r of tile m; the labels of rows 16m + 4g + i
    // come from lane 4g + i
    // (every tile's state, perspective and labels are requested before any
    // of them is waited for; data row 0 stands in for rows past the batch)
    bool has[MT];
    RowFeat rf[MT];
    float yv[MT][4];
    uint32_t src[MT];
    uint4 st[MT];
    uint32_t pq[MT];
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m) {
        const uint32_t myrow = row0 + 16u * m + r;
        has[m] = myrow < a.n_rows;
        src[m] = has[m] ? vn_train_row(a, myrow) : 0u;
        st[m] = a.states[src[m]];
        pq[m] = a.persp[src[m]];
    }
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m)
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i) {
            const uint32_t row = row0 + 16u * m + 4u * g + i;
            const uint32_t sr = (uint32_t)__shfl((int)src[m], (int)(4u * g + i), 64);
            yv[m][i] = row < a.n_rows ? a.labels[sr] : 0.0f;
        }
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m) {
        if (has[m]) {
            rf[m] = row_features(st[m], pq[m]);
        } else {
            rf[m].ok = false;
        }
        if (has[m] && !rf[m].ok && wv == 0u) atomicOr(&g_error_word, kErrState);
        if (!rf[m].ok) rf[m] = no_row();
    }

    // ---- layer 1: h1 = bf16(relu(W1 x + b1)), columns of this wavefront ----
    floatx4 acc1[MT][JJ];
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m) {
        bf16x8 xa[5];
#pragma unroll
        for (uint32_t s = 0; s < 5u; ++s) xa[s] = feature8(rf[m], s, g);
#pragma unroll
        for (uint32_t jj = 0; jj < JJ; ++jj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (uint32_t s = 0; s < 5u; ++s) acc = mfma16(xa[s], w1f[jj][s], acc);
            acc1[m][jj] = acc;
        }
    }
    // second-layer weights, requested while the first layer's products run
    bf16x8 w2f[JJ][8];
#pragma unroll
    for (uint32_t jj = 0; jj < JJ; ++jj)
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s)
            w2f[jj][s] = load8(P.w2b + (((JJ * wv + jj) * 8u + s) * 64u + lane) * 8u);
    // X^T (internal feature order) for the weight gradient: the 5 MT (feature
    // block, row tile) pairs split over the wavefronts
    for (uint32_t idx = wv; idx < 5u * MT; idx += NW) {
        const uint32_t s = idx % 5u, m = idx / 5u;
        bool hm = false;
        RowFeat rm = rf[0];
#pragma unroll
        for (uint32_t mm = 0; mm < MT; ++mm)
            if (mm == m) {
                hm = has[mm];
                rm = rf[mm];
            }
        if (hm) {
            const uint32_t fb = feature_word(rm, s) >> (8u * g);
            const uint32_t myrow = row0 + 16u * m + r;
#pragma unroll
            for (uint32_t i = 0; i < 8u; ++i)
                a.xt[vn_act_idx(32u * s + 8u * g + i, myrow, a.n_rows)] =
                    ((fb >> i) & 1u) ? (uint16_t)0x3F80u : (uint16_t)0u;
        }
    }
    uint32_t h1pos[MT];   // bit 4jj+i: h1 of row 16m+4g+i, column 16(JJ wv+jj)+r is positive
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m) {
        h1pos[m] = 0u;
#pragma unroll
        for (uint32_t jj = 0; jj < JJ; ++jj) {
            const uint32_t j = JJ * wv + jj;
            uint16_t hq[4];
#pragma unroll
            for (uint32_t i = 0; i < 4u; ++i) {
                const float h = acc1[m][jj][i] + b1v[jj];
                hq[i] = bf16_bits(h > 0.0f ? h : 0.0f);
                hs[16u * m + 4u * g + i][16u * j + r] = hq[i];
                h1pos[m] |= (uint32_t)(h > 0.0f) << (4u * jj + i);
            }
            const uint32_t rr = row0 + 16u * m + 4u * g;
            if (rr + 3u < a.n_rows) {
                const uint2 packed = make_uint2((uint32_t)hq[0] | ((uint32_t)hq[1] << 16),
                                                (uint32_t)hq[2] | ((uint32_t)hq[3] << 16));
                *reinterpret_cast<uint2 *>(a.h1t + vn_act_idx(16u * j + r, rr, a.n_rows)) = packed;
            }
        }
    }
    lds_barrier();

    // ---- layer 2: h2 = bf16(relu(W2 h1 + b2)), z = w3 . h2 + b3 ------------
    floatx4 acc2[MT][JJ];
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m) {
        bf16x8 ha[8];
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s) ha[s] = load8(&hs[16u * m + r][32u * s + 8u * g]);
#pragma unroll
        for (uint32_t jj = 0; jj < JJ; ++jj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (uint32_t s = 0; s < 8u; ++s) acc = mfma16(ha[s], w2f[jj][s], acc);
            acc2[m][jj] = acc;
        }
    }
    // transposed second-layer weights for the data gradient, requested now
    bf16x8 w2tf[JJ][8];
#pragma unroll
    for (uint32_t jj = 0; jj < JJ; ++jj)
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s)
            w2tf[jj][s] = load8(P.w2tb + (((JJ * wv + jj) * 8u + s) * 64u + lane) * 8u);
    floatx4 h2[MT][JJ];
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m) {
        float zpart[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (uint32_t jj = 0; jj < JJ; ++jj) {
#pragma unroll
            for (uint32_t i = 0; i < 4u; ++i) {
                const float h = acc2[m][jj][i] + b2v[jj];
                h2[m][jj][i] = bf16_round(h > 0.0f ? h : 0.0f);
                zpart[i] += h2[m][jj][i] * w3v[jj];
            }
        }
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i)
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) zpart[i] += __shfl_xor(zpart[i], off, 64);
        if (r == 0u) {
#pragma unroll
            for (uint32_t i = 0; i < 4u; ++i) zred[wv][16u * m + 4u * g + i] = zpart[i];
        }
    }
    lds_barrier();   // zred complete; every wavefront has read h1 from hs
    float dz[MT][4], err2 = 0.0f, dsum = 0.0f;
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m) {
#pragma unroll
        for (uint32_t i = 0; i < 4u; ++i) {
            const uint32_t lr = 16u * m + 4u * g + i;
            float z = zred[0][lr];
#pragma unroll
            for (uint32_t w = 1; w < NW; ++w) z += zred[w][lr];
            const float v = 1.0f / (1.0f + expf(-(z + b3)));
            const uint32_t row = row0 + lr;
            float d = 0.0f;
            if (row < a.n_rows) {
                const float e = v - yv[m][i];
                err2 += e * e;
                d = 2.0f * e * a.inv_batch * v * (1.0f - v);
            }
            dz[m][i] = d;
            dsum += d;
        }
    }
    // this workgroup's partials, one column of stride gridDim.x each
    float *part = a.part + tb;
    const size_t pst = nb;
    if (wv == 0u) {
        float l4 = r == 0u ? err2 : 0.0f, d3 = r == 0u ? dsum : 0.0f;
        for (int off = 1; off < 64; off <<= 1) {
            l4 += __shfl_xor(l4, off, 64);
            d3 += __shfl_xor(d3, off, 64);
        }
        if (lane == 0) {
            part[0] = l4;
            part[pst] = d3;
        }
    }

    // ---- dh2 = dz w3 (h2 > 0); w3 and b2 gradients ---------------------------
#pragma unroll
    for (uint32_t jj = 0; jj < JJ; ++jj) {
        const uint32_t col = 16u * (JJ * wv + jj) + r;
        const float w3 = w3v[jj];
        float dw3 = 0.0f, db2 = 0.0f;
#pragma unroll
        for (uint32_t m = 0; m < MT; ++m) {
            uint16_t dq[4];
#pragma unroll
            for (uint32_t i = 0; i < 4u; ++i) {
                dw3 += dz[m][i] * h2[m][jj][i];
                const float d = h2[m][jj][i] > 0.0f ? dz[m][i] * w3 : 0.0f;
                dq[i] = bf16_bits(d);
                db2 += bf16_to_f(dq[i]);
                hs[16u * m + 4u * g + i][col] = dq[i];
            }
            const uint32_t rr = row0 + 16u * m + 4u * g;
            if (rr + 3u < a.n_rows) {
                const uint2 packed = make_uint2((uint32_t)dq[0] | ((uint32_t)dq[1] << 16),
                                                (uint32_t)dq[2] | ((uint32_t)dq[3] << 16));
                *reinterpret_cast<uint2 *>(a.dh2t + vn_act_idx(col, rr, a.n_rows)) = packed;
            }
        }
        dw3 += __shfl_xor(dw3, 16, 64);
        dw3 += __shfl_xor(dw3, 32, 64);
        db2 += __shfl_xor(db2, 16, 64);
        db2 += __shfl_xor(db2, 32, 64);
        if (g == 0u) {
            part[(2u + col) * pst] = dw3;
            part[(2u + 256u + col) * pst] = db2;
        }
    }
    lds_barrier();   // dh2 tiles complete

    // ---- dh1 = (dh2 W2) * (h1 > 0), columns of this wavefront ----------------
    float db1[JJ];
#pragma unroll
    for (uint32_t jj = 0; jj < JJ; ++jj) db1[jj] = 0.0f;
#pragma unroll
    for (uint32_t m = 0; m < MT; ++m) {
        bf16x8 da[8];
#pragma unroll
        for (uint32_t s = 0; s < 8u; ++s) da[s] = load8(&hs[16u * m + r][32u * s + 8u * g]);
#pragma unroll
        for (uint32_t jj = 0; jj < JJ; ++jj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (uint32_t s = 0; s < 8u; ++s) acc = mfma16(da[s], w2tf[jj][s], acc);
            const uint32_t col = 16u * (JJ * wv + jj) + r;
            uint16_t dq[4];
#pragma unroll
            for (uint32_t i = 0; i < 4u; ++i) {
                const float d = ((h1pos[m] >> (4u * jj + i)) & 1u) ? acc[i] : 0.0f;
                dq[i] = bf16_bits(d);
                db1[jj] += bf16_to_f(dq[i]);
            }
            const uint32_t rr = row0 + 16u * m + 4u * g;
            if (rr + 3u < a.n_rows) {
                const uint2 packed = make_uint2((uint32_t)dq[0] | ((uint32_t)dq[1] << 16),
                                                (uint32_t)dq[2] | ((uint32_t)dq[3] << 16));
                *reinterpret_cast<uint2 *>(a.dh1t + vn_act_idx(col, rr, a.n_rows)) = packed;
            }
        }
    }
#pragma unroll
    for (uint32_t jj = 0; jj < JJ; ++jj) {
        const uint32_t col = 16u * (JJ * wv + jj) + r;
        float d = db1[jj];
        d += __shfl_xor(d, 16, 64);
        d += __shfl_xor(d, 32, 64);
        if (g == 0u) part[(2u + 512u + col) * pst] = d;
    }
}

// Adam (Kingma and Ba, 2015) for parameter k (canonical order) with gradient
// gk, on the float32 master weight and moments; the bf16 shadow the products
// read is refreshed from the updated weight.  `p` is the internal feature
// index of a W1 weight (its column in the shadow), unused otherwise.
// beta1, beta2 and their complements 1 - beta1, 1 - beta2 are each the
// float nearest the exact value (1 - 0.999f computed in float would be
// 1.3e-5 away from 0.001 in relative terms)
struct VnAdam {
    float lr, beta1, beta2, eps, c1, c2, omb1, omb2;
};

__device__ __forceinline__ void vn_adam_one(const VnPtrs &P, const VnAdam &h, uint32_t k,
                                            uint32_t p, float gk, float *grad_out)
{
    if (grad_out) grad_out[k] = gk;
    const float m = h.beta1 * P.m[k] + h.omb1 * gk;
    const float v = h.beta2 * P.v[k] + h.omb2 * gk * gk;
    P.m[k] = m;
    P.v[k] = v;
    const float w = P.master[k] - h.lr * (m / h.c1) / (sqrtf(v / h.c2) + h.eps);
    P.master[k] = w;
    const uint16_t b = bf16_bits(w);
    if (k < kOffB1) {
        P.w1b[vn_frag(k / kVnIn, p, 5u)] = b;
    } else if (k >= kOffW2 && k < kOffB2) {
        const uint32_t kk = k - kOffW2, n = kk / kVnH, i = kk % kVnH;
        P.w2b[vn_frag(n, i, 8u)] = b;
        P.w2tb[vn_frag(i, n, 8u)] = b;
    } else if (k >= kOffW3 && k < kOffB3) {
        P.w3b[k - kOffW3] = b;
    }
}

struct VnGradArgs {
    void *net;
    const uint16_t *xt, *h1t, *dh1t, *dh2t;   // fragment layout (vn_act_idx), batch K
    uint32_t K, slices, k_slice;             // slice length: a multiple of 32
    float *grad;                             // slice s of the weight gradients at s * kVnPad
    const float *part;                       // column-major partials of the row workgroups
    uint32_t n_parts;
    VnAdam h;
    float inv_batch;
    float *grad_out, *loss_out;
};

// The weight gradients, and the Adam step of the parameters outside W1 and
// W2, in one launch of single-wavefront workgroups.  Workgroups [0, 104 S):
// one 32 x 32 tile of dW2 = dh2^T h1 or dW1 = dh1^T x and one of S batch
// slices each (split K, so that enough wavefronts stream the activations at
// once); the partial tile goes to its slice's copy of the gradient.
// Workgroup b takes slice b % S: with S = 8, consecutive workgroups going to
// the 8 XCDs in turn, each XCD streams one slice of the activations (1/8 of
// them, small enough to stay in its L2) instead of all of them.
// Workgroups [104 S, 104 S + 770): one column of the rows kernel's partials
// each (loss, b3, w3, b2, b1), summed by lane l over tiles l, l + 64, ... and
// then across the lanes in a fixed order, followed by that parameter's Adam
// step (those parameters are read by no other workgroup of the launch).
constexpr uint32_t kVnChunk = 4u;        // k steps whose operands are loaded together

__global__ void __launch_bounds__(64) vn_grad_kernel(VnGradArgs a)
{
    const VnPtrs P = vn_ptrs(a.net);
    const uint32_t lane = threadIdx.x, r = lane & 15u, g = lane >> 4;
    const uint32_t n_tile_groups = kVnGradTiles * a.slices;
    if (blockIdx.x >= n_tile_groups) {
        const uint32_t col = blockIdx.x - n_tile_groups;
        if (col >= kPartWords) return;
        const float *pc = a.part + (size_t)col * a.n_parts;
        float acc = 0.0f;
        for (uint32_t w0 = 0; w0 < a.n_parts; w0 += 512u) {
            // eight loads in flight, then the additions in index order
            float x[8];
#pragma unroll
            for (uint32_t u = 0; u < 8u; ++u) {
                const uint32_t w = w0 + 64u * u + lane;
                x[u] = w < a.n_parts ? pc[w] : 0.0f;
            }
#pragma unroll
            for (uint32_t u = 0; u < 8u; ++u)
                if (w0 + 64u * u + lane < a.n_parts) acc += x[u];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane != 0u) return;
        if (col == 0u) {
            if (a.loss_out) *a.loss_out = acc * a.inv_batch;
            return;
        }
        const uint32_t k = col == 1u ? kOffB3
                         : col < 258u ? kOffW3 + (col - 2u)
                         : col < 514u ? kOffB2 + (col - 258u)
                                      : kOffB1 + (col - 514u);
        vn_adam_one(P, a.h, k, 0u, acc, a.grad_out);
        return;
    }

    const uint32_t tile = blockIdx.x / a.slices, slice = blockIdx.x % a.slices;
    const bool w2 = tile < kVnTilesW2;
    const uint32_t t = w2 ? tile : tile - kVnTilesW2;
    const uint32_t ntn = w2 ? 8u : 5u;                    // 32-wide column tiles
    const uint32_t mt = t / ntn, nt = t % ntn;
    const uint32_t ldo = w2 ? kVnH : kVnIn, off = w2 ? kOffW2 : kOffW1;
    const uint16_t *at = w2 ? a.dh2t : a.dh1t;
    const uint16_t *bt = w2 ? a.h1t : a.xt;
    const uint32_t kb = slice * a.k_slice;
    // operand fragments of the 16-feature tiles 2mt, 2mt + 1 (A) and 2nt,
    // 2nt + 1 (B) at the slice's first k step; a k step is 512 elements on
    const uint16_t *ap0 = at + vn_act_idx(32u * mt, kb, a.K) + 8u * lane;
    const uint16_t *ap1 = at + vn_act_idx(32u * mt + 16u, kb, a.K) + 8u * lane;
    const uint16_t *bp0 = bt + vn_act_idx(32u * nt, kb, a.K) + 8u * lane;
    const uint16_t *bp1 = bt + vn_act_idx(32u * nt + 16u, kb, a.K) + 8u * lane;

    floatx4 acc[2][2];
#pragma unroll
    for (uint32_t x = 0; x < 2u; ++x)
#pragma unroll
        for (uint32_t y = 0; y < 2u; ++y) acc[x][y] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    // operands of kVnChunk k steps are requested one chunk ahead of the
    // products that use them
    const uint32_t nsteps = a.k_slice / 32u, nfull = nsteps / kVnChunk;
    bf16x8 fa[kVnChunk][2], fb[kVnChunk][2];
    auto load_chunk = [&](uint32_t c, bf16x8 (&A)[kVnChunk][2], bf16x8 (&B)[kVnChunk][2]) {
#pragma unroll
        for (uint32_t u = 0; u < kVnChunk; ++u) {
            const uint32_t k0 = 512u * (c * kVnChunk + u);
            A[u][0] = load8(ap0 + k0);
            A[u][1] = load8(ap1 + k0);
            B[u][0] = load8(bp0 + k0);
            B[u][1] = load8(bp1 + k0);
        }
    };
    auto run_chunk = [&](bf16x8 (&A)[kVnChunk][2], bf16x8 (&B)[kVnChunk][2]) {
#pragma unroll
        for (uint32_t u = 0; u < kVnChunk; ++u)
#pragma unroll
            for (uint32_t x = 0; x < 2u; ++x)
#pragma unroll
                for (uint32_t y = 0; y < 2u; ++y) acc[x][y] = mfma16(A[u][x], B[u][y], acc[x][y]);
    };
    // two operand buffers used in turn (no register copies between chunks,
    // which would wait for the loads just issued)
    if (nfull > 0u) {
        bf16x8 ga_[kVnChunk][2], gb_[kVnChunk][2];
        load_chunk(0u, fa, fb);
        uint32_t c = 0;
        for (; c + 2u < nfull; c += 2u) {
            load_chunk(c + 1u, ga_, gb_);
            run_chunk(fa, fb);
            load_chunk(c + 2u, fa, fb);
            run_chunk(ga_, gb_);
        }
        if (c + 1u < nfull) {
            load_chunk(c + 1u, ga_, gb_);
            run_chunk(fa, fb);
            run_chunk(ga_, gb_);
        } else {
            run_chunk(fa, fb);
        }
    }
    for (uint32_t s = nfull * kVnChunk; s < nsteps; ++s) {
        const uint32_t k0 = 512u * s;
        const bf16x8 a0 = load8(ap0 + k0), a1 = load8(ap1 + k0);
        const bf16x8 b0 = load8(bp0 + k0), b1 = load8(bp1 + k0);
        acc[0][0] = mfma16(a0, b0, acc[0][0]);
        acc[0][1] = mfma16(a0, b1, acc[0][1]);
        acc[1][0] = mfma16(a1, b0, acc[1][0]);
        acc[1][1] = mfma16(a1, b1, acc[1][1]);
    }

    float *o = a.grad + (size_t)slice * kVnPad + off;
#pragma unroll
    for (uint32_t x = 0; x < 2u; ++x)
#pragma unroll
        for (uint32_t y = 0; y < 2u; ++y)
#pragma unroll
            for (uint32_t i = 0; i < 4u; ++i)
                o[(size_t)(32u * mt + 16u * x + 4u * g + i) * ldo + 32u * nt + 16u * y + r] =
                    acc[x][y][i];

}

// Adam for the weights of W1 and W2: the S slices' partial gradients summed
// in slice order (the W1 gradient is laid out in the internal feature order).
__global__ void vn_adam_w_kernel(void *net, const float *grad, uint32_t slices, VnAdam h,
                                 float *grad_out)
{
    const VnPtrs P = vn_ptrs(net);
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kOffB1 + kVnH * kVnH) return;
    const bool w1 = e < kOffB1;
    const uint32_t k = w1 ? e : kOffW2 + (e - kOffB1);          // canonical index
    const uint32_t p = w1 ? vn_perm(k % kVnIn) : 0u;
    const uint32_t kg = w1 ? (k / kVnIn) * kVnIn + p : k;
    // the (at most eight) slices' loads in flight together, then summed in order
    float x[kVnMaxSlices];
#pragma unroll
    for (uint32_t sl = 0; sl < kVnMaxSlices; ++sl)
        x[sl] = sl < slices ? grad[(size_t)sl * kVnPad + kg] : 0.0f;
    float gk = x[0];
#pragma unroll
    for (uint32_t sl = 1; sl < kVnMaxSlices; ++sl)
        if (sl < slices) gk += x[sl];
    vn_adam_one(P, h, k, p, gk, grad_out);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
size_t vn_bytes() { return (size_t)kVnBytes; }

// batch slices of the weight-gradient products: up to 8, each a multiple of
// 32 rows
static constexpr uint32_t vn_wgrad_slices(uint32_t batch)
{
    uint32_t s = kVnMaxSlices;
    while (s > 1u && (batch / 32u) % s != 0u) s >>= 1;
    return s;
}

// xt (160 x B), h1t, dh1t, dh2t (256 x B) bf16; grad[NPAD] fp32 per slice;
// partials of the row workgroups (at most one column per 16 rows, and one
// spare row)
static constexpr size_t vn_ws_bytes(uint32_t batch)
{
    return (size_t)batch * (160u + 3u * 256u) * 2u + (size_t)vn_wgrad_slices(batch) * kVnPad * 4u +
           (size_t)((batch + 15u) / 16u + 1u) * kPartWords * 4u + 256u;
}

size_t vn_train_ws_bytes(uint32_t batch) { return vn_ws_bytes(batch); }

hipError_t launch_vn_init(void *net, uint32_t k0, uint32_t k1, hipStream_t st)
{
    const float bw1 = sqrtf(6.0f / 148.0f), bw2 = sqrtf(6.0f / 256.0f), bw3 = 1.0f / 16.0f;
    hipLaunchKernelGGL(vn_init_kernel, dim3((kVnPad + 255u) / 256u), dim3(256), 0, st, net, k0, k1,
                       bw1, bw2, bw3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(vn_shadow_kernel, dim3(65536u / 256u), dim3(256), 0, st, net);
    return hipGetLastError();
}

hipError_t launch_vn_shadow(void *net, hipStream_t st)
{
    hipLaunchKernelGGL(vn_shadow_kernel, dim3(65536u / 256u), dim3(256), 0, st, net);
    return hipGetLastError();
}

hipError_t launch_vn_infer(const void *net, const uint4 *states, const uint8_t *persp, uint32_t n,
                           float *v_out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    VnRowsArgs a = {};
    a.net = net;
    a.states = states;
    a.persp = persp;
    a.n_rows = n;
    a.v_out = v_out;
    hipLaunchKernelGGL(vn_infer_kernel, dim3((n + 15u) / 16u), dim3(64), 0, st, net, states, persp, n,
                       v_out);
    return hipGetLastError();
}

hipError_t launch_vn_train_step(void *net, const uint4 *states, const uint8_t *persp,
                                const float *labels, uint32_t n_data, uint32_t perm_a,
                                uint32_t perm_b, uint32_t row_base, uint32_t batch, float lr,
                                float c1, float c2, void *ws, float *loss_out, float *grad_out,
                                hipStream_t st)
{
    uint8_t *w = (uint8_t *)ws;
    VnRowsArgs a = {};
    a.net = net;
    a.states = states;
    a.persp = persp;
    a.labels = labels;
    a.n_rows = batch;
    a.n_data = n_data;
    a.n_mask = (n_data & (n_data - 1u)) == 0u ? n_data - 1u : 0u;
    a.perm_a = perm_a;
    a.perm_b = perm_b;
    a.row_base = row_base;
    a.xt = (uint16_t *)w;
    a.h1t = a.xt + (size_t)160u * batch;
    a.dh1t = a.h1t + (size_t)256u * batch;
    a.dh2t = a.dh1t + (size_t)256u * batch;
    float *grad = (float *)(a.dh2t + (size_t)256u * batch);
    const uint32_t slices = vn_wgrad_slices(batch);
    a.part = grad + (size_t)slices * kVnPad;
    a.inv_batch = 1.0f / (float)batch;
    // 32-row workgroups of two tiles (the batch is a multiple of 32): each
    // weight fragment serves two products (25.9 against 26.8 us per step of
    // 8192 rows with one tile per workgroup)
    const uint32_t waves = batch / 32u;
    hipLaunchKernelGGL(vn_rows_kernel<2>, dim3(waves), dim3(512), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    VnGradArgs ga = {};
    ga.net = net;
    ga.xt = a.xt;
    ga.h1t = a.h1t;
    ga.dh1t = a.dh1t;
    ga.dh2t = a.dh2t;
    ga.K = batch;
    ga.slices = slices;
    ga.k_slice = batch / slices;
    ga.grad = grad;
    ga.part = a.part;
    ga.n_parts = waves;
    ga.h = VnAdam{lr, 0.9f, 0.999f, 1e-8f, c1, c2, (float)(1.0 - 0.9), (float)(1.0 - 0.999)};
    ga.inv_batch = a.inv_batch;
    ga.grad_out = grad_out;
    ga.loss_out = loss_out;
    hipLaunchKernelGGL(vn_grad_kernel, dim3(kVnGradTiles * slices + kPartWords), dim3(64), 0, st,
                       ga);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr uint32_t n_w = kOffB1 + kVnH * kVnH;
    hipLaunchKernelGGL(vn_adam_w_kernel, dim3((n_w + 255u) / 256u), dim3(256), 0, st, net, grad,
                       slices, ga.h, grad_out);
    return hipGetLastError();
}

__global__ void vn_set_params_kernel(void *net, const float *params)
{
    VnPtrs P = vn_ptrs(net);
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kVnPad) return;
    P.master[k] = k < kVnParams ? params[k] : 0.0f;
    P.m[k] = 0.0f;
    P.v[k] = 0.0f;
}

__global__ void vn_get_params_kernel(const void *net, float *params)
{
    const VnPtrs P = vn_ptrs(const_cast<void *>(net));
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kVnParams) params[k] = P.master[k];
}

__global__ void vn_get_moments_kernel(const void *net, float *m, float *v)
{
    const VnPtrs P = vn_ptrs(const_cast<void *>(net));
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kVnParams) return;
    m[k] = P.m[k];
    v[k] = P.v[k];
}

// perspective of a training pair and its playout win-rate label
__global__ void vn_labels_kernel(const uint4 *states, uint32_t n, uint32_t playouts, uint32_t k0,
                                 uint32_t k1, uint32_t base, const uint32_t *seat_wins,
                                 uint8_t *persp, float *labels)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t P = ((states[i].x >> 26) & 3u) + 1u;
    const Words w = philox(0u, 0xFFFFFFFCu, 0u, base + i, k0, k1);
    const uint32_t q = pick(w.w0, P);
    persp[i] = (uint8_t)q;
    labels[i] = (float)seat_wins[(size_t)i * 4u + q] / (float)playouts;
}

hipError_t launch_vn_set_params(void *net, const float *params, hipStream_t st)
{
    hipLaunchKernelGGL(vn_set_params_kernel, dim3((kVnPad + 255u) / 256u), dim3(256), 0, st, net,
                       params);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_vn_shadow(net, st);
}

hipError_t launch_vn_get_params(const void *net, float *params, hipStream_t st)
{
    hipLaunchKernelGGL(vn_get_params_kernel, dim3((kVnParams + 255u) / 256u), dim3(256), 0, st, net,
                       params);
    return hipGetLastError();
}

hipError_t launch_vn_get_moments(const void *net, float *m, float *v, hipStream_t st)
{
    hipLaunchKernelGGL(vn_get_moments_kernel, dim3((kVnParams + 255u) / 256u), dim3(256), 0, st,
                       net, m, v);
    return hipGetLastError();
}

hipError_t launch_vn_labels(const uint4 *states, uint32_t n, uint32_t playouts, uint32_t k0,
                            uint32_t k1, uint32_t index_base, const uint32_t *seat_wins,
                            uint8_t *persp, float *labels, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(vn_labels_kernel, dim3((n + 255u) / 256u), dim3(256), 0, st, states, n,
                       playouts, k0, k1, index_base, seat_wins, persp, labels);
    return hipGetLastError();
}

}  // namespace dvc
