// Learned edge proposal: per-(edge, view) features, the 32-64-64-1 MLP on the
// BF16 matrix cores (forward and backward), and per-view softmax
// cross-entropy.
//
// The thesis samples edges by importance (Ch. 5, Importance Sampling the
// Edges) with a hand-built pdf; this network proposes a per-view distribution
// over edges that the renderer mixes with that pdf, trained on the boundary
// magnitudes the renderer itself harvests.
//
// Arithmetic: inputs and weight matrices are rounded to BF16 (nearest even);
// hidden activations and all gradients stay FP32 and enter the matrix cores
// as a sum of three BF16 terms (hi + mid + lo, exact to ~2^-24); every MFMA
// accumulates in FP32. Biases, logits and the softmax are FP32.
//
// MFMA v_mfma_f32_16x16x32_bf16 (one wave): A is 16 x 32, B is 32 x 16, C/D
// is 16 x 16. Lane l holds row (l & 15) of A and column (l & 15) of B, eight
// consecutive k each (k = 8 (l >> 4) + j); C/D lane l holds column (l & 15),
// rows 4 (l >> 4) + i, i < 4. A and B place k identically, so the product
// does not depend on the order of k within a lane group.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "dr_host.h"

namespace dr {
namespace {

constexpr int kNF = 32, kHid = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 32 * 64, OFF_W2 = OFF_B1 + 64, OFF_B2 = OFF_W2 + 64 * 64, OFF_W3 = OFF_B2 + 64,
              OFF_B3 = OFF_W3 + 64, NPAR = OFF_B3 + 1;
static_assert(NPAR == DR_MLP_PARAMS, "parameter layout");
constexpr float kNdcClamp = 8.0f;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);      // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_round(float x) { return __uint_as_float((uint32_t)bf16_bits(x) << 16); }

__device__ inline bf16x8 pack8(const float v[8]) {
    s16x8 s;
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] = (short)bf16_bits(v[j]);
    return __builtin_bit_cast(bf16x8, s);
}

// x = hi + mid + lo, each a BF16 number
__device__ inline void split8(const float v[8], bf16x8& hi, bf16x8& mi, bf16x8& lo) {
    float r1[8], r2[8], r3[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float h = bf16_round(v[j]);
        r1[j] = h;
        float rem = v[j] - h;
        float m = bf16_round(rem);
        r2[j] = m;
        r3[j] = rem - m;
    }
    hi = pack8(r1);
    mi = pack8(r2);
    lo = pack8(r3);
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

__device__ inline float group16_sum(float v) {
    // sum over the 16 lanes sharing (lane >> 4)
    for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float across_groups_sum(float v) {
    // sum over the 4 lanes sharing (lane & 15)
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
__device__ inline v3 face_unit_normal(const float* P, const int* I, int f) {
    v3 p0 = ld3(P, I[3 * f]), p1 = ld3(P, I[3 * f + 1]), p2 = ld3(P, I[3 * f + 2]);
    return nrm(cross(p1 - p0, p2 - p0));
}

__global__ void k_edge_features(SceneView s, Cam k, float* __restrict__ X) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.E) return;
    int4 e = s.edges[i];
    v3 A = ld3(s.P, e.x), B = ld3(s.P, e.y);
    v3 da = A - k.c, db = B - k.c;
    v3 qa = {dot(da, k.r), dot(da, k.u), dot(da, k.f)};
    v3 qb = {dot(db, k.r), dot(db, k.u), dot(db, k.f)};
    bool has1 = e.w >= 0;
    v3 n0 = face_unit_normal(s.P, s.I, e.z);
    v3 n1 = has1 ? face_unit_normal(s.P, s.I, e.w) : v3{0.0f, 0.0f, 0.0f};
    float f[kNF];
    f[0] = qa.x; f[1] = qa.y; f[2] = qa.z;
    f[3] = qb.x; f[4] = qb.y; f[5] = qb.z;
    f[6] = dot(n0, k.r); f[7] = dot(n0, k.u); f[8] = dot(n0, k.f);
    f[9] = dot(n1, k.r); f[10] = dot(n1, k.u); f[11] = dot(n1, k.f);
    f[12] = A.x; f[13] = A.y; f[14] = A.z;
    f[15] = B.x; f[16] = B.y; f[17] = B.z;
    f[18] = s.alb[e.z];
    f[19] = has1 ? s.alb[e.w] : 0.0f;
    f[20] = s.emi[e.z];
    f[21] = has1 ? s.emi[e.w] : 0.0f;
    f[22] = has1 ? 0.0f : 1.0f;
    f[23] = has1 ? dot(n0, n1) : 0.0f;
    float za = fmaxf(qa.z, k.nearc), zb = fmaxf(qb.z, k.nearc);
    f[24] = fminf(fmaxf(qa.x / (za * k.th * k.asp), -kNdcClamp), kNdcClamp);
    f[25] = fminf(fmaxf(qa.y / (za * k.th), -kNdcClamp), kNdcClamp);
    f[26] = fminf(fmaxf(qb.x / (zb * k.th * k.asp), -kNdcClamp), kNdcClamp);
    f[27] = fminf(fmaxf(qb.y / (zb * k.th), -kNdcClamp), kNdcClamp);
    f[28] = len(B - A);
    f[29] = f[30] = f[31] = 0.0f;
    float4* out = reinterpret_cast<float4*>(X + (size_t)i * kNF);
#pragma unroll
    for (int q = 0; q < kNF / 4; ++q) out[q] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
}

// ---------------------------------------------------------------------------
// network (one wave per block; each wave owns its LDS tiles)
// ---------------------------------------------------------------------------
struct Weights {
    bf16x8 B1[4];          // W1 tiles: k = 8g + j, n = 16 nt + c
    bf16x8 B2[2][4];       // W2 tiles: k = 32 ks + 8g + j, n = 16 nt + c
    float b1[4], b2[4], w3[4], b3;
};

__device__ inline void load_weights(const float* __restrict__ th, int g, int c, Weights& w) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = th[OFF_W1 + (8 * g + j) * kHid + 16 * nt + c];
        w.B1[nt] = pack8(v);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = th[OFF_W2 + (32 * ks + 8 * g + j) * kHid + 16 * nt + c];
            w.B2[ks][nt] = pack8(v);
        }
        w.b1[nt] = th[OFF_B1 + 16 * nt + c];
        w.b2[nt] = th[OFF_B2 + 16 * nt + c];
        w.w3[nt] = bf16_round(th[OFF_W3 + 16 * nt + c]);
    }
    w.b3 = th[OFF_B3];
}

// Forward of 16 rows starting at r0 (rows >= n read as zero input). On return
// a1/a2 hold the pre-activations and h2 the second hidden layer in C/D layout
// (rows 4g + i, column 16 nt + c); hs[16][65] holds the first hidden layer.
__device__ inline void forward16(const Weights& w, const float* __restrict__ X, int n, int r0, int g, int c, float* hs,
                                 float a1[4][4], float a2[4][4]) {
    float xv[8];
    int row = r0 + c;
#pragma unroll
    for (int j = 0; j < 8; ++j) xv[j] = row < n ? X[(size_t)row * kNF + 8 * g + j] : 0.0f;
    bf16x8 ax = pack8(xv);
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = mfma(ax, w.B1[nt], zero);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a1[nt][i] = acc[i] + w.b1[nt];
            hs[(4 * g + i) * 65 + 16 * nt + c] = fmaxf(a1[nt][i], 0.0f);
        }
    }
    __syncthreads();
    f32x4 acc2[4] = {zero, zero, zero, zero};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = hs[c * 65 + 32 * ks + 8 * g + j];
        bf16x8 hi, mi, lo;
        split8(v, hi, mi, lo);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            acc2[nt] = mfma(hi, w.B2[ks][nt], acc2[nt]);
            acc2[nt] = mfma(mi, w.B2[ks][nt], acc2[nt]);
            acc2[nt] = mfma(lo, w.B2[ks][nt], acc2[nt]);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) a2[nt][i] = acc2[nt][i] + w.b2[nt];
}

__global__ __launch_bounds__(64) void k_mlp_forward(const float* __restrict__ th, const float* __restrict__ X, int n,
                                                    float* __restrict__ z) {
    __shared__ float hs[16 * 65];
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    Weights w;
    load_weights(th, g, c, w);
    int tiles = (n + 15) / 16;
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        int r0 = 16 * t;
        float a1[4][4], a2[4][4];
        forward16(w, X, n, r0, g, c, hs, a1, a2);
        float zp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) zp[i] += fmaxf(a2[nt][i], 0.0f) * w.w3[nt];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = group16_sum(zp[i]);
            int row = r0 + 4 * g + i;
            if (c == 0 && row < n) z[row] = s + w.b3;
        }
        __syncthreads();     // hs is rewritten by the next tile
    }
}

// Backward: per 32-row tile, recompute the forward of both 16-row halves, then
// g2 = dz w3 [a2 > 0], g1 = (g2 W2^T) [a1 > 0], and the weight gradients as
// GEMMs contracted over the tile's 32 rows. Accumulates into grad (zeroed by
// the caller) with one atomic add per entry per wave.
__global__ __launch_bounds__(64) void k_mlp_backward(const float* __restrict__ th, const float* __restrict__ X, int n,
                                                     const float* __restrict__ dz, float* __restrict__ grad) {
    __shared__ float h1s[32 * 65], g2s[32 * 65], g1s[32 * 65];
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    Weights w;
    load_weights(th, g, c, w);
    bf16x8 W2T[2][4];      // B[k = unit 32 ks + 8g + j][n = feature 16 nt + c] = W2[feature][unit]
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = th[OFF_W2 + (16 * nt + c) * kHid + 32 * ks + 8 * g + j];
            W2T[ks][nt] = pack8(v);
        }
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 dW2[4][4], dW1[2][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) dW2[a][b] = zero;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) dW1[a][b] = zero;
    float dW3[4] = {0, 0, 0, 0}, db2[4] = {0, 0, 0, 0}, db1[4] = {0, 0, 0, 0}, db3 = 0.0f;
    int tiles = (n + 31) / 32;
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        int r0 = 32 * t;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            int rh = r0 + 16 * half;
            float* hs = h1s + 16 * half * 65;
            float a1[4][4], a2[4][4];
            forward16(w, X, n, rh, g, c, hs, a1, a2);
            float dzv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int row = rh + 4 * g + i;
                dzv[i] = row < n ? dz[row] : 0.0f;
                if (c == 0) db3 += dzv[i];
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    dW3[nt] += fmaxf(a2[nt][i], 0.0f) * dzv[i];
                    float gg = a2[nt][i] > 0.0f ? dzv[i] * w.w3[nt] : 0.0f;
                    db2[nt] += gg;
                    g2s[(16 * half + 4 * g + i) * 65 + 16 * nt + c] = gg;
                }
            __syncthreads();
            f32x4 acc[4] = {zero, zero, zero, zero};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = g2s[(16 * half + c) * 65 + 32 * ks + 8 * g + j];
                bf16x8 hi, mi, lo;
                split8(v, hi, mi, lo);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    acc[nt] = mfma(hi, W2T[ks][nt], acc[nt]);
                    acc[nt] = mfma(mi, W2T[ks][nt], acc[nt]);
                    acc[nt] = mfma(lo, W2T[ks][nt], acc[nt]);
                }
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float gg = a1[nt][i] > 0.0f ? acc[nt][i] : 0.0f;
                    db1[nt] += gg;
                    g1s[(16 * half + 4 * g + i) * 65 + 16 * nt + c] = gg;
                }
            __syncthreads();
        }
        // dW2[f][u] += sum over the 32 rows of h1[row][f] g2[row][u]
        // (A: f = 16 mt + c, k = row 8g + j; B: k = row 8g + j, u = 16 nt + c)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = h1s[(8 * g + j) * 65 + 16 * mt + c];
            bf16x8 ah, am, al;
            split8(v, ah, am, al);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = g2s[(8 * g + j) * 65 + 16 * nt + c];
                bf16x8 bh, bm, bl;
                split8(v, bh, bm, bl);
                f32x4 d = dW2[mt][nt];
                d = mfma(ah, bh, d);
                d = mfma(ah, bm, d);
                d = mfma(am, bh, d);
                d = mfma(ah, bl, d);
                d = mfma(al, bh, d);
                d = mfma(am, bm, d);
                dW2[mt][nt] = d;
            }
        }
        // dW1[f][k] += sum over the 32 rows of bf16(X)[row][f] g1[row][k]
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                int row = r0 + 8 * g + j;
                v[j] = row < n ? X[(size_t)row * kNF + 16 * mt + c] : 0.0f;
            }
            bf16x8 ax = pack8(v);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = g1s[(8 * g + j) * 65 + 16 * nt + c];
                bf16x8 bh, bm, bl;
                split8(v, bh, bm, bl);
                f32x4 d = dW1[mt][nt];
                d = mfma(ax, bh, d);
                d = mfma(ax, bm, d);
                d = mfma(ax, bl, d);
                dW1[mt][nt] = d;
            }
        }
        __syncthreads();     // the LDS tiles are rewritten by the next tile
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = dW2[mt][nt][i];
                if (v != 0.0f) atomicAdd(&grad[OFF_W2 + (16 * mt + 4 * g + i) * kHid + 16 * nt + c], v);
            }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = dW1[mt][nt][i];
                if (v != 0.0f) atomicAdd(&grad[OFF_W1 + (16 * mt + 4 * g + i) * kHid + 16 * nt + c], v);
            }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        float a = across_groups_sum(dW3[nt]), b = across_groups_sum(db2[nt]), d = across_groups_sum(db1[nt]);
        if (g == 0) {
            if (a != 0.0f) atomicAdd(&grad[OFF_W3 + 16 * nt + c], a);
            if (b != 0.0f) atomicAdd(&grad[OFF_B2 + 16 * nt + c], b);
            if (d != 0.0f) atomicAdd(&grad[OFF_B1 + 16 * nt + c], d);
        }
    }
    float s3 = across_groups_sum(group16_sum(db3));
    if (lane == 0 && s3 != 0.0f) atomicAdd(&grad[OFF_B3], s3);
}

// ---------------------------------------------------------------------------
// softmax cross-entropy per view (one block per view)
// ---------------------------------------------------------------------------
__device__ inline float block_reduce(float v, float* sh, bool is_max) {
    for (int o = 32; o > 0; o >>= 1) {
        float u = __shfl_xor(v, o, 64);
        v = is_max ? fmaxf(v, u) : v + u;
    }
    int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[wv] = v;
    __syncthreads();
    float r = sh[0];
    for (int i = 1; i < nw; ++i) r = is_max ? fmaxf(r, sh[i]) : r + sh[i];
    return r;
}

__global__ void k_view_target_sum(const float* __restrict__ target, const int* __restrict__ off, float* __restrict__ tsum) {
    __shared__ float sh[4];
    int v = blockIdx.x, lo = off[v], hi = off[v + 1];
    float s = 0.0f;
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) s += target[i];
    s = block_reduce(s, sh, false);
    if (threadIdx.x == 0) tsum[v] = s;
}

__global__ void k_softmax_xent(const float* __restrict__ z, const float* __restrict__ target, const int* __restrict__ off,
                               int nv, const float* __restrict__ tsum, float* __restrict__ p, float* __restrict__ dz,
                               float* __restrict__ vloss) {
    __shared__ float sh[4];
    int v = blockIdx.x, lo = off[v], hi = off[v + 1];
    int used = 0;
    for (int u = 0; u < nv; ++u) used += (off[u + 1] > off[u] && tsum[u] > 0.0f) ? 1 : 0;
    float mx = -3.0e38f;
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) mx = fmaxf(mx, z[i]);
    mx = block_reduce(mx, sh, true);
    float se = 0.0f;
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) se += expf(z[i] - mx);
    se = block_reduce(se, sh, false);
    float lse = logf(se);
    float ts = tsum[v];
    bool on = hi > lo && ts > 0.0f;
    float l = 0.0f;
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        float pi = expf(z[i] - mx) / se;
        if (p) p[i] = pi;
        float t = on ? target[i] / ts : 0.0f;
        if (dz) dz[i] = on ? (pi - t) / (float)used : 0.0f;
        if (t > 0.0f) l -= t * (z[i] - mx - lse);
    }
    l = block_reduce(l, sh, false);
    if (threadIdx.x == 0 && vloss) vloss[v] = on ? l : 0.0f;
}

__global__ void k_zero(float* __restrict__ x, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0f;
}

int grid_for(int tiles, int cap) { return tiles < 1 ? 1 : (tiles < cap ? tiles : cap); }

// Per-view target sums of drMlpSoftmaxXentNoAlloc: one device-resident array
// per GPU, held until the process ends. In host code the name stands for a
// host-side shadow, not a device address: kernels and copies take the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float xent_scratch[DR_XENT_MAX_VIEWS];

constexpr int kMaxDevices = 64;
std::mutex xent_mu;
float* xent_ptr[kMaxDevices] = {};

// Device address of xent_scratch on the current device (looked up once per
// device, with that device current), or nullptr on failure.
float* xent_scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(xent_mu);
    if (!xent_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(xent_scratch)) != hipSuccess || !p) return nullptr;
        xent_ptr[dev] = static_cast<float*>(p);
    }
    return xent_ptr[dev];
}

}  // namespace
}  // namespace dr

using namespace dr;

extern "C" drStatus drEdgeFeatures(drScene s, const drCamera* c, float* features, hipStream_t st) {
    if (!s || !c || !features || c->width <= 0 || c->height <= 0 || !(c->near_clip > 0.0f)) return DR_ERROR_INVALID_VALUE;
    Cam cam = make_cam(*c);
    SceneView sv = s->view();
    k_edge_features<<<(s->E + 127) / 128, 128, 0, st>>>(sv, cam, features);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

extern "C" drStatus drMlpForward(const float* theta, const float* x, int32_t n, float* logits, hipStream_t st) {
    if (!theta || n < 0 || (n > 0 && (!x || !logits))) return DR_ERROR_INVALID_VALUE;
    if (n == 0) return DR_SUCCESS;
    int tiles = (n + 15) / 16;
    k_mlp_forward<<<grid_for(tiles, 4096), 64, 0, st>>>(theta, x, n, logits);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

extern "C" drStatus drMlpBackward(const float* theta, const float* x, int32_t n, const float* d_logits, float* grad,
                                  hipStream_t st) {
    if (!theta || !grad || n < 0 || (n > 0 && (!x || !d_logits))) return DR_ERROR_INVALID_VALUE;
    k_zero<<<(NPAR + 255) / 256, 256, 0, st>>>(grad, NPAR);
    if (n > 0) {
        int tiles = (n + 31) / 32;
        k_mlp_backward<<<grid_for(tiles, 1024), 64, 0, st>>>(theta, x, n, d_logits, grad);
    }
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

extern "C" drStatus drMlpSoftmaxXent(const float* logits, const float* target, const int32_t* offsets, int32_t n_views,
                                     float* prob, float* d_logits, float* view_loss, float* scratch, hipStream_t st) {
    if (!logits || !offsets || n_views < 0 || (n_views > 0 && !scratch) || ((d_logits || view_loss) && !target))
        return DR_ERROR_INVALID_VALUE;
    if (n_views == 0) return DR_SUCCESS;
    if (target) k_view_target_sum<<<n_views, 256, 0, st>>>(target, offsets, scratch);
    else k_zero<<<(n_views + 255) / 256, 256, 0, st>>>(scratch, n_views);
    k_softmax_xent<<<n_views, 256, 0, st>>>(logits, target, offsets, n_views, scratch, prob, d_logits, view_loss);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

extern "C" drStatus drMlpSoftmaxXentNoAlloc(const float* logits, const float* target, const int32_t* offsets,
                                            int32_t n_views, float* prob, float* d_logits, float* view_loss,
                                            hipStream_t st) {
    if (!logits || !offsets || n_views < 0 || n_views > DR_XENT_MAX_VIEWS || ((d_logits || view_loss) && !target))
        return DR_ERROR_INVALID_VALUE;
    if (n_views == 0) return DR_SUCCESS;
    float* scratch = xent_scratch_ptr();
    if (!scratch) return DR_ERROR_DEVICE;
    // every entry the softmax reads, [0, n_views), is written first by one of
    // these two kernels: nothing left by an earlier call is used
    if (target) k_view_target_sum<<<n_views, 256, 0, st>>>(target, offsets, scratch);
    else k_zero<<<(n_views + 255) / 256, 256, 0, st>>>(scratch, n_views);
    k_softmax_xent<<<n_views, 256, 0, st>>>(logits, target, offsets, n_views, scratch, prob, d_logits, view_loss);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}
