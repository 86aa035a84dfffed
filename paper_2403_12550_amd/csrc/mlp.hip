// Learned warm start: a PointNet-style pose regressor over a frame pair.
//
// Not part of the paper (its tracker starts each registration from the
// previous pose); this is the project's extension.  Network, per pair of
// N = 4096 rows X_r = [source point r ; target point r] (centred, scaled):
//     H1 = relu(X W1 + b1)   6 -> 64      (FP32 VALU: K = 6 is too thin for MFMA)
//     H2 = relu(H1 W2 + b2) 64 -> 128     (bf16 MFMA 16x16x32, FP32 accumulation)
//     H3 = relu(H2 W3 + b3) 128 -> 256    (bf16 MFMA 16x16x32, FP32 accumulation)
//     g  = max over rows of H3             (lowest row index among equal maxima)
//     z  = relu(g W4 + b4)  256 -> 128    (FP32)
//     y  = z W5 + b5        128 -> 6      (FP32): [rotation vector ; translation]
// Storage: X, W1..W3 and the hidden activations H1, H2 are bf16 (round to
// nearest even); everything else is FP32.
//
// The forward pass is the dense part (0.34 GFLOP per pair) and runs on the
// matrix cores.  Its backward pass is sparse: the max-pool passes gradient
// to at most 256 rows per pair, so the backward kernel recomputes those rows
// with FP32 vector arithmetic and writes one gradient vector per pair; a
// fixed-order reduction over pairs and the Adam update follow.
#include <float.h>

#include "common.hpp"
#include "launch.hpp"

namespace gicp {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRows = GICP_MLP_POINTS;   // rows per pair
constexpr int kSplits = 16;              // workgroups per pair in the forward pass
constexpr int kRowsPerSplit = kRows / kSplits;
constexpr int kTile = 64;                // rows per tile
constexpr int kH1Stride = 64 + 8;        // bf16 elements per LDS row (padding against bank conflicts)
constexpr int kH2Stride = 128 + 8;
static_assert(kRowsPerSplit % kTile == 0, "tiles must cover a split");

// Flat parameter layout (FP32): W1[6][64] b1[64] W2[64][128] b2[128]
// W3[128][256] b3[256] W4[256][128] b4[128] W5[128][6] b5[6].
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + 6 * 64;
constexpr int kOffW2 = kOffB1 + 64, kOffB2 = kOffW2 + 64 * 128;
constexpr int kOffW3 = kOffB2 + 128, kOffB3 = kOffW3 + 128 * 256;
constexpr int kOffW4 = kOffB3 + 256, kOffB4 = kOffW4 + 256 * 128;
constexpr int kOffW5 = kOffB4 + 128, kOffB5 = kOffW5 + 128 * 6;
static_assert(kOffB5 + 6 == GICP_MLP_PARAMS, "parameter layout");

// bf16 copies of W2 and W3 in MFMA fragment order: fragment (n_tile, k_step)
// holds, for lane l, W[k_step*32 + 8*(l/16) + i][n_tile*16 + l%16], i = 0..7
// (the B operand of v_mfma_f32_16x16x32_bf16), 16 bytes per lane.
constexpr int kW2Frags = 8 * 2;    // 128 columns / 16, 64 rows / 32
constexpr int kW3Frags = 16 * 4;   // 256 columns / 16, 128 rows / 32
static_assert((kW2Frags + kW3Frags) * 64 * 8 == GICP_MLP_BF16, "fragment layout");

// Cache per pair written by the forward pass for the backward pass:
// g[256], argmax row[256] (int bits), A4[128] (pre-activation of z).
constexpr int kCache = 256 + 256 + 128;
static_assert(kCache == GICP_MLP_CACHE, "cache layout");

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);   // round to nearest, ties to even (finite inputs)
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float((uint32_t)bf16_bits(x) << 16); }
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// (value, row) order of the max-pool: larger value first, then lower row.
__device__ __forceinline__ bool pool_better(float v, int r, float bv, int br) {
    return v > bv || (v == bv && r < br);
}

// ---------------------------------------------------------------------------
// parameter draw: SplitMix64 of the counter seed * 2^32 + j
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int fan_in_of(int j, bool& is_weight) {
    is_weight = true;
    if (j < kOffB1) return 6;
    if (j < kOffW2) { is_weight = false; return 1; }
    if (j < kOffB2) return 64;
    if (j < kOffW3) { is_weight = false; return 1; }
    if (j < kOffB3) return 128;
    if (j < kOffW4) { is_weight = false; return 1; }
    if (j < kOffB4) return 256;
    if (j < kOffW5) { is_weight = false; return 1; }
    if (j < kOffB5) return 128;
    is_weight = false;
    return 1;
}

__global__ void k_mlp_init(uint64_t seed, float* __restrict__ params, float* __restrict__ m, float* __restrict__ v) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= GICP_MLP_PARAMS) return;
    bool w;
    const int fan = fan_in_of(j, w);
    float p = 0.f;
    if (w) {
        const uint64_t z = splitmix64((seed << 32) + (uint64_t)j);
        const double u = (double)(z >> 11) * 0x1.0p-53;
        p = (float)(sqrt(6.0 / fan) * (2.0 * u - 1.0));
    }
    params[j] = p;
    if (m) m[j] = 0.f;
    if (v) v[j] = 0.f;
}

// bf16 fragment copies of W2 and W3 from the FP32 parameters.
__global__ void k_mlp_fragments(const float* __restrict__ params, uint16_t* __restrict__ wb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // element of the fragment array
    if (e >= GICP_MLP_BF16) return;
    const int i = e & 7, lane = (e >> 3) & 63, frag = e >> 9;
    int k, n;
    float w;
    if (frag < kW2Frags) {
        const int nt = frag / 2, ks = frag % 2;
        k = ks * 32 + 8 * (lane / 16) + i;
        n = nt * 16 + lane % 16;
        w = params[kOffW2 + k * 128 + n];
    } else {
        const int f = frag - kW2Frags, nt = f / 4, ks = f % 4;
        k = ks * 32 + 8 * (lane / 16) + i;
        n = nt * 16 + lane % 16;
        w = params[kOffW3 + k * 256 + n];
    }
    wb[e] = bf16_bits(w);
}

// ---------------------------------------------------------------------------
// input packing: rows [(s - c) * SCALE ; (t - c) * SCALE], c = FP64 mean of
// the chosen target points; one workgroup per pair
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_pack(const gicp_mlp_pair* __restrict__ pairs, uint16_t* __restrict__ X,
                                                  double* __restrict__ centres, int* __restrict__ err) {
    __shared__ double s_sum[3][256];
    const gicp_mlp_pair P = pairs[blockIdx.x];
    double sx = 0, sy = 0, sz = 0;
    bool bad = false;
    for (int r = threadIdx.x; r < kRows; r += 256) {
        int32_t t = P.tgt_idx[r];
        if (t < 0 || t >= P.n_tgt) {
            bad = true;
            t = 0;
        }
        sx += (double)P.tgt[t];
        sy += (double)P.tgt[P.n_tgt + t];
        sz += (double)P.tgt[2 * P.n_tgt + t];
    }
    s_sum[0][threadIdx.x] = sx;
    s_sum[1][threadIdx.x] = sy;
    s_sum[2][threadIdx.x] = sz;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int a = 0; a < 3; ++a) s_sum[a][threadIdx.x] += s_sum[a][threadIdx.x + h];
        __syncthreads();
    }
    const double cx = s_sum[0][0] / kRows, cy = s_sum[1][0] / kRows, cz = s_sum[2][0] / kRows;
    if (threadIdx.x == 0 && centres) {
        centres[3 * blockIdx.x] = cx;
        centres[3 * blockIdx.x + 1] = cy;
        centres[3 * blockIdx.x + 2] = cz;
    }
    uint16_t* out = X + (int64_t)blockIdx.x * kRows * 6;
    for (int r = threadIdx.x; r < kRows; r += 256) {
        int32_t s = P.src_idx[r], t = P.tgt_idx[r];
        if (s < 0 || s >= P.n_src) {
            bad = true;
            s = 0;
        }
        if (t < 0 || t >= P.n_tgt) t = 0;
        const double v[6] = {((double)P.src[s] - cx) * GICP_MLP_SCALE,
                             ((double)P.src[P.n_src + s] - cy) * GICP_MLP_SCALE,
                             ((double)P.src[2 * P.n_src + s] - cz) * GICP_MLP_SCALE,
                             ((double)P.tgt[t] - cx) * GICP_MLP_SCALE,
                             ((double)P.tgt[P.n_tgt + t] - cy) * GICP_MLP_SCALE,
                             ((double)P.tgt[2 * P.n_tgt + t] - cz) * GICP_MLP_SCALE};
#pragma unroll
        for (int c = 0; c < 6; ++c) out[r * 6 + c] = bf16_bits((float)v[c]);
    }
    if (bad) atomicOr(err, kErrIndex);
}

// ---------------------------------------------------------------------------
// forward, shared layers + partial max-pool: workgroup = (pair, split) of
// kRowsPerSplit rows in tiles of 64; wave w owns layer-2 columns
// [32w, 32w+32) and layer-3 columns [64w, 64w+64).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_shared(const uint16_t* __restrict__ X, const float* __restrict__ params,
                                                    const bf16x8* __restrict__ wfrag, float* __restrict__ pmax,
                                                    int* __restrict__ parg) {
    __shared__ float s_w1[6 * 64];
    __shared__ float s_b1[64];
    __shared__ __attribute__((aligned(16))) uint16_t s_h1[kTile * kH1Stride];
    __shared__ __attribute__((aligned(16))) uint16_t s_h2[kTile * kH2Stride];
    const int pair = blockIdx.x / kSplits, split = blockIdx.x % kSplits;
    const int tid = threadIdx.x, w = tid / 64, l = tid % 64;
    const int lr = l % 16, lq = l / 16;
    for (int j = tid; j < 6 * 64; j += 256) s_w1[j] = bf16_round(params[kOffW1 + j]);
    if (tid < 64) s_b1[tid] = params[kOffB1 + tid];
    // resident B fragments and biases of this wave's columns
    bf16x8 f2[2][2], f3[4][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) f2[j][ks] = wfrag[((2 * w + j) * 2 + ks) * 64 + l];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) f3[j][ks] = wfrag[kW2Frags * 64 + ((4 * w + j) * 4 + ks) * 64 + l];
    float bias2[2], bias3[4];
#pragma unroll
    for (int j = 0; j < 2; ++j) bias2[j] = params[kOffB2 + (2 * w + j) * 16 + lr];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias3[j] = params[kOffB3 + (4 * w + j) * 16 + lr];
    float best[4];
    int barg[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        best[j] = -FLT_MAX;
        barg[j] = 0x7FFFFFFF;
    }
    const uint16_t* Xp = X + (int64_t)pair * kRows * 6;
    for (int t = 0; t < kRowsPerSplit / kTile; ++t) {
        const int row0 = split * kRowsPerSplit + t * kTile;
        __syncthreads();   // s_w1 ready; the previous tile's layer 3 has read s_h2
        // layer 1 (VALU): thread -> row tid/4, outputs 16 * (tid%4) .. +16
        {
            const int r = tid / 4, o0 = 16 * (tid % 4);
            float x[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) x[c] = bf16_value(Xp[(row0 + r) * 6 + c]);
#pragma unroll
            for (int o = 0; o < 16; ++o) {
                float a = s_b1[o0 + o];
#pragma unroll
                for (int c = 0; c < 6; ++c) a += x[c] * s_w1[c * 64 + o0 + o];
                s_h1[r * kH1Stride + o0 + o] = bf16_bits(fmaxf(a, 0.f));
            }
        }
        __syncthreads();
        // layer 2 (MFMA): 4 row tiles x 2 column tiles x 2 k-steps
        f32x4 acc2[4][2];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc2[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&s_h1[(m * 16 + lr) * kH1Stride + ks * 32 + 8 * lq]);
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc2[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, f2[j][ks], acc2[m][j], 0, 0, 0);
            }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    s_h2[(m * 16 + 4 * lq + i) * kH2Stride + (2 * w + j) * 16 + lr] =
                        bf16_bits(fmaxf(acc2[m][j][i] + bias2[j], 0.f));
        __syncthreads();
        // layer 3 (MFMA): 4 row tiles x 4 column tiles x 4 k-steps, then the
        // running max over this lane's rows
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 acc3[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc3[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&s_h2[(m * 16 + lr) * kH2Stride + ks * 32 + 8 * lq]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc3[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, f3[j][ks], acc3[j], 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = fmaxf(acc3[j][i] + bias3[j], 0.f);
                    const int r = row0 + m * 16 + 4 * lq + i;   // increasing along (t, m, i)
                    if (v > best[j]) {
                        best[j] = v;
                        barg[j] = r;
                    }
                }
        }
    }
    // combine the four row quarters of each column (lanes lr, lr+16, lr+32, lr+48)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float ov = __shfl_xor(best[j], o);
            const int orr = __shfl_xor(barg[j], o);
            if (pool_better(ov, orr, best[j], barg[j])) {
                best[j] = ov;
                barg[j] = orr;
            }
        }
        if (lq == 0) {
            const int64_t o = ((int64_t)pair * kSplits + split) * 256 + (4 * w + j) * 16 + lr;
            pmax[o] = best[j];
            parg[o] = barg[j];
        }
    }
}

// Rodrigues' formula for R = exp([w]x) (FP64).
__device__ void rotvec_matrix(const double w[3], double R[9]) {
    const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    const double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double a, b;
    if (th < 1e-12) {
        a = 1.0;
        b = 0.5;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / (th * th);
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double kk = 0;
            for (int q = 0; q < 3; ++q) kk += K[3 * i + q] * K[3 * q + j];
            R[3 * i + j] = (i == j ? 1.0 : 0.0) + a * K[3 * i + j] + b * kk;
        }
}

// ---------------------------------------------------------------------------
// forward, head: one workgroup per pair.  Combines the split maxima, runs the
// two FP32 head layers, writes y, the backward cache and (optionally) the
// relative pose decoded in the original coordinates.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_head(const float* __restrict__ params, const float* __restrict__ pmax,
                                                  const int* __restrict__ parg, const double* __restrict__ centres,
                                                  float* __restrict__ y, float* __restrict__ cache,
                                                  double* __restrict__ poses) {
    __shared__ float s_g[256];
    __shared__ float s_z[128];
    __shared__ float s_y[6];
    const int pair = blockIdx.x, c = threadIdx.x;
    float bv = -FLT_MAX;
    int br = 0x7FFFFFFF;
    for (int s = 0; s < kSplits; ++s) {
        const int64_t o = ((int64_t)pair * kSplits + s) * 256 + c;
        const float v = pmax[o];
        const int r = parg[o];
        if (pool_better(v, r, bv, br)) {
            bv = v;
            br = r;
        }
    }
    s_g[c] = bv;
    float* ca = cache ? cache + (int64_t)pair * kCache : nullptr;
    if (ca) {
        ca[c] = bv;
        ca[256 + c] = __int_as_float(br);
    }
    __syncthreads();
    if (c < 128) {
        float a = params[kOffB4 + c];
        for (int q = 0; q < 256; ++q) a += s_g[q] * params[kOffW4 + q * 128 + c];
        if (ca) ca[512 + c] = a;
        s_z[c] = fmaxf(a, 0.f);
    }
    __syncthreads();
    if (c < 6) {
        float a = params[kOffB5 + c];
        for (int q = 0; q < 128; ++q) a += s_z[q] * params[kOffW5 + q * 6 + c];
        s_y[c] = a;
        if (y) y[pair * 6 + c] = a;
    }
    __syncthreads();
    if (c == 0 && poses && centres) {
        // pose in the centred frame is [R, t']; in the original one t = t' - (R - I) c
        const double w[3] = {s_y[0], s_y[1], s_y[2]};
        double R[9];
        rotvec_matrix(w, R);
        const double* cc = centres + 3 * pair;
        double* T = poses + 16 * pair;
        for (int i = 0; i < 3; ++i) {
            double rc = 0;
            for (int j = 0; j < 3; ++j) {
                T[4 * i + j] = R[3 * i + j];
                rc += (R[3 * i + j] - (i == j ? 1.0 : 0.0)) * cc[j];
            }
            T[4 * i + 3] = (double)s_y[3 + i] - rc;
        }
        T[12] = 0;
        T[13] = 0;
        T[14] = 0;
        T[15] = 1;
    }
}

// ---------------------------------------------------------------------------
// backward: one workgroup per pair; writes the pair's full gradient vector
// (every entry, zeros included) and its loss term.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_backward(const uint16_t* __restrict__ X, const float* __restrict__ params,
                                                      const float* __restrict__ cache, const float* __restrict__ y,
                                                      const float* __restrict__ ystar, int B,
                                                      float* __restrict__ gpair, float* __restrict__ lpair) {
    __shared__ float s_dy[6];
    __shared__ float s_z[128], s_dA4[128];
    __shared__ float s_dg[256];
    __shared__ int s_row[256], s_ch[256];   // channels sorted by argmax row
    __shared__ float s_x[6], s_a1[64], s_h1[64], s_a2[128], s_h2[128], s_dA2[128], s_dA1[64];
    __shared__ float s_dA3[256];
    __shared__ int s_nu;
    const int pair = blockIdx.x, tid = threadIdx.x;
    const float* ca = cache + (int64_t)pair * kCache;
    float* G = gpair + (int64_t)pair * GICP_MLP_PARAMS;
    // loss term and dy = (y - y*) / B
    if (tid < 6) s_dy[tid] = (y[pair * 6 + tid] - ystar[pair * 6 + tid]) / (float)B;
    if (tid == 0) {
        float e = 0;
        for (int i = 0; i < 6; ++i) {
            const float d = y[pair * 6 + i] - ystar[pair * 6 + i];
            e += d * d;
        }
        lpair[pair] = 0.5f * e / (float)B;
    }
    __syncthreads();
    // head: W5, b5, then dA4
    if (tid < 128) {
        const float a4 = ca[512 + tid];
        const float z = fmaxf(a4, 0.f);
        s_z[tid] = z;
        float d = 0;
        for (int i = 0; i < 6; ++i) {
            d += params[kOffW5 + tid * 6 + i] * s_dy[i];
            G[kOffW5 + tid * 6 + i] = z * s_dy[i];
        }
        s_dA4[tid] = a4 > 0.f ? d : 0.f;
    }
    if (tid < 6) G[kOffB5 + tid] = s_dy[tid];
    __syncthreads();
    // W4, b4 and dg
    {
        const float g = ca[tid];
        float d = 0;
        for (int j = 0; j < 128; ++j) {
            G[kOffW4 + tid * 128 + j] = g * s_dA4[j];
            d += params[kOffW4 + tid * 128 + j] * s_dA4[j];
        }
        s_dg[tid] = d;
        if (tid < 128) G[kOffB4 + tid] = s_dA4[tid];
        const int r = __float_as_int(ca[256 + tid]);
        s_row[tid] = (r >= 0 && r < kRows) ? r : 0;   // a cache not written by the forward pass stays in bounds
        s_ch[tid] = tid;
    }
    // zero the shared-layer gradients that are accumulated over rows
    for (int j = tid; j < kOffW3; j += 256) G[j] = 0.f;   // W1 b1 W2 b2
    for (int j = tid; j < 256; j += 256) G[kOffB3 + j] = 0.f;
    __syncthreads();
    // sort the 256 (row, channel) pairs by row, then channel (bitonic, in LDS)
    for (int k = 2; k <= 256; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int ixj = tid ^ j;
            if (ixj > tid) {
                const bool up = (tid & k) == 0;
                const int ra = s_row[tid], rb = s_row[ixj], ca_ = s_ch[tid], cb = s_ch[ixj];
                const bool gt = ra > rb || (ra == rb && ca_ > cb);
                if (gt == up) {
                    s_row[tid] = rb;
                    s_row[ixj] = ra;
                    s_ch[tid] = cb;
                    s_ch[ixj] = ca_;
                }
            }
            __syncthreads();
        }
    // walk the distinct rows in increasing order
    const uint16_t* Xp = X + (int64_t)pair * kRows * 6;
    int pos = 0;
    while (pos < 256) {
        const int r = s_row[pos];
        int end = pos + 1;
        while (end < 256 && s_row[end] == r) ++end;   // uniform: every thread reads the same LDS
        // recompute the row's forward values (bf16 storage as in the forward pass)
        if (tid < 6) s_x[tid] = bf16_value(Xp[r * 6 + tid]);
        __syncthreads();
        if (tid < 64) {
            float a = params[kOffB1 + tid];
            for (int c = 0; c < 6; ++c) a += s_x[c] * bf16_round(params[kOffW1 + c * 64 + tid]);
            s_a1[tid] = a;
            s_h1[tid] = bf16_round(fmaxf(a, 0.f));
        }
        __syncthreads();
        if (tid < 128) {
            float a = params[kOffB2 + tid];
            for (int c = 0; c < 64; ++c) a += s_h1[c] * bf16_round(params[kOffW2 + c * 128 + tid]);
            s_a2[tid] = a;
            s_h2[tid] = bf16_round(fmaxf(a, 0.f));
        }
        __syncthreads();
        // the row's channels: dA3 = dg * [A3 > 0]; W3 column and b3 entry
        for (int q = pos + (tid >> 7); q < end; q += 2) {
            const int ch = s_ch[q];
            const int k = tid & 127;
            // A3 of (row, ch) by a 128-lane reduction would need LDS; every
            // lane of the half computes it (128 products)
            float a = params[kOffB3 + ch];
            for (int c = 0; c < 128; ++c) a += s_h2[c] * bf16_round(params[kOffW3 + c * 256 + ch]);
            const float d = a > 0.f ? s_dg[ch] : 0.f;
            G[kOffW3 + k * 256 + ch] = s_h2[k] * d;
            if (k == 0) {
                G[kOffB3 + ch] = d;
                s_dA3[ch] = d;
            }
        }
        __syncthreads();
        // dH2 -> dA2; W2, b2
        if (tid < 128) {
            float d = 0;
            for (int q = pos; q < end; ++q) {
                const int ch = s_ch[q];
                d += bf16_round(params[kOffW3 + tid * 256 + ch]) * s_dA3[ch];
            }
            s_dA2[tid] = s_a2[tid] > 0.f ? d : 0.f;
        }
        __syncthreads();
        for (int e = tid; e < 64 * 128; e += 256) {
            const int c = e / 128, j = e % 128;
            G[kOffW2 + e] += s_h1[c] * s_dA2[j];
        }
        if (tid < 128) G[kOffB2 + tid] += s_dA2[tid];
        // dH1 -> dA1; W1, b1
        if (tid < 64) {
            float d = 0;
            for (int j = 0; j < 128; ++j) d += bf16_round(params[kOffW2 + tid * 128 + j]) * s_dA2[j];
            s_dA1[tid] = s_a1[tid] > 0.f ? d : 0.f;
        }
        __syncthreads();
        for (int e = tid; e < 6 * 64; e += 256) {
            const int c = e / 64, j = e % 64;
            G[kOffW1 + e] += s_x[c] * s_dA1[j];
        }
        if (tid < 64) G[kOffB1 + tid] += s_dA1[tid];
        __syncthreads();
        pos = end;
    }
    (void)s_nu;
}

// grad[j] = sum over pairs of gpair[pair][j], in pair order.
__global__ void k_mlp_reduce(const float* __restrict__ gpair, const float* __restrict__ lpair, int B,
                             float* __restrict__ grad, float* __restrict__ loss) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < GICP_MLP_PARAMS) {
        float s = 0;
        for (int b = 0; b < B; ++b) s += gpair[(int64_t)b * GICP_MLP_PARAMS + j];
        grad[j] = s;
    }
    if (j == 0 && loss) {
        float e = 0;
        for (int b = 0; b < B; ++b) e += lpair[b];
        *loss = e;
    }
}

// Adam (Kingma & Ba, Algorithm 1) with bias correction; FP32 state.
__global__ void k_mlp_adam(float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ grad, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= GICP_MLP_PARAMS) return;
    const float g = grad[j];
    const float mj = b1 * m[j] + (1.f - b1) * g;
    const float vj = b2 * v[j] + (1.f - b2) * g * g;
    m[j] = mj;
    v[j] = vj;
    params[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

}  // namespace

constexpr int kMlpThreads = 256;

hipError_t launch_mlp_init(uint64_t seed, float* params, float* m, float* v, uint16_t* wb, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_init, dim3((GICP_MLP_PARAMS + kMlpThreads - 1) / kMlpThreads), dim3(kMlpThreads), 0, s,
                       seed, params, m, v);
    hipLaunchKernelGGL(k_mlp_fragments, dim3((GICP_MLP_BF16 + kMlpThreads - 1) / kMlpThreads), dim3(kMlpThreads), 0,
                       s, (const float*)params, wb);
    return hipGetLastError();
}

hipError_t launch_mlp_fragments(const float* params, uint16_t* wb, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_fragments, dim3((GICP_MLP_BF16 + kMlpThreads - 1) / kMlpThreads), dim3(kMlpThreads), 0,
                       s, params, wb);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(int B, const gicp_mlp_pair* pairs, uint16_t* X, double* centres, int* err,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(B), dim3(256), 0, s, pairs, X, centres, err);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(int B, const uint16_t* X, const float* params, const uint16_t* wb, float* pmax,
                              int* parg, const double* centres, float* y, float* cache, double* poses,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_shared, dim3(B * kSplits), dim3(256), 0, s, X, params,
                       reinterpret_cast<const bf16x8*>(wb), pmax, parg);
    hipLaunchKernelGGL(k_mlp_head, dim3(B), dim3(256), 0, s, params, (const float*)pmax, (const int*)parg, centres, y,
                       cache, poses);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(int B, const uint16_t* X, const float* params, const float* cache, const float* y,
                               const float* ystar, float* gpair, float* lpair, float* grad, float* loss,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_backward, dim3(B), dim3(256), 0, s, X, params, cache, y, ystar, B, gpair, lpair);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((GICP_MLP_PARAMS + kMlpThreads - 1) / kMlpThreads), dim3(kMlpThreads), 0,
                       s, (const float*)gpair, (const float*)lpair, B, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, int t, float lr, uint16_t* wb,
                           hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - pow(0.9, t)), c2 = (float)(1.0 - pow(0.999, t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((GICP_MLP_PARAMS + kMlpThreads - 1) / kMlpThreads), dim3(kMlpThreads), 0, s,
                       params, m, v, grad, lr, b1, b2, eps, c1, c2);
    return launch_mlp_fragments(params, wb, s);
}

int mlp_splits() { return kSplits; }

}  // namespace gicp
