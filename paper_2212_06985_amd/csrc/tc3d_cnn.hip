// Learned per-edge prior for BP: a translation-invariant periodic 3D CNN, four
// 3x3x3 convolutions 8 -> 32 -> 32 -> 32 -> 3 with ReLU between them, BF16
// weights and activations, FP32 accumulation on the gfx950 matrix cores.
//
//   input   row g = s*N + v (shot s, site v), 8 BF16 channels: the measured
//           syndrome bits of faces f(v,0..2) this cycle, the working-syndrome
//           bits those faces kept at the end of the previous cycle, 2 zeros
//   layer   y[v][co] = b[co] + sum_{d, ci} W[d][ci][co] x[v + off(d)][ci],
//           off(d) = (d%3 - 1, d/3%3 - 1, d/9 - 1), coordinates mod L
//   output  z[v][c] = logit of an error on edge e(v,c); the BP prior
//           llr0 = -z is written straight into BP's [W][3N][64] layout
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16: a
// wavefront computes 16 rows x 16 output channels per instruction; its A
// operand is the 16-byte channel chunk of one neighbour row (for 32 input
// channels one offset per K step, for 8 input channels four offsets per K
// step), its B operand a 16-byte column chunk of the packed weights held in
// LDS. The backward pass uses the same kernel with the taps reversed and the
// weights transposed (dX[u] = sum_d W[d]^T dY[u - off(d)]), and a separate
// weight-gradient kernel (a GEMM over rows, staged transposed in LDS).
#include <math.h>

#include "tc3d_device.hpp"
#include "tc3d_internal.hpp"

namespace tc3d {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kCh[5] = {8, 32, 32, 32, 3};
constexpr int kConvWaves = 8;
constexpr int kConvBlock = 64 * kConvWaves;

// ------------------------------------------------------ parameter layout
// FP32 parameter vector: for each layer W [27][cin][cout] then b [cout].
__host__ __device__ constexpr int64_t param_offset(int layer) {
    int64_t o = 0;
    for (int l = 0; l < layer; ++l) o += 27 * kCh[l] * kCh[l + 1] + kCh[l + 1];
    return o;
}
constexpr int64_t kParams = param_offset(4);

// Packed BF16 weight blocks, each [KS][NT][16][32]: a K step t, an output
// tile nt, output column n, K index k. Forward blocks for layers 1-4, then
// backward-data blocks for layers 4, 3, 2 (taps reversed, weights
// transposed: input channels = that layer's outputs, outputs = its inputs).
struct Block {
    int layer;   // 0..3
    int bwd;     // 0 forward, 1 backward-data
    int cin_k;   // channels of the conv input as the kernel sees it (8 or 32)
    int cin;     // real input channels of this conv
    int cout;    // real output channels of this conv
    int ks, nt;  // K steps, output tiles of 16
};

__host__ __device__ constexpr Block block_of(int i) {
    // i: 0..3 forward layer i; 4..6 backward of layer 3, 2, 1 (0-based)
    if (i < 4) {
        const int cin = kCh[i], cout = kCh[i + 1];
        const int cin_k = cin == 8 ? 8 : 32;
        return Block{i, 0, cin_k, cin, cout, cin_k == 32 ? 27 : 7, (cout + 15) / 16};
    }
    const int layer = 7 - i;  // 3, 2, 1
    const int cin = kCh[layer + 1], cout = kCh[layer];
    const int cin_k = cin <= 8 ? 8 : 32;
    return Block{layer, 1, cin_k, cin, cout, cin_k == 32 ? 27 : 7, (cout + 15) / 16};
}

__host__ __device__ constexpr int64_t block_elems(int i) {
    return (int64_t)block_of(i).ks * block_of(i).nt * 16 * 32;
}
__host__ __device__ constexpr int64_t block_offset(int i) {
    int64_t o = 0;
    for (int j = 0; j < i; ++j) o += block_elems(j);
    return o;
}
constexpr int kBlocks = 7;
constexpr int64_t kPackedElems = block_offset(kBlocks);
// biases follow the BF16 blocks as FP32 [4][32] (zero beyond cout)
constexpr int64_t kBiasOffsetBytes = ((kPackedElems * 2 + 255) / 256) * 256;
constexpr int64_t kPackedBytes = kBiasOffsetBytes + 4 * 32 * 4;

__device__ __forceinline__ int off_x(int d) { return d % 3 - 1; }
__device__ __forceinline__ int off_y(int d) { return (d / 3) % 3 - 1; }
__device__ __forceinline__ int off_z(int d) { return d / 9 - 1; }

__device__ __forceinline__ int wrap(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

// ----------------------------------------------------------- packing
__global__ void k_pack(const float* __restrict__ params, bf16* __restrict__ packed,
                       float* __restrict__ bias) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4 * 32) {
        const int l = (int)(i / 32), c = (int)(i % 32);
        bias[i] = c < kCh[l + 1] ? params[param_offset(l) + 27 * kCh[l] * kCh[l + 1] + c] : 0.f;
    }
    if (i >= kPackedElems) return;
    int b = 0;
    while (b + 1 < kBlocks && i >= block_offset(b + 1)) ++b;
    const Block B = block_of(b);
    int64_t r = i - block_offset(b);
    const int k = (int)(r % 32);
    r /= 32;
    const int n = (int)(r % 16);
    r /= 16;
    const int nt = (int)(r % B.nt);
    const int t = (int)(r / B.nt);
    const int d = B.cin_k == 32 ? t : 4 * t + k / 8;
    const int c = B.cin_k == 32 ? k : k % 8;  // input channel of this conv
    const int o = 16 * nt + n;                // output channel of this conv
    float v = 0.f;
    if (d < 27 && c < B.cin && o < B.cout) {
        const int lin = kCh[B.layer], lout = kCh[B.layer + 1];
        const float* W = params + param_offset(B.layer);
        if (!B.bwd)  // W[d][c][o]
            v = W[((int64_t)d * lin + c) * lout + o];
        else  // reversed tap, transposed: input channel c is the layer's output
            v = W[((int64_t)(26 - d) * lin + o) * lout + c];
    }
    packed[i] = (bf16)v;
}

// ---------------------------------------------------------- input rows
// x0[g][8] from the bit planes of this cycle's syndrome and the previous
// cycle's final working syndrome (nullptr: zeros).
__global__ void k_cnn_input(const uint64_t* __restrict__ syn, const uint64_t* __restrict__ prev,
                            int64_t ld, int N, int64_t R, bf16* __restrict__ x0) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= R) return;
    const int64_t s = g / N;
    const int v = (int)(g - s * N);
    const int64_t w = s >> 6;
    const int bit = (int)(s & 63);
    bf16x8 o;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        o[n] = (bf16)(float)((syn[((int64_t)n * N + v) * ld + w] >> bit) & 1u);
        o[3 + n] = prev ? (bf16)(float)((prev[((int64_t)n * N + v) * ld + w] >> bit) & 1u)
                        : (bf16)0.f;
    }
    o[6] = (bf16)0.f;
    o[7] = (bf16)0.f;
    *reinterpret_cast<bf16x8*>(x0 + g * 8) = o;
}

// ------------------------------------------------------------ conv (MFMA)
enum { EPI_RELU = 0, EPI_LLR = 1, EPI_MASK = 2 };

// x [R][CIN] BF16 (CIN = 8 or 32); packed block [KS][NT][16][32].
//  EPI_RELU: y = relu(acc + bias) as BF16 [R][NT*16]
//  EPI_LLR : llr[(s/64)*3N + c*N + v][s%64] = -(acc + bias) for c < 3
//  EPI_MASK: y = acc where mask_act > 0 else 0, BF16 [R][NT*16]
// Every variant reads x[v + off(d)]; the backward-data blocks carry the
// reversed taps in their packing.
template <int CIN, int NT, int EPI>
__global__ __launch_bounds__(kConvBlock) void k_conv(
    const bf16* __restrict__ x, const bf16* __restrict__ wp, const float* __restrict__ bias,
    const bf16* __restrict__ mask_act, bf16* __restrict__ y, float* __restrict__ llr, int L,
    int N, uint32_t R, uint32_t n_tiles) {
    constexpr int KS = CIN == 32 ? 27 : 7;
    constexpr int WELEMS = KS * NT * 16 * 32;
    __shared__ __attribute__((aligned(16))) bf16 wl[WELEMS];
    for (int i = threadIdx.x * 8; i < WELEMS; i += kConvBlock * 8)
        *reinterpret_cast<bf16x8*>(wl + i) = *reinterpret_cast<const bf16x8*>(wp + i);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int r16 = lane & 15, q = lane >> 4;
    const int LL = L * L;
    for (uint32_t tile = blockIdx.x * kConvWaves + wave; tile < n_tiles;
         tile += gridDim.x * kConvWaves) {
        // A row of this lane
        const uint32_t g = tile * 16 + r16;
        const uint32_t gc = g < R ? g : R - 1;
        const uint32_t s = gc / (uint32_t)N;
        const int v = (int)(gc - s * (uint32_t)N);
        const int vx = v % L, vy = (v / L) % L, vz = v / LL;
        const bf16* xs = x + (int64_t)s * N * CIN;
        f32x4 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            const int d = CIN == 32 ? t : 4 * t + q;
            bf16x8 a;
            if (d < 27) {
                const int ux = wrap(vx + off_x(d), L), uy = wrap(vy + off_y(d), L),
                          uz = wrap(vz + off_z(d), L);
                const int u = ux + L * (uy + L * uz);
                a = *reinterpret_cast<const bf16x8*>(xs + (int64_t)u * CIN + (CIN == 32 ? 8 * q : 0));
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) a[j] = (bf16)0.f;
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const bf16x8 b =
                    *reinterpret_cast<const bf16x8*>(wl + ((t * NT + nt) * 16 + r16) * 32 + 8 * q);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nt], 0, 0, 0);
            }
        }
        // lane holds D[row 4q + i][column r16 + 16 nt]
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int col = 16 * nt + r16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t row = tile * 16 + 4 * q + i;
                if (row >= R) continue;
                float val = acc[nt][i];
                if constexpr (EPI == EPI_RELU) {
                    val = fmaxf(val + bias[col], 0.f);
                    y[(int64_t)row * (NT * 16) + col] = (bf16)val;
                } else if constexpr (EPI == EPI_MASK) {
                    const float m = (float)mask_act[(int64_t)row * (NT * 16) + col];
                    y[(int64_t)row * (NT * 16) + col] = m > 0.f ? (bf16)val : (bf16)0.f;
                } else {
                    if (col < 3) {
                        const uint32_t rs = row / (uint32_t)N;
                        const int rv = (int)(row - rs * (uint32_t)N);
                        const int64_t e = (int64_t)col * N + rv;
                        llr[((int64_t)(rs >> 6) * 3 * N + e) * 64 + (rs & 63)] = -(val + bias[col]);
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------ loss and dz
// Binary cross-entropy with logits z = -llr against the error bits of the
// target plane; dy[g][c] = (sigmoid(z) - t) / count for c < 3, 0 for 3..7.
// Per-block partial sums of the mean loss (fixed order) go to
// loss_part[blockIdx].
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ llr,
                                             const uint64_t* __restrict__ target, int64_t ld,
                                             int N, uint32_t R, float inv_count,
                                             bf16* __restrict__ dy, float* __restrict__ loss_part) {
    __shared__ float red[256];
    const uint32_t g = blockIdx.x * 256 + threadIdx.x;
    float acc = 0.f;
    if (g < R) {
        const uint32_t s = g / (uint32_t)N;
        const int v = (int)(g - s * (uint32_t)N);
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = (bf16)0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t e = (int64_t)c * N + v;
            const float z = -llr[((int64_t)(s >> 6) * 3 * N + e) * 64 + (s & 63)];
            const float t = (float)((target[e * ld + (s >> 6)] >> (s & 63)) & 1u);
            const float sp = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));
            acc += sp - t * z;
            o[c] = (bf16)((1.f / (1.f + expf(-z)) - t) * inv_count);
        }
        *reinterpret_cast<bf16x8*>(dy + (int64_t)g * 8) = o;
    }
    red[threadIdx.x] = acc * inv_count;  // partial of the mean
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// -------------------------------------------------- weight gradient
// dW[d][ci][co] = sum_g x[g + off(d)][ci] dy[g][co]; db[co] = sum_g dy[g][co].
// A workgroup walks chunks of 256 rows; for each chunk it stages dy^T and,
// per offset, x^T of the neighbour rows in LDS, then MFMA tiles (ci x co of
// 16 x 16) accumulate over the chunk's rows. Work items (tile, offset) are
// dealt round-robin to the 4 wavefronts. Partials per workgroup are written
// to part[block][27][CI][CO] and part_b[block][CO] and summed in a fixed
// order by k_reduce.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(const bf16* __restrict__ x,
                                               const bf16* __restrict__ dy, int L, int N,
                                               uint32_t R, uint32_t n_chunks,
                                               float* __restrict__ part,
                                               float* __restrict__ part_b) {
    constexpr int CIP = CIN < 16 ? 16 : CIN;   // padded M
    constexpr int COP = COUT < 16 ? 16 : 32;   // padded N
    constexpr int DYC = COUT <= 8 ? 8 : 32;    // stored channels of dy rows
    constexpr int MT = CIP / 16, NT = COP / 16, TILES = MT * NT;
    constexpr int ITEMS = 27 * TILES;
    constexpr int PER_WAVE = (ITEMS + 3) / 4;
    constexpr int STR = 256 + 8;  // LDS row stride (bf16), padded
    __shared__ __attribute__((aligned(16))) bf16 dyT[COP][STR];
    __shared__ __attribute__((aligned(16))) bf16 xT[CIP][STR];
    __shared__ float bred[256][COP > 16 ? 32 : 16];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r16 = lane & 15, q = lane >> 4;
    const int LL = L * L;
    f32x4 acc[PER_WAVE];
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[COP];
#pragma unroll
    for (int c = 0; c < COP; ++c) bsum[c] = 0.f;
    // zero the padding rows of the transposed tiles once
    for (int c = CIN; c < CIP; ++c) xT[c][tid] = (bf16)0.f;
    for (int c = COUT; c < COP; ++c) dyT[c][tid] = (bf16)0.f;
    for (uint32_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        const uint32_t g = chunk * 256 + tid;
        const bool ok = g < R;
        uint32_t s = 0;
        int vx = 0, vy = 0, vz = 0;
        if (ok) {
            s = g / (uint32_t)N;
            const int v = (int)(g - s * (uint32_t)N);
            vx = v % L;
            vy = (v / L) % L;
            vz = v / LL;
        }
        __syncthreads();
        // dy^T
#pragma unroll
        for (int c = 0; c < COUT; ++c) {
            const float val = ok ? (float)dy[(int64_t)g * DYC + c] : 0.f;
            dyT[c][tid] = (bf16)val;
            bsum[c] += val;
        }
        for (int d = 0; d < 27; ++d) {
            // x^T of the neighbour rows at offset d
            if (ok) {
                const int ux = wrap(vx + off_x(d), L), uy = wrap(vy + off_y(d), L),
                          uz = wrap(vz + off_z(d), L);
                const int64_t row = (int64_t)s * N + ux + L * (uy + L * uz);
#pragma unroll
                for (int c8 = 0; c8 < CIN; c8 += 8) {
                    const bf16x8 v8 = *reinterpret_cast<const bf16x8*>(x + row * CIN + c8);
#pragma unroll
                    for (int j = 0; j < 8; ++j) xT[c8 + j][tid] = v8[j];
                }
            } else {
#pragma unroll
                for (int c = 0; c < CIN; ++c) xT[c][tid] = (bf16)0.f;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < PER_WAVE; ++j) {
                const int item = wave + 4 * j;
                if (item >= ITEMS || item / TILES != d) continue;
                const int tile = item % TILES;
                const int mt = tile / NT, nt = tile % NT;
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) {
                    const bf16x8 a =
                        *reinterpret_cast<const bf16x8*>(&xT[16 * mt + r16][32 * ks + 8 * q]);
                    const bf16x8 b =
                        *reinterpret_cast<const bf16x8*>(&dyT[16 * nt + r16][32 * ks + 8 * q]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
                }
            }
            __syncthreads();
        }
    }
    // partial weight gradient of this workgroup: lane holds D[ci 4q+i][co r16]
    float* pb = part + (int64_t)blockIdx.x * 27 * CIN * COUT;
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j) {
        const int item = wave + 4 * j;
        if (item >= ITEMS) continue;
        const int d = item / TILES, tile = item % TILES;
        const int mt = tile / NT, nt = tile % NT;
        const int co = 16 * nt + r16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ci = 16 * mt + 4 * q + i;
            if (ci < CIN && co < COUT) pb[((int64_t)d * CIN + ci) * COUT + co] = acc[j][i];
        }
    }
    // bias partial: sum of the per-thread sums in a fixed order
#pragma unroll
    for (int c = 0; c < COP; ++c) bred[tid][c] = bsum[c];
    __syncthreads();
    if (tid < COUT) {
        float sum = 0.f;
        for (int t = 0; t < 256; ++t) sum += bred[t][tid];
        part_b[(int64_t)blockIdx.x * COUT + tid] = sum;
    }
}

// out[i] = sum over blocks b of part[b][i], in block order.
__global__ void k_reduce(const float* __restrict__ part, int64_t n, int nblocks,
                         float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * n + i];
    out[i] = s;
}

// Adam on the FP32 parameters (bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float c1,
                       float c2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_copy_words(uint64_t* __restrict__ dst, int64_t ld_d,
                             const uint64_t* __restrict__ src, int64_t ld_s, int64_t rows,
                             int64_t nw) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * nw) return;
    const int64_t r = idx / nw, w = idx - r * nw;
    dst[r * ld_d + w] = src[r * ld_s + w];
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workspace of a CNN pass over R rows.
struct CnnWs {
    bf16* x0;    // [R][8]
    bf16* a[3];  // post-ReLU activations of layers 1-3, [R][32] each
    bf16* dy8;   // [R][8]: d loss / d logits (training)
    bf16* dyb[2];  // [R][32] ping-pong gradients (training)
    float* part;   // weight-gradient partials (training)
    float* part_b;
    float* loss_part;
};

constexpr int kWgradBlocks = 512;

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

size_t cnn_ws_bytes(int64_t R, int training) {
    size_t b = align_up((size_t)R * 8 * 2) + 3 * align_up((size_t)R * 32 * 2);
    if (training) {
        b += align_up((size_t)R * 8 * 2) + 2 * align_up((size_t)R * 32 * 2);
        b += align_up((size_t)kWgradBlocks * 27 * 32 * 32 * 4);
        b += align_up((size_t)kWgradBlocks * 32 * 4);
        b += align_up((size_t)cdiv(R, 256) * 4);
    }
    return b;
}

CnnWs carve(void* ws, int64_t R, int training) {
    CnnWs w{};
    char* p = (char*)ws;
    w.x0 = (bf16*)p;
    p += align_up((size_t)R * 8 * 2);
    for (int i = 0; i < 3; ++i) {
        w.a[i] = (bf16*)p;
        p += align_up((size_t)R * 32 * 2);
    }
    if (training) {
        w.dy8 = (bf16*)p;
        p += align_up((size_t)R * 8 * 2);
        for (int i = 0; i < 2; ++i) {
            w.dyb[i] = (bf16*)p;
            p += align_up((size_t)R * 32 * 2);
        }
        w.part = (float*)p;
        p += align_up((size_t)kWgradBlocks * 27 * 32 * 32 * 4);
        w.part_b = (float*)p;
        p += align_up((size_t)kWgradBlocks * 32 * 4);
        w.loss_part = (float*)p;
    }
    return w;
}

int conv_grid(int64_t tiles) {
    const int64_t g = cdiv(tiles, kConvWaves);
    return (int)(g < 2048 ? g : 2048);
}

template <int CIN, int NT, int EPI>
int launch_conv(const Ctx& c, const bf16* x, const bf16* wp, const float* bias,
                const bf16* mask_act, bf16* y, float* llr, Geo g, int64_t R) {
    const int64_t tiles = cdiv(R, 16);
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_conv<CIN, NT, EPI><<<dim3(conv_grid(tiles)), dim3(kConvBlock), 0, c.stream>>>(
        x, wp, bias, mask_act, y, llr, g.L, g.N, (uint32_t)R, (uint32_t)tiles);
    return after_launch(c);
}

const bf16* blk(const void* packed, int i) { return (const bf16*)packed + block_offset(i); }
const float* bias_of(const void* packed, int layer) {
    return (const float*)((const char*)packed + kBiasOffsetBytes) + 32 * layer;
}

// Forward pass: x0 from the syndromes, then the four layers; writes llr.
int cnn_forward_impl(const Ctx& c, Geo g, const uint64_t* syn, const uint64_t* prev, int64_t ld,
                     int64_t R, const void* packed, float* llr, const CnnWs& w) {
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_cnn_input<<<dim3((unsigned)cdiv(R, 256)), dim3(256), 0, c.stream>>>(syn, prev, ld, g.N, R,
                                                                           w.x0);
    if ((rc = after_launch(c))) return rc;
    if ((rc = launch_conv<8, 2, EPI_RELU>(c, w.x0, blk(packed, 0), bias_of(packed, 0), nullptr,
                                          w.a[0], nullptr, g, R)))
        return rc;
    if ((rc = launch_conv<32, 2, EPI_RELU>(c, w.a[0], blk(packed, 1), bias_of(packed, 1), nullptr,
                                           w.a[1], nullptr, g, R)))
        return rc;
    if ((rc = launch_conv<32, 2, EPI_RELU>(c, w.a[1], blk(packed, 2), bias_of(packed, 2), nullptr,
                                           w.a[2], nullptr, g, R)))
        return rc;
    return launch_conv<32, 1, EPI_LLR>(c, w.a[2], blk(packed, 3), bias_of(packed, 3), nullptr,
                                       nullptr, llr, g, R);
}

template <int CIN, int COUT>
int launch_wgrad(const Ctx& c, const bf16* x, const bf16* dy, Geo g, int64_t R, const CnnWs& w,
                 float* grad_layer) {
    const int64_t chunks = cdiv(R, 256);
    const int nb = (int)(chunks < kWgradBlocks ? chunks : kWgradBlocks);
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_wgrad<CIN, COUT><<<dim3(nb), dim3(256), 0, c.stream>>>(x, dy, g.L, g.N, (uint32_t)R,
                                                            (uint32_t)chunks, w.part, w.part_b);
    if ((rc = after_launch(c))) return rc;
    const int64_t nw = 27 * CIN * COUT;
    if ((rc = before_launch(c, TC3D_K_CNN))) return rc;
    k_reduce<<<dim3((unsigned)cdiv(nw, 256)), dim3(256), 0, c.stream>>>(w.part, nw, nb,
                                                                         grad_layer);
    if ((rc = after_launch(c))) return rc;
    if ((rc = before_launch(c, TC3D_K_CNN))) return rc;
    k_reduce<<<dim3(1), dim3(64), 0, c.stream>>>(w.part_b, COUT, nb, grad_layer + nw);
    return after_launch(c);
}

}  // namespace

// ------------------------------------------------------------ entry points
int64_t cnn_param_count() { return kParams; }
size_t cnn_packed_bytes() { return (size_t)kPackedBytes; }
size_t cnn_workspace_bytes(int64_t R, int training) { return cnn_ws_bytes(R, training); }

int cnn_pack(const Ctx& c, const float* params, void* packed) {
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_pack<<<dim3((unsigned)cdiv(kPackedElems, 256)), dim3(256), 0, c.stream>>>(
        params, (bf16*)packed, (float*)((char*)packed + kBiasOffsetBytes));
    return after_launch(c);
}

int cnn_forward(const Ctx& c, Geo g, const uint64_t* syn, const uint64_t* prev, int64_t ld,
                int64_t R, const void* packed, float* llr, void* ws) {
    const CnnWs w = carve(ws, R, 0);
    return cnn_forward_impl(c, g, syn, prev, ld, R, packed, llr, w);
}

int cnn_loss_grad(const Ctx& c, Geo g, const uint64_t* syn, const uint64_t* prev,
                  const uint64_t* target, int64_t ld, int64_t R, const void* packed, float* llr,
                  float* grad, float* loss, void* ws) {
    const CnnWs w = carve(ws, R, 1);
    int rc = cnn_forward_impl(c, g, syn, prev, ld, R, packed, llr, w);
    if (rc) return rc;
    const float inv_count = (float)(1.0 / ((double)R * 3.0));
    const int64_t lb = cdiv(R, 256);
    if ((rc = before_launch(c, TC3D_K_CNN))) return rc;
    k_bce<<<dim3((unsigned)lb), dim3(256), 0, c.stream>>>(llr, target, ld, g.N, (uint32_t)R,
                                                          inv_count, w.dy8, w.loss_part);
    if ((rc = after_launch(c))) return rc;
    if ((rc = before_launch(c, TC3D_K_CNN))) return rc;
    k_reduce<<<dim3(1), dim3(64), 0, c.stream>>>(w.loss_part, 1, (int)lb, loss);
    if ((rc = after_launch(c))) return rc;
    // layer 4 (32 -> 3): weight gradient, then dy of layer 3 through its ReLU
    if ((rc = launch_wgrad<32, 3>(c, w.a[2], w.dy8, g, R, w, grad + param_offset(3)))) return rc;
    if ((rc = launch_conv<8, 2, EPI_MASK>(c, w.dy8, blk(packed, 4), nullptr, w.a[2], w.dyb[0],
                                          nullptr, g, R)))
        return rc;
    // layer 3 (32 -> 32)
    if ((rc = launch_wgrad<32, 32>(c, w.a[1], w.dyb[0], g, R, w, grad + param_offset(2))))
        return rc;
    if ((rc = launch_conv<32, 2, EPI_MASK>(c, w.dyb[0], blk(packed, 5), nullptr, w.a[1],
                                           w.dyb[1], nullptr, g, R)))
        return rc;
    // layer 2 (32 -> 32)
    if ((rc = launch_wgrad<32, 32>(c, w.a[0], w.dyb[1], g, R, w, grad + param_offset(1))))
        return rc;
    if ((rc = launch_conv<32, 2, EPI_MASK>(c, w.dyb[1], blk(packed, 6), nullptr, w.a[0],
                                           w.dyb[0], nullptr, g, R)))
        return rc;
    // layer 1 (8 -> 32): weight gradient only
    return launch_wgrad<8, 32>(c, w.x0, w.dyb[0], g, R, w, grad + param_offset(0));
}

int cnn_adam(const Ctx& c, float* params, const float* grad, float* m, float* v, int step,
             float lr, float b1, float b2, float eps, void* packed) {
    const double c1 = 1.0 - pow((double)b1, step), c2 = 1.0 - pow((double)b2, step);
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_adam<<<dim3((unsigned)cdiv(kParams, 256)), dim3(256), 0, c.stream>>>(
        params, grad, m, v, kParams, lr, b1, b2, (float)c1, (float)c2, eps);
    if ((rc = after_launch(c))) return rc;
    return cnn_pack(c, params, packed);
}

int copy_plane(const Ctx& c, Plane dst, CPlane src, int64_t rows, int64_t nw) {
    if (nw == 0 || rows == 0) return TC3D_OK;
    int rc = before_launch(c, TC3D_K_APPLY);
    if (rc) return rc;
    k_copy_words<<<dim3((unsigned)cdiv(rows * nw, 256)), dim3(256), 0, c.stream>>>(
        dst.p, dst.ld, src.p, src.ld, rows, nw);
    return after_launch(c);
}

}  // namespace tc3d
