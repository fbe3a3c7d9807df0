// Learned per-edge prior for BP: a translation-invariant periodic 3D CNN, four
// 3x3x3 convolutions 8 -> 32 -> 32 -> 32 -> 3 with ReLU between them, BF16
// weights and activations, FP32 accumulation on the gfx950 matrix cores.
//
//   rows    g = (w N + v) 64 + l for shot s = 64 w + l at site v: the 64
//           shots of a bit-plane word are adjacent, as in BP's message layout
//   input   8 BF16 channels per row: the measured syndrome bits of faces
//           f(v,0..2) this cycle, the working-syndrome bits those faces kept
//           at the end of the previous cycle, 2 zeros
//   layer   y[v][co] = b[co] + sum_{d, ci} W[d][ci][co] x[v + off(d)][ci],
//           off(d) = (d%3 - 1, d/3%3 - 1, d/9 - 1), coordinates mod L
//   output  z[v][c] = logit of an error on edge e(v,c); the BP prior
//           llr0 = -z is written straight into BP's [W][3N][64] layout
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16 with the
// weights as the A operand (16 output channels x 32 input channels of one
// tap, or of the three x-taps of one (dy, dz) column for 8 input channels),
// read from LDS in lane order, and the activations of 16 shots at one site as
// the B operand: each B fragment is one contiguous 16-row slab. A wavefront
// reuses every slab it loads from registers for all the output sites of its
// tile the slab neighbours:
//   k_convz (the forward 32-channel layers) walks a column of NX x BY sites
//   along z; each input plane is loaded once and feeds the three output
//   planes around it, whose accumulators stay in registers: 7 slab loads per
//   output site for the 32 -> 32 layers instead of 27;
//   k_conv (the 8 -> 32 layer and the backward pass) owns NX x BY sites of
//   one plane and loads the NX + 2 slabs of each of its 3 (BY + 2)
//   neighbouring pencil columns once.
// The backward pass uses k_conv with the taps reversed and the weights
// transposed (dX[u] = sum_d W[d]^T dY[u - off(d)]), and a separate
// weight-gradient kernel (a GEMM over rows, staged transposed in LDS).
#include <math.h>

#include <atomic>

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

// Packed BF16 weight blocks, each [KS][NT][64][8]: K step t, output tile nt,
// then one MFMA A fragment in lane order (lane = 16 q + n holds output
// channel 16 nt + n, K indices 8 q .. 8 q + 7). With 32 input channels K step
// t is tap t and k the input channel; with 8 input channels K step t is the
// (dy, dz) column t (taps 3t, 3t+1, 3t+2, i.e. dx = -1, 0, 1) and k = 8 dx' +
// c, dx' = k / 8 = 3 being zero padding. Forward blocks for layers 1-4, then
// backward-data blocks for layers 4, 3, 2 (taps reversed, weights transposed:
// input channels = that layer's outputs, outputs = its inputs).
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
        return Block{i, 0, cin_k, cin, cout, cin_k == 32 ? 27 : 9, (cout + 15) / 16};
    }
    const int layer = 7 - i;  // 3, 2, 1
    const int cin = kCh[layer + 1], cout = kCh[layer];
    const int cin_k = cin <= 8 ? 8 : 32;
    return Block{layer, 1, cin_k, cin, cout, cin_k == 32 ? 27 : 9, (cout + 15) / 16};
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


__device__ __forceinline__ int wrap(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

// ----------------------------------------------------------- packing
// The last layer is packed blended with the channel prior l0 at strength
// beta: its weights scale by beta and its biases become beta b - (1 - beta)
// l0, so that the prior -z of the packed network is l0 + beta (llr - l0).
__global__ void k_pack(const float* __restrict__ params, float beta, float l0,
                       bf16* __restrict__ packed, float* __restrict__ bias) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4 * 32) {
        const int l = (int)(i / 32), c = (int)(i % 32);
        const float b =
            c < kCh[l + 1] ? params[param_offset(l) + 27 * kCh[l] * kCh[l + 1] + c] : 0.f;
        bias[i] = l == 3 && c < kCh[l + 1] ? beta * b - (1.0f - beta) * l0 : b;
    }
    if (i >= kPackedElems) return;
    int b = 0;
    while (b + 1 < kBlocks && i >= block_offset(b + 1)) ++b;
    const Block B = block_of(b);
    int64_t r = i - block_offset(b);
    const int j = (int)(r % 8);
    r /= 8;
    const int lane = (int)(r % 64);
    r /= 64;
    const int n = lane % 16, k = 8 * (lane / 16) + j;
    const int nt = (int)(r % B.nt);
    const int t = (int)(r / B.nt);
    const int d = B.cin_k == 32 ? t : (k / 8 < 3 ? 3 * t + k / 8 : 27);
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
    if (B.layer == 3) v *= beta;
    packed[i] = (bf16)v;
}

// ---------------------------------------------------------- input rows
// x0[g][8] for the rows of shot groups sg0 .. sg0 + n_sg - 1 (row g = (w N +
// v) 64 + l, shot 64 w + l) from the bit planes of this cycle's syndrome and
// the previous cycle's final working syndrome (nullptr: zeros).
__global__ void k_cnn_input(const uint64_t* __restrict__ syn, const uint64_t* __restrict__ prev,
                            int64_t ld, int N, int64_t sg0, int64_t n_sg, bf16* __restrict__ x0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_sg * 16 * N) return;
    const int64_t sgl = t / (16 * (int64_t)N);
    const int64_t rem = t - sgl * 16 * N;
    const int v = (int)(rem >> 4);
    const int64_t sg = sg0 + sgl;
    const int64_t w = sg >> 2;
    const int bit = (int)((sg & 3) * 16 + (rem & 15));
    const int64_t g = (w * N + v) * 64 + bit;
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

int launch_input(const Ctx& c, Geo g, const uint64_t* syn, const uint64_t* prev, int64_t ld,
                 int64_t sg0, int64_t n_sg, bf16* x0) {
    const int64_t n = n_sg * 16 * (int64_t)g.N;
    if (n == 0) return TC3D_OK;
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_cnn_input<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream>>>(syn, prev, ld, g.N,
                                                                               sg0, n_sg, x0);
    return after_launch(c);
}

// ------------------------------------------------------------ conv (MFMA)
enum { EPI_RELU = 0, EPI_LLR = 1, EPI_MASK = 2 };

// Work item of a k_conv wavefront: 16 shots (group sg, shots 16 sg .. 16 sg +
// 15), the BY pencils y0 .. y0 + BY - 1 at one z and the run of NX sites
// x0 .. x0 + NX - 1 along x (both clipped at L). Items are numbered with the
// x-run fastest, then the y-group, z and the shot group, so that consecutive
// items share most of their neighbour slabs.
struct ConvItems {
    int L, N, nxr;       // lattice, sites, x-runs per pencil
    uint32_t n_items;    // n_sg L ceil(L / BY) nxr, for shot groups sg0 .. sg0 + n_sg - 1
    uint32_t sg0;
};


// x rows [R][CIN] BF16 (CIN = 8 or 32); packed block [KS][2][64][8]. Used for
// the 8 -> 32 forward layer and the backward-data convolutions.
//  EPI_RELU: y = relu(acc + bias) as BF16 [R][32]
//  EPI_MASK: y = acc where mask_act > 0 else 0, BF16 [R][32]
// Every variant reads x[v + off(d)]; the backward-data blocks carry the
// reversed taps in their packing.
template <int CIN, int EPI, int NX, int BY>
__global__ __launch_bounds__(kConvBlock) void k_conv(
    const bf16* __restrict__ x, const bf16* __restrict__ wp, const float* __restrict__ bias,
    const bf16* __restrict__ mask_act, bf16* __restrict__ y, ConvItems it) {
    static_assert(EPI == EPI_RELU || EPI == EPI_MASK, "the 32 -> 3 layer runs in k_convz");
    constexpr int NT = 2;
    constexpr int KS = CIN == 32 ? 27 : 9;
    constexpr int WELEMS = KS * NT * 64 * 8;
    constexpr int NB = CIN == 32 ? NX + 2 : NX;  // B fragments per pencil column
    constexpr int NC = 3 * (BY + 2);             // pencil columns (dz, dy') per item
    __shared__ __attribute__((aligned(16))) bf16 wl[WELEMS];
    for (int i = threadIdx.x * 8; i < WELEMS; i += kConvBlock * 8)
        *reinterpret_cast<bf16x8*>(wl + i) = *reinterpret_cast<const bf16x8*>(wp + i);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int r16 = lane & 15, q = lane >> 4;
    const int L = it.L, N = it.N;
    const int ny = (L + BY - 1) / BY;
    // per-lane channel block of the A/B fragments and output channels
    float bv[NT][4];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            bv[mt][i] = (EPI == EPI_MASK) ? 0.f : bias[16 * mt + 4 * q + i];
    const int64_t G = gridDim.x;
    const int64_t lb = xcd_block(blockIdx.x, G);
    for (int64_t base = lb * kConvWaves; base < it.n_items; base += G * kConvWaves) {
        const uint32_t item = (uint32_t)(base + wave);
        if (item >= it.n_items) break;
        // wave-uniform decode: x-run, then BY-pencil row group, z, shot group
        uint32_t t = item;
        const int xr = (int)(t % (uint32_t)it.nxr);
        t /= (uint32_t)it.nxr;
        const int y0 = BY * (int)(t % (uint32_t)ny);
        t /= (uint32_t)ny;
        const int zz = (int)(t % (uint32_t)L);
        const uint32_t sg = it.sg0 + t / (uint32_t)L;
        const int64_t w = sg >> 2;
        const int l0 = 16 * (int)(sg & 3);
        const int x0 = xr * NX;
        // row (w, v, l) = (w N + v) 64 + l; lane part of every fragment address
        const int64_t wrow = w * N;
        const int lane_off = (l0 + r16) * CIN + (CIN == 32 ? 8 * q : 0);
        f32x4 acc[BY][NX][NT];
#pragma unroll
        for (int by = 0; by < BY; ++by)
#pragma unroll
            for (int i = 0; i < NX; ++i)
#pragma unroll
                for (int mt = 0; mt < NT; ++mt) acc[by][i][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        // the B slabs of pencil column c: dz = c / (BY + 2) - 1, rows y0 - 1 .. y0 + BY
        auto load_col = [&](int c, bf16x8 (&b)[NB]) {
            const int uy = wrap(y0 + c % (BY + 2) - 1, L), uz = wrap(zz + c / (BY + 2) - 1, L);
            const int64_t pencil = (wrow + (int64_t)L * (uy + (int64_t)L * uz)) * 64;
            if constexpr (CIN == 32) {
                // slabs x0 - 1 .. x0 + NX
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const int ux = wrap(x0 - 1 + i, L);
                    const bf16* src = x + (pencil + (int64_t)ux * 64) * CIN;
                    b[i] = *reinterpret_cast<const bf16x8*>(src + lane_off);
                }
            } else {
                // lane group q reads site x + q - 1 (q = 3: zero padding)
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    if (q < 3) {
                        const int ux = wrap(x0 + i + q - 1, L);
                        b[i] = *reinterpret_cast<const bf16x8*>(
                            x + (pencil + (int64_t)ux * 64) * CIN + lane_off);
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) b[i][e] = (bf16)0.f;
                    }
                }
            }
        };
        // apply column c to every output pencil y0 + by it is a (dy, dz) neighbour of:
        // taps j = 3 (dz + 1) + (dy + 1) with dy = dy' - by
        auto mma_col = [&](int c, const bf16x8 (&b)[NB]) {
            const int dzi = c / (BY + 2), dyp = c % (BY + 2) - 1;
#pragma unroll
            for (int by = 0; by < BY; ++by) {
                const int dy = dyp - by;
                if (dy < -1 || dy > 1) continue;
                const int j = 3 * dzi + dy + 1;
                if constexpr (CIN == 32) {
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        bf16x8 a[NT];
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt)
                            a[mt] = *reinterpret_cast<const bf16x8*>(
                                wl + (((3 * j + dx) * NT + mt) * 64 + lane) * 8);
#pragma unroll
                        for (int i = 0; i < NX; ++i)
#pragma unroll
                            for (int mt = 0; mt < NT; ++mt)
                                acc[by][i][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    a[mt], b[i + dx], acc[by][i][mt], 0, 0, 0);
                    }
                } else {
                    bf16x8 a[NT];
#pragma unroll
                    for (int mt = 0; mt < NT; ++mt)
                        a[mt] = *reinterpret_cast<const bf16x8*>(
                            wl + ((j * NT + mt) * 64 + lane) * 8);
#pragma unroll
                    for (int i = 0; i < NX; ++i)
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt)
                            acc[by][i][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                a[mt], b[i], acc[by][i][mt], 0, 0, 0);
                }
            }
        };
        // software pipeline: the slabs of column c + 1 are in flight while the
        // matrix cores work on column c
        bf16x8 b0[NB], b1[NB];
        load_col(0, b0);
#pragma unroll
        for (int c = 0; c < NC; c += 2) {
            if (c + 1 < NC) load_col(c + 1, b1);
            mma_col(c, b0);
            if (c + 1 < NC) {
                if (c + 2 < NC) load_col(c + 2, b0);
                mma_col(c + 1, b1);
            }
        }
        // epilogue: lane holds D[channel 16 mt + 4 q + i][shot l0 + r16] of site
        // (x0 + i, y0 + by)
#pragma unroll
        for (int by = 0; by < BY; ++by) {
            if (y0 + by >= L) break;
            const int64_t vrow = (int64_t)L * (y0 + by + (int64_t)L * zz);
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                if (x0 + i >= L) break;
                const int64_t v = vrow + x0 + i;
                const int64_t row = (wrow + v) * 64 + l0 + r16;
#pragma unroll
                for (int mt = 0; mt < NT; ++mt) {
                    const int64_t o = row * 32 + 16 * mt + 4 * q;
                    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                    bf16x4 out;
                    if constexpr (EPI == EPI_RELU) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            out[e] = (bf16)fmaxf(acc[by][i][mt][e] + bv[mt][e], 0.f);
                    } else {
                        const bf16x4 m = *reinterpret_cast<const bf16x4*>(mask_act + o);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            out[e] = (float)m[e] > 0.f ? (bf16)acc[by][i][mt][e] : (bf16)0.f;
                    }
                    *reinterpret_cast<bf16x4*>(y + o) = out;
                }
            }
        }
    }
}

// ------------------------------------- conv marching along z (MFMA)
// The forward 32-channel layers walk columns of sites along z instead: a
// wavefront owns NX x BY sites of an (x, y) column over a segment of zs
// consecutive planes, for 16 shots. Every input plane of the segment and
// its two neighbours is loaded once, row by row ((NX + 2)(BY + 2) slabs),
// and feeds the output planes below, at and above it. Their accumulators
// stay in registers as a ring of three: after input plane z the output
// plane z - 1 has all 27 taps and is written. That is (NX + 2)(BY + 2)
// (zs + 2) / (NX BY zs) slab loads per output site, 7 for 2 x 1 sites and 12
// planes, against 12 when every output plane loads its three input planes
// itself (k_conv with 2 x 2 sites).
constexpr int kConvZWaves = 8;
constexpr int kConvZBlock = 64 * kConvZWaves;

struct ConvZItems {
    int L, N;
    int nxr, ny, nzs, zs;  // x-runs, y-groups, z-segments of zs planes (the last may be short)
    uint32_t n_items;      // n_sg nzs ny nxr, for shot groups sg0 .. sg0 + n_sg - 1
    uint32_t sg0;
};

template <int EPI, int NX, int BY>
__global__ __launch_bounds__(kConvZBlock) void k_convz(
    const bf16* __restrict__ x, const bf16* __restrict__ wp, const float* __restrict__ bias,
    bf16* __restrict__ y, float* __restrict__ llr, ConvZItems it) {
    static_assert(EPI == EPI_RELU || EPI == EPI_LLR, "forward layers only");
    constexpr int CIN = 32;
    constexpr int NT = EPI == EPI_LLR ? 1 : 2;
    constexpr int WELEMS = 27 * NT * 64 * 8;
    constexpr int NB = NX + 2;  // slabs per row
    constexpr int NR = BY + 2;  // rows per input plane
    __shared__ __attribute__((aligned(16))) bf16 wl[WELEMS];
    for (int i = threadIdx.x * 8; i < WELEMS; i += kConvZBlock * 8)
        *reinterpret_cast<bf16x8*>(wl + i) = *reinterpret_cast<const bf16x8*>(wp + i);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int r16 = lane & 15, q = lane >> 4;
    const int L = it.L, N = it.N;
    const int64_t G = gridDim.x;
    const int64_t lb = xcd_block(blockIdx.x, G);
    for (int64_t base = lb * kConvZWaves; base < it.n_items; base += G * kConvZWaves) {
        const uint32_t item = (uint32_t)(base + wave);
        if (item >= it.n_items) break;
        // wave-uniform decode: x-run, y-group, z-segment, shot group
        uint32_t t = item;
        const int xr = (int)(t % (uint32_t)it.nxr);
        t /= (uint32_t)it.nxr;
        const int y0 = BY * (int)(t % (uint32_t)it.ny);
        t /= (uint32_t)it.ny;
        const int z0 = it.zs * (int)(t % (uint32_t)it.nzs);
        t /= (uint32_t)it.nzs;
        const uint32_t sg = it.sg0 + t;
        const int zn = L - z0 < it.zs ? L - z0 : it.zs;  // output planes of this segment
        const int64_t w = sg >> 2;
        const int l0 = 16 * (int)(sg & 3);
        const int x0 = xr * NX;
        const int64_t wrow = w * N;
        const int lane_off = (l0 + r16) * CIN + 8 * q;
        int ux[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) ux[i] = wrap(x0 - 1 + i, L);
        // acc[k]: output plane zi - 1 + k of the current input plane zi
        f32x4 acc[3][BY][NX][NT];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int by = 0; by < BY; ++by)
#pragma unroll
                for (int i = 0; i < NX; ++i)
#pragma unroll
                    for (int mt = 0; mt < NT; ++mt) acc[k][by][i][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        // step s: input plane zi = z0 - 1 + s / NR, row y0 - 1 + s % NR
        auto load_row = [&](int s, bf16x8 (&b)[NB]) {
            const int uz = wrap(z0 - 1 + s / NR, L), uy = wrap(y0 - 1 + s % NR, L);
            const int64_t pencil = (wrow + (int64_t)L * (uy + (int64_t)L * uz)) * 64;
#pragma unroll
            for (int i = 0; i < NB; ++i)
                b[i] = *reinterpret_cast<const bf16x8*>(x + (pencil + (int64_t)ux[i] * 64) * CIN +
                                                        lane_off);
        };
        auto store_plane = [&](int zo, const f32x4 (&a)[BY][NX][NT]) {
            // the bias is read here, once per plane, to keep it out of the
            // registers the accumulator ring needs
            float bv[NT][4];
#pragma unroll
            for (int mt = 0; mt < NT; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) bv[mt][i] = bias[16 * mt + 4 * q + i];
#pragma unroll
            for (int by = 0; by < BY; ++by) {
                if (y0 + by >= L) break;
                const int64_t vrow = (int64_t)L * (y0 + by + (int64_t)L * zo);
#pragma unroll
                for (int i = 0; i < NX; ++i) {
                    if (x0 + i >= L) break;
                    const int64_t v = vrow + x0 + i;
                    if constexpr (EPI == EPI_LLR) {
                        if (q == 0) {
#pragma unroll
                            for (int c = 0; c < 3; ++c)
                                llr[((w * 3 + c) * N + v) * 64 + l0 + r16] =
                                    -(a[by][i][0][c] + bv[0][c]);
                        }
                    } else {
                        const int64_t row = (wrow + v) * 64 + l0 + r16;
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt) {
                            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                            bf16x4 out;
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                out[e] = (bf16)fmaxf(a[by][i][mt][e] + bv[mt][e], 0.f);
                            *reinterpret_cast<bf16x4*>(y + row * 32 + 16 * mt + 4 * q) = out;
                        }
                    }
                }
            }
        };
        auto step = [&](int s, const bf16x8 (&b)[NB]) {
            const int p = s / NR, r = s % NR;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int oz = p - 2 + k;  // output plane z0 + oz, tap dz = 1 - k
                if (oz < 0 || oz >= zn) continue;
#pragma unroll
                for (int by = 0; by < BY; ++by) {
                    const int dy = r - 1 - by;
                    if (dy < -1 || dy > 1) continue;
                    const int tap0 = 3 * (dy + 1) + 9 * (2 - k);
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        bf16x8 a[NT];
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt)
                            a[mt] = *reinterpret_cast<const bf16x8*>(
                                wl + (((tap0 + dx) * NT + mt) * 64 + lane) * 8);
#pragma unroll
                        for (int i = 0; i < NX; ++i)
#pragma unroll
                            for (int mt = 0; mt < NT; ++mt)
                                acc[k][by][i][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    a[mt], b[i + dx], acc[k][by][i][mt], 0, 0, 0);
                    }
                }
            }
            if (r == NR - 1) {
                // input plane done: output plane zi - 1 has all its taps
                if (p >= 2 && p - 2 < zn) store_plane(z0 + p - 2, acc[0]);
#pragma unroll
                for (int by = 0; by < BY; ++by)
#pragma unroll
                    for (int i = 0; i < NX; ++i)
#pragma unroll
                        for (int mt = 0; mt < NT; ++mt) {
                            acc[0][by][i][mt] = acc[1][by][i][mt];
                            acc[1][by][i][mt] = acc[2][by][i][mt];
                            acc[2][by][i][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
                        }
            }
        };
        // software pipeline over rows: the next row's slabs are in flight
        // while the matrix cores work on the current one
        const int n_steps = (zn + 2) * NR;
        bf16x8 b0[NB], b1[NB];
        load_row(0, b0);
        for (int s = 0; s < n_steps; s += 2) {
            if (s + 1 < n_steps) load_row(s + 1, b1);
            step(s, b0);
            if (s + 1 < n_steps) {
                if (s + 2 < n_steps) load_row(s + 2, b0);
                step(s + 1, b1);
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
        const int l = (int)(g & 63);
        const uint32_t wv = g >> 6;
        const uint32_t w = wv / (uint32_t)N;
        const int v = (int)(wv - w * (uint32_t)N);
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = (bf16)0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t e = (int64_t)c * N + v;
            const float z = -llr[((int64_t)w * 3 * N + e) * 64 + l];
            const float t = (float)((target[e * ld + w] >> l) & 1u);
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
// The contraction runs over rows, i.e. over the 64 shots of each site-word,
// so both MFMA operands need 8 consecutive shots of one channel per lane,
// while activations are stored channel-contiguous for the forward pass.
// k_rows_to_shots makes a shot-contiguous copy of x and of dy first
// ([(w N + v) C + c][64 shots]); k_wgradP then reads every fragment with one
// 16-byte load.

// One 256-thread workgroup per 256 / (8 C) site-words, staged through LDS.
template <int C>
__global__ __launch_bounds__(256) void k_rows_to_shots(const bf16* __restrict__ in,
                                                       bf16* __restrict__ out, int64_t n_sw) {
    constexpr int TPS = 8 * C;      // threads per site-word: 16 bytes each way
    constexpr int SPB = 256 / TPS;  // site-words per workgroup
    constexpr int STR = C + 2;      // LDS row stride (bf16)
    __shared__ bf16 t[SPB][64][STR];
    const int tid = threadIdx.x;
    const int s = tid / TPS, r = tid % TPS;
    const int64_t sw = (int64_t)blockIdx.x * SPB + s;
    if (sw < n_sw) {
        // row r / (C / 8) of the site-word, channels 8 (r % (C / 8)) .. + 7
        const int row = r / (C / 8), c8 = 8 * (r % (C / 8));
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(in + (sw * 64 + row) * C + c8);
#pragma unroll
        for (int e = 0; e < 8; ++e) t[s][row][c8 + e] = v[e];
    }
    __syncthreads();
    if (sw < n_sw) {
        // channel r / 8, shots 8 (r % 8) .. + 7
        const int ch = r / 8, l8 = 8 * (r % 8);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = t[s][l8 + e][ch];
        *reinterpret_cast<bf16x8*>(out + (sw * C + ch) * 64 + l8) = o;
    }
}

// MFMA 16x16x32 with M = ci, N = co and K = 32 shots of one site: an A lane
// (ci = 16 mt + lane % 16, shots 8 (lane / 16) ..) is a 16-byte load of a
// neighbour site's x copy, a B lane likewise of this site's dy copy. A
// workgroup walks x-pencils; wavefront c of its 9 owns the (dy, dz) column c
// (dy = c % 3 - 1, dz = c / 3 - 1) and the three offsets d = 3 c + dx. Along
// the pencil it keeps the x copies of sites x - 1, x, x + 1 of the neighbour
// pencil in registers and loads one new site per step, so a site's x
// fragments feed three offsets: 8 loads per 24 MFMAs. Wavefront 0 also owns
// the bias gradient, as the product of an all-ones A with dy. Each workgroup
// walks a contiguous range of pencils and writes its partial sums to
// part[block][27][CIN][COUT] and part_b[block][COUT]; k_reduce8 adds the
// partials in a fixed order.
template <int CIN, int COUT, int CXS, int CYS>
__global__ __launch_bounds__(576) void k_wgradP(const bf16* __restrict__ xT,
                                                const bf16* __restrict__ dyT, int L, int N,
                                                int64_t n_pencils, int64_t per_block,
                                                float* __restrict__ part,
                                                float* __restrict__ part_b) {
    constexpr int MT = CIN > 16 ? 2 : 1, NT = COUT > 16 ? 2 : 1;
    const int lane = threadIdx.x & 63;
    const int col = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int r16 = lane & 15, q = lane >> 4;
    const int dy = col % 3 - 1, dz = col / 3 - 1;
    f32x4 acc[3][MT][NT];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[k][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 accb[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) accb[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ones, zero;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        ones[e] = (bf16)1.f;
        zero[e] = (bf16)0.f;
    }
    const int64_t LL = (int64_t)L * L;
    const int64_t p0 = (int64_t)blockIdx.x * per_block;
    const int64_t p1 = p0 + per_block < n_pencils ? p0 + per_block : n_pencils;
    for (int64_t pn = p0; pn < p1; ++pn) {
        const int64_t w = pn / LL;
        const int r = (int)(pn - w * LL);
        const int y = r % L, z = r / L;
        const int uy = wrap(y + dy, L), uz = wrap(z + dz, L);
        // site x = 0 of the neighbour pencil and of this pencil
        const bf16* xs = xT + (w * N + (int64_t)L * (uy + (int64_t)L * uz)) * CXS * 64;
        const bf16* ds = dyT + (w * N + (int64_t)L * (y + (int64_t)L * z)) * CYS * 64;
        auto load_x = [&](int x, bf16x8 (&a)[MT][2]) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int ci = 16 * mt + r16;
#pragma unroll
                for (int kb = 0; kb < 2; ++kb)
                    a[mt][kb] = ci < CXS ? *reinterpret_cast<const bf16x8*>(
                                               xs + ((int64_t)x * CXS + ci) * 64 + 32 * kb + 8 * q)
                                         : zero;
            }
        };
        bf16x8 am[MT][2], a0[MT][2], ap[MT][2], b[NT][2];
        load_x(L - 1, am);
        load_x(0, a0);
        for (int x = 0; x < L; ++x) {
            load_x(x + 1 < L ? x + 1 : 0, ap);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = 16 * nt + r16;
#pragma unroll
                for (int kb = 0; kb < 2; ++kb)
                    b[nt][kb] = co < CYS ? *reinterpret_cast<const bf16x8*>(
                                               ds + ((int64_t)x * CYS + co) * 64 + 32 * kb + 8 * q)
                                         : zero;
            }
            if (col == 0) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb)
                        accb[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ones, b[nt][kb],
                                                                           accb[nt], 0, 0, 0);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb) {
                        acc[0][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            am[mt][kb], b[nt][kb], acc[0][mt][nt], 0, 0, 0);
                        acc[1][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            a0[mt][kb], b[nt][kb], acc[1][mt][nt], 0, 0, 0);
                        acc[2][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            ap[mt][kb], b[nt][kb], acc[2][mt][nt], 0, 0, 0);
                    }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    am[mt][kb] = a0[mt][kb];
                    a0[mt][kb] = ap[mt][kb];
                }
        }
    }
    // lane holds D[ci = 16 mt + 4 q + i][co = 16 nt + r16] of offset 3 col + dx
    float* pb = part + (int64_t)blockIdx.x * 27 * CIN * COUT;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const int d = 3 * col + dx;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = 16 * nt + r16;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int ci = 16 * mt + 4 * q + i;
                    if (ci < CIN && co < COUT)
                        pb[((int64_t)d * CIN + ci) * COUT + co] = acc[dx][mt][nt][i];
                }
            }
    }
    if (col == 0 && q == 0) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int co = 16 * nt + r16;
            if (co < COUT) part_b[(int64_t)blockIdx.x * COUT + co] = accb[nt][0];
        }
    }
}

// out[i] = sum_b part[b][i] in a fixed order: 8 threads per output each add
// every 8th partial (consecutive outputs across lanes, so loads coalesce),
// then the 8 sums are added in order.
__global__ __launch_bounds__(256) void k_reduce8(const float* __restrict__ part, int64_t n,
                                                 int nblocks, float* __restrict__ out) {
    __shared__ float s[8][32];
    const int ii = threadIdx.x % 32, k = threadIdx.x / 32;
    const int64_t i = (int64_t)blockIdx.x * 32 + ii;
    float acc = 0.f;
    if (i < n)
        for (int b = k; b < nblocks; b += 8) acc += part[(int64_t)b * n + i];
    s[k][ii] = acc;
    __syncthreads();
    if (k == 0 && i < n) {
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) t += s[j][ii];
        out[i] = t;
    }
}

// *out = sum of part[0 .. n - 1] in a fixed order: thread t adds every 256th
// value from t on, then a tree over the 256 sums.
__global__ __launch_bounds__(256) void k_sum(const float* __restrict__ part, int64_t n,
                                             float* __restrict__ out) {
    __shared__ float s[256];
    float acc = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
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
    bf16* xT;      // shot-contiguous copies for the weight gradient, [R / 64][32][64]
    bf16* dyT;
    float* part;   // weight-gradient partials (training)
    float* part_b;
    float* loss_part;
};

constexpr int kWgradBlocks = 512;

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

size_t cnn_ws_bytes(int64_t R, int training) {
    size_t b = align_up((size_t)R * 8 * 2) + 3 * align_up((size_t)R * 32 * 2);
    if (training) {
        b += align_up((size_t)R * 8 * 2) + 4 * align_up((size_t)R * 32 * 2);
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
        w.xT = (bf16*)p;
        p += align_up((size_t)R * 32 * 2);
        w.dyT = (bf16*)p;
        p += align_up((size_t)R * 32 * 2);
        w.part = (float*)p;
        p += align_up((size_t)kWgradBlocks * 27 * 32 * 32 * 4);
        w.part_b = (float*)p;
        p += align_up((size_t)kWgradBlocks * 32 * 4);
        w.loss_part = (float*)p;
    }
    return w;
}

// Wavefront shape of k_conv, chosen by timing.
template <int CIN, int EPI>
struct ConvShape {
    static constexpr int NX = 2;  // sites per wavefront run along x
    static constexpr int BY = 2;  // y-pencils per wavefront
};

// Workgroups of a persistent conv launch: as many as the GPU holds at once
// (occupancy times compute units), found once per device. A grid of several
// rounds of workgroups re-stages the weights and leaves a ragged last round.
template <typename K>
int resident_blocks(K kernel, int block, std::atomic<int>* cache, int n_cache) {
    constexpr int kFallback = 512;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= n_cache) return kFallback;
    int c = cache[dev].load(std::memory_order_relaxed);
    if (c == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            per_cu < 1 || cus < 1)
            return kFallback;
        c = per_cu * cus;
        cache[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

// Rows of shot groups sg0 .. sg0 + n_sg - 1 (16 shots each); one wavefront
// item per (shot group, pencil, x-run).
template <int CIN, int EPI>
int launch_conv(const Ctx& c, const bf16* x, const bf16* wp, const float* bias,
                const bf16* mask_act, bf16* y, Geo g, int64_t sg0, int64_t n_sg) {
    ConvItems it;
    it.L = g.L;
    it.N = g.N;
    constexpr int NX = ConvShape<CIN, EPI>::NX, BY = ConvShape<CIN, EPI>::BY;
    it.nxr = (g.L + NX - 1) / NX;
    const int64_t items = n_sg * (int64_t)g.L * ((g.L + BY - 1) / BY) * it.nxr;
    if (items >= (1ll << 32) || sg0 + n_sg >= (1ll << 32)) return TC3D_EINVAL;
    if (items == 0) return TC3D_OK;
    it.n_items = (uint32_t)items;
    it.sg0 = (uint32_t)sg0;
    const int64_t blocks = cdiv(items, kConvWaves);
    static std::atomic<int> resident[64];
    const int cap = resident_blocks(k_conv<CIN, EPI, NX, BY>, kConvBlock, resident, 64);
    const int grid = (int)(blocks < cap ? blocks : cap);
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_conv<CIN, EPI, NX, BY><<<dim3(grid), dim3(kConvBlock), 0, c.stream>>>(
        x, wp, bias, mask_act, y, it);
    return after_launch(c);
}

// Shape of the z-marching forward convolutions (x-sites x y-pencils), chosen
// by timing: the ring of three output planes must leave 4 wavefronts per SIMD,
// which 2 x 1 sites of 32 channels do (111 registers) and 2 x 2 do not; the
// 32 -> 3 layer holds a third of the accumulators and affords 2 x 2.
template <int EPI>
struct ConvZShape {
    static constexpr int NX = 2;
    static constexpr int BY = EPI == EPI_LLR ? 2 : 1;
};

// Planes per z-segment: long segments load fewer extra planes ((zs + 2) / zs)
// but make fewer work items; take the length that minimises the rounds of
// resident wavefronts times the planes each item walks.
int choose_zs(int L, int64_t columns, int64_t slots) {
    int best = L;
    int64_t best_cost = -1;
    for (int zs = L; zs >= 1; --zs) {
        const int64_t rounds = cdiv(columns * cdiv(L, zs), slots);
        const int64_t cost = rounds * (zs + 2);
        if (best_cost < 0 || cost < best_cost) {
            best = zs;
            best_cost = cost;
        }
    }
    return best;
}

// Forward 32-channel layer over shot groups sg0 .. sg0 + n_sg - 1, marching
// along z; one wavefront item per (shot group, z-segment, y-group, x-run).
template <int EPI>
int launch_convz(const Ctx& c, const bf16* x, const bf16* wp, const float* bias, bf16* y,
                 float* llr, Geo g, int64_t sg0, int64_t n_sg) {
    constexpr int NX = ConvZShape<EPI>::NX, BY = ConvZShape<EPI>::BY;
    ConvZItems it;
    it.L = g.L;
    it.N = g.N;
    it.nxr = (g.L + NX - 1) / NX;
    it.ny = (g.L + BY - 1) / BY;
    static std::atomic<int> resident[64];
    const int cap = resident_blocks(k_convz<EPI, NX, BY>, kConvZBlock, resident, 64);
    const int64_t columns = n_sg * it.ny * it.nxr;
    it.zs = choose_zs(g.L, columns, (int64_t)cap * kConvZWaves);
    it.nzs = (g.L + it.zs - 1) / it.zs;
    const int64_t items = columns * it.nzs;
    if (items >= (1ll << 32) || sg0 + n_sg >= (1ll << 32)) return TC3D_EINVAL;
    if (items == 0) return TC3D_OK;
    it.n_items = (uint32_t)items;
    it.sg0 = (uint32_t)sg0;
    const int64_t blocks = cdiv(items, kConvZWaves);
    const int grid = (int)(blocks < cap ? blocks : cap);
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_convz<EPI, NX, BY><<<dim3(grid), dim3(kConvZBlock), 0, c.stream>>>(x, wp, bias, y, llr, it);
    return after_launch(c);
}

// Shot groups per pass of the forward network. A pass keeps its input and
// output activations (2 x 16 x N x 64 bytes per group) within the 256 MB
// Infinity Cache, so the neighbour re-reads of the convolutions are served
// from it rather than from HBM: 64 to 128 MB of input per pass (96 MB timed
// best where the count below does not decide). Within that range take the
// count whose z-marching 32 -> 32 launches fill the resident wavefronts best:
// time per group ~ rounds x (zs + 2) / groups.
constexpr int64_t kPassBytesLo = 64ll << 20, kPassBytesHi = 128ll << 20;
int64_t groups_per_pass(Geo g, int64_t n_sg) {
    const int64_t per = (int64_t)g.N * 16 * 64;
    int64_t hi = kPassBytesHi / per < 1 ? 1 : kPassBytesHi / per;
    if (hi > n_sg) hi = n_sg < 1 ? 1 : n_sg;
    int64_t lo = kPassBytesLo / per < 1 ? 1 : kPassBytesLo / per;
    if (lo > hi) lo = hi;
    constexpr int NX = ConvZShape<EPI_RELU>::NX, BY = ConvZShape<EPI_RELU>::BY;
    static std::atomic<int> resident[64];
    const int64_t slots =
        (int64_t)resident_blocks(k_convz<EPI_RELU, NX, BY>, kConvZBlock, resident, 64) *
        kConvZWaves;
    const int64_t cols = cdiv(g.L, BY) * cdiv(g.L, NX);  // z-columns per shot group
    int64_t best = (96ll << 20) / per;
    if (best < lo) best = lo;
    if (best > hi) best = hi;
    int64_t best_cost = -1;  // rounds x (zs + 2) of the best count
    for (int64_t gp = lo; gp <= hi; ++gp) {
        const int zs = choose_zs(g.L, gp * cols, slots);
        const int64_t cost = cdiv(gp * cols * cdiv(g.L, zs), slots) * (zs + 2);
        // cost / gp < best_cost / best, in integers
        if (best_cost < 0 || cost * best < best_cost * gp) {
            best = gp;
            best_cost = cost;
        }
    }
    return best;
}

const bf16* blk(const void* packed, int i) { return (const bf16*)packed + block_offset(i); }
const float* bias_of(const void* packed, int layer) {
    return (const float*)((const char*)packed + kBiasOffsetBytes) + 32 * layer;
}

// Forward pass over passes of a few shot groups each: input rows from the
// syndromes, then the four layers; writes llr. Rows of every shot group are
// written, so the weight gradient of the first layer can read x0 afterwards.
int cnn_forward_impl(const Ctx& c, Geo g, const uint64_t* syn, const uint64_t* prev, int64_t ld,
                     int64_t R, const void* packed, float* llr, const CnnWs& w) {
    int rc;
    const int64_t n_sg = R / (16 * (int64_t)g.N);
    const int64_t per = groups_per_pass(g, n_sg);
    for (int64_t sg0 = 0; sg0 < n_sg; sg0 += per) {
        const int64_t k = n_sg - sg0 < per ? n_sg - sg0 : per;
        if ((rc = launch_input(c, g, syn, prev, ld, sg0, k, w.x0))) return rc;
        if ((rc = launch_conv<8, EPI_RELU>(c, w.x0, blk(packed, 0), bias_of(packed, 0), nullptr,
                                           w.a[0], g, sg0, k)))
            return rc;
        if ((rc = launch_convz<EPI_RELU>(c, w.a[0], blk(packed, 1), bias_of(packed, 1), w.a[1],
                                         nullptr, g, sg0, k)))
            return rc;
        if ((rc = launch_convz<EPI_RELU>(c, w.a[1], blk(packed, 2), bias_of(packed, 2), w.a[2],
                                         nullptr, g, sg0, k)))
            return rc;
        if ((rc = launch_convz<EPI_LLR>(c, w.a[2], blk(packed, 3), bias_of(packed, 3), nullptr,
                                        llr, g, sg0, k)))
            return rc;
    }
    return TC3D_OK;
}

template <int C>
int launch_rows_to_shots(const Ctx& c, const bf16* in, bf16* out, int64_t n_sw) {
    constexpr int SPB = 256 / (8 * C);
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_rows_to_shots<C><<<dim3((unsigned)cdiv(n_sw, SPB)), dim3(256), 0, c.stream>>>(in, out,
                                                                                   n_sw);
    return after_launch(c);
}

// Weight and bias gradient of one layer from its input rows x ([R][CIN]) and
// output gradient rows dy ([R][8] for the 3-channel layer, else [R][32]).
template <int CIN, int COUT>
int launch_wgrad(const Ctx& c, const bf16* x, const bf16* dy, Geo g, int64_t R, const CnnWs& w,
                 float* grad_layer) {
    constexpr int CXS = CIN, CYS = COUT == 3 ? 8 : 32;  // stored channels of the rows
    const int64_t n_sw = R / 64;
    if (n_sw == 0) return TC3D_OK;
    int rc;
    if ((rc = launch_rows_to_shots<CXS>(c, x, w.xT, n_sw))) return rc;
    if ((rc = launch_rows_to_shots<CYS>(c, dy, w.dyT, n_sw))) return rc;
    const int64_t n_pencils = n_sw / g.L;  // W L^2 x-pencils
    const int64_t per = cdiv(n_pencils, kWgradBlocks);
    const int nb = (int)cdiv(n_pencils, per);
    if ((rc = before_launch(c, TC3D_K_CNN))) return rc;
    k_wgradP<CIN, COUT, CXS, CYS><<<dim3(nb), dim3(576), 0, c.stream>>>(
        w.xT, w.dyT, g.L, g.N, n_pencils, per, w.part, w.part_b);
    if ((rc = after_launch(c))) return rc;
    const int64_t nw = 27 * CIN * COUT;
    if ((rc = before_launch(c, TC3D_K_CNN))) return rc;
    k_reduce8<<<dim3((unsigned)cdiv(nw, 32)), dim3(256), 0, c.stream>>>(w.part, nw, nb,
                                                                        grad_layer);
    if ((rc = after_launch(c))) return rc;
    if ((rc = before_launch(c, TC3D_K_CNN))) return rc;
    k_reduce8<<<dim3((unsigned)cdiv(COUT, 32)), dim3(256), 0, c.stream>>>(w.part_b, COUT, nb,
                                                                          grad_layer + nw);
    return after_launch(c);
}

}  // namespace

// ------------------------------------------------------------ entry points
int64_t cnn_param_count() { return kParams; }
size_t cnn_packed_bytes() { return (size_t)kPackedBytes; }
size_t cnn_workspace_bytes(int64_t R, int training) { return cnn_ws_bytes(R, training); }

int cnn_pack(const Ctx& c, const float* params, float beta, float l0, void* packed) {
    int rc = before_launch(c, TC3D_K_CNN);
    if (rc) return rc;
    k_pack<<<dim3((unsigned)cdiv(kPackedElems, 256)), dim3(256), 0, c.stream>>>(
        params, beta, l0, (bf16*)packed, (float*)((char*)packed + kBiasOffsetBytes));
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
    k_sum<<<dim3(1), dim3(256), 0, c.stream>>>(w.loss_part, lb, loss);
    if ((rc = after_launch(c))) return rc;
    // layer 4 (32 -> 3): weight gradient, then dy of layer 3 through its ReLU
    if ((rc = launch_wgrad<32, 3>(c, w.a[2], w.dy8, g, R, w, grad + param_offset(3)))) return rc;
    const int64_t n_sg = R / (16 * (int64_t)g.N);
    if ((rc = launch_conv<8, EPI_MASK>(c, w.dy8, blk(packed, 4), nullptr, w.a[2], w.dyb[0], g,
                                       0, n_sg)))
        return rc;
    // layer 3 (32 -> 32)
    if ((rc = launch_wgrad<32, 32>(c, w.a[1], w.dyb[0], g, R, w, grad + param_offset(2))))
        return rc;
    if ((rc = launch_conv<32, EPI_MASK>(c, w.dyb[0], blk(packed, 5), nullptr, w.a[1],
                                        w.dyb[1], g, 0, n_sg)))
        return rc;
    // layer 2 (32 -> 32)
    if ((rc = launch_wgrad<32, 32>(c, w.a[0], w.dyb[1], g, R, w, grad + param_offset(1))))
        return rc;
    if ((rc = launch_conv<32, EPI_MASK>(c, w.dyb[1], blk(packed, 6), nullptr, w.a[0],
                                        w.dyb[0], g, 0, n_sg)))
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
    return cnn_pack(c, params, 1.0f, 0.0f, packed);
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
