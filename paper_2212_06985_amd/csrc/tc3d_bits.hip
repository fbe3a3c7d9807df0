// Bit-sliced kernels: 64 shots per uint64 word, one work item per
// (lattice row, word). Noise (Sections 3.1, 4.1), syndrome (Section 2),
// flip / p-flip decisions (Sections 3.1, 3.2) and the majority-vote readout.
#include "tc3d_device.hpp"
#include "tc3d_internal.hpp"

namespace tc3d {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_noise(uint64_t* __restrict__ plane, int64_t ld,
                                                  int64_t rows, int64_t nw, uint64_t word0,
                                                  uint32_t tag, uint32_t cycle, uint32_t th,
                                                  uint32_t k0, uint32_t k1) {
    const int64_t G = gridDim.x;
    const int64_t blk = xcd_block(blockIdx.x, G);
    const int64_t idx = blk * kBlock + threadIdx.x;
    if (idx >= rows * nw) return;
    const int64_t row = idx / nw, w = idx - row * nw;
    const uint64_t bits = bernoulli_word((uint32_t)row, cycle, word0 + (uint64_t)w, tag, th, k0, k1);
    plane[row * ld + w] ^= bits;
}

// dst[f] (=|^=) XOR of src over the four members of face f, optionally with
// check-outcome noise (tag 1) XORed in.
__global__ __launch_bounds__(kBlock) void k_syndrome(const uint64_t* __restrict__ src,
                                                     int64_t ld_src, uint64_t* __restrict__ dst,
                                                     int64_t ld_dst, int64_t nw, int L, int N,
                                                     int xor_into, uint32_t th, uint64_t word0,
                                                     uint32_t cycle, uint32_t k0, uint32_t k1) {
    const int64_t G = gridDim.x;
    const int64_t blk = xcd_block(blockIdx.x, G);
    const int64_t idx = blk * kBlock + threadIdx.x;
    const int64_t rows = 3 * (int64_t)N;
    if (idx >= rows * nw) return;
    const int64_t f = idx / nw, w = idx - f * nw;
    const int n = (int)(f / N), v = (int)(f - (int64_t)n * N);
    int m[4];
    face_members(n, coord_of(v, L), L, N, m);
    uint64_t s = src[m[0] * ld_src + w] ^ src[m[1] * ld_src + w] ^ src[m[2] * ld_src + w] ^
                 src[m[3] * ld_src + w];
    if (th) s ^= bernoulli_word((uint32_t)f, cycle, word0 + (uint64_t)w, 1u, th, k0, k1);
    uint64_t* o = dst + f * ld_dst + w;
    *o = xor_into ? (*o ^ s) : s;
}

// Decision pass of one sweep. a..d: the four checks of the edge, one bit per
// shot. At least 3 of 4 unsatisfied -> flip; exactly 2 -> flip if p-flip and
// the coin is 1. corr ^= F; F stored for the check update.
__global__ __launch_bounds__(kBlock) void k_sweep(const uint64_t* __restrict__ syn, int64_t ld_s,
                                                  uint64_t* __restrict__ corr, int64_t ld_c,
                                                  uint64_t* __restrict__ fpl, int64_t ld_f,
                                                  int64_t nw, int L, int N, int pflip,
                                                  int cls, uint64_t word0, uint32_t cycle,
                                                  uint32_t sweep, uint32_t k0, uint32_t k1) {
    const int64_t G = gridDim.x;
    const int64_t blk = xcd_block(blockIdx.x, G);
    const int64_t idx = blk * kBlock + threadIdx.x;
    const int64_t rows = 3 * (int64_t)N;
    if (idx >= rows * nw) return;
    const int64_t e = idx / nw, w = idx - e * nw;
    const int ax = (int)(e / N), v = (int)(e - (int64_t)ax * N);
    const Coord cv = coord_of(v, L);
    if (cls >= 0) {
        // subset sweep: only edges of class cls = 4 ax + 2 (v_b & 1) + (v_c & 1),
        // b < c the other two axes, may flip
        const int cb = ax == 0 ? cv.y : cv.x, cc = ax == 2 ? cv.y : cv.z;
        if (4 * ax + 2 * (cb & 1) + (cc & 1) != cls) {
            fpl[e * ld_f + w] = 0;
            return;
        }
    }
    int f[4];
    edge_faces(ax, cv, L, N, f);
    const uint64_t a = syn[f[0] * ld_s + w], b = syn[f[1] * ld_s + w];
    const uint64_t c = syn[f[2] * ld_s + w], d = syn[f[3] * ld_s + w];
    const uint64_t ab = a & b, cd = c & d;
    uint64_t F = (ab & (c | d)) | (cd & (a | b));
    if (pflip) {
        const uint64_t eq2 = ((a ^ b) & (c ^ d)) | (ab & ~(c | d)) | (cd & ~(a | b));
        F |= eq2 & coin_word((uint32_t)e, cycle, word0 + (uint64_t)w, sweep, k0, k1);
    }
    corr[e * ld_c + w] ^= F;
    fpl[e * ld_f + w] = F;
}

__global__ __launch_bounds__(kBlock) void k_xor(uint64_t* __restrict__ dst, int64_t ld_d,
                                                const uint64_t* __restrict__ src, int64_t ld_s,
                                                int64_t rows, int64_t nw) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= rows * nw) return;
    const int64_t r = idx / nw, w = idx - r * nw;
    dst[r * ld_d + w] ^= src[r * ld_s + w];
}

// Plain streaming copy, 16 bytes per lane (byte-counter calibration and the
// read + write ceiling the BP kernel is compared with).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_stream_copy(u32x4* __restrict__ dst,
                                                        const u32x4* __restrict__ src, int64_t n,
                                                        int nontemporal) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const u32x4 v = src[i];
    if (nontemporal)
        __builtin_nontemporal_store(v, dst + i);
    else
        dst[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_clear(uint64_t* __restrict__ dst, int64_t ld,
                                                  int64_t rows, int64_t nw) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= rows * nw) return;
    const int64_t r = idx / nw, w = idx - r * nw;
    dst[r * ld + w] = 0;
}

// Majority-vote readout in two passes.
// Pass 1, one work item per (axis d, logical Z string s, word w), w fastest so
// that a wavefront's loads of one edge row are contiguous: the parity word of
// the string (XOR of its L edge words) goes to par[(w 3 + d) L^2 + s]. String
// s = i L + j holds the edges e(v + t unit(d), d), t = 0 .. L-1, where v has
// coordinate i on axis (d+1) mod 3, j on axis (d+2) mod 3 and 0 on axis d.
__global__ __launch_bounds__(kBlock) void k_string_parity(const uint64_t* __restrict__ err,
                                                          int64_t ld, int L, int N, int64_t nw,
                                                          uint64_t* __restrict__ par) {
    const int64_t LL = (int64_t)L * L;
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 3 * LL * nw) return;
    const int64_t w = idx % nw, rest = idx / nw;
    const int64_t s = rest % LL;
    const int d = (int)(rest / LL);
    const int64_t i = s / L, j = s - (s / L) * L;
    const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    const int64_t st = d == 0 ? 1 : (d == 1 ? L : LL);
    const int64_t s1 = d1 == 0 ? 1 : (d1 == 1 ? L : LL);
    const int64_t s2 = d2 == 0 ? 1 : (d2 == 1 ? L : LL);
    const uint64_t* row = err + ((int64_t)d * N + i * s1 + j * s2) * ld + w;
    uint64_t p = 0;
    for (int t = 0; t < L; ++t) p ^= row[t * st * ld];
    par[(w * 3 + d) * LL + s] = p;
}

// Pass 2, one workgroup per word, wavefront 4 d + q for axis d: each lane
// loads the parity word of one string (64 consecutive strings per step, every
// fourth step for wavefront q) and 64 ballots count, for each shot of the word,
// its odd strings among them; lane k keeps the count of shot 64 w + k. The 12
// partial counts meet in LDS; wavefront 0 applies the majority rule.
constexpr int kReadoutParts = 4;

__global__ __launch_bounds__(64 * 3 * kReadoutParts) void k_string_count(
    const uint64_t* __restrict__ par, int L, int64_t n_shots, uint8_t* __restrict__ mask,
    int32_t* __restrict__ odd) {
    __shared__ int part_count[3 * kReadoutParts][64];
    const int64_t w = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int d = wave / kReadoutParts, q = wave % kReadoutParts;
    const int64_t LL = (int64_t)L * L;
    const uint64_t* col = par + (w * 3 + d) * LL;
    int cnt = 0;
    for (int64_t c0 = 64 * (int64_t)q; c0 < LL; c0 += 64 * kReadoutParts) {
        const int64_t s = c0 + lane;
        const uint64_t p = s < LL ? col[s] : 0ull;
#pragma unroll 8
        for (int k = 0; k < 64; ++k) {
            const int n = __popcll(__ballot((p >> k) & 1ull));
            cnt += lane == k ? n : 0;
        }
    }
    part_count[wave][lane] = cnt;
    __syncthreads();
    if (wave != 0) return;
    const int64_t shot = w * 64 + lane;
    if (shot >= n_shots) return;
    uint32_t bits = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int total = 0;
#pragma unroll
        for (int k = 0; k < kReadoutParts; ++k) total += part_count[a * kReadoutParts + k][lane];
        if (2 * (int64_t)total >= LL) bits |= 1u << a;
        if (odd) odd[shot * 3 + a] = total;
    }
    mask[shot] = (uint8_t)bits;
}

inline int64_t blocks_for(int64_t items) { return (items + kBlock - 1) / kBlock; }

}  // namespace

int launch_noise(const Ctx& c, Geo g, Plane plane, int64_t nw, uint64_t word0, uint32_t tag,
                 uint32_t cycle, uint32_t th, uint64_t seed) {
    if (th == 0 || nw == 0) return TC3D_OK;
    const int64_t rows = 3 * (int64_t)g.N;
    int rc = before_launch(c, TC3D_K_NOISE);
    if (rc) return rc;
    k_noise<<<dim3((unsigned)blocks_for(rows * nw)), dim3(kBlock), 0, c.stream>>>(
        plane.p, plane.ld, rows, nw, word0, tag, cycle, th, (uint32_t)seed,
        (uint32_t)(seed >> 32));
    return after_launch(c);
}

int launch_syndrome(const Ctx& c, Geo g, CPlane src, Plane dst, int64_t nw, int xor_into,
                    uint32_t th_meas, uint64_t word0, uint32_t cycle, uint64_t seed) {
    if (nw == 0) return TC3D_OK;
    const int64_t rows = 3 * (int64_t)g.N;
    int rc = before_launch(c, TC3D_K_SYNDROME);
    if (rc) return rc;
    k_syndrome<<<dim3((unsigned)blocks_for(rows * nw)), dim3(kBlock), 0, c.stream>>>(
        src.p, src.ld, dst.p, dst.ld, nw, g.L, g.N, xor_into, th_meas, word0, cycle,
        (uint32_t)seed, (uint32_t)(seed >> 32));
    return after_launch(c);
}

int launch_sweep_decide(const Ctx& c, Geo g, CPlane syn, Plane corr, Plane fplane, int64_t nw,
                        int pflip, uint64_t word0, uint32_t cycle, uint32_t sweep,
                        uint64_t seed, int cls) {
    if (nw == 0) return TC3D_OK;
    const int64_t rows = 3 * (int64_t)g.N;
    int rc = before_launch(c, TC3D_K_SWEEP);
    if (rc) return rc;
    k_sweep<<<dim3((unsigned)blocks_for(rows * nw)), dim3(kBlock), 0, c.stream>>>(
        syn.p, syn.ld, corr.p, corr.ld, fplane.p, fplane.ld, nw, g.L, g.N, pflip, cls, word0,
        cycle, sweep, (uint32_t)seed, (uint32_t)(seed >> 32));
    return after_launch(c);
}

int launch_xor(const Ctx& c, Plane dst, CPlane src, int64_t rows, int64_t nw) {
    if (nw == 0 || rows == 0) return TC3D_OK;
    int rc = before_launch(c, TC3D_K_APPLY);
    if (rc) return rc;
    k_xor<<<dim3((unsigned)blocks_for(rows * nw)), dim3(kBlock), 0, c.stream>>>(
        dst.p, dst.ld, src.p, src.ld, rows, nw);
    return after_launch(c);
}

int launch_stream_copy(const Ctx& c, void* dst, const void* src, int64_t n16, int nontemporal) {
    if (n16 == 0) return TC3D_OK;
    int rc = before_launch(c, TC3D_K_APPLY);
    if (rc) return rc;
    k_stream_copy<<<dim3((unsigned)blocks_for(n16)), dim3(kBlock), 0, c.stream>>>(
        (u32x4*)dst, (const u32x4*)src, n16, nontemporal);
    return after_launch(c);
}

int launch_clear(const Ctx& c, Plane dst, int64_t rows, int64_t nw) {
    if (nw == 0 || rows == 0) return TC3D_OK;
    int rc = before_launch(c, TC3D_K_APPLY);
    if (rc) return rc;
    k_clear<<<dim3((unsigned)blocks_for(rows * nw)), dim3(kBlock), 0, c.stream>>>(dst.p, dst.ld,
                                                                                   rows, nw);
    return after_launch(c);
}

int64_t readout_scratch_words(Geo g, int64_t nw) { return 3 * (int64_t)g.L * g.L * nw; }

int launch_readout(const Ctx& c, Geo g, CPlane err, int64_t n_shots, uint8_t* mask,
                   int32_t* odd, uint64_t* par) {
    if (n_shots == 0) return TC3D_OK;
    const int64_t nw = (n_shots + 63) / 64;
    int rc = before_launch(c, TC3D_K_READOUT);
    if (rc) return rc;
    k_string_parity<<<dim3((unsigned)blocks_for(readout_scratch_words(g, nw))), dim3(kBlock), 0,
                      c.stream>>>(err.p, err.ld, g.L, g.N, nw, par);
    rc = after_launch(c);
    if (rc) return rc;
    rc = before_launch(c, TC3D_K_READOUT);
    if (rc) return rc;
    k_string_count<<<dim3((unsigned)nw), dim3(64 * 3 * kReadoutParts), 0, c.stream>>>(
        par, g.L, n_shots, mask, odd);
    return after_launch(c);
}

}  // namespace tc3d
