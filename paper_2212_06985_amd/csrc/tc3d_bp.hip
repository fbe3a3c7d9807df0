// FP32 belief propagation on the Tanner graph of the 3D toric code's Z checks
// (Section 4.1: LLR definition, factor-to-variable rule, variable-to-factor
// rule, posterior), flooding schedule, with the measurement-error variables
// folded into a constant factor K = 1 - 2q of every check product.
//
// State between iterations is only the factor-to-variable messages nu, FP32,
// [12][L^3][S_pad] with row (4n + k) * L^3 + v = message of face f(v,n) to its
// member k; the shot index is the fastest dimension, so a wavefront (64 lanes
// = 64 consecutive shots of one site) reads and writes 256 contiguous bytes
// per message row.
//
// One iteration is one kernel: a wavefront owns site v and its three faces.
// It rebuilds the posterior l of the 9 edges its faces touch from the old
// messages (E4: l = l0 + sum of the 4 incoming messages), forms the
// variable-to-factor messages mu = l - nu_old (E3 written as a difference),
// and writes the new messages of its faces (E2). The posterior needs messages
// of neighbouring sites; those reads are served by the caches because
// neighbouring sites of the same shot word are processed by the same XCD at
// nearly the same time.
#include "tc3d_device.hpp"
#include "tc3d_internal.hpp"

namespace tc3d {

namespace {

constexpr int kWaves = 4;  // sites per workgroup, one wavefront each
constexpr int kBlock = 64 * kWaves;

struct Src {
    const float* __restrict__ nu;    // NU_LOAD
    const uint64_t* __restrict__ syn;
    int64_t ld_syn;
    const float* __restrict__ llr0;  // nullptr: scalar prior
    float l0, nu1;
    int N;
    int64_t s_pad, s, w;
    int lane;
};

// Old message of face f(site, n) to member k.
template <int MODE>
__device__ __forceinline__ float nu_old(const Src& S, int n, int k, int site) {
    if constexpr (MODE == NU_ZERO) {
        return 0.0f;
    } else if constexpr (MODE == NU_SIGMA) {
        const uint64_t word = S.syn[((int64_t)n * S.N + site) * S.ld_syn + S.w];
        return ((word >> S.lane) & 1u) ? -S.nu1 : S.nu1;
    } else {
        return S.nu[((int64_t)(4 * n + k) * S.N + site) * S.s_pad + S.s];
    }
}

// Posterior of edge e(w, c) at the old state (E4).
template <int MODE>
__device__ __forceinline__ float edge_llr(const Src& S, int c, Coord cw, int L) {
    const int w = site_of(cw.x, cw.y, cw.z, L);
    float l = S.llr0 ? S.llr0[((int64_t)c * S.N + w) * S.s_pad + S.s] : S.l0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d == c) continue;
        const int n = 3 - c - d;
        const int k = c < d ? 0 : 2;
        l += nu_old<MODE>(S, n, k, w) + nu_old<MODE>(S, n, k + 1, shift(cw, d, -1, L));
    }
    return l;
}

// tanh(mu/2) = 1 - 2 / (1 + e^mu)
__device__ __forceinline__ float tanh_half(float mu) {
    const float e = __builtin_amdgcn_exp2f(mu * 1.4426950408889634f);
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
}

// 2 atanh(y) = ln((1 + y) / (1 - y)), |y| <= K < 1
__device__ __forceinline__ float two_atanh(float y) {
    const float r = (1.0f + y) * __builtin_amdgcn_rcpf(1.0f - y);
    return 0.69314718055994531f * __builtin_amdgcn_logf(r);
}

struct Item {
    int v;
    Coord cv;
    bool ok;
};

__device__ __forceinline__ Item item_of(const Src& S, int L, int64_t n_sg, int64_t& w_out,
                                        int64_t& s_out, int& lane_out) {
    const int64_t G = gridDim.x;
    const int64_t lb = xcd_block(blockIdx.x, G);
    const int64_t w = lb / n_sg;
    const int64_t sg = lb - w * n_sg;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    Item it;
    it.v = (int)(sg * kWaves + wave);
    it.ok = it.v < S.N;
    it.cv = coord_of(it.ok ? it.v : 0, L);
    lane_out = (int)(threadIdx.x & 63);
    w_out = w;
    s_out = w * 64 + lane_out;
    return it;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_bp_iter(Src S, int L, int64_t n_sg, float K,
                                                    float* __restrict__ nu_out) {
    Item it = item_of(S, L, n_sg, S.w, S.s, S.lane);
    if (!it.ok) return;
    const Coord cv = it.cv;
    const int v = it.v;
    const Coord cxp{inc(cv.x, L), cv.y, cv.z};
    const Coord cyp{cv.x, inc(cv.y, L), cv.z};
    const Coord czp{cv.x, cv.y, inc(cv.z, L)};
    // posteriors of the 9 edges touched by the faces of v
    const float lx = edge_llr<MODE>(S, 0, cv, L);
    const float ly = edge_llr<MODE>(S, 1, cv, L);
    const float lz = edge_llr<MODE>(S, 2, cv, L);
    const float lx_yp = edge_llr<MODE>(S, 0, cyp, L);
    const float lx_zp = edge_llr<MODE>(S, 0, czp, L);
    const float ly_xp = edge_llr<MODE>(S, 1, cxp, L);
    const float ly_zp = edge_llr<MODE>(S, 1, czp, L);
    const float lz_xp = edge_llr<MODE>(S, 2, cxp, L);
    const float lz_yp = edge_llr<MODE>(S, 2, cyp, L);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        float lm[4];
        if (n == 2) {  // spans x, y
            lm[0] = lx; lm[1] = lx_yp; lm[2] = ly; lm[3] = ly_xp;
        } else if (n == 1) {  // spans x, z
            lm[0] = lx; lm[1] = lx_zp; lm[2] = lz; lm[3] = lz_xp;
        } else {  // spans y, z
            lm[0] = ly; lm[1] = ly_zp; lm[2] = lz; lm[3] = lz_yp;
        }
        float t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = tanh_half(lm[k] - nu_old<MODE>(S, n, k, v));
        const uint64_t sw = S.syn[((int64_t)n * S.N + v) * S.ld_syn + S.w];
        const float sK = ((sw >> S.lane) & 1u) ? -K : K;
        const float a01 = sK * (t[0] * t[1]);
        const float a23 = sK * (t[2] * t[3]);
        float* o = nu_out + ((int64_t)(4 * n) * S.N + v) * S.s_pad + S.s;
        const int64_t row = (int64_t)S.N * S.s_pad;
        o[0] = two_atanh(t[1] * a23);
        o[row] = two_atanh(t[0] * a23);
        o[2 * row] = two_atanh(t[3] * a01);
        o[3 * row] = two_atanh(t[2] * a01);
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_bp_post(Src S, int L, int64_t n_sg,
                                                    uint64_t* __restrict__ corr, int64_t ld_c,
                                                    float* __restrict__ post) {
    Item it = item_of(S, L, n_sg, S.w, S.s, S.lane);
    if (!it.ok) return;
    float l[3];
    l[0] = edge_llr<MODE>(S, 0, it.cv, L);
    l[1] = edge_llr<MODE>(S, 1, it.cv, L);
    l[2] = edge_llr<MODE>(S, 2, it.cv, L);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = (int64_t)c * S.N + it.v;
        if (post) post[e * S.s_pad + S.s] = l[c];
        const uint64_t flips = __ballot(l[c] < 0.0f);
        if (corr && S.lane == 0) corr[e * ld_c + S.w] = flips;
    }
}

Src make_src(Geo g, const BpArgs& a, const float* nu) {
    Src S;
    S.nu = nu;
    S.syn = a.syn.p;
    S.ld_syn = a.syn.ld;
    S.llr0 = a.llr0;
    S.l0 = a.l0;
    S.nu1 = a.nu1;
    S.N = g.N;
    S.s_pad = a.s_pad;
    S.s = S.w = 0;
    S.lane = 0;
    return S;
}

}  // namespace

int launch_bp_iter(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu_in,
                   float* nu_out, int kclass) {
    if (a.nw == 0) return TC3D_OK;
    const int64_t n_sg = (g.N + kWaves - 1) / kWaves;
    const int64_t blocks = n_sg * a.nw;
    if (blocks > 0x7fffffff) return TC3D_EINVAL;
    int rc = before_launch(c, kclass);
    if (rc) return rc;
    const Src S = make_src(g, a, nu_in);
    const dim3 grid((unsigned)blocks), block(kBlock);
    if (mode == NU_ZERO)
        k_bp_iter<NU_ZERO><<<grid, block, 0, c.stream>>>(S, g.L, n_sg, a.K, nu_out);
    else if (mode == NU_SIGMA)
        k_bp_iter<NU_SIGMA><<<grid, block, 0, c.stream>>>(S, g.L, n_sg, a.K, nu_out);
    else
        k_bp_iter<NU_LOAD><<<grid, block, 0, c.stream>>>(S, g.L, n_sg, a.K, nu_out);
    return after_launch(c);
}

int launch_bp_post(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu, Plane corr,
                   float* post) {
    if (a.nw == 0) return TC3D_OK;
    const int64_t n_sg = (g.N + kWaves - 1) / kWaves;
    const int64_t blocks = n_sg * a.nw;
    if (blocks > 0x7fffffff) return TC3D_EINVAL;
    int rc = before_launch(c, TC3D_K_BP_POST);
    if (rc) return rc;
    const Src S = make_src(g, a, nu);
    const dim3 grid((unsigned)blocks), block(kBlock);
    if (mode == NU_ZERO)
        k_bp_post<NU_ZERO><<<grid, block, 0, c.stream>>>(S, g.L, n_sg, corr.p, corr.ld, post);
    else if (mode == NU_SIGMA)
        k_bp_post<NU_SIGMA><<<grid, block, 0, c.stream>>>(S, g.L, n_sg, corr.p, corr.ld, post);
    else
        k_bp_post<NU_LOAD><<<grid, block, 0, c.stream>>>(S, g.L, n_sg, corr.p, corr.ld, post);
    return after_launch(c);
}

}  // namespace tc3d
