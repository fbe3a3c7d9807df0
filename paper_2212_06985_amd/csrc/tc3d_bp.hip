// FP32 belief propagation on the Tanner graph of the 3D toric code's Z checks
// (Section 4.1: LLR definition, factor-to-variable rule, variable-to-factor
// rule, posterior), flooding schedule, with the measurement-error variables
// folded into a constant factor K = 1 - 2q of every check product.
//
// State between iterations is only the factor-to-variable messages nu, FP32,
// [L^3][12][S_pad] with row 12 v + 4n + k = message of face f(v,n) to its
// member k; the shot index is the fastest dimension, so a wavefront (64 lanes
// = 64 consecutive shots of one site) reads and writes 256 contiguous bytes
// per message row, and the 12 rows of a site are S_pad floats apart. Each
// access is a wave-uniform 64-bit site base (scalar registers) plus a 32-bit
// per-lane offset for the row, kept in 12 vector registers.
//
// One iteration is one kernel: a wavefront owns site v and its three faces.
// It rebuilds the posterior l of the 9 edges its faces touch from the old
// messages (E4: l = l0 + sum of the 4 incoming messages), forms the
// variable-to-factor messages mu = l - nu_old (E3 written as a difference),
// and writes the new messages of its faces (E2). The posterior needs 24
// messages of neighbouring sites; those come from L2 because each XCD walks
// one shot word at a time through tile columns (T x T sites in x-y, z running
// slowest inside the column), which keeps every neighbour within T*T sites of
// the wavefront that first loaded it.
#include "tc3d_device.hpp"
#include "tc3d_internal.hpp"

namespace tc3d {

namespace {

constexpr int kWaves = 4;  // sites per workgroup, one wavefront each
constexpr int kBlock = 64 * kWaves;

// Division of a non-negative n < 2^31 by an invariant d >= 1 with one
// multiply-high and a shift (Granlund and Montgomery, "Division by invariant
// integers using multiplication", PLDI 1994): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, n / d = (mulhi(m, n) + n) >> l.
struct FastDiv {
    uint32_t d, m, l;
};

FastDiv fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    f.l = 0;
    while ((1ull << f.l) < d) ++f.l;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << f.l) - d)) / d + 1);
    return f;
}

__device__ __forceinline__ uint32_t div_of(uint32_t n, const FastDiv& f) {
    const uint32_t t = __umulhi(n, f.m);
    return (uint32_t)(((uint64_t)t + n) >> f.l);
}

// Site order of one shot word: tile columns of T x T sites, z outermost
// inside a column, x fastest. Sites outside the lattice (when T does not
// divide L) are skipped. Logical indices stay below 2^31 (checked on launch).
struct Tiling {
    int L, T, nT;
    uint32_t per_word;          // nT * nT * T * T * L logical sites
    FastDiv n_sg;               // site groups of kWaves per word
    FastDiv col, plane, row, tiles_x;  // T*T*L, T*T, T, nT
};

struct Src {
    const float* __restrict__ nu;    // NU_LOAD
    const uint64_t* __restrict__ syn;
    int64_t ld_syn;
    const float* __restrict__ llr0;  // nullptr: scalar prior
    float l0, nu1;
    int N;
    int64_t s_pad;
};

struct Item {
    bool ok;
    int x, y, z, v;
    int64_t w;  // word of the batch
    int lane;
};

__device__ __forceinline__ Item item_of(const Tiling& tl) {
    Item it;
    const uint32_t lb = (uint32_t)xcd_block(blockIdx.x, gridDim.x);
    const uint32_t w = div_of(lb, tl.n_sg);
    const uint32_t sg = lb - w * tl.n_sg.d;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    it.w = w;
    it.lane = (int)(threadIdx.x & 63);
    const uint32_t i = sg * kWaves + wave;
    const uint32_t tile = div_of(i, tl.col);
    const uint32_t r = i - tile * tl.col.d;
    const uint32_t z = div_of(r, tl.plane);
    const uint32_t r2 = r - z * tl.plane.d;
    const uint32_t yy = div_of(r2, tl.row), xx = r2 - yy * tl.row.d;
    const uint32_t ty = div_of(tile, tl.tiles_x), tx = tile - ty * tl.tiles_x.d;
    it.z = (int)z;
    it.x = (int)(tx * tl.T + xx);
    it.y = (int)(ty * tl.T + yy);
    it.ok = i < tl.per_word && it.x < tl.L && it.y < tl.L;
    it.v = it.ok ? site_of(it.x, it.y, it.z, tl.L) : 0;
    return it;
}

// Reads of one shot word: a wave-uniform site base plus a per-lane offset.
template <int MODE>
struct Reader {
    const char* __restrict__ base;  // (char*)(nu + 64 w) (NU_LOAD)
    const uint64_t* __restrict__ syn;
    int64_t ld_syn, w, site_bytes;
    uint32_t voff[12];  // byte offset of row `slot` for this lane
    int N, lane;
    float nu1;

    // old message of face f(site, slot / 4) to member slot % 4
    __device__ __forceinline__ float operator()(int slot, int site) const {
        if constexpr (MODE == NU_ZERO) {
            return 0.0f;
        } else if constexpr (MODE == NU_SIGMA) {
            const uint64_t word = syn[((int64_t)(slot >> 2) * N + site) * ld_syn + w];
            return ((word >> lane) & 1u) ? -nu1 : nu1;
        } else {
            const char* sb = base + (int64_t)site * site_bytes;
            return *reinterpret_cast<const float*>(sb + voff[slot]);
        }
    }
};

template <int MODE>
__device__ __forceinline__ Reader<MODE> reader_of(const Src& S, const Item& it) {
    Reader<MODE> R;
    R.base = S.nu ? reinterpret_cast<const char*>(S.nu + it.w * 64) : nullptr;
    R.syn = S.syn;
    R.ld_syn = S.ld_syn;
    R.w = it.w;
    R.site_bytes = 12 * S.s_pad * 4;
#pragma unroll
    for (int k = 0; k < 12; ++k) R.voff[k] = (uint32_t)((k * S.s_pad + it.lane) * 4);
    R.N = S.N;
    R.lane = it.lane;
    R.nu1 = S.nu1;
    return R;
}

__device__ __forceinline__ float prior(const Src& S, const Item& it, int c, int site) {
    if (!S.llr0) return S.l0;
    const float* row = S.llr0 + ((int64_t)c * S.N + site) * S.s_pad + it.w * 64;
    return row[it.lane];
}

// Neighbour sites of v = (x,y,z) by offset.
struct Nbr {
    int xm, xp, ym, yp, zm, zp;                    // v -/+ unit
    int yp_zm, zp_ym, xp_zm, zp_xm, xp_ym, yp_xm;  // diagonal
};

__device__ __forceinline__ Nbr neighbours(const Item& it, int L) {
    const int x = it.x, y = it.y, z = it.z;
    const int xm = dec(x, L), xp = inc(x, L), ym = dec(y, L), yp = inc(y, L);
    const int zm = dec(z, L), zp = inc(z, L);
    Nbr n;
    n.xm = site_of(xm, y, z, L);
    n.xp = site_of(xp, y, z, L);
    n.ym = site_of(x, ym, z, L);
    n.yp = site_of(x, yp, z, L);
    n.zm = site_of(x, y, zm, L);
    n.zp = site_of(x, y, zp, L);
    n.yp_zm = site_of(x, yp, zm, L);
    n.zp_ym = site_of(x, ym, zp, L);
    n.xp_zm = site_of(xp, y, zm, L);
    n.zp_xm = site_of(xm, y, zp, L);
    n.xp_ym = site_of(xp, ym, z, L);
    n.yp_xm = site_of(xm, yp, z, L);
    return n;
}

// The check rule E2 for one face from its four member posteriors lm and old
// messages own: with a_k = e^{mu_k}, tanh(mu_k/2) = (a_k - 1)/(a_k + 1), so
// the product over the other three members is N_k / D_k with N_k, D_k the
// leave-one-out products of (a-1) and (a+1), and
//   2 atanh(sK N_k / D_k) = ln((D_k + sK N_k) / (D_k - sK N_k)).
// mu is clamped to +-20, where tanh(mu/2) already equals +-1 in FP32.
__device__ __forceinline__ void check_rule(const float lm[4], const float own[4], float sK,
                                           float out[4]) {
    float am[4], ap[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float mu = fminf(fmaxf(lm[k] - own[k], -20.0f), 20.0f);
        const float a = __builtin_amdgcn_exp2f(mu * 1.4426950408889634f);
        am[k] = a - 1.0f;
        ap[k] = a + 1.0f;
    }
    const float n01 = am[0] * am[1], n23 = am[2] * am[3];
    const float d01 = ap[0] * ap[1], d23 = ap[2] * ap[3];
    const float sn01 = sK * n01, sn23 = sK * n23;
    float Nk[4], Dk[4];
    Nk[0] = am[1] * sn23; Dk[0] = ap[1] * d23;
    Nk[1] = am[0] * sn23; Dk[1] = ap[0] * d23;
    Nk[2] = am[3] * sn01; Dk[2] = ap[3] * d01;
    Nk[3] = am[2] * sn01; Dk[3] = ap[2] * d01;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float r = (Dk[k] + Nk[k]) * __builtin_amdgcn_rcpf(Dk[k] - Nk[k]);
        out[k] = 0.69314718055994531f * __builtin_amdgcn_logf(r);
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_bp_iter(Src S, Tiling tl, float K,
                                                    float* __restrict__ nu_out) {
    const Item it = item_of(tl);
    if (!it.ok) return;
    const int L = tl.L;
    const Reader<MODE> R = reader_of<MODE>(S, it);
    const Nbr nb = neighbours(it, L);
    const int v = it.v;
    float own[12];
#pragma unroll
    for (int s = 0; s < 12; ++s) own[s] = R(s, v);
    // posteriors (E4) of the 9 edges touched by the faces of v
    const float lx = prior(S, it, 0, v) + own[8] + own[4] + R(9, nb.ym) + R(5, nb.zm);
    const float ly = prior(S, it, 1, v) + own[10] + own[0] + R(11, nb.xm) + R(1, nb.zm);
    const float lz = prior(S, it, 2, v) + own[6] + own[2] + R(7, nb.xm) + R(3, nb.ym);
    const float lx_yp =
        prior(S, it, 0, nb.yp) + R(8, nb.yp) + R(4, nb.yp) + own[9] + R(5, nb.yp_zm);
    const float lx_zp =
        prior(S, it, 0, nb.zp) + R(8, nb.zp) + R(4, nb.zp) + R(9, nb.zp_ym) + own[5];
    const float ly_xp =
        prior(S, it, 1, nb.xp) + R(10, nb.xp) + R(0, nb.xp) + own[11] + R(1, nb.xp_zm);
    const float ly_zp =
        prior(S, it, 1, nb.zp) + R(10, nb.zp) + R(0, nb.zp) + R(11, nb.zp_xm) + own[1];
    const float lz_xp =
        prior(S, it, 2, nb.xp) + R(6, nb.xp) + R(2, nb.xp) + own[7] + R(3, nb.xp_ym);
    const float lz_yp =
        prior(S, it, 2, nb.yp) + R(6, nb.yp) + R(2, nb.yp) + R(7, nb.yp_xm) + own[3];
    char* outb = reinterpret_cast<char*>(nu_out + it.w * 64) + (int64_t)v * R.site_bytes;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        float lm[4];
        if (n == 2) {  // normal z, spans x, y
            lm[0] = lx; lm[1] = lx_yp; lm[2] = ly; lm[3] = ly_xp;
        } else if (n == 1) {  // normal y, spans x, z
            lm[0] = lx; lm[1] = lx_zp; lm[2] = lz; lm[3] = lz_xp;
        } else {  // normal x, spans y, z
            lm[0] = ly; lm[1] = ly_zp; lm[2] = lz; lm[3] = lz_yp;
        }
        const uint64_t sw = S.syn[((int64_t)n * S.N + v) * S.ld_syn + it.w];
        const float sK = ((sw >> it.lane) & 1u) ? -K : K;
        float out[4];
        check_rule(lm, own + 4 * n, sK, out);
#pragma unroll
        for (int k = 0; k < 4; ++k) *reinterpret_cast<float*>(outb + R.voff[4 * n + k]) = out[k];
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_bp_post(Src S, Tiling tl,
                                                    uint64_t* __restrict__ corr, int64_t ld_c,
                                                    float* __restrict__ post) {
    const Item it = item_of(tl);
    if (!it.ok) return;
    const Reader<MODE> R = reader_of<MODE>(S, it);
    const Nbr nb = neighbours(it, tl.L);
    const int v = it.v;
    float l[3];
    l[0] = prior(S, it, 0, v) + R(8, v) + R(4, v) + R(9, nb.ym) + R(5, nb.zm);
    l[1] = prior(S, it, 1, v) + R(10, v) + R(0, v) + R(11, nb.xm) + R(1, nb.zm);
    l[2] = prior(S, it, 2, v) + R(6, v) + R(2, v) + R(7, nb.xm) + R(3, nb.ym);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = (int64_t)c * S.N + v;
        if (post) {
            float* row = post + e * S.s_pad + it.w * 64;
            row[it.lane] = l[c];
        }
        const uint64_t flips = __ballot(l[c] < 0.0f);
        if (corr && it.lane == 0) corr[e * ld_c + it.w] = flips;
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
    return S;
}

// Tile edge: the request if given, else L up to 16, else the largest divisor
// of L in [8, 16], else 16 with the overhanging sites skipped.
int tile_of(int L, int req) {
    if (req > 0) return req < L ? req : L;
    if (L <= 16) return L;
    for (int t = 16; t >= 8; --t)
        if (L % t == 0) return t;
    return 16;
}

// Returns false when the launch's logical indices would not fit 31 bits.
bool tiling_of(Geo g, const BpArgs& a, Tiling* out) {
    Tiling tl;
    tl.L = g.L;
    tl.T = tile_of(g.L, a.tile);
    tl.nT = (g.L + tl.T - 1) / tl.T;
    const int64_t per_word = (int64_t)tl.nT * tl.nT * tl.T * tl.T * g.L;
    const int64_t n_sg = (per_word + kWaves - 1) / kWaves;
    if (n_sg * a.nw > 0x7fffffff || per_word + kWaves > 0x7fffffff) return false;
    tl.per_word = (uint32_t)per_word;
    tl.n_sg = fastdiv((uint32_t)n_sg);
    tl.col = fastdiv((uint32_t)(tl.T * tl.T * g.L));
    tl.plane = fastdiv((uint32_t)(tl.T * tl.T));
    tl.row = fastdiv((uint32_t)tl.T);
    tl.tiles_x = fastdiv((uint32_t)tl.nT);
    *out = tl;
    return true;
}

}  // namespace

int launch_bp_iter(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu_in,
                   float* nu_out, int kclass) {
    if (a.nw == 0) return TC3D_OK;
    Tiling tl;
    if (!tiling_of(g, a, &tl)) return TC3D_EINVAL;
    const int64_t blocks = (int64_t)tl.n_sg.d * a.nw;
    int rc = before_launch(c, kclass);
    if (rc) return rc;
    const Src S = make_src(g, a, nu_in);
    const dim3 grid((unsigned)blocks), block(kBlock);
    if (mode == NU_ZERO)
        k_bp_iter<NU_ZERO><<<grid, block, 0, c.stream>>>(S, tl, a.K, nu_out);
    else if (mode == NU_SIGMA)
        k_bp_iter<NU_SIGMA><<<grid, block, 0, c.stream>>>(S, tl, a.K, nu_out);
    else
        k_bp_iter<NU_LOAD><<<grid, block, 0, c.stream>>>(S, tl, a.K, nu_out);
    return after_launch(c);
}

int launch_bp_post(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu, Plane corr,
                   float* post) {
    if (a.nw == 0) return TC3D_OK;
    Tiling tl;
    if (!tiling_of(g, a, &tl)) return TC3D_EINVAL;
    const int64_t blocks = (int64_t)tl.n_sg.d * a.nw;
    int rc = before_launch(c, TC3D_K_BP_POST);
    if (rc) return rc;
    const Src S = make_src(g, a, nu);
    const dim3 grid((unsigned)blocks), block(kBlock);
    if (mode == NU_ZERO)
        k_bp_post<NU_ZERO><<<grid, block, 0, c.stream>>>(S, tl, corr.p, corr.ld, post);
    else if (mode == NU_SIGMA)
        k_bp_post<NU_SIGMA><<<grid, block, 0, c.stream>>>(S, tl, corr.p, corr.ld, post);
    else
        k_bp_post<NU_LOAD><<<grid, block, 0, c.stream>>>(S, tl, corr.p, corr.ld, post);
    return after_launch(c);
}

}  // namespace tc3d
