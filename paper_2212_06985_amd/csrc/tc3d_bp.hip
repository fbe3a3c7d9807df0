// FP32 belief propagation on the Tanner graph of the 3D toric code's Z checks
// (Section 4.1: LLR definition, factor-to-variable rule, variable-to-factor
// rule, posterior), flooding schedule, with the measurement-error variables
// folded into a constant factor K = 1 - 2q of every check product.
//
// Messages are kept in multiplicative form: the state between iterations is
// b = e^nu for every factor-to-variable message nu. Then
//   * the posterior e^l of an edge is e^{l0} times the product of its four
//     incoming b (E4), and the variable-to-factor message e^mu towards one
//     check is e^{l0} times the product of the other three (E3);
//   * with a = e^mu, tanh(mu/2) = (a - 1)/(a + 1), so the check rule E2 for
//     member k is b_k = (D_k + sK N_k) / (D_k - sK N_k), where N_k and D_k are
//     the products of (a - 1) and (a + 1) over the other three members and
//     sK = (-1)^s K (because e^{2 atanh y} = (1 + y)/(1 - y));
//   * the hard decision l < 0 is e^l < 1.
// An iteration therefore needs one reciprocal per message and no exp or log.
// e^mu is clamped to [e^-20, e^20], where tanh(mu/2) is already +-1 in FP32.
//
// Layout: FP32 [W][L^3][12][64]: the messages of one 64-shot word are
// contiguous, row (w L^3 + v) 12 + 4n + k = message of face f(v,n) to its
// member k for the 64 shots of word w. A wavefront (64 lanes = the 64 shots
// of one word at one site) reads and writes 256 contiguous bytes per row and
// a site's rows are adjacent, so the accesses of a word spread over every L2
// and HBM channel. Each access is a wave-uniform site base (scalar
// registers) plus a per-lane row offset held in vector registers; neighbour
// sites are v plus per-axis steps with the periodic wrap folded in.
//
// Per-edge priors (the learned prior) cost loads, not arithmetic: the check
// rules of a site need the priors of its own three edges and of six edges of
// its neighbours. Inside a whole decode the prior of edge e(v,a) is therefore
// folded into one message that site v stores (slot 8 for a = x, 10 for y, 6
// for z): the neighbours read that message anyway, and only the check that
// excludes it needs the prior by itself, from its own site. The one-step
// entry point keeps the plain state.
//
// One iteration is one kernel: a wavefront owns site v and its three faces.
// The inputs of its 12 check-member messages need 6 of its own messages and
// 24 messages of neighbouring sites; those come from L2 because each XCD
// walks one shot word at a time through tile columns (T x T sites in x-y, z
// running slowest inside the column; T = L by default, i.e. plain memory
// order), with the message stores streaming past L2 so that the rows loaded
// for neighbours stay resident.
#include <atomic>

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

// Site order of one shot word: tile columns of TX x TY sites, z outermost
// inside a column, x fastest. Sites outside the lattice (when a tile edge
// does not divide L) are skipped. Logical indices stay below 2^31 (checked
// on launch).
struct Tiling {
    int L, TX, TY, nTX, nTY;
    uint32_t per_word;          // nTX * nTY * TX * TY * L logical sites
    FastDiv n_sg;               // site groups of kWaves per word
    FastDiv col, plane, row, tiles_x;  // TX*TY*L, TX*TY, TX, nTX
    uint32_t xq, xr;            // grid size G: G / 8 and G % 8 (blocks per XCD)
};

// The grid of a launch over nw words (set before the launch).
int64_t set_grid(Tiling& tl, int64_t nw) {
    const int64_t blocks = (int64_t)tl.n_sg.d * nw;
    tl.xq = (uint32_t)(blocks >> 3);
    tl.xr = (uint32_t)(blocks & 7);
    return blocks;
}

struct Src {
    const float* __restrict__ nu;    // NU_LOAD
    const uint64_t* __restrict__ syn;
    int64_t ld_syn;
    const float* __restrict__ llr0;  // nullptr: scalar prior
    float a0;          // e^{l0} of the scalar prior
    float b1, b1_inv;  // e^{+-nu1}
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
    // hardware block b -> logical block: the blocks each XCD runs (b % 8) are
    // a contiguous range (the 32-bit form of xcd_block, grid from the host)
    const uint32_t b = blockIdx.x, j = b & 7, bi = b >> 3;
    const uint32_t lb = j < tl.xr ? j * (tl.xq + 1) + bi : tl.xr + j * tl.xq + bi;
    const uint32_t w = div_of(lb, tl.n_sg);
    const uint32_t sg = lb - w * tl.n_sg.d;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    it.w = w;
    it.lane = (int)(threadIdx.x & 63);
    const uint32_t i = sg * kWaves + wave;
    // tile columns (a uniform branch: whole planes need no tile index)
    uint32_t tile = 0, r = i, tx = 0, ty = 0;
    if (tl.nTX * tl.nTY != 1) {
        tile = div_of(i, tl.col);
        r = i - tile * tl.col.d;
        ty = div_of(tile, tl.tiles_x);
        tx = tile - ty * tl.tiles_x.d;
    }
    const uint32_t z = div_of(r, tl.plane);
    const uint32_t r2 = r - z * tl.plane.d;
    const uint32_t yy = div_of(r2, tl.row), xx = r2 - yy * tl.row.d;
    it.z = (int)z;
    it.x = (int)(tx * tl.TX + xx);
    it.y = (int)(ty * tl.TY + yy);
    it.ok = i < tl.per_word && it.x < tl.L && it.y < tl.L;
    it.v = it.ok ? site_of(it.x, it.y, it.z, tl.L) : 0;
    return it;
}

// Bit `lane` of a 64-shot syndrome word, read as the 32-bit half that holds
// it. The address differs between the two halves of the wavefront, so this is
// a vector load: those return in order and can all be in flight together,
// while scalar loads of a whole word return out of order and make the wave
// wait for each batch in turn.
__device__ __forceinline__ uint32_t shot_bit(const uint64_t* word, int lane) {
    const uint32_t h = reinterpret_cast<const uint32_t*>(word)[lane >> 5];
    return (h >> (lane & 31)) & 1u;
}

// Reads of one shot word: a wave-uniform site base plus a per-lane offset.
template <int MODE>
struct Reader {
    const char* __restrict__ base;  // (char*)(nu + 64 w) (NU_LOAD)
    const uint64_t* __restrict__ syn_w;  // syndrome plane + word w (NU_SIGMA)
    int64_t ld_syn, face_plane, w, site_bytes;
    uint32_t voff[12];  // byte offset of row `slot` for this lane
    int N, lane;
    float b1, b1_inv;  // e^{+-nu1}: first-iteration messages (NU_SIGMA)

    // e^nu of the old message of face f(site, slot / 4) to member slot % 4
    __device__ __forceinline__ float operator()(int slot, int site) const {
        if constexpr (MODE == NU_ZERO) {
            return 1.0f;
        } else if constexpr (MODE == NU_SIGMA) {
            return shot_bit(syn_w + (slot >> 2) * face_plane + (int64_t)site * ld_syn, lane)
                       ? b1_inv : b1;
        } else {
            const char* sb = base + (int64_t)site * site_bytes;
            return *reinterpret_cast<const float*>(sb + voff[slot]);
        }
    }
};

// First float of word w in an [W][rows][64] array.
__device__ __forceinline__ int64_t word_base(int64_t w, int64_t rows) { return w * rows * 64; }

template <int MODE>
__device__ __forceinline__ Reader<MODE> reader_of(const Src& S, const Item& it) {
    Reader<MODE> R;
    R.base = S.nu ? reinterpret_cast<const char*>(S.nu + word_base(it.w, 12 * (int64_t)S.N))
                  : nullptr;
    R.syn_w = S.syn + it.w;
    R.ld_syn = S.ld_syn;
    R.face_plane = (int64_t)S.N * S.ld_syn;
    R.w = it.w;
    R.site_bytes = 12 * 64 * 4;
#pragma unroll
    for (int k = 0; k < 12; ++k) R.voff[k] = (uint32_t)((k * 64 + it.lane) * 4);
    R.N = S.N;
    R.lane = it.lane;
    R.b1 = S.b1;
    R.b1_inv = S.b1_inv;
    return R;
}

// e^{l0} of edge e(site, c); per-edge priors are clamped to +-40 nats.
template <bool EDGE_PRIOR>
__device__ __forceinline__ float prior(const Src& S, const Item& it, int c, int site) {
    if constexpr (!EDGE_PRIOR) return S.a0;
    const float* row =
        S.llr0 + word_base(it.w, 3 * (int64_t)S.N) + ((int64_t)c * S.N + site) * 64;
    const float l = fminf(fmaxf(row[it.lane], -40.0f), 40.0f);
    return __builtin_amdgcn_exp2f(l * 1.4426950408889634f);
}

// The check rule E2 of one face in multiplicative form: a[k] = e^{mu_k} of
// its four members (clamped), out[k] = e^{nu_k} of the new messages.
__device__ __forceinline__ void check_rule(const float a_in[4], float sK, float out[4]) {
    float am[4], ap[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float a = fminf(fmaxf(a_in[k], 2.0611536e-9f), 4.85165195e8f);  // e^-+20
        am[k] = a - 1.0f;
        ap[k] = a + 1.0f;
    }
    const float sn01 = sK * (am[0] * am[1]), sn23 = sK * (am[2] * am[3]);
    const float d01 = ap[0] * ap[1], d23 = ap[2] * ap[3];
    float Nk[4], Dk[4];
    Nk[0] = am[1] * sn23; Dk[0] = ap[1] * d23;
    Nk[1] = am[0] * sn23; Dk[1] = ap[0] * d23;
    Nk[2] = am[3] * sn01; Dk[2] = ap[3] * d01;
    Nk[3] = am[2] * sn01; Dk[3] = ap[2] * d01;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = (Dk[k] + Nk[k]) * __builtin_amdgcn_rcpf(Dk[k] - Nk[k]);
}

// |l| < 1e-3 for the posterior e^l: e^-0.001 < e^l < e^0.001.
__device__ __forceinline__ bool near_tie(float el) {
    return el > 0.99900050f && el < 1.00100050f;
}

// Damping (DAMP): nu = (1 - g) nu_new + g nu_old, i.e. e^nu =
// (e^nu_new)^(1 - g) (e^nu_old)^g, formed with the hardware's base-2 log and
// exp. Only with the scalar prior.
__device__ __forceinline__ float damped(float b_new, float b_old, float g) {
    return __builtin_amdgcn_exp2f((1.0f - g) * __builtin_amdgcn_logf(b_new) +
                                  g * __builtin_amdgcn_logf(b_old));
}

// Sites v + (dx, dy, dz), -2 <= d <= 1, as index and as byte offset of the
// site's message rows inside one shot word (12 rows of 256 B). The wrapped
// coordinates and their scaled forms are formed once per wavefront, so a
// site costs two scalar adds per form.
struct Site {
    int v;
    uint32_t off;
};

struct Pos {
    int xs[4], ys[4], zs[4];        // wrapped coordinate c + d at [d + 2]
    int yl[4], zl[4];               // L y', L^2 z'
    uint32_t xo[4], yo[4], zo[4];   // byte offsets 3072 x', 3072 L y', 3072 L^2 z'
    __device__ __forceinline__ Site at(int dx, int dy, int dz) const {
        return Site{xs[dx + 2] + yl[dy + 2] + zl[dz + 2], xo[dx + 2] + yo[dy + 2] + zo[dz + 2]};
    }
};

// Sites v + (dx, dy, dz), |d| <= 1, for one site: v's index and row offset
// plus, per axis, the step to the previous and the next site with the
// periodic wrap folded in (offsets modulo 2^32).
struct Steps {
    int v;
    uint32_t off;
    int di[3][3];         // index step, [axis][d + 1]
    uint32_t doff[3][3];  // 3072 x the index step
    __device__ __forceinline__ Site at(int dx, int dy, int dz) const {
        return Site{v + di[0][dx + 1] + di[1][dy + 1] + di[2][dz + 1],
                    off + doff[0][dx + 1] + doff[1][dy + 1] + doff[2][dz + 1]};
    }
};

__device__ __forceinline__ Steps steps_of(const Item& it, int L) {
    Steps s;
    const int c[3] = {it.x, it.y, it.z};
    int stride = 1;
    s.v = it.v;
    s.off = 3072u * (uint32_t)it.v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.di[a][0] = c[a] == 0 ? (L - 1) * stride : -stride;
        s.di[a][1] = 0;
        s.di[a][2] = c[a] == L - 1 ? (1 - L) * stride : stride;
#pragma unroll
        for (int d = 0; d < 3; ++d) s.doff[a][d] = 3072u * (uint32_t)s.di[a][d];
        stride *= L;
    }
    return s;
}

__device__ __forceinline__ int wrap(int t, int L) { return t < 0 ? t + L : (t >= L ? t - L : t); }

__device__ __forceinline__ Pos pos_of_xy(int x, int y, int L) {
    Pos p;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        p.xs[d] = wrap(x + d - 2, L);
        p.ys[d] = wrap(y + d - 2, L);
        p.yl[d] = L * p.ys[d];
        p.xo[d] = 3072u * (uint32_t)p.xs[d];
        p.yo[d] = 3072u * (uint32_t)p.yl[d];
    }
    return p;
}

__device__ __forceinline__ void set_z(Pos& p, int z, int L) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        p.zs[d] = wrap(z + d - 2, L);
        p.zl[d] = L * L * p.zs[d];
        p.zo[d] = 3072u * (uint32_t)p.zl[d];
    }
}

// Message loads of one shot word by the site's 32-bit byte offset inside the
// word (L^3 * 3072 < 2^32, i.e. L <= 111): a 64-bit word base plus the offset
// (one 64-bit scalar add per site), the lane's offset in a vector register and
// the slot's row. Buffer loads with the site's offset as their scalar offset
// need fewer scalar instructions but ran 1% slower.
struct OffReader {
    const char* base;
    uint32_t lane4;
    __device__ __forceinline__ float operator()(int slot, const Site& s) const {
        return *reinterpret_cast<const float*>(base + s.off + lane4 + slot * 256);
    }
};

// The reader by site index: 64-bit site addresses (NU_LOAD) or the first
// iteration's messages from the syndrome (NU_SIGMA).
template <int MODE>
struct IdxReader {
    Reader<MODE> R;
    __device__ __forceinline__ float operator()(int slot, const Site& s) const {
        return R(slot, s.v);
    }
};

// One site of one iteration: its three faces' check rules (E2) from the
// incoming messages (E3), stored through W. LOC locates the neighbouring
// sites (Steps or Pos), R reads the old state.
// FOLD: 0 plain state in and out; 1 plain in, folded out (the first
// iteration of a decode with per-edge priors); 2 folded in and out.
template <int MODE, bool EP, int FOLD, bool DAMP, class LOC, class RD, class WR>
__device__ __forceinline__ void iter_site(const Src& S, const Item& it, const LOC& p, const RD& R,
                                          const WR& W, float K, float g) {
    const Site v = p.at(0, 0, 0);
    const Site xm = p.at(-1, 0, 0), xp = p.at(1, 0, 0), ym = p.at(0, -1, 0),
               yp = p.at(0, 1, 0), zm = p.at(0, 0, -1), zp = p.at(0, 0, 1);
    const Site yp_zm = p.at(0, 1, -1), zp_ym = p.at(0, -1, 1), xp_zm = p.at(1, 0, -1),
               zp_xm = p.at(-1, 0, 1), xp_ym = p.at(1, -1, 0), yp_xm = p.at(-1, 1, 0);
    // syndrome bits of the three faces of v (read first, with the messages)
    uint32_t sbit[3];
#pragma unroll
    for (int n = 0; n < 3; ++n)
        sbit[n] = shot_bit(S.syn + ((int64_t)n * S.N + v.v) * S.ld_syn + it.w, it.lane);
    // own messages to the members k = 0, 2 of each face (the others are the
    // excluded message of the member-k check and are not needed)
    const float o0 = R(0, v), o2 = R(2, v), o4 = R(4, v), o6 = R(6, v), o8 = R(8, v),
                o10 = R(10, v);
    // e^{l0} of the three edges at v, and the two incoming messages from
    // faces of other sites for each of them (each is a member of two of v's faces)
    const float ex = prior<EP>(S, it, 0, v.v), ey = prior<EP>(S, it, 1, v.v),
                ez = prior<EP>(S, it, 2, v.v);
    const float fx = R(9, ym) * R(5, zm);
    const float fy = R(11, xm) * R(1, zm);
    const float fz = R(7, xm) * R(3, ym);
    const float px = ex * fx, py = ey * fy, pz = ez * fz;
    // e^{mu} of the six edges that are a member of one face of v
    float a_x_yp, a_x_zp, a_y_xp, a_y_zp, a_z_xp, a_z_yp;
    if constexpr (FOLD == 2) {  // slots 8, 10, 6 of each site carry its edges' priors
        a_x_yp = R(8, yp) * R(4, yp) * R(5, yp_zm);
        a_x_zp = R(8, zp) * R(4, zp) * R(9, zp_ym);
        a_y_xp = R(10, xp) * R(0, xp) * R(1, xp_zm);
        a_y_zp = R(10, zp) * R(0, zp) * R(11, zp_xm);
        a_z_xp = R(6, xp) * R(2, xp) * R(3, xp_ym);
        a_z_yp = R(6, yp) * R(2, yp) * R(7, yp_xm);
    } else {
        a_x_yp = prior<EP>(S, it, 0, yp.v) * R(8, yp) * R(4, yp) * R(5, yp_zm);
        a_x_zp = prior<EP>(S, it, 0, zp.v) * R(8, zp) * R(4, zp) * R(9, zp_ym);
        a_y_xp = prior<EP>(S, it, 1, xp.v) * R(10, xp) * R(0, xp) * R(1, xp_zm);
        a_y_zp = prior<EP>(S, it, 1, zp.v) * R(10, zp) * R(0, zp) * R(11, zp_xm);
        a_z_xp = prior<EP>(S, it, 2, xp.v) * R(6, xp) * R(2, xp) * R(3, xp_ym);
        a_z_yp = prior<EP>(S, it, 2, yp.v) * R(6, yp) * R(2, yp) * R(7, yp_xm);
    }
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        float a[4];
        if (n == 2) {  // normal z: e(v,x), e(v+y,x), e(v,y), e(v+x,y)
            a[0] = px * o4; a[1] = a_x_yp; a[2] = py * o0; a[3] = a_y_xp;
        } else if (n == 1) {  // normal y: e(v,x), e(v+z,x), e(v,z), e(v+x,z)
            a[0] = FOLD == 2 ? fx * o8 : px * o8; a[1] = a_x_zp; a[2] = pz * o2;
            a[3] = a_z_xp;
        } else {  // normal x: e(v,y), e(v+z,y), e(v,z), e(v+y,z)
            a[0] = FOLD == 2 ? fy * o10 : py * o10; a[1] = a_y_zp;
            a[2] = FOLD == 2 ? fz * o6 : pz * o6; a[3] = a_z_yp;
        }
        const float sK = sbit[n] ? -K : K;
        float out[4];
        check_rule(a, sK, out);
        if constexpr (DAMP) {
#pragma unroll
            for (int k = 0; k < 4; ++k) out[k] = damped(out[k], R(4 * n + k, v), g);
        }
        if constexpr (FOLD != 0) {  // slots 8, 10, 6 carry the priors of e(v,x), e(v,y), e(v,z)
            if (n == 2) {
                out[0] *= ex;
                out[2] *= ey;
            } else if (n == 1) {
                out[2] *= ez;
            }
        }
        // streaming stores: the new messages are read again only in the next
        // iteration, so they should not evict the neighbour rows from L2
#pragma unroll
        for (int k = 0; k < 4; ++k) W(out[k], 4 * n + k, v);
    }
}

// Stores by 64-bit site address.
struct PtrWriter {
    char* base;  // (char*)(b_out + 64 * 12 N w)
    uint32_t lane4;
    __device__ __forceinline__ void operator()(float x, int slot, const Site& s) const {
        __builtin_nontemporal_store(
            x, reinterpret_cast<float*>(base + (int64_t)s.v * 3072 + lane4 + slot * 256));
    }
};

template <int MODE, bool EP, int FOLD, bool DAMP = false>
__global__ __launch_bounds__(kBlock) void k_bp_iter(Src S, Tiling tl, float K, float g,
                                                    float* __restrict__ b_out) {
    static_assert(FOLD == 0 || EP, "only per-edge priors are folded");
    static_assert(!DAMP || (!EP && FOLD == 0), "damping goes with the scalar prior");
    const Item it = item_of(tl);
    if (!it.ok) return;
    const Steps p = steps_of(it, tl.L);
    const PtrWriter W{reinterpret_cast<char*>(b_out + word_base(it.w, 12 * (int64_t)S.N)),
                      (uint32_t)it.lane * 4u};
    const IdxReader<MODE> R{reader_of<MODE>(S, it)};
    iter_site<MODE, EP, FOLD, DAMP>(S, it, p, R, W, K, g);
}

template <int MODE, bool EP, bool FOLDED>
__global__ __launch_bounds__(kBlock) void k_bp_post(Src S, Tiling tl,
                                                    uint64_t* __restrict__ corr, int64_t ld_c,
                                                    float* __restrict__ post,
                                                    unsigned long long* __restrict__ ties) {
    const Item it = item_of(tl);
    if (!it.ok) return;
    const IdxReader<MODE> R{reader_of<MODE>(S, it)};
    const Steps p = steps_of(it, tl.L);
    const Site sv = p.at(0, 0, 0), xm = p.at(-1, 0, 0), ym = p.at(0, -1, 0), zm = p.at(0, 0, -1);
    const int v = it.v;
    // e^l = e^{l0} times the four incoming messages (E4); in a folded state
    // slots 8, 10, 6 already carry the factor e^{l0}
    const float ex = FOLDED ? 1.0f : prior<EP>(S, it, 0, v);
    const float ey = FOLDED ? 1.0f : prior<EP>(S, it, 1, v);
    const float ez = FOLDED ? 1.0f : prior<EP>(S, it, 2, v);
    float el[3];
    el[0] = ex * R(8, sv) * R(4, sv) * R(9, ym) * R(5, zm);
    el[1] = ey * R(10, sv) * R(0, sv) * R(11, xm) * R(1, zm);
    el[2] = ez * R(6, sv) * R(2, sv) * R(7, xm) * R(3, ym);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = (int64_t)c * S.N + v;
        if (post) {
            float* row = post + word_base(it.w, 3 * (int64_t)S.N) + e * 64;
            row[it.lane] = 0.69314718055994531f * __builtin_amdgcn_logf(el[c]);
        }
        const uint64_t flips = __ballot(el[c] < 1.0f);
        if (corr && it.lane == 0) corr[e * ld_c + it.w] = flips;
    }
    if (ties) {  // posteriors within 1e-3 nats of the decision boundary
        int n = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) n += __popcll(__ballot(near_tie(el[c])));
        if (n && it.lane == 0) atomicAdd(ties, (unsigned long long)n);
    }
}

// ------------------------------------------- last iteration with the posterior
// The decision after iteration T needs, for each edge of site v, only the four
// messages that iteration sends into the edge (E4): from two faces of v and
// from one face each of v - unit(d) for the two other axes d. So iteration T
// and the posterior can be one pass over the state of iteration T - 1: a
// wavefront evaluates the check rule of v's three faces and, for the single
// member it needs, of the six faces f(v-x, 1), f(v-x, 2), f(v-y, 0),
// f(v-y, 2), f(v-z, 0), f(v-z, 1), each with its inputs formed by the same
// products in the same order as k_bp_iter forms them at the face's own site.
// The decision and posterior are bit-identical to k_bp_iter followed by
// k_bp_post, while iteration T's messages (16 B per edge and shot) are
// neither written nor read back; the price is about twice the loads, which
// L2 serves, and the check rules of the neighbouring faces. Undamped; per-edge
// priors in the folded form of a whole decode.

// e^{mu} of the four members of face f(u, n), u = v + (ox, oy, oz), as
// k_bp_iter forms them at u: with the scalar prior a0 = e^{l0} (EP false),
// or (EP) from a folded state, where slots 8, 10, 6 carry the per-edge priors
// and only the products px, py, pz need a prior of u's own edges.
template <bool EP, class RD>
__device__ __forceinline__ void face_inputs(const RD& R, const Src& S, const Item& it,
                                            const Pos& p, int ox, int oy, int oz, int n,
                                            float a[4]) {
    const float a0 = S.a0;
    const Site u = p.at(ox, oy, oz);
    const Site u_xm = p.at(ox - 1, oy, oz), u_ym = p.at(ox, oy - 1, oz),
               u_zm = p.at(ox, oy, oz - 1);
    // the products of the two incoming messages from faces of other sites
    const float fx = R(9, u_ym) * R(5, u_zm);
    const float fy = R(11, u_xm) * R(1, u_zm);
    const float fz = R(7, u_xm) * R(3, u_ym);
    if (n == 2) {  // members e(u,x), e(u+y,x), e(u,y), e(u+x,y)
        const Site u_yp = p.at(ox, oy + 1, oz), u_xp = p.at(ox + 1, oy, oz);
        const Site u_yp_zm = p.at(ox, oy + 1, oz - 1), u_xp_zm = p.at(ox + 1, oy, oz - 1);
        if constexpr (EP) {
            a[0] = (prior<true>(S, it, 0, u.v) * fx) * R(4, u);
            a[1] = R(8, u_yp) * R(4, u_yp) * R(5, u_yp_zm);
            a[2] = (prior<true>(S, it, 1, u.v) * fy) * R(0, u);
            a[3] = R(10, u_xp) * R(0, u_xp) * R(1, u_xp_zm);
        } else {
            a[0] = (a0 * fx) * R(4, u);
            a[1] = a0 * R(8, u_yp) * R(4, u_yp) * R(5, u_yp_zm);
            a[2] = (a0 * fy) * R(0, u);
            a[3] = a0 * R(10, u_xp) * R(0, u_xp) * R(1, u_xp_zm);
        }
    } else if (n == 1) {  // members e(u,x), e(u+z,x), e(u,z), e(u+x,z)
        const Site u_zp = p.at(ox, oy, oz + 1), u_xp = p.at(ox + 1, oy, oz);
        const Site u_zp_ym = p.at(ox, oy - 1, oz + 1), u_xp_ym = p.at(ox + 1, oy - 1, oz);
        if constexpr (EP) {
            a[0] = fx * R(8, u);
            a[1] = R(8, u_zp) * R(4, u_zp) * R(9, u_zp_ym);
            a[2] = (prior<true>(S, it, 2, u.v) * fz) * R(2, u);
            a[3] = R(6, u_xp) * R(2, u_xp) * R(3, u_xp_ym);
        } else {
            a[0] = (a0 * fx) * R(8, u);
            a[1] = a0 * R(8, u_zp) * R(4, u_zp) * R(9, u_zp_ym);
            a[2] = (a0 * fz) * R(2, u);
            a[3] = a0 * R(6, u_xp) * R(2, u_xp) * R(3, u_xp_ym);
        }
    } else {  // members e(u,y), e(u+z,y), e(u,z), e(u+y,z)
        const Site u_zp = p.at(ox, oy, oz + 1), u_yp = p.at(ox, oy + 1, oz);
        const Site u_zp_xm = p.at(ox - 1, oy, oz + 1), u_yp_xm = p.at(ox - 1, oy + 1, oz);
        if constexpr (EP) {
            a[0] = fy * R(10, u);
            a[1] = R(10, u_zp) * R(0, u_zp) * R(11, u_zp_xm);
            a[2] = fz * R(6, u);
            a[3] = R(6, u_yp) * R(2, u_yp) * R(7, u_yp_xm);
        } else {
            a[0] = (a0 * fy) * R(10, u);
            a[1] = a0 * R(10, u_zp) * R(0, u_zp) * R(11, u_zp_xm);
            a[2] = (a0 * fz) * R(6, u);
            a[3] = a0 * R(6, u_yp) * R(2, u_yp) * R(7, u_yp_xm);
        }
    }
}

// New messages of face f(u, n) (the caller keeps the members it needs).
template <bool EP, class RD>
__device__ __forceinline__ void face_messages(const RD& R, const Src& S, const Item& it,
                                              const uint64_t* syn_w, const Pos& p, float K,
                                              int ox, int oy, int oz, int n, float out[4]) {
    float a[4];
    face_inputs<EP>(R, S, it, p, ox, oy, oz, n, a);
    const Site u = p.at(ox, oy, oz);
    const uint32_t s = shot_bit(syn_w + ((int64_t)n * S.N + u.v) * S.ld_syn, it.lane);
    check_rule(a, s ? -K : K, out);
}

// A wavefront walks ZR consecutive planes of one (x, y) column: the messages
// of f(v-z, 0) and f(v-z, 1) that a site needs are those its predecessor in
// the column computed for its own faces, so only the first site of the run
// recomputes them, and the column's addresses change by one plane per step.
// Item z indexes the runs (ceil(L / ZR) per column).
// EP: the state is folded (per-edge priors); the new messages that a folded
// state keeps with their edge's prior (slots 8, 10, 6) enter the posterior
// with it, as k_bp_post<.., true, true> reads them.
// OFF: stored messages read by 32-bit offsets inside a word (L <= 111), else
// by 64-bit site addresses.
template <int MODE, int ZR, bool EP, bool OFF>
__global__ __launch_bounds__(kBlock) void k_bp_final(Src S, Tiling tl, float K,
                                                     uint64_t* __restrict__ corr, int64_t ld_c,
                                                     float* __restrict__ post,
                                                     unsigned long long* __restrict__ ties) {
    const Item it = item_of(tl);
    if (!it.ok) return;
    const int L = tl.L;
    const int z0 = it.z * ZR;
    Pos p = pos_of_xy(it.x, it.y, L);
    const uint64_t* syn_w = S.syn + it.w;
    const float a0 = S.a0;
    int n_ties = 0;
    auto walk = [&](const auto& R) {
        float t[4];
        set_z(p, z0, L);
        face_messages<EP>(R, S, it, syn_w, p, K, 0, 0, -1, 0, t);
        float zc0 = t[1];  // message of f(v-z, 0) to e(v, y)
        face_messages<EP>(R, S, it, syn_w, p, K, 0, 0, -1, 1, t);
        float zc1 = t[1];  // message of f(v-z, 1) to e(v, x)
#pragma unroll 1
        for (int z = z0; z < z0 + ZR && z < L; ++z) {
            if (z != z0) set_z(p, z, L);
            float f0[4], f1[4], f2[4], xm1[4], xm2[4], ym0[4], ym2[4];
            face_messages<EP>(R, S, it, syn_w, p, K, 0, 0, 0, 0, f0);
            face_messages<EP>(R, S, it, syn_w, p, K, 0, 0, 0, 1, f1);
            face_messages<EP>(R, S, it, syn_w, p, K, 0, 0, 0, 2, f2);
            face_messages<EP>(R, S, it, syn_w, p, K, -1, 0, 0, 1, xm1);
            face_messages<EP>(R, S, it, syn_w, p, K, -1, 0, 0, 2, xm2);
            face_messages<EP>(R, S, it, syn_w, p, K, 0, -1, 0, 0, ym0);
            face_messages<EP>(R, S, it, syn_w, p, K, 0, -1, 0, 2, ym2);
            // the products k_bp_post forms from the stored slots 8 4 | 9 5,
            // 10 0 | 11 1 and 6 2 | 7 3
            const int v = p.at(0, 0, 0).v;
            float el[3];
            if constexpr (EP) {  // slots 8, 10, 6 folded with their edge's prior
                el[0] = 1.0f * (f2[0] * prior<true>(S, it, 0, v)) * f1[0] * ym2[1] * zc1;
                el[1] = 1.0f * (f2[2] * prior<true>(S, it, 1, v)) * f0[0] * xm2[3] * zc0;
                el[2] = 1.0f * (f1[2] * prior<true>(S, it, 2, v)) * f0[2] * xm1[3] * ym0[3];
            } else {
                el[0] = a0 * f2[0] * f1[0] * ym2[1] * zc1;
                el[1] = a0 * f2[2] * f0[0] * xm2[3] * zc0;
                el[2] = a0 * f1[2] * f0[2] * xm1[3] * ym0[3];
            }
            zc0 = f0[1];
            zc1 = f1[1];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int64_t e = (int64_t)c * S.N + v;
                if (post) {
                    float* row = post + word_base(it.w, 3 * (int64_t)S.N) + e * 64;
                    row[it.lane] = 0.69314718055994531f * __builtin_amdgcn_logf(el[c]);
                }
                const uint64_t flips = __ballot(el[c] < 1.0f);
                if (corr && it.lane == 0) corr[e * ld_c + it.w] = flips;
                if (ties) n_ties += __popcll(__ballot(near_tie(el[c])));
            }
        }
    };
    if constexpr (MODE == NU_LOAD && OFF) {
        const OffReader R{reinterpret_cast<const char*>(S.nu + word_base(it.w, 12 * (int64_t)S.N)),
                          (uint32_t)it.lane * 4u};
        walk(R);
    } else {
        IdxReader<MODE> R{reader_of<MODE>(S, it)};
        walk(R);
    }
    if (ties && n_ties && it.lane == 0) atomicAdd(ties, (unsigned long long)n_ties);
}

// ---------------------------------------------- one shot per workgroup in LDS
// On small lattices the whole message state of one shot, 12 FP32 per site,
// fits a CU's LDS (83 KB at L = 12, 132 KB at L = 14). A workgroup then runs
// a whole decode for one shot: the first iteration's messages from the
// syndrome, iterations 2 .. T and the posterior, with HBM traffic only for the
// syndrome bits in and the correction bits out. Each thread owns sites
// t, t + 1024, t + 2048 (SPT of them) and evaluates exactly the expressions of
// k_bp_iter and k_bp_post, in the same order, so the decode is bit-identical
// to the streaming kernels; the state is laid out [slot][site], so that the
// lanes of a wavefront read consecutive words.
constexpr int kLdsThreads = 1024;
constexpr int kLdsMaxSites = 3 * kLdsThreads;  // L <= 14

template <int SPT>
__global__ __launch_bounds__(kLdsThreads) void k_bp_lds(
    const uint64_t* __restrict__ syn, int64_t ld_syn, int L, float a0, float b1, float b1_inv,
    float K, int more_iters, uint64_t* __restrict__ corr, int64_t ld_c, float* __restrict__ post,
    unsigned long long* __restrict__ ties) {
    extern __shared__ float m[];  // [12][N]
    const int N = L * L * L;
    const int64_t w = blockIdx.x >> 6;
    const int bit = (int)(blockIdx.x & 63);
    const int t = (int)threadIdx.x;
    int xyz[SPT];
    uint32_t sbit[SPT][3];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int v = t + k * kLdsThreads;
        xyz[k] = -1;
        if (v < N) {
            const int x = v % L, y = (v / L) % L, z = v / (L * L);
            xyz[k] = x | (y << 8) | (z << 16);
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                sbit[k][n] = (uint32_t)(syn[((int64_t)n * N + v) * ld_syn + w] >> bit) & 1u;
                // the first iteration's messages, implied by the check's syndrome bit
                const float b = sbit[k][n] ? b1_inv : b1;
#pragma unroll
                for (int j = 0; j < 4; ++j) m[(4 * n + j) * N + v] = b;
            }
        }
    }
    __syncthreads();
    auto R = [&](int slot, int site) { return m[slot * N + site]; };
    for (int it = 0; it < more_iters; ++it) {
        float out[SPT][12];
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            if (xyz[k] < 0) continue;
            const int x = xyz[k] & 255, y = (xyz[k] >> 8) & 255, z = xyz[k] >> 16;
            const int xm = dec(x, L), xp = inc(x, L), ym = dec(y, L), yp = inc(y, L);
            const int zm = dec(z, L), zp = inc(z, L);
            const int v = site_of(x, y, z, L);
            const int s_xm = site_of(xm, y, z, L), s_xp = site_of(xp, y, z, L);
            const int s_ym = site_of(x, ym, z, L), s_yp = site_of(x, yp, z, L);
            const int s_zm = site_of(x, y, zm, L), s_zp = site_of(x, y, zp, L);
            const float o0 = R(0, v), o2 = R(2, v), o4 = R(4, v), o6 = R(6, v), o8 = R(8, v),
                        o10 = R(10, v);
            const float fx = R(9, s_ym) * R(5, s_zm);
            const float fy = R(11, s_xm) * R(1, s_zm);
            const float fz = R(7, s_xm) * R(3, s_ym);
            const float px = a0 * fx, py = a0 * fy, pz = a0 * fz;
            const float a_x_yp = a0 * R(8, s_yp) * R(4, s_yp) * R(5, site_of(x, yp, zm, L));
            const float a_x_zp = a0 * R(8, s_zp) * R(4, s_zp) * R(9, site_of(x, ym, zp, L));
            const float a_y_xp = a0 * R(10, s_xp) * R(0, s_xp) * R(1, site_of(xp, y, zm, L));
            const float a_y_zp = a0 * R(10, s_zp) * R(0, s_zp) * R(11, site_of(xm, y, zp, L));
            const float a_z_xp = a0 * R(6, s_xp) * R(2, s_xp) * R(3, site_of(xp, ym, z, L));
            const float a_z_yp = a0 * R(6, s_yp) * R(2, s_yp) * R(7, site_of(xm, yp, z, L));
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                float a[4];
                if (n == 2) {
                    a[0] = px * o4; a[1] = a_x_yp; a[2] = py * o0; a[3] = a_y_xp;
                } else if (n == 1) {
                    a[0] = px * o8; a[1] = a_x_zp; a[2] = pz * o2; a[3] = a_z_xp;
                } else {
                    a[0] = py * o10; a[1] = a_y_zp; a[2] = pz * o6; a[3] = a_z_yp;
                }
                const float sK = sbit[k][n] ? -K : K;
                check_rule(a, sK, &out[k][4 * n]);
            }
        }
        __syncthreads();  // every read of the old state is done
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            if (xyz[k] < 0) continue;
            const int v = t + k * kLdsThreads;
#pragma unroll
            for (int slot = 0; slot < 12; ++slot) m[slot * N + v] = out[k][slot];
        }
        __syncthreads();  // the new state is complete
    }
    // posterior and hard decision (E4), as k_bp_post
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        if (xyz[k] < 0) continue;
        const int x = xyz[k] & 255, y = (xyz[k] >> 8) & 255, z = xyz[k] >> 16;
        const int v = site_of(x, y, z, L);
        const int s_xm = site_of(dec(x, L), y, z, L), s_ym = site_of(x, dec(y, L), z, L);
        const int s_zm = site_of(x, y, dec(z, L), L);
        float el[3];
        el[0] = a0 * R(8, v) * R(4, v) * R(9, s_ym) * R(5, s_zm);
        el[1] = a0 * R(10, v) * R(0, v) * R(11, s_xm) * R(1, s_zm);
        el[2] = a0 * R(6, v) * R(2, v) * R(7, s_xm) * R(3, s_ym);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t e = (int64_t)c * N + v;
            if (post)
                post[(w * 3 * (int64_t)N + e) * 64 + bit] =
                    0.69314718055994531f * __builtin_amdgcn_logf(el[c]);
            if (el[c] < 1.0f) atomicOr((unsigned long long*)(corr + e * ld_c + w), 1ull << bit);
            if (ties && near_tie(el[c])) atomicAdd(ties, 1ull);
        }
    }
}

Src make_src(Geo g, const BpArgs& a, const float* nu) {
    Src S;
    S.nu = nu;
    S.syn = a.syn.p;
    S.ld_syn = a.syn.ld;
    S.llr0 = a.llr0;
    S.a0 = a.a0;
    S.b1 = a.b1;
    S.b1_inv = a.b1_inv;
    S.N = g.N;
    S.s_pad = a.s_pad;
    return S;
}

// Tile of the traversal. req = 0: the library's choice, whole x-y planes in
// memory order up to L = 64 and bands of 8 rows above; req > 0: req x req
// columns; req < 0: bands of whole x rows, -req rows high. Smaller tiles and
// bands shorten the z reuse distance (one tile plane instead of a whole
// plane); bands keep whole x rows, i.e. long contiguous DRAM runs. Up to
// L = 64 the rows a plane traversal re-reads are still in the Infinity Cache
// when they are needed again; from L = 72 they are not, and bands of 8 rows
// made the iteration 5% (L = 72) to 18% (L = 128) faster.
constexpr int kBandMinL = 72, kBandRows = 8;

void tile_of(int L, int req, int* tx, int* ty) {
    if (req == 0 && L >= kBandMinL) req = -kBandRows;
    const int r = req < 0 ? -req : req;
    const int t = r < L ? r : L;
    *tx = req > 0 ? t : L;
    *ty = req != 0 ? t : L;
}

// Returns false when the launch's logical indices would not fit 31 bits.
bool tiling_of(Geo g, const BpArgs& a, Tiling* out) {
    Tiling tl;
    tl.L = g.L;
    tile_of(g.L, a.tile, &tl.TX, &tl.TY);
    tl.nTX = (g.L + tl.TX - 1) / tl.TX;
    tl.nTY = (g.L + tl.TY - 1) / tl.TY;
    const int64_t per_word = (int64_t)tl.nTX * tl.nTY * tl.TX * tl.TY * g.L;
    const int64_t n_sg = (per_word + kWaves - 1) / kWaves;
    if (n_sg * a.nw > 0x7fffffff || per_word + kWaves > 0x7fffffff) return false;
    tl.per_word = (uint32_t)per_word;
    tl.n_sg = fastdiv((uint32_t)n_sg);
    tl.col = fastdiv((uint32_t)(tl.TX * tl.TY * g.L));
    tl.plane = fastdiv((uint32_t)(tl.TX * tl.TY));
    tl.row = fastdiv((uint32_t)tl.TX);
    tl.tiles_x = fastdiv((uint32_t)tl.nTX);
    *out = tl;
    return true;
}

}  // namespace

// Residency of the kernels that read stored messages. The iterations run
// faster with four workgroups (16 wavefronts) per CU than with the 32
// wavefronts their registers allow: 4.08 instead of 4.19 ms at L = 48 (2048
// shots) and 1.92 instead of 2.03 ms at L = 12 (65,536 shots), measured in one
// run; three or five per CU are between. The posterior is fastest with six
// (2.14 instead of 2.20 ms at L = 48). The cap is dynamic LDS that the kernel
// does not touch: just over 1/(n+1) of the CU's LDS per workgroup, so n fit
// and n + 1 do not. 0 (no cap) when the device cannot be queried.
static constexpr int kLoadIterBlocksPerCu = 4;
static constexpr int kLoadPostBlocksPerCu = 6;
static constexpr int kLoadFinalBlocksPerCu = 4;  // 3, 5, 6 and uncapped measured slower
static std::atomic<int> g_cu_lds[64];

static size_t residency_lds(int blocks_per_cu) {
    if (blocks_per_cu >= 8) return 0;  // no cap: the registers allow 8
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int per_cu = g_cu_lds[dev].load(std::memory_order_relaxed);
    if (per_cu == 0) {
        if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                  dev) != hipSuccess ||
            per_cu < 4096)
            return 0;
        g_cu_lds[dev].store(per_cu, std::memory_order_relaxed);
    }
    int b = per_cu / (blocks_per_cu + 1) + 1024;  // > 1/(n+1) of the CU
    if (b > per_cu / blocks_per_cu) b = per_cu / blocks_per_cu;  // <= 1/n
    return (size_t)b;
}

namespace {
template <int MODE, bool EP, int FOLD, bool DAMP = false>
void iter_kernel(dim3 grid, size_t lds, hipStream_t st, const Src& S, const Tiling& tl, float K,
                 float damp, float* out) {
    k_bp_iter<MODE, EP, FOLD, DAMP><<<grid, dim3(kBlock), lds, st>>>(S, tl, K, damp, out);
}
}  // namespace

// One word of messages addressable with 32-bit offsets (L <= 111).
static bool word_fits_32(Geo g) { return (int64_t)g.N * 3072 < ((int64_t)1 << 32); }

int launch_bp_iter(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu_in,
                   float* nu_out, int kclass) {
    if (a.nw == 0) return TC3D_OK;
    Tiling tl;
    if (!tiling_of(g, a, &tl)) return TC3D_EINVAL;
    const int64_t blocks = set_grid(tl, a.nw);
    int rc = before_launch(c, kclass);
    if (rc) return rc;
    const Src S = make_src(g, a, nu_in);
    const dim3 grid((unsigned)blocks);
    const size_t lds =
        mode == NU_LOAD ? residency_lds(a.occupancy ? a.occupancy : kLoadIterBlocksPerCu) : 0;
    const float damp = a.damp;
    const hipStream_t st = c.stream;
    const float K = a.K;
    if (a.llr0) {
        if (damp != 0.0f) return TC3D_EINVAL;  // damping goes with the scalar prior
        if (mode == NU_ZERO && a.fold)
            iter_kernel<NU_ZERO, true, 1>(grid, 0, st, S, tl, K, damp, nu_out);
        else if (mode == NU_ZERO)
            iter_kernel<NU_ZERO, true, 0>(grid, 0, st, S, tl, K, damp, nu_out);
        else if (mode == NU_LOAD && a.fold)
            iter_kernel<NU_LOAD, true, 2>(grid, lds, st, S, tl, K, damp, nu_out);
        else if (mode == NU_LOAD)
            iter_kernel<NU_LOAD, true, 0>(grid, lds, st, S, tl, K, damp, nu_out);
        else
            return TC3D_EINVAL;  // the syndrome-implied first state needs a scalar prior
    } else if (damp != 0.0f) {
        if (mode == NU_ZERO)
            iter_kernel<NU_ZERO, false, 0, true>(grid, 0, st, S, tl, K, damp, nu_out);
        else if (mode == NU_SIGMA)
            iter_kernel<NU_SIGMA, false, 0, true>(grid, 0, st, S, tl, K, damp, nu_out);
        else
            iter_kernel<NU_LOAD, false, 0, true>(grid, lds, st, S, tl, K, damp, nu_out);
    } else {
        if (mode == NU_ZERO)
            iter_kernel<NU_ZERO, false, 0>(grid, 0, st, S, tl, K, damp, nu_out);
        else if (mode == NU_SIGMA)
            iter_kernel<NU_SIGMA, false, 0>(grid, 0, st, S, tl, K, damp, nu_out);
        else
            iter_kernel<NU_LOAD, false, 0>(grid, lds, st, S, tl, K, damp, nu_out);
    }
    return after_launch(c);
}

bool bp_final_fits(Geo g, const BpArgs& a) {
    // undamped, per-edge priors folded into the state
    (void)g;
    return (!a.llr0 || a.fold) && a.damp == 0.0f;
}

// Planes each wavefront of the fused last iteration walks (1, 2, 4 and 16
// measured slower at L = 48; unrolling the walk by 2 too).
static constexpr int kFinalRun = 8;

namespace {
// Work items of k_bp_final: (x, y, run of zr planes) per word, x fastest.
bool final_tiling(Geo g, int64_t nw, int zr, Tiling* out) {
    Tiling tl;
    const int L = g.L;
    const int64_t runs = (L + zr - 1) / zr;
    const int64_t per_word = (int64_t)L * L * runs;
    const int64_t n_sg = (per_word + kWaves - 1) / kWaves;
    if (n_sg * nw > 0x7fffffff || per_word + kWaves > 0x7fffffff) return false;
    tl.L = L;
    tl.TX = tl.TY = L;
    tl.nTX = tl.nTY = 1;
    tl.per_word = (uint32_t)per_word;
    tl.n_sg = fastdiv((uint32_t)n_sg);
    tl.col = fastdiv((uint32_t)per_word);
    tl.plane = fastdiv((uint32_t)(L * L));
    tl.row = fastdiv((uint32_t)L);
    tl.tiles_x = fastdiv(1u);
    *out = tl;
    return true;
}
}  // namespace

int launch_bp_final(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu, Plane corr,
                    float* post) {
    if (!bp_final_fits(g, a)) return TC3D_EINVAL;
    if (a.nw == 0) return TC3D_OK;
    Tiling tl;
    if (!final_tiling(g, a.nw, kFinalRun, &tl)) return TC3D_EINVAL;
    const int64_t blocks = set_grid(tl, a.nw);
    int rc = before_launch(c, TC3D_K_BP_POST);
    if (rc) return rc;
    const Src S = make_src(g, a, nu);
    const dim3 grid((unsigned)blocks), block(kBlock);
    const size_t lds =
        mode == NU_LOAD ? residency_lds(a.occupancy ? a.occupancy : kLoadFinalBlocksPerCu) : 0;
    const bool off = word_fits_32(g);
    if (a.llr0 && mode == NU_LOAD && off)
        k_bp_final<NU_LOAD, kFinalRun, true, true>
            <<<grid, block, lds, c.stream>>>(S, tl, a.K, corr.p, corr.ld, post, a.ties);
    else if (a.llr0 && mode == NU_LOAD)
        k_bp_final<NU_LOAD, kFinalRun, true, false>
            <<<grid, block, lds, c.stream>>>(S, tl, a.K, corr.p, corr.ld, post, a.ties);
    else if (a.llr0)
        return TC3D_EINVAL;  // a folded state is always stored
    else if (mode == NU_SIGMA)
        k_bp_final<NU_SIGMA, kFinalRun, false, false>
            <<<grid, block, 0, c.stream>>>(S, tl, a.K, corr.p, corr.ld, post, a.ties);
    else if (mode == NU_LOAD && off)
        k_bp_final<NU_LOAD, kFinalRun, false, true>
            <<<grid, block, lds, c.stream>>>(S, tl, a.K, corr.p, corr.ld, post, a.ties);
    else if (mode == NU_LOAD)
        k_bp_final<NU_LOAD, kFinalRun, false, false>
            <<<grid, block, lds, c.stream>>>(S, tl, a.K, corr.p, corr.ld, post, a.ties);
    else
        return TC3D_EINVAL;
    return after_launch(c);
}

bool bp_resident_fits(Geo g, const float* llr0, int64_t nw) {
    return !llr0 && g.N <= kLdsMaxSites && nw > 0 && nw <= (int64_t)1 << 24;
}

bool bp_resident_used(Geo g, const BpArgs& a) {
    return (a.path == TC3D_BP_AUTO || a.path == TC3D_BP_RESIDENT) && a.damp == 0.0f &&
           bp_resident_fits(g, a.llr0, a.nw);
}

static std::atomic<int> g_lds_opted[64];  // 1: the kernels may use their LDS size there

int bp_resident_prepare() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return TC3D_EHIP;
    if (g_lds_opted[dev].load(std::memory_order_relaxed)) return TC3D_OK;
    const int bytes = (int)(12 * kLdsMaxSites * sizeof(float));
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bp_lds<1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bp_lds<2>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bp_lds<3>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
        return TC3D_EHIP;
    g_lds_opted[dev].store(1, std::memory_order_relaxed);
    return TC3D_OK;
}

namespace {
template <int SPT>
int launch_lds(const Ctx& c, Geo g, const BpArgs& a, int32_t iters, Plane corr, float* post) {
    const size_t lds = (size_t)12 * g.N * sizeof(float);
    int rc = bp_resident_prepare();
    if (rc) return rc;
    rc = launch_clear(c, corr, 3 * (int64_t)g.N, a.nw);
    if (rc) return rc;
    rc = before_launch(c, TC3D_K_BP_ITER);
    if (rc) return rc;
    k_bp_lds<SPT><<<dim3((unsigned)(64 * a.nw)), dim3(kLdsThreads), lds, c.stream>>>(
        a.syn.p, a.syn.ld, g.L, a.a0, a.b1, a.b1_inv, a.K, iters - 1, corr.p, corr.ld, post,
        a.ties);
    return after_launch(c);
}
}  // namespace

int launch_bp_resident(const Ctx& c, Geo g, const BpArgs& a, int32_t iters, Plane corr,
                       float* post) {
    if (!bp_resident_fits(g, a.llr0, a.nw) || iters < 1) return TC3D_EINVAL;
    const int spt = (g.N + kLdsThreads - 1) / kLdsThreads;
    if (spt == 1) return launch_lds<1>(c, g, a, iters, corr, post);
    if (spt == 2) return launch_lds<2>(c, g, a, iters, corr, post);
    return launch_lds<3>(c, g, a, iters, corr, post);
}

int launch_bp_post(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu, Plane corr,
                   float* post) {
    if (a.nw == 0) return TC3D_OK;
    Tiling tl;
    if (!tiling_of(g, a, &tl)) return TC3D_EINVAL;
    const int64_t blocks = set_grid(tl, a.nw);
    int rc = before_launch(c, TC3D_K_BP_POST);
    if (rc) return rc;
    const Src S = make_src(g, a, nu);
    const dim3 grid((unsigned)blocks), block(kBlock);
    const size_t lds = mode == NU_LOAD ? residency_lds(kLoadPostBlocksPerCu) : 0;
    unsigned long long* ties = a.ties;
    if (a.llr0) {
        if (mode != NU_LOAD) return TC3D_EINVAL;  // a posterior follows a stored iteration
        if (a.fold)
            k_bp_post<NU_LOAD, true, true>
                <<<grid, block, lds, c.stream>>>(S, tl, corr.p, corr.ld, post, ties);
        else
            k_bp_post<NU_LOAD, true, false>
                <<<grid, block, lds, c.stream>>>(S, tl, corr.p, corr.ld, post, ties);
    } else {
        if (mode == NU_SIGMA)
            k_bp_post<NU_SIGMA, false, false>
                <<<grid, block, 0, c.stream>>>(S, tl, corr.p, corr.ld, post, ties);
        else if (mode == NU_LOAD)
            k_bp_post<NU_LOAD, false, false>
                <<<grid, block, lds, c.stream>>>(S, tl, corr.p, corr.ld, post, ties);
        else
            return TC3D_EINVAL;
    }
    return after_launch(c);
}

}  // namespace tc3d
