// Belief propagation with meta-check factors: the extension of the check
// factor graph that Section 4.1 describes and leaves out (and that the
// closing discussion names as a likely improvement). Besides the qubits and
// the Z checks the graph has
//   * one measurement-error variable m_f per check f (prior lm = ln((1-q)/q)),
//     a member of its check and of the two cubes that contain f;
//   * one meta-check per cube: the six measurement variables of its faces
//     must have the parity mu_c of the six measured outcomes (a valid
//     syndrome is closed, so every cube's true parity is even).
// Messages, flooding schedule (variable-to-factor ones clamped to +-30 nats:
// the cube loops feed back and the messages grow without bound):
//   qubit e -> check f   Q   = l0 + the other three checks' nu
//   m_f -> check f       M   = lm + kappa from both cubes of f
//   m_f -> cube c        R   = lm + lambda_f + kappa from f's other cube
//   check f -> qubit e   nu  = (-1)^{s_f} 2 atanh(tanh(M/2) prod_{e' != e} tanh(Q/2))
//   check f -> m_f       lambda = (-1)^{s_f} 2 atanh(prod_e tanh(Q/2))
//   cube c -> m_f        kappa  = (-1)^{mu_c} 2 atanh(prod_{f' != f} tanh(R/2))
//   posterior            l_e = l0 + the four nu
// In FP64 and in multiplicative form (every message is kept as e^msg;
// tanh(x/2) = (e^x - 1)/(e^x + 1) and e^{2 atanh y} = (1 + y)/(1 - y)), so an
// iteration needs divisions only.
//
// State: FP64 [W][L^3][21][64], per site v and word w the 64 shots of
//   slots 0..11   e^nu of face f(v, s/4) to member s%4 (the member order of
//                 the plain BP kernel),
//   slots 12..14  e^lambda of face f(v, n),
//   slots 15..20  e^kappa of cube v to its face slot j: j = 2n the face
//                 f(v, n), j = 2n+1 the face f(v + unit(n), n).
// A wavefront is one site of one word (lane = shot).
#include "tc3d_device.hpp"
#include "tc3d_internal.hpp"

namespace tc3d {

namespace {

constexpr int kMetaWaves = 4;
constexpr int kMetaBlock = 64 * kMetaWaves;
constexpr int kSlots = 21;
constexpr double kLo = 9.357622968840175e-14;  // e^-30
constexpr double kHi = 1.0686474581524463e13;  // e^30

__device__ __forceinline__ double clampd(double a) { return fmin(fmax(a, kLo), kHi); }
// tanh(x/2) of a = e^x
__device__ __forceinline__ double th(double a) { return (a - 1.0) / (a + 1.0); }
// e^{2 atanh y}
__device__ __forceinline__ double ex(double y) { return (1.0 + y) / (1.0 - y); }

struct MetaSrc {
    const double* __restrict__ in;  // nullptr: first iteration (all factor messages 1)
    const uint64_t* __restrict__ syn;
    int64_t ld;
    int L, N;
    int64_t nw;
    double a0, am;  // e^{l0}, e^{lm}
};

struct MetaItem {
    bool ok;
    int x, y, z, v, lane;
    int64_t w;
};

__device__ __forceinline__ MetaItem meta_item(const MetaSrc& S) {
    MetaItem it;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = lb * kMetaWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    it.lane = (int)(threadIdx.x & 63);
    it.ok = i < S.nw * S.N;
    const int64_t ii = it.ok ? i : 0;
    it.w = ii / S.N;
    it.v = (int)(ii - it.w * S.N);
    it.x = it.v % S.L;
    it.y = (it.v / S.L) % S.L;
    it.z = it.v / (S.L * S.L);
    return it;
}

struct MetaReader {
    const double* __restrict__ base;  // in + word w
    int lane;
    __device__ __forceinline__ double operator()(int slot, int site) const {
        if (!base) return 1.0;
        return base[((int64_t)site * kSlots + slot) * 64 + lane];
    }
};

__device__ __forceinline__ int bit_of(const MetaSrc& S, const MetaItem& it, int n, int site) {
    return (int)((S.syn[((int64_t)n * S.N + site) * S.ld + it.w] >> it.lane) & 1u);
}

__global__ __launch_bounds__(kMetaBlock) void k_bp_meta_iter(MetaSrc S, double* __restrict__ out) {
    const MetaItem it = meta_item(S);
    if (!it.ok) return;
    const MetaReader R{S.in ? S.in + it.w * (int64_t)S.N * kSlots * 64 : nullptr, it.lane};
    const int L = S.L, v = it.v, x = it.x, y = it.y, z = it.z;
    const int xm = site_of(dec(x, L), y, z, L), xp = site_of(inc(x, L), y, z, L);
    const int ym = site_of(x, dec(y, L), z, L), yp = site_of(x, inc(y, L), z, L);
    const int zm = site_of(x, y, dec(z, L), L), zp = site_of(x, y, inc(z, L), L);
    const int yp_zm = site_of(x, inc(y, L), dec(z, L), L), zp_ym = site_of(x, dec(y, L), inc(z, L), L);
    const int xp_zm = site_of(inc(x, L), y, dec(z, L), L), zp_xm = site_of(dec(x, L), y, inc(z, L), L);
    const int xp_ym = site_of(inc(x, L), dec(y, L), z, L), yp_xm = site_of(dec(x, L), inc(y, L), z, L);
    const int nm[3] = {xm, ym, zm}, np[3] = {xp, yp, zp};

    // ---- qubit -> check, e^Q (E3), as in the plain kernel
    const double o0 = R(0, v), o2 = R(2, v), o4 = R(4, v), o6 = R(6, v), o8 = R(8, v),
                 o10 = R(10, v);
    const double px = S.a0 * R(9, ym) * R(5, zm);
    const double py = S.a0 * R(11, xm) * R(1, zm);
    const double pz = S.a0 * R(7, xm) * R(3, ym);
    const double a_x_yp = S.a0 * R(8, yp) * R(4, yp) * R(5, yp_zm);
    const double a_x_zp = S.a0 * R(8, zp) * R(4, zp) * R(9, zp_ym);
    const double a_y_xp = S.a0 * R(10, xp) * R(0, xp) * R(1, xp_zm);
    const double a_y_zp = S.a0 * R(10, zp) * R(0, zp) * R(11, zp_xm);
    const double a_z_xp = S.a0 * R(6, xp) * R(2, xp) * R(3, xp_ym);
    const double a_z_yp = S.a0 * R(6, yp) * R(2, yp) * R(7, yp_xm);

    double* ob = out + ((it.w * (int64_t)S.N + v) * kSlots) * 64 + it.lane;
    int s_own[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        double a[4];
        if (n == 2) {
            a[0] = px * o4; a[1] = a_x_yp; a[2] = py * o0; a[3] = a_y_xp;
        } else if (n == 1) {
            a[0] = px * o8; a[1] = a_x_zp; a[2] = pz * o2; a[3] = a_z_xp;
        } else {
            a[0] = py * o10; a[1] = a_y_zp; a[2] = pz * o6; a[3] = a_z_yp;
        }
        double t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = th(clampd(a[k]));
        s_own[n] = bit_of(S, it, n, v);
        const double sg = s_own[n] ? -1.0 : 1.0;
        // m_f -> check: lm + kappa of cube v (slot 2n) and of cube v - unit(n) (slot 2n+1)
        const double tm = th(clampd(S.am * R(15 + 2 * n, v) * R(16 + 2 * n, nm[n])));
        const double t01 = t[0] * t[1], t23 = t[2] * t[3];
        const double lo[4] = {t[1] * t23, t[0] * t23, t[3] * t01, t[2] * t01};
#pragma unroll
        for (int k = 0; k < 4; ++k) ob[(4 * n + k) * 64] = ex(sg * tm * lo[k]);
        ob[(12 + n) * 64] = ex(sg * t01 * t23);
    }

    // ---- cube v -> its six measurement variables
    double r[6];
    int par = 0;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        // lower face f(v,n): its other cube is v - unit(n) (slot 2n+1 there)
        r[2 * n] = th(clampd(S.am * R(12 + n, v) * R(16 + 2 * n, nm[n])));
        // upper face f(v+unit(n), n): its other cube is v + unit(n) (slot 2n there)
        r[2 * n + 1] = th(clampd(S.am * R(12 + n, np[n]) * R(15 + 2 * n, np[n])));
        par ^= s_own[n] ^ bit_of(S, it, n, np[n]);
    }
    const double sc = par ? -1.0 : 1.0;
    double pre[6], suf[6];
    pre[0] = 1.0;
#pragma unroll
    for (int j = 1; j < 6; ++j) pre[j] = pre[j - 1] * r[j - 1];
    suf[5] = 1.0;
#pragma unroll
    for (int j = 4; j >= 0; --j) suf[j] = suf[j + 1] * r[j + 1];
#pragma unroll
    for (int j = 0; j < 6; ++j) ob[(15 + j) * 64] = ex(sc * pre[j] * suf[j]);
}

// Posterior and hard decision from the last state (E4): e^l = e^{l0} times
// the four incoming e^nu; flip where e^l < 1. post: FP64 [W][3N][64] or null.
__global__ __launch_bounds__(kMetaBlock) void k_bp_meta_post(MetaSrc S,
                                                            uint64_t* __restrict__ corr,
                                                            int64_t ld_c,
                                                            double* __restrict__ post) {
    const MetaItem it = meta_item(S);
    if (!it.ok) return;
    const MetaReader R{S.in + it.w * (int64_t)S.N * kSlots * 64, it.lane};
    const int L = S.L, v = it.v, x = it.x, y = it.y, z = it.z;
    const int xm = site_of(dec(x, L), y, z, L), ym = site_of(x, dec(y, L), z, L),
              zm = site_of(x, y, dec(z, L), L);
    double el[3];
    el[0] = S.a0 * R(8, v) * R(4, v) * R(9, ym) * R(5, zm);
    el[1] = S.a0 * R(10, v) * R(0, v) * R(11, xm) * R(1, zm);
    el[2] = S.a0 * R(6, v) * R(2, v) * R(7, xm) * R(3, ym);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = (int64_t)c * S.N + v;
        if (post) post[(it.w * 3 * (int64_t)S.N + e) * 64 + it.lane] = log(el[c]);
        const uint64_t flips = __ballot(el[c] < 1.0);
        if (corr && it.lane == 0) corr[e * ld_c + it.w] = flips;
    }
}

MetaSrc meta_src(Geo g, CPlane syn, int64_t nw, double p_dec, double q_dec, const double* in) {
    MetaSrc S;
    S.in = in;
    S.syn = syn.p;
    S.ld = syn.ld;
    S.L = g.L;
    S.N = g.N;
    S.nw = nw;
    S.a0 = (1.0 - p_dec) / p_dec;
    S.am = (1.0 - q_dec) / q_dec;
    return S;
}

int64_t meta_blocks(Geo g, int64_t nw) { return (nw * g.N + kMetaWaves - 1) / kMetaWaves; }

}  // namespace

size_t bp_meta_state_bytes(Geo g, int64_t nw) { return (size_t)nw * g.N * kSlots * 64 * 8; }

int launch_bp_meta_iter(const Ctx& c, Geo g, CPlane syn, int64_t nw, double p_dec, double q_dec,
                        const double* in, double* out) {
    if (nw == 0) return TC3D_OK;
    int rc = before_launch(c, in ? TC3D_K_BP_ITER : TC3D_K_BP_FIRST);
    if (rc) return rc;
    const MetaSrc S = meta_src(g, syn, nw, p_dec, q_dec, in);
    k_bp_meta_iter<<<dim3((unsigned)meta_blocks(g, nw)), dim3(kMetaBlock), 0, c.stream>>>(S, out);
    return after_launch(c);
}

int launch_bp_meta_post(const Ctx& c, Geo g, CPlane syn, int64_t nw, double p_dec,
                        double q_dec, const double* state, Plane corr, double* post) {
    if (nw == 0) return TC3D_OK;
    int rc = before_launch(c, TC3D_K_BP_POST);
    if (rc) return rc;
    const MetaSrc S = meta_src(g, syn, nw, p_dec, q_dec, state);
    k_bp_meta_post<<<dim3((unsigned)meta_blocks(g, nw)), dim3(kMetaBlock), 0, c.stream>>>(
        S, corr.p, corr.ld, post);
    return after_launch(c);
}

int bp_meta_run(const Ctx& c, Geo g, CPlane syn, int64_t nw, double p_dec, double q_dec,
                int32_t iters, double* buf0, double* buf1, Plane corr, double* post) {
    double* bufs[2] = {buf0, buf1};
    const double* cur = nullptr;
    int nb = 0;
    for (int32_t i = 0; i < iters; ++i) {
        int rc = launch_bp_meta_iter(c, g, syn, nw, p_dec, q_dec, cur, bufs[nb]);
        if (rc) return rc;
        cur = bufs[nb];
        nb ^= 1;
    }
    return launch_bp_meta_post(c, g, syn, nw, p_dec, q_dec, cur, corr, post);
}

}  // namespace tc3d
