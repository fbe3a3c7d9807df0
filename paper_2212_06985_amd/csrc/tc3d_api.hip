// C ABI (include/tc3d.h): argument checks, workspace carving, the BP
// iteration schedule and the multi-cycle loop. Every step of the decoding
// path runs in the kernels of tc3d_bits.hip and tc3d_bp.hip.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <vector>

#include "tc3d_internal.hpp"

namespace tc3d {

// ------------------------------------------------------------------- timer
Timer::~Timer() {
    for (auto& s : slots_) {
        if (s.start) (void)hipEventDestroy(s.start);
        if (s.stop) (void)hipEventDestroy(s.stop);
    }
    if (first_) (void)hipEventDestroy(first_);
    if (last_) (void)hipEventDestroy(last_);
}

int Timer::drain(Slot& s) {
    if (!s.pending) return TC3D_OK;
    if (hipEventSynchronize(s.stop) != hipSuccess) return TC3D_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s.start, s.stop) != hipSuccess) return TC3D_EHIP;
    ms_[s.kclass] += ms;
    s.pending = false;
    return TC3D_OK;
}

int Timer::close() {
    if (!open_) return TC3D_OK;
    Slot& s = slots_[cur_];
    if (hipEventRecord(s.stop, stream_) != hipSuccess) return TC3D_EHIP;
    s.pending = true;
    open_ = false;
    return TC3D_OK;
}

int Timer::begin(int kclass) {
    constexpr size_t kSlots = 512;
    if (!first_) {
        if (hipEventCreate(&first_) != hipSuccess || hipEventCreate(&last_) != hipSuccess)
            return TC3D_EHIP;
        if (hipEventRecord(first_, stream_) != hipSuccess) return TC3D_EHIP;
    }
    launches_[kclass] += 1;
    if (open_ && slots_[cur_].kclass == kclass) return TC3D_OK;  // the run continues
    int rc = close();
    if (rc) return rc;
    if (slots_.size() < kSlots) {
        Slot s;
        if (hipEventCreate(&s.start) != hipSuccess || hipEventCreate(&s.stop) != hipSuccess)
            return TC3D_EHIP;
        slots_.push_back(s);
    }
    cur_ = (int)(next_ % slots_.size());
    next_++;
    Slot& s = slots_[cur_];
    rc = drain(s);  // reuse: wait for the interval recorded kSlots intervals ago
    if (rc) return rc;
    s.kclass = kclass;
    if (hipEventRecord(s.start, stream_) != hipSuccess) return TC3D_EHIP;
    open_ = true;
    return TC3D_OK;
}

int Timer::end() { return TC3D_OK; }

int Timer::finish(tc3d_timing* out) {
    int rc = close();
    if (rc) return rc;
    if (first_ && hipEventRecord(last_, stream_) != hipSuccess) return TC3D_EHIP;
    for (auto& s : slots_) {
        rc = drain(s);
        if (rc) return rc;
    }
    memset(out, 0, sizeof(*out));
    for (int k = 0; k < TC3D_K_COUNT; ++k) {
        out->ms[k] = ms_[k];
        out->launches[k] = launches_[k];
    }
    if (first_) {
        if (hipEventSynchronize(last_) != hipSuccess) return TC3D_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, first_, last_) != hipSuccess) return TC3D_EHIP;
        out->total_ms = ms;
    }
    return TC3D_OK;
}

int before_launch(const Ctx& c, int kclass) {
    return c.timer ? c.timer->begin(kclass) : TC3D_OK;
}

int after_launch(const Ctx& c) {
    if (hipGetLastError() != hipSuccess) return TC3D_EHIP;
    return c.timer ? c.timer->end() : TC3D_OK;
}

namespace {

constexpr int32_t kMaxL = 512;
constexpr int kMaxSweeps = 32;

bool lattice_ok(const tc3d_lattice* lat) {
    if (!lat || lat->L < 3 || lat->L > kMaxL) return false;
    const int64_t N = (int64_t)lat->L * lat->L * lat->L;
    return lat->n_sites == N && lat->n_edges == 3 * N && lat->n_faces == 3 * N;
}

Geo geo_of(const tc3d_lattice* lat) { return Geo{lat->L, (int)lat->n_sites}; }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int64_t words_of(int64_t shots) { return (shots + 63) / 64; }

uint32_t threshold_of(double prob) {
    if (!(prob > 0.0)) return 0;
    const double t = floor(prob * 4294967296.0);
    return t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t plane_bytes(const tc3d_lattice* lat, int64_t nw) {
    return round_up((size_t)lat->n_edges * (size_t)nw * 8, 256);
}

size_t nu_bytes(const tc3d_lattice* lat, int64_t n_shots) {
    return round_up((size_t)12 * (size_t)lat->n_sites * (size_t)(64 * words_of(n_shots)) * 4,
                    256);
}

// BP schedule (Section 4.1): `iters` flooding iterations, then the hard
// decision. With a scalar prior the first iteration's messages are
// (-1)^s * nu1 for every check, so they are not stored: the second iteration
// reads them straight from the syndrome.
int bp_run(const Ctx& c, Geo g, const BpArgs& args, int32_t iters, float* buf0, float* buf1,
           Plane corr, float* post, const float* warm = nullptr,
           const float** final_state = nullptr) {
    int rc;
    // a whole decode keeps its state to itself, so per-edge priors can be
    // folded into it (the one-step entry point keeps the plain state)
    BpArgs a = args;
    a.fold = a.llr0 != nullptr;
    if (c.stats) {
        a.ties = c.stats->d_ties;
        c.stats->decisions += 3 * (int64_t)g.N * a.s_pad;
    }
    if (final_state) *final_state = nullptr;
    // small lattices: the whole decode of a shot inside one workgroup's LDS
    if (a.path == TC3D_BP_RESIDENT && (!bp_resident_fits(g, a.llr0, a.nw) || warm || final_state))
        return TC3D_EINVAL;
    if (iters >= 1 && !warm && !final_state && bp_resident_used(g, a))
        return launch_bp_resident(c, g, a, iters, corr, post);
    int mode;
    const float* cur = nullptr;
    float* bufs[2] = {buf0, buf1};
    int nb = 0;
    int32_t first = 2;  // the first iteration launched
    if (warm) {
        // every iteration reads stored messages, the first those the previous
        // cycle ended with
        cur = warm;
        nb = warm == buf0 ? 1 : 0;
        mode = NU_LOAD;
        first = 1;
    } else if (!a.llr0) {
        mode = NU_SIGMA;
    } else {
        rc = launch_bp_iter(c, g, a, NU_ZERO, nullptr, bufs[nb], TC3D_K_BP_FIRST);
        if (rc) return rc;
        cur = bufs[nb];
        nb ^= 1;
        mode = NU_LOAD;
    }
    // the last iteration and the posterior in one pass, unless the caller
    // keeps the final messages or asks for the two launches
    const bool fuse = a.path != TC3D_BP_STREAMING_SPLIT && bp_final_fits(g, a) &&
                      !final_state && iters >= first;
    for (int32_t it = first; it <= iters - (fuse ? 1 : 0); ++it) {
        rc = launch_bp_iter(c, g, a, mode, cur, bufs[nb],
                            mode == NU_SIGMA ? TC3D_K_BP_FIRST : TC3D_K_BP_ITER);
        if (rc) return rc;
        cur = bufs[nb];
        nb ^= 1;
        mode = NU_LOAD;
    }
    if (fuse) return launch_bp_final(c, g, a, mode, cur, corr, post);
    if (final_state) *final_state = mode == NU_LOAD ? cur : nullptr;
    return launch_bp_post(c, g, a, mode, cur, corr, post);
}

bool prob_ok(double p) { return p >= 0.0 && p <= 1.0; }

}  // namespace

BpArgs make_bp_args(CPlane syn, const float* llr0, float l0, float K, int64_t nw, int tile,
                    int path, float damp) {
    BpArgs a;
    a.syn = syn;
    a.llr0 = llr0;
    a.l0 = l0;
    a.K = K;
    const double t = tanh(0.5 * (double)l0);
    // the first iteration's messages (from the priors), damped towards 0
    const double nu1 = (1.0 - (double)damp) * 2.0 * atanh((double)K * t * t * t);
    a.a0 = (float)exp((double)l0);
    a.b1 = (float)exp(nu1);
    a.b1_inv = (float)exp(-nu1);
    a.nw = nw;
    a.s_pad = 64 * nw;
    a.tile = tile;
    a.fold = false;
    a.path = path;
    a.ties = nullptr;
    a.damp = damp;
    a.occupancy = 0;
    return a;
}

namespace {

int check_run(const tc3d_lattice* lat, const tc3d_run_params* prm) {
    if (!lattice_ok(lat) || !prm) return TC3D_EINVAL;
    if (!(prm->p >= 0.0 && prm->p < 0.5) || !(prm->q >= 0.0 && prm->q < 0.5)) return TC3D_EINVAL;
    if (prm->noisy_cycles < 0 || prm->n_sweeps < 0 || prm->n_sweeps > kMaxSweeps ||
        prm->bp_iters < 0 || prm->n_shots < 0 || prm->batch_shots < 0 || prm->bp_tile < -kMaxL ||
        prm->bp_tile > kMaxL)
        return TC3D_EINVAL;
    if (prm->perfect_final != 0 && prm->perfect_final != 1) return TC3D_EINVAL;
    if (prm->bp_meta != 0 && prm->bp_meta != 1) return TC3D_EINVAL;
    if (prm->bp_path < TC3D_BP_AUTO || prm->bp_path > TC3D_BP_STREAMING_SPLIT) return TC3D_EINVAL;
    if (prm->bp_warm != 0 && prm->bp_warm != 1) return TC3D_EINVAL;
    if (!(prm->bp_damp >= 0.0 && prm->bp_damp < 1.0)) return TC3D_EINVAL;
    // the readings of BP as damped or warm-started apply to the paper's BP
    if ((prm->bp_warm || prm->bp_damp > 0.0) && prm->bp_meta) return TC3D_EINVAL;
    // a warm start continues from stored messages, which one iteration never writes
    if (prm->bp_warm && prm->bp_iters == 1) return TC3D_EINVAL;
    if ((prm->flags & ~(uint32_t)TC3D_RUN_GRAPH) != 0) return TC3D_EINVAL;
    if (prm->bp_occupancy < 0 || prm->bp_occupancy > 8) return TC3D_EINVAL;
    // cycle indices of this call stay below 2^32
    if ((uint64_t)prm->cycle0 + (uint64_t)prm->noisy_cycles + 1 > 0xffffffffull)
        return TC3D_EINVAL;
    // subset sweeps: within the schedule, and an edge colouring needs L even
    if (prm->subset_mask != 0 &&
        ((prm->n_sweeps < 32 && (prm->subset_mask >> prm->n_sweeps) != 0) || lat->L % 2 != 0))
        return TC3D_EINVAL;
    if (prm->shot0 % 64 != 0 || prm->batch_shots % 64 != 0) return TC3D_EINVAL;
    if (prm->shot0 + (uint64_t)prm->n_shots >= (1ull << 34)) return TC3D_EINVAL;
    if (prm->bp_iters > 0 && !(prm->p_dec > 0.0 && prm->p_dec < 0.5 && prm->q_dec > 0.0 &&
                               prm->q_dec < 0.5))
        return TC3D_EINVAL;
    return TC3D_OK;
}

// One BP state buffer for nw words: FP32 messages, or the FP64 state of BP
// with meta-checks.
size_t bp_state_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm, int64_t nw) {
    return prm->bp_meta ? round_up(bp_meta_state_bytes(geo_of(lat), nw), 256)
                        : nu_bytes(lat, 64 * nw);
}

size_t llr_bytes(const tc3d_lattice* lat, int64_t nw) {
    return round_up((size_t)nw * 64 * (size_t)lat->n_edges * 4, 256);
}

// The paper's BP decoded by the resident kernel keeps its messages in LDS
// and needs no BP state in the workspace.
bool run_bp_resident(const tc3d_lattice* lat, const tc3d_run_params* prm, bool cnn) {
    return prm->bp_iters > 0 && !prm->bp_meta && !cnn &&
           (prm->bp_path == TC3D_BP_AUTO || prm->bp_path == TC3D_BP_RESIDENT) &&
           !prm->bp_warm && prm->bp_damp == 0.0 && bp_resident_fits(geo_of(lat), nullptr, 1);
}

// BP state buffers of a batch of nw words (two, or none).
size_t run_bp_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm, int64_t nw, bool cnn) {
    if (prm->bp_iters <= 0 || run_bp_resident(lat, prm, cnn)) return 0;
    return 2 * bp_state_bytes(lat, prm, nw);
}

// Words decoded together. With the CNN prior a batch also holds the CNN's
// activations and its rows (64 words N) must stay below 2^31.
int64_t batch_words(const tc3d_lattice* lat, const tc3d_run_params* prm, bool cnn) {
    const int64_t W = words_of(prm->n_shots);
    if (W == 0) return 0;
    int64_t nb;
    if (prm->batch_shots > 0) {
        nb = std::min<int64_t>(W, prm->batch_shots / 64);
    } else {
        size_t per_word = (cnn ? 4 : 3) * plane_bytes(lat, 1) + run_bp_bytes(lat, prm, 1, cnn);
        if (cnn) per_word += llr_bytes(lat, 1) + cnn_workspace_bytes(64 * lat->n_sites, 0);
        const size_t budget = (size_t)24 << 30;
        nb = std::max<int64_t>(1, std::min<int64_t>(W, (int64_t)(budget / per_word)));
    }
    if (cnn) nb = std::min<int64_t>(nb, std::max<int64_t>(1, 0x7fffffffLL / (64 * lat->n_sites)));
    return nb;
}

// The last 256 bytes of a run's workspace hold its counters (timed runs).
constexpr size_t kCounterBytes = 256;

size_t run_ws_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm, int64_t* nb_out,
                    bool cnn) {
    const int64_t nb = batch_words(lat, prm, cnn);
    if (nb_out) *nb_out = nb;
    if (nb == 0) return kCounterBytes;
    size_t b = 3 * plane_bytes(lat, nb);  // syn, corr, flips (also the readout's scratch)
    b += run_bp_bytes(lat, prm, nb, cnn);
    if (cnn)  // previous working syndrome, priors, CNN activations
        b += plane_bytes(lat, nb) + llr_bytes(lat, nb) +
             round_up(cnn_workspace_bytes(64 * nb * lat->n_sites, 0), 256);
    return b + kCounterBytes;
}

// packed == nullptr: the paper's BP prior; else the CNN prior every cycle.
// Every argument check of run_impl, without launching anything.
int run_validate(const tc3d_lattice* lat, const tc3d_run_params* prm, const void* packed,
                 const uint64_t* err, const uint8_t* mask, const int32_t* odd, const void* ws,
                 size_t ws_bytes) {
    int rc = check_run(lat, prm);
    if (rc) return rc;
    const bool cnn = packed != nullptr;
    // the CNN prior changes every cycle (and is folded into the messages), so
    // it takes neither reading
    if (cnn && (prm->bp_iters <= 0 || prm->bp_meta || prm->bp_damp > 0.0 || prm->bp_warm))
        return TC3D_EINVAL;
    if (prm->bp_path == TC3D_BP_RESIDENT && prm->bp_iters > 0 && !run_bp_resident(lat, prm, cnn))
        return TC3D_EINVAL;
    if (prm->n_shots == 0) return TC3D_OK;
    if (!err || !mask) return TC3D_EINVAL;
    if (!aligned(err, 8) || (odd && !aligned(odd, 4)) || (cnn && !aligned(packed, 256)))
        return TC3D_EALIGN;
    const size_t need = run_ws_bytes(lat, prm, nullptr, cnn);
    if (!ws || ws_bytes < need) return TC3D_EWORKSPACE;
    if (!aligned(ws, 256)) return TC3D_EALIGN;
    return TC3D_OK;
}

int run_impl(const tc3d_lattice* lat, const tc3d_run_params* prm, const void* packed,
             uint64_t* err, uint8_t* mask, int32_t* odd, void* ws, size_t ws_bytes,
             const Ctx& c) {
    int rc = run_validate(lat, prm, packed, err, mask, odd, ws, ws_bytes);
    if (rc) return rc;
    if (prm->n_shots == 0) return TC3D_OK;
    const bool cnn = packed != nullptr;
    int64_t nb = 0;
    const size_t ws_need = run_ws_bytes(lat, prm, &nb, cnn);
    const Geo g = geo_of(lat);
    const int64_t W = words_of(prm->n_shots);
    const int64_t rows = lat->n_edges;
    char* base = (char*)ws;
    uint64_t* syn = (uint64_t*)base;
    uint64_t* corr = (uint64_t*)(base + plane_bytes(lat, nb));
    uint64_t* flips = (uint64_t*)(base + 2 * plane_bytes(lat, nb));
    float* nu0 = nullptr;
    float* nu1 = nullptr;
    char* next = base + 3 * plane_bytes(lat, nb);
    if (run_bp_bytes(lat, prm, nb, cnn) > 0) {
        nu0 = (float*)next;
        nu1 = (float*)(next + bp_state_bytes(lat, prm, nb));
        next += 2 * bp_state_bytes(lat, prm, nb);
    }
    if (c.stats) {  // a timed run counts BP near-ties on the device
        c.stats->d_ties = (unsigned long long*)(base + ws_need - kCounterBytes);
        if ((rc = launch_clear(c, Plane{(uint64_t*)c.stats->d_ties, 1}, 1, 1))) return rc;
    }
    uint64_t* prev = nullptr;
    float* llr = nullptr;
    void* cnn_ws = nullptr;
    if (cnn) {
        prev = (uint64_t*)next;
        next += plane_bytes(lat, nb);
        llr = (float*)next;
        next += llr_bytes(lat, nb);
        cnn_ws = next;
    }
    const int32_t cycles = prm->noisy_cycles + prm->perfect_final;
    const uint32_t th_p = threshold_of(prm->p), th_q = threshold_of(prm->q);
    const float l0 = (float)log((1.0 - prm->p_dec) / prm->p_dec);
    const float K = (float)(1.0 - 2.0 * prm->q_dec);
    const int n_subset = __builtin_popcount(prm->subset_mask);
    for (int64_t w0 = 0; w0 < W; w0 += nb) {
        const int64_t bw = std::min(nb, W - w0);
        const uint64_t gword0 = prm->shot0 / 64 + (uint64_t)w0;
        const Plane E{err + w0, W}, S{syn, bw}, C{corr, bw}, F{flips, bw};
        const CPlane cE{err + w0, W}, cS{syn, bw}, cC{corr, bw}, cF{flips, bw};
        const float* warm = nullptr;  // the messages the previous cycle's BP ended with
        // a resumed run's CNN input needs the working syndrome the previous
        // cycle ended with: H e of the residual plus that cycle's check-outcome
        // noise (the sweeps' corrections cancel in H e), a noisy cycle
        if (cnn && prm->cycle0 > 0 &&
            (rc = launch_syndrome(c, g, cE, Plane{prev, bw}, bw, 0, th_q, gword0,
                                  prm->cycle0 - 1, prm->seed)))
            return rc;
        for (int32_t t = 0; t < cycles; ++t) {
            const bool noisy = t < prm->noisy_cycles;
            const uint32_t tp = (noisy || prm->final_qubit_noise) ? th_p : 0u;
            const uint32_t tq = noisy ? th_q : 0u;
            const uint32_t cyc = prm->cycle0 + (uint32_t)t;  // cycle of the whole experiment
            if ((rc = launch_noise(c, g, E, bw, gword0, 0u, cyc, tp, prm->seed))) return rc;
            if ((rc = launch_syndrome(c, g, cE, S, bw, 0, tq, gword0, cyc, prm->seed)))
                return rc;
            if (prm->bp_iters > 0) {
                if (cnn &&
                    (rc = cnn_forward(c, g, syn, (t == 0 && prm->cycle0 == 0) ? nullptr : prev,
                                      bw, 64 * bw * g.N, packed, llr, cnn_ws)))
                    return rc;
                if (prm->bp_meta) {
                    if ((rc = bp_meta_run(c, g, cS, bw, prm->p_dec, prm->q_dec, prm->bp_iters,
                                          (double*)nu0, (double*)nu1, C, nullptr)))
                        return rc;
                } else {
                    BpArgs a = make_bp_args(cS, cnn ? llr : nullptr, l0, K, bw, prm->bp_tile,
                                            prm->bp_path, (float)prm->bp_damp);
                    a.occupancy = prm->bp_occupancy;
                    if ((rc = bp_run(c, g, a, prm->bp_iters, nu0, nu1, C, nullptr, warm,
                                     prm->bp_warm ? &warm : nullptr)))
                        return rc;
                }
                if ((rc = launch_syndrome(c, g, cC, S, bw, 1, 0u, 0, 0, 0))) return rc;
            } else {
                if ((rc = launch_clear(c, C, rows, bw))) return rc;
            }
            for (int32_t k = 0, j = 0; k < prm->n_sweeps; ++k) {
                const bool sub = (prm->subset_mask >> k) & 1u;
                const int pf = sub ? 1 : (int)((prm->pflip_mask >> k) & 1u);
                const int cls = sub ? (int)(((uint64_t)j++ + (uint64_t)cyc * n_subset) % 12u) : -1;
                if ((rc = launch_sweep_decide(c, g, cS, C, F, bw, pf, gword0, cyc, (uint32_t)k,
                                              prm->seed, cls)))
                    return rc;
                if ((rc = launch_syndrome(c, g, cF, S, bw, 1, 0u, 0, 0, 0))) return rc;
            }
            if (cnn && (rc = copy_plane(c, Plane{prev, bw}, cS, rows, bw))) return rc;
            if ((rc = launch_xor(c, E, cC, rows, bw))) return rc;
        }
        const int64_t shots_b = std::min<int64_t>(64 * bw, prm->n_shots - 64 * w0);
        // the flip plane (3 L^3 rows) holds the 3 L^2 string parities
        if ((rc = launch_readout(c, g, cE, shots_b, mask + 64 * w0,
                                 odd ? odd + 3 * 64 * w0 : nullptr, flips)))
            return rc;
    }
    return TC3D_OK;
}

// run_impl captured into one HIP graph on a library stream (a capture cannot
// start on the legacy default stream), launched on `stream` and waited for.
// Every argument is checked first, so nothing half-captured is left behind.
int run_graph(const tc3d_lattice* lat, const tc3d_run_params* prm, uint64_t* err,
              uint8_t* mask, int32_t* odd, void* ws, size_t ws_bytes, hipStream_t stream) {
    int rc = run_validate(lat, prm, nullptr, err, mask, odd, ws, ws_bytes);
    if (rc || prm->n_shots == 0) return rc;
    if ((rc = bp_resident_prepare())) return rc;
    hipStream_t cap = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return TC3D_EHIP;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return TC3D_EHIP;
    }
    // the captured work starts after what is already on `stream`
    if (hipEventRecord(ev, stream) != hipSuccess || hipStreamWaitEvent(cap, ev, 0) != hipSuccess)
        rc = TC3D_EHIP;
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    if (!rc && hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        rc = TC3D_EHIP;
    if (!rc) {
        const Ctx c{cap, nullptr};
        rc = run_impl(lat, prm, nullptr, err, mask, odd, ws, ws_bytes, c);
        if (hipStreamEndCapture(cap, &g) != hipSuccess && !rc) rc = TC3D_EHIP;
    }
    if (!rc && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) rc = TC3D_EHIP;
    if (!rc && hipGraphLaunch(ex, stream) != hipSuccess) rc = TC3D_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess && !rc) rc = TC3D_EHIP;
    if (ex) (void)hipGraphExecDestroy(ex);
    if (g) (void)hipGraphDestroy(g);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(cap);
    return rc;
}

// run_impl with HIP-event timing and the BP near-tie counter; blocks.
int run_timed(const tc3d_lattice* lat, const tc3d_run_params* prm, const void* packed,
              uint64_t* err, uint8_t* mask, int32_t* odd, void* ws, size_t ws_bytes,
              hipStream_t stream, tc3d_timing* timing) {
    Timer tm(stream);
    RunStats st;
    const Ctx c{stream, &tm, &st};
    int rc = run_impl(lat, prm, packed, err, mask, odd, ws, ws_bytes, c);
    unsigned long long ties = 0;
    if (!rc && st.d_ties &&
        hipMemcpyAsync(&ties, st.d_ties, sizeof(ties), hipMemcpyDeviceToHost, stream) !=
            hipSuccess)
        rc = TC3D_EHIP;
    const int rc2 = tm.finish(timing);
    if (hipStreamSynchronize(stream) != hipSuccess && !rc) rc = TC3D_EHIP;
    timing->bp_decisions = st.decisions;
    timing->bp_near_ties = (int64_t)ties;
    return rc ? rc : rc2;
}

}  // namespace

// Scratch of tc3d_run_cycles_noalloc: a fixed array in device memory, one
// copy per device, held until the process ends. 128 MiB holds one 64-shot
// word of the streaming BP state up to L = 24 and whole batches at smaller L.
// Every step of run_impl writes its scratch before reading it, so nothing
// in it needs clearing between calls.
constexpr size_t kNoallocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch[kMaxDevices];

// Device address of the current device's copy of the array, looked up once
// per device on the first call there (in host code the array's name only
// stands in for it).
int scratch_of_current_device(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TC3D_EHIP;
    void* p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TC3D_EHIP;
        g_scratch[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return TC3D_OK;
}
}  // namespace
}  // namespace tc3d

using namespace tc3d;

extern "C" {

int tc3d_make_lattice(int32_t L, tc3d_lattice* out) {
    if (!out || L < 3 || L > kMaxL) return TC3D_EINVAL;
    const int64_t N = (int64_t)L * L * L;
    out->L = L;
    out->reserved = 0;
    out->n_sites = N;
    out->n_edges = 3 * N;
    out->n_faces = 3 * N;
    return TC3D_OK;
}

int tc3d_sample_noise(const tc3d_lattice* lat, uint64_t* plane, int32_t kind, double prob,
                      uint64_t seed, uint32_t cycle, uint64_t shot0, int64_t n_shots,
                      void* stream) {
    if (!lattice_ok(lat) || (kind != 0 && kind != 1) || !prob_ok(prob) || n_shots < 0 ||
        shot0 % 64 != 0 || shot0 + (uint64_t)n_shots >= (1ull << 34))
        return TC3D_EINVAL;
    if (n_shots == 0) return TC3D_OK;
    if (!plane) return TC3D_EINVAL;
    if (!aligned(plane, 8)) return TC3D_EALIGN;
    const int64_t nw = words_of(n_shots);
    const Ctx c{(hipStream_t)stream, nullptr};
    return launch_noise(c, geo_of(lat), Plane{plane, nw}, nw, shot0 / 64, (uint32_t)kind, cycle,
                        threshold_of(prob), seed);
}

int tc3d_syndrome(const tc3d_lattice* lat, const uint64_t* err, uint64_t* syn,
                  int64_t n_words, int32_t xor_into, void* stream) {
    if (!lattice_ok(lat) || n_words < 0) return TC3D_EINVAL;
    if (n_words == 0) return TC3D_OK;
    if (!err || !syn) return TC3D_EINVAL;
    if (!aligned(err, 8) || !aligned(syn, 8)) return TC3D_EALIGN;
    const Ctx c{(hipStream_t)stream, nullptr};
    return launch_syndrome(c, geo_of(lat), CPlane{err, n_words}, Plane{syn, n_words}, n_words,
                           xor_into ? 1 : 0, 0u, 0, 0, 0);
}

int tc3d_apply_correction(const tc3d_lattice* lat, uint64_t* err, const uint64_t* corr,
                          int64_t n_words, void* stream) {
    if (!lattice_ok(lat) || n_words < 0) return TC3D_EINVAL;
    if (n_words == 0) return TC3D_OK;
    if (!err || !corr) return TC3D_EINVAL;
    if (!aligned(err, 8) || !aligned(corr, 8)) return TC3D_EALIGN;
    const Ctx c{(hipStream_t)stream, nullptr};
    return launch_xor(c, Plane{err, n_words}, CPlane{corr, n_words}, lat->n_edges, n_words);
}

size_t tc3d_sweep_workspace_bytes(const tc3d_lattice* lat, int64_t n_words) {
    if (!lattice_ok(lat) || n_words < 0) return 0;
    return plane_bytes(lat, n_words);
}

static int sweep_common(const tc3d_lattice* lat, uint64_t* syn, uint64_t* corr, int64_t n_words,
                        int pflip, uint64_t seed, uint32_t cycle, uint32_t sweep, uint64_t shot0,
                        void* ws, size_t ws_bytes, void* stream, int cls = -1) {
    if (!lattice_ok(lat) || n_words < 0 || shot0 % 64 != 0) return TC3D_EINVAL;
    if (n_words == 0) return TC3D_OK;
    if (!syn || !corr) return TC3D_EINVAL;
    if (!aligned(syn, 8) || !aligned(corr, 8)) return TC3D_EALIGN;
    if (!ws || ws_bytes < plane_bytes(lat, n_words)) return TC3D_EWORKSPACE;
    if (!aligned(ws, 256)) return TC3D_EALIGN;
    const Ctx c{(hipStream_t)stream, nullptr};
    const Geo g = geo_of(lat);
    uint64_t* F = (uint64_t*)ws;
    int rc = launch_sweep_decide(c, g, CPlane{syn, n_words}, Plane{corr, n_words},
                                 Plane{F, n_words}, n_words, pflip, shot0 / 64, cycle, sweep, seed,
                                 cls);
    if (rc) return rc;
    return launch_syndrome(c, g, CPlane{F, n_words}, Plane{syn, n_words}, n_words, 1, 0u, 0, 0, 0);
}

int tc3d_flip_sweep(const tc3d_lattice* lat, uint64_t* syn, uint64_t* corr, int64_t n_words,
                    void* ws, size_t ws_bytes, void* stream) {
    return sweep_common(lat, syn, corr, n_words, 0, 0, 0, 0, 0, ws, ws_bytes, stream);
}

int tc3d_pflip_sweep(const tc3d_lattice* lat, uint64_t* syn, uint64_t* corr, int64_t n_words,
                     uint64_t seed, uint32_t cycle, uint32_t sweep, uint64_t shot0, void* ws,
                     size_t ws_bytes, void* stream) {
    return sweep_common(lat, syn, corr, n_words, 1, seed, cycle, sweep, shot0, ws, ws_bytes,
                        stream);
}

int tc3d_subset_pflip_sweep(const tc3d_lattice* lat, uint64_t* syn, uint64_t* corr,
                            int64_t n_words, uint64_t seed, uint32_t cycle, uint32_t sweep,
                            uint64_t shot0, int32_t edge_class, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!lattice_ok(lat) || lat->L % 2 != 0 || edge_class < 0 || edge_class >= 12)
        return TC3D_EINVAL;
    return sweep_common(lat, syn, corr, n_words, 1, seed, cycle, sweep, shot0, ws, ws_bytes,
                        stream, edge_class);
}

size_t tc3d_bp_workspace_bytes(const tc3d_lattice* lat, int64_t n_shots) {
    if (!lattice_ok(lat) || n_shots < 0) return 0;
    return 2 * nu_bytes(lat, n_shots);
}

static bool bp_scalars_ok(float l0, float K) {
    return isfinite(l0) && fabsf(l0) <= 40.0f && K >= 0.0f && K < 1.0f;
}

int tc3d_bp_decode(const tc3d_lattice* lat, const uint64_t* syn, int64_t n_shots,
                   const float* llr0, float llr0_scalar, float meas_factor, int32_t iters,
                   int32_t bp_path, uint64_t* corr_out, float* post_out, void* ws,
                   size_t ws_bytes, void* stream) {
    if (!lattice_ok(lat) || n_shots < 0 || iters < 1 || !bp_scalars_ok(llr0_scalar, meas_factor) ||
        bp_path < TC3D_BP_AUTO || bp_path > TC3D_BP_STREAMING_SPLIT)
        return TC3D_EINVAL;
    if (bp_path == TC3D_BP_RESIDENT && !bp_resident_fits(geo_of(lat), llr0, 1)) return TC3D_EINVAL;
    if (n_shots == 0) return TC3D_OK;
    if (!syn || !corr_out) return TC3D_EINVAL;
    if (!aligned(syn, 8) || !aligned(corr_out, 8) || (llr0 && !aligned(llr0, 4)) ||
        (post_out && !aligned(post_out, 4)))
        return TC3D_EALIGN;
    const size_t half = nu_bytes(lat, n_shots);
    if (!ws || ws_bytes < 2 * half) return TC3D_EWORKSPACE;
    if (!aligned(ws, 256)) return TC3D_EALIGN;
    const int64_t nw = words_of(n_shots);
    const Ctx c{(hipStream_t)stream, nullptr};
    const BpArgs a =
        make_bp_args(CPlane{syn, nw}, llr0, llr0_scalar, meas_factor, nw, 0, bp_path);
    float* b0 = (float*)ws;
    float* b1 = (float*)((char*)ws + half);
    return bp_run(c, geo_of(lat), a, iters, b0, b1, Plane{corr_out, nw}, post_out);
}

int tc3d_bp_step(const tc3d_lattice* lat, const uint64_t* syn, int64_t n_shots,
                 const float* llr0, float llr0_scalar, float meas_factor, float damp,
                 const float* nu_in, float* nu_out, float* post_out, void* stream) {
    if (!lattice_ok(lat) || n_shots < 0 || !bp_scalars_ok(llr0_scalar, meas_factor) ||
        !(damp >= 0.0f && damp < 1.0f) || (damp > 0.0f && llr0))
        return TC3D_EINVAL;
    if (n_shots == 0) return TC3D_OK;
    if (!syn || !nu_out || nu_in == nu_out) return TC3D_EINVAL;
    if (!aligned(syn, 8) || !aligned(nu_out, 4) || (nu_in && !aligned(nu_in, 4)) ||
        (llr0 && !aligned(llr0, 4)) || (post_out && !aligned(post_out, 4)))
        return TC3D_EALIGN;
    const int64_t nw = words_of(n_shots);
    const Ctx c{(hipStream_t)stream, nullptr};
    const Geo g = geo_of(lat);
    const BpArgs a = make_bp_args(CPlane{syn, nw}, llr0, llr0_scalar, meas_factor, nw, 0,
                                  TC3D_BP_STREAMING, damp);
    int rc = launch_bp_iter(c, g, a, nu_in ? NU_LOAD : NU_ZERO, nu_in, nu_out,
                            nu_in ? TC3D_K_BP_ITER : TC3D_K_BP_FIRST);
    if (rc || !post_out) return rc;
    // posterior of the new state; no correction plane (the store is skipped)
    return launch_bp_post(c, g, a, NU_LOAD, nu_out, Plane{nullptr, nw}, post_out);
}

static bool probs_open(double p_dec, double q_dec) {
    return p_dec > 0.0 && p_dec < 0.5 && q_dec > 0.0 && q_dec < 0.5;
}

size_t tc3d_bp_meta_workspace_bytes(const tc3d_lattice* lat, int64_t n_shots) {
    if (!lattice_ok(lat) || n_shots < 0) return 0;
    return 2 * round_up(bp_meta_state_bytes(geo_of(lat), words_of(n_shots)), 256);
}

int tc3d_bp_meta_decode(const tc3d_lattice* lat, const uint64_t* syn, int64_t n_shots,
                        double p_dec, double q_dec, int32_t iters, uint64_t* corr_out,
                        double* post_out, void* ws, size_t ws_bytes, void* stream) {
    if (!lattice_ok(lat) || n_shots < 0 || iters < 1 || !probs_open(p_dec, q_dec))
        return TC3D_EINVAL;
    if (n_shots == 0) return TC3D_OK;
    if (!syn || !corr_out) return TC3D_EINVAL;
    if (!aligned(syn, 8) || !aligned(corr_out, 8) || (post_out && !aligned(post_out, 8)))
        return TC3D_EALIGN;
    const int64_t nw = words_of(n_shots);
    const Geo g = geo_of(lat);
    const size_t half = round_up(bp_meta_state_bytes(g, nw), 256);
    if (!ws || ws_bytes < 2 * half) return TC3D_EWORKSPACE;
    if (!aligned(ws, 256)) return TC3D_EALIGN;
    const Ctx c{(hipStream_t)stream, nullptr};
    return bp_meta_run(c, g, CPlane{syn, nw}, nw, p_dec, q_dec, iters, (double*)ws,
                       (double*)((char*)ws + half), Plane{corr_out, nw}, post_out);
}

int tc3d_bp_meta_step(const tc3d_lattice* lat, const uint64_t* syn, int64_t n_shots,
                      double p_dec, double q_dec, const double* state_in, double* state_out,
                      double* post_out, void* stream) {
    if (!lattice_ok(lat) || n_shots < 0 || !probs_open(p_dec, q_dec)) return TC3D_EINVAL;
    if (n_shots == 0) return TC3D_OK;
    if (!syn || !state_out || state_in == state_out) return TC3D_EINVAL;
    if (!aligned(syn, 8) || !aligned(state_out, 8) || (state_in && !aligned(state_in, 8)) ||
        (post_out && !aligned(post_out, 8)))
        return TC3D_EALIGN;
    const int64_t nw = words_of(n_shots);
    const Ctx c{(hipStream_t)stream, nullptr};
    const Geo g = geo_of(lat);
    int rc = launch_bp_meta_iter(c, g, CPlane{syn, nw}, nw, p_dec, q_dec, state_in, state_out);
    if (rc || !post_out) return rc;
    return launch_bp_meta_post(c, g, CPlane{syn, nw}, nw, p_dec, q_dec, state_out,
                               Plane{nullptr, nw}, post_out);
}

size_t tc3d_logical_check_workspace_bytes(const tc3d_lattice* lat, int64_t n_shots) {
    if (!lattice_ok(lat) || n_shots < 0) return 0;
    return round_up((size_t)readout_scratch_words(geo_of(lat), words_of(n_shots)) * 8 + 8, 256);
}

int tc3d_logical_check(const tc3d_lattice* lat, const uint64_t* err, int64_t n_shots,
                       uint8_t* mask_out, int32_t* odd_out, void* ws, size_t ws_bytes,
                       void* stream) {
    if (!lattice_ok(lat) || n_shots < 0) return TC3D_EINVAL;
    if (n_shots == 0) return TC3D_OK;
    if (!err || !mask_out) return TC3D_EINVAL;
    if (!aligned(err, 8) || (odd_out && !aligned(odd_out, 4))) return TC3D_EALIGN;
    if (!ws || ws_bytes < tc3d_logical_check_workspace_bytes(lat, n_shots))
        return TC3D_EWORKSPACE;
    if (!aligned(ws, 256)) return TC3D_EALIGN;
    const Ctx c{(hipStream_t)stream, nullptr};
    return launch_readout(c, geo_of(lat), CPlane{err, words_of(n_shots)}, n_shots, mask_out,
                          odd_out, (uint64_t*)ws);
}

size_t tc3d_run_workspace_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm) {
    if (check_run(lat, prm)) return 0;
    return run_ws_bytes(lat, prm, nullptr, false);
}

int tc3d_run_cycles(const tc3d_lattice* lat, const tc3d_run_params* prm, uint64_t* err_state,
                    uint8_t* mask_out, int32_t* odd_out, void* ws, size_t ws_bytes,
                    void* stream) {
    if (prm && (prm->flags & TC3D_RUN_GRAPH))
        return run_graph(lat, prm, err_state, mask_out, odd_out, ws, ws_bytes,
                         (hipStream_t)stream);
    const Ctx c{(hipStream_t)stream, nullptr};
    return run_impl(lat, prm, nullptr, err_state, mask_out, odd_out, ws, ws_bytes, c);
}

int tc3d_run_cycles_timed(const tc3d_lattice* lat, const tc3d_run_params* prm,
                          uint64_t* err_state, uint8_t* mask_out, int32_t* odd_out, void* ws,
                          size_t ws_bytes, void* stream, tc3d_timing* timing) {
    if (!timing) return TC3D_EINVAL;
    return run_timed(lat, prm, nullptr, err_state, mask_out, odd_out, ws, ws_bytes,
                     (hipStream_t)stream, timing);
}

// ------------------------------------------------------------------ CNN prior
int64_t tc3d_cnn_param_count(void) { return cnn_param_count(); }

size_t tc3d_cnn_packed_bytes(void) { return cnn_packed_bytes(); }

int tc3d_cnn_pack(const float* params, float beta, float l0, void* packed, void* stream) {
    if (!params || !packed || !(beta >= 0.0f && beta <= 1.0f) || !isfinite(l0) ||
        fabsf(l0) > 40.0f)
        return TC3D_EINVAL;
    if (!aligned(params, 4) || !aligned(packed, 256)) return TC3D_EALIGN;
    const Ctx c{(hipStream_t)stream, nullptr};
    return cnn_pack(c, params, beta, l0, packed);
}

static int64_t cnn_rows(const tc3d_lattice* lat, int64_t n_shots) {
    const int64_t R = 64 * words_of(n_shots) * lat->n_sites;
    return R < 0x7fffffffLL ? R : -1;
}

size_t tc3d_cnn_workspace_bytes(const tc3d_lattice* lat, int64_t n_shots, int32_t training) {
    if (!lattice_ok(lat) || n_shots <= 0) return 0;
    const int64_t R = cnn_rows(lat, n_shots);
    if (R < 0) return 0;
    return cnn_workspace_bytes(R, training ? 1 : 0);
}

static int cnn_common_checks(const tc3d_lattice* lat, const uint64_t* syn, const uint64_t* prev,
                             int64_t n_shots, const void* packed, const float* llr, void* ws,
                             size_t ws_bytes, int training) {
    if (!lattice_ok(lat) || n_shots <= 0 || !syn || !packed || !llr) return TC3D_EINVAL;
    if (!aligned(syn, 8) || (prev && !aligned(prev, 8)) || !aligned(packed, 256) ||
        !aligned(llr, 4))
        return TC3D_EALIGN;
    const int64_t R = cnn_rows(lat, n_shots);
    if (R < 0) return TC3D_EINVAL;
    if (!ws || ws_bytes < cnn_workspace_bytes(R, training)) return TC3D_EWORKSPACE;
    if (!aligned(ws, 256)) return TC3D_EALIGN;
    return TC3D_OK;
}

int tc3d_cnn_forward(const tc3d_lattice* lat, const uint64_t* syn, const uint64_t* prev,
                     int64_t n_shots, const void* packed, float* llr_out, void* ws,
                     size_t ws_bytes, void* stream) {
    int rc = cnn_common_checks(lat, syn, prev, n_shots, packed, llr_out, ws, ws_bytes, 0);
    if (rc) return rc;
    const Ctx c{(hipStream_t)stream, nullptr};
    return cnn_forward(c, geo_of(lat), syn, prev, words_of(n_shots), cnn_rows(lat, n_shots),
                       packed, llr_out, ws);
}

int tc3d_cnn_loss_grad(const tc3d_lattice* lat, const uint64_t* syn, const uint64_t* prev,
                       const uint64_t* target, int64_t n_shots, const void* packed,
                       float* llr_out, float* grad, float* loss, void* ws, size_t ws_bytes,
                       void* stream) {
    int rc = cnn_common_checks(lat, syn, prev, n_shots, packed, llr_out, ws, ws_bytes, 1);
    if (rc) return rc;
    if (!target || !grad || !loss) return TC3D_EINVAL;
    if (!aligned(target, 8) || !aligned(grad, 4) || !aligned(loss, 4)) return TC3D_EALIGN;
    const Ctx c{(hipStream_t)stream, nullptr};
    return cnn_loss_grad(c, geo_of(lat), syn, prev, target, words_of(n_shots),
                         cnn_rows(lat, n_shots), packed, llr_out, grad, loss, ws);
}

int tc3d_cnn_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                  float beta1, float beta2, float eps, void* packed, void* stream) {
    if (!params || !grad || !m || !v || !packed || step < 1 || !(lr > 0.f) ||
        !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return TC3D_EINVAL;
    if (!aligned(params, 4) || !aligned(grad, 4) || !aligned(m, 4) || !aligned(v, 4) ||
        !aligned(packed, 256))
        return TC3D_EALIGN;
    const Ctx c{(hipStream_t)stream, nullptr};
    return cnn_adam(c, params, grad, m, v, step, lr, beta1, beta2, eps, packed);
}

size_t tc3d_run_cnn_workspace_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm) {
    if (check_run(lat, prm) || prm->bp_iters <= 0) return 0;
    return run_ws_bytes(lat, prm, nullptr, true);
}

int tc3d_run_cycles_cnn(const tc3d_lattice* lat, const tc3d_run_params* prm, const void* packed,
                        uint64_t* err_state, uint8_t* mask_out, int32_t* odd_out, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!packed) return TC3D_EINVAL;
    const Ctx c{(hipStream_t)stream, nullptr};
    return run_impl(lat, prm, packed, err_state, mask_out, odd_out, ws, ws_bytes, c);
}

int tc3d_run_cycles_cnn_timed(const tc3d_lattice* lat, const tc3d_run_params* prm,
                              const void* packed, uint64_t* err_state, uint8_t* mask_out,
                              int32_t* odd_out, void* ws, size_t ws_bytes, void* stream,
                              tc3d_timing* timing) {
    if (!packed || !timing) return TC3D_EINVAL;
    return run_timed(lat, prm, packed, err_state, mask_out, odd_out, ws, ws_bytes,
                     (hipStream_t)stream, timing);
}

// A run that allocates nothing: its scratch is the array above.
int tc3d_run_cycles_noalloc(const tc3d_lattice* lat, const tc3d_run_params* prm,
                            uint64_t* err_state, uint8_t* mask_out, int32_t* odd_out,
                            void* stream) {
    int rc = check_run(lat, prm);
    if (rc) return rc;
    tc3d_run_params p = *prm;
    if (p.batch_shots == 0 && p.n_shots > 0) {
        // the largest batch whose workspace fits the array (results do not
        // depend on the batch)
        int64_t lo = 0, hi = words_of(p.n_shots);
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            p.batch_shots = 64 * mid;
            if (run_ws_bytes(lat, &p, nullptr, false) <= kNoallocScratchBytes)
                lo = mid;
            else
                hi = mid - 1;
        }
        if (lo == 0) return TC3D_EWORKSPACE;  // one word does not fit: L too large
        p.batch_shots = 64 * lo;
    }
    if (run_ws_bytes(lat, &p, nullptr, false) > kNoallocScratchBytes) return TC3D_EWORKSPACE;
    void* ws = nullptr;
    if ((rc = scratch_of_current_device(&ws))) return rc;
    const Ctx c{(hipStream_t)stream, nullptr};
    return run_impl(lat, &p, nullptr, err_state, mask_out, odd_out, ws, kNoallocScratchBytes, c);
}

// ------------------------------------------------------------ batched jobs
static constexpr int32_t kMaxJobs = 4096;
static constexpr int kMaxJobStreams = 8;

size_t tc3d_run_jobs_workspace_bytes(const tc3d_job* jobs, int32_t n_jobs) {
    if (!jobs || n_jobs <= 0 || n_jobs > kMaxJobs) return 0;
    size_t b = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        tc3d_lattice lat;
        if (tc3d_make_lattice(jobs[i].L, &lat) || check_run(&lat, &jobs[i].prm)) return 0;
        b += round_up(run_ws_bytes(&lat, &jobs[i].prm, nullptr, false), 256);
    }
    return b;
}

namespace {
// Streams and events of one tc3d_run_jobs call, released on every exit path.
struct JobStreams {
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> ev;  // ev[0]: fork; ev[1 + j]: join of stream j
    ~JobStreams() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto x : s)
            if (x) (void)hipStreamDestroy(x);
    }
};
}  // namespace

int tc3d_run_jobs(const tc3d_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                  int32_t flags, void* stream) {
    if (!jobs || n_jobs <= 0 || n_jobs > kMaxJobs) return TC3D_EINVAL;
    if (flags & ~(TC3D_JOBS_CONCURRENT | TC3D_JOBS_GRAPH)) return TC3D_EINVAL;
    if (!ws || !aligned(ws, 256)) return ws ? TC3D_EALIGN : TC3D_EWORKSPACE;
    // validate everything before the first launch (nothing half-enqueued,
    // nothing half-captured)
    std::vector<tc3d_lattice> lats((size_t)n_jobs);
    std::vector<size_t> off((size_t)n_jobs), len((size_t)n_jobs);
    size_t total = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const tc3d_job& j = jobs[i];
        if (j.reserved != 0 || tc3d_make_lattice(j.L, &lats[i])) return TC3D_EINVAL;
        int rc = check_run(&lats[i], &j.prm);
        if (rc) return rc;
        len[i] = round_up(run_ws_bytes(&lats[i], &j.prm, nullptr, false), 256);
        off[i] = total;
        total += len[i];
        if (total > ws_bytes) return TC3D_EWORKSPACE;
        rc = run_validate(&lats[i], &j.prm, nullptr, j.err_state, j.mask_out, j.odd_out,
                          (char*)ws + off[i], len[i]);
        if (rc) return rc;
    }
    const hipStream_t origin = (hipStream_t)stream;
    const bool graph = (flags & TC3D_JOBS_GRAPH) != 0;
    const int n_str = (flags & TC3D_JOBS_CONCURRENT) ? std::min(n_jobs, kMaxJobStreams) : 1;
    // stream 0 of js.s is the capture stream in graph mode (a capture cannot
    // start on the legacy default stream, which `stream` may be)
    JobStreams js;
    js.s.assign((size_t)n_str + 1, nullptr);
    js.ev.assign((size_t)n_str + 1, nullptr);
    for (auto& x : js.s)
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) return TC3D_EHIP;
    for (auto& e : js.ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return TC3D_EHIP;
    const hipStream_t head = graph ? js.s[0] : origin;
    if (graph) {
        const int prc = bp_resident_prepare();
        if (prc) return prc;
    }
    if (graph && hipStreamBeginCapture(head, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return TC3D_EHIP;
    int rc = TC3D_OK;
    // fork: every job stream starts after the work already on `head`
    if (hipEventRecord(js.ev[0], head) != hipSuccess) rc = TC3D_EHIP;
    for (int k = 1; k <= n_str && !rc; ++k)
        if (hipStreamWaitEvent(js.s[k], js.ev[0], 0) != hipSuccess) rc = TC3D_EHIP;
    for (int32_t i = 0; i < n_jobs && !rc; ++i) {
        const tc3d_job& j = jobs[i];
        const Ctx c{js.s[1 + (size_t)(i % n_str)], nullptr};
        rc = run_impl(&lats[i], &j.prm, nullptr, j.err_state, j.mask_out, j.odd_out,
                      (char*)ws + off[i], len[i], c);
    }
    // join: `head` continues after every job
    for (int k = 1; k <= n_str; ++k) {
        if (hipEventRecord(js.ev[k], js.s[k]) != hipSuccess && !rc) rc = TC3D_EHIP;
        if (hipStreamWaitEvent(head, js.ev[k], 0) != hipSuccess && !rc) rc = TC3D_EHIP;
    }
    if (graph) {
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(head, &g) != hipSuccess && !rc) rc = TC3D_EHIP;
        hipGraphExec_t ex = nullptr;
        if (!rc && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) rc = TC3D_EHIP;
        if (!rc && hipGraphLaunch(ex, origin) != hipSuccess) rc = TC3D_EHIP;
        if (hipStreamSynchronize(origin) != hipSuccess && !rc) rc = TC3D_EHIP;
        if (ex) (void)hipGraphExecDestroy(ex);
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (hipStreamSynchronize(origin) != hipSuccess && !rc) rc = TC3D_EHIP;
    return rc;
}

// ------------------------------------------------------------- autotuning
size_t tc3d_autotune_workspace_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm) {
    if (!lattice_ok(lat) || !prm || check_run(lat, prm) || prm->n_shots <= 0) return 0;
    tc3d_run_params p = *prm;
    p.batch_shots = 0;
    p.bp_path = TC3D_BP_STREAMING;  // the candidate that needs the most
    return plane_bytes(lat, words_of(prm->n_shots)) + round_up((size_t)prm->n_shots, 256) +
           round_up(run_ws_bytes(lat, &p, nullptr, false), 256);
}

int tc3d_autotune(const tc3d_lattice* lat, tc3d_run_params* prm, int32_t probe_cycles,
                  void* ws, size_t ws_bytes, tc3d_tune_choice* out, int32_t max_out,
                  int32_t* n_out, void* stream) {
    if (!lattice_ok(lat) || !prm || probe_cycles < 1 || probe_cycles > 64 || max_out < 0 ||
        (max_out > 0 && !out))
        return TC3D_EINVAL;
    int rc = check_run(lat, prm);
    if (rc) return rc;
    if (prm->n_shots <= 0) return TC3D_EINVAL;
    if (!ws || ws_bytes < tc3d_autotune_workspace_bytes(lat, prm)) return TC3D_EWORKSPACE;
    if (!aligned(ws, 256)) return TC3D_EALIGN;
    const hipStream_t st = (hipStream_t)stream;
    const int64_t W = words_of(prm->n_shots);
    char* base = (char*)ws;
    uint64_t* err = (uint64_t*)base;
    uint8_t* mask = (uint8_t*)(base + plane_bytes(lat, W));
    char* rws = (char*)mask + round_up((size_t)prm->n_shots, 256);
    const size_t rws_bytes = ws_bytes - (size_t)(rws - base);

    tc3d_run_params probe = *prm;
    probe.noisy_cycles = probe_cycles;
    probe.perfect_final = 0;
    probe.batch_shots = 0;
    probe.flags = 0;
    const Ctx plain{st, nullptr};
    // warm-up (first launches, code-object loading)
    if ((rc = launch_clear(plain, Plane{err, W}, lat->n_edges, W))) return rc;
    if ((rc = run_impl(lat, &probe, nullptr, err, mask, nullptr, rws, rws_bytes, plain)))
        return rc;
    int32_t n = 0;
    double best = 1e300;
    tc3d_run_params best_prm = probe;
    // times one candidate; keeps it when it is the fastest so far
    auto trial = [&](const tc3d_run_params& cand) -> int {
        if (run_ws_bytes(lat, &cand, nullptr, false) > rws_bytes) return TC3D_OK;  // skip
        int r = launch_clear(plain, Plane{err, W}, lat->n_edges, W);
        if (r) return r;
        Timer tm(st);
        const Ctx c{st, &tm};
        if ((r = run_impl(lat, &cand, nullptr, err, mask, nullptr, rws, rws_bytes, c))) return r;
        tc3d_timing tmg;
        if ((r = tm.finish(&tmg))) return r;
        if (n < max_out)
            out[n] = tc3d_tune_choice{cand.bp_tile, cand.bp_path, cand.batch_shots, tmg.total_ms,
                                      cand.bp_occupancy, 0};
        ++n;
        if (tmg.total_ms < best) {
            best = tmg.total_ms;
            best_prm = cand;
        }
        return TC3D_OK;
    };
    const bool bp = prm->bp_iters > 0 && !prm->bp_meta;
    // 1. the BP iteration schedule: resident decode or streaming iterations
    tc3d_run_params cand = probe;
    if (bp && run_bp_resident(lat, &probe, false)) {
        for (int32_t path : {TC3D_BP_AUTO, TC3D_BP_STREAMING}) {
            cand.bp_path = path;
            if ((rc = trial(cand))) return rc;
        }
    } else {
        if ((rc = trial(cand))) return rc;
    }
    // 2.-3. the streaming kernels' traversal and occupancy
    if (bp && !run_bp_resident(lat, &best_prm, false)) {
        cand = best_prm;
        for (int32_t t : {4, 8, 12, 16, 24, 32, -4, -8, -12, -16}) {
            if ((t < 0 ? -t : t) >= lat->L) continue;
            cand.bp_tile = t;
            if ((rc = trial(cand))) return rc;
        }
        cand = best_prm;
        for (int32_t occ : {3, 5, 6, 8}) {
            cand.bp_occupancy = occ;
            if ((rc = trial(cand))) return rc;
        }
    }
    // 4. the batch
    int64_t nb_auto = 0;
    (void)run_ws_bytes(lat, &best_prm, &nb_auto, false);
    cand = best_prm;
    for (int64_t b : {nb_auto / 2, nb_auto / 4}) {
        if (b < 1 || b == nb_auto) continue;
        cand.batch_shots = 64 * b;
        if ((rc = trial(cand))) return rc;
    }
    if (n_out) *n_out = n;
    prm->bp_tile = best_prm.bp_tile;
    prm->bp_path = best_prm.bp_path;
    prm->bp_occupancy = best_prm.bp_occupancy;
    prm->batch_shots = best_prm.batch_shots ? best_prm.batch_shots : 64 * nb_auto;
    return TC3D_OK;
}

int tc3d_stream_copy(void* dst, const void* src, int64_t n_bytes, int32_t nontemporal,
                     void* stream) {
    if (n_bytes < 0 || n_bytes % 16 != 0 || (nontemporal != 0 && nontemporal != 1))
        return TC3D_EINVAL;
    if (n_bytes == 0) return TC3D_OK;
    if (!dst || !src) return TC3D_EINVAL;
    if (!aligned(dst, 16) || !aligned(src, 16)) return TC3D_EALIGN;
    const uintptr_t s = (uintptr_t)src, d = (uintptr_t)dst;
    if (s < d + (uintptr_t)n_bytes && d < s + (uintptr_t)n_bytes) return TC3D_EINVAL;  // overlap
    const Ctx c{(hipStream_t)stream, nullptr};
    return launch_stream_copy(c, dst, src, n_bytes / 16, nontemporal);
}

#ifndef TC3D_BUILD_ID
#define TC3D_BUILD_ID "unknown"
#endif

const char* tc3d_build_id(void) { return TC3D_BUILD_ID; }

const char* tc3d_strerror(int code) {
    switch (code) {
        case TC3D_OK: return "ok";
        case TC3D_EINVAL: return "invalid argument";
        case TC3D_EALIGN: return "misaligned pointer";
        case TC3D_EHIP: return "HIP launch or runtime error";
        case TC3D_EWORKSPACE: return "workspace missing or too small";
        default: return "unknown error";
    }
}

}  // extern "C"
