// Internal launch interface shared by the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "tc3d.h"

namespace tc3d {

// Optional HIP-event timing (used by tc3d_run_cycles_timed). Consecutive
// launches of one kernel class share one pair of events: an event pair per
// launch costs a few microseconds of GPU time each, which the CNN path, with
// hundreds of short launches per cycle, would feel (about 9%).
class Timer {
  public:
    explicit Timer(hipStream_t s) : stream_(s) {}
    ~Timer();
    int begin(int kclass);  // before a launch: opens an interval unless one of this class is open
    int end();              // after a launch (the interval stays open)
    int finish(tc3d_timing* out);  // closes the last interval, waits for all events, sums them

  private:
    struct Slot {
        hipEvent_t start = nullptr, stop = nullptr;
        int kclass = -1;
        bool pending = false;
    };
    int drain(Slot& s);
    int close();  // records the stop event of the open interval
    hipStream_t stream_;
    std::vector<Slot> slots_;
    size_t next_ = 0;
    int cur_ = -1;
    bool open_ = false;  // slot cur_ has its start event and awaits its stop
    hipEvent_t first_ = nullptr, last_ = nullptr;
    double ms_[TC3D_K_COUNT] = {};
    int64_t launches_[TC3D_K_COUNT] = {};
};

// Counters a timed run reports besides kernel times.
struct RunStats {
    unsigned long long* d_ties = nullptr;  // device counter of BP near-ties
    int64_t decisions = 0;                 // BP hard decisions enqueued
};

struct Ctx {
    hipStream_t stream;
    Timer* timer;              // nullptr: no timing
    RunStats* stats = nullptr;  // nullptr: no counters
};

// A bit plane view: rows x nw words, row stride ld words.
struct Plane {
    uint64_t* p;
    int64_t ld;
};
struct CPlane {
    const uint64_t* p;
    int64_t ld;
};

struct Geo {
    int L;
    int N;  // L^3
};

// ---------------------------------------------------------------- bit planes
// plane[row][w] ^= Bernoulli bits of (row, cycle, global word word0 + w, tag).
int launch_noise(const Ctx& c, Geo g, Plane plane, int64_t nw, uint64_t word0, uint32_t tag,
                 uint32_t cycle, uint32_t th, uint64_t seed);
// dst (faces) = / ^= H src (edges), optionally XOR check-outcome noise.
int launch_syndrome(const Ctx& c, Geo g, CPlane src, Plane dst, int64_t nw, int xor_into,
                    uint32_t th_meas, uint64_t word0, uint32_t cycle, uint64_t seed);
// F = flip (pflip=0) or p-flip decisions; corr ^= F; F written to fplane.
// One flip / p-flip decision pass; cls >= 0 restricts it to one edge class
// (the subset sweep), cls < 0 lets every edge flip.
int launch_sweep_decide(const Ctx& c, Geo g, CPlane syn, Plane corr, Plane fplane, int64_t nw,
                        int pflip, uint64_t word0, uint32_t cycle, uint32_t sweep,
                        uint64_t seed, int cls = -1);
// dst ^= src over rows x nw.
int launch_xor(const Ctx& c, Plane dst, CPlane src, int64_t rows, int64_t nw);
// dst = 0 over rows x nw.
int launch_clear(const Ctx& c, Plane dst, int64_t rows, int64_t nw);
// dst[i] = src[i] for n16 16-byte elements (non-temporal stores if asked).
int launch_stream_copy(const Ctx& c, void* dst, const void* src, int64_t n16, int nontemporal);
// Majority-vote readout of n_shots shots of an edge plane; par is scratch of
// readout_scratch_words(g, nw) words (the parities of the logical strings).
int64_t readout_scratch_words(Geo g, int64_t nw);
int launch_readout(const Ctx& c, Geo g, CPlane err, int64_t n_shots, uint8_t* mask,
                   int32_t* odd, uint64_t* par);

// ----------------------------------------------------------------------- BP
enum NuMode { NU_ZERO = 0, NU_SIGMA = 1, NU_LOAD = 2 };

struct BpArgs {
    CPlane syn;          // face plane
    const float* llr0;   // [3N][S_pad] per-edge priors (nats) or nullptr
    float l0;            // scalar prior (nats) when llr0 == nullptr
    float K;             // measurement factor 1 - 2q
    float a0;            // e^{l0}
    float b1, b1_inv;    // e^{+-nu1}, nu1 = 2 atanh(K tanh(l0/2)^3) (NU_SIGMA only)
    int64_t nw;          // words in the batch
    int64_t s_pad;       // 64 * nw
    int tile;            // site-tile edge of the traversal order (0: automatic)
    bool fold;           // per-edge priors folded into the stored state (see tc3d_bp.hip)
    int path;            // TC3D_BP_AUTO / _STREAMING / _RESIDENT / _STREAMING_SPLIT
    unsigned long long* ties;  // device counter of posteriors |l| < 1e-3, or nullptr
    float damp;          // damping g: nu = (1 - g) nu_new + g nu_old (0: none)
    int occupancy;       // workgroups per CU of the stored-message iterations (0: default)
};

// Fills the derived fields of BpArgs (in double precision, then rounded).
BpArgs make_bp_args(CPlane syn, const float* llr0, float l0, float K, int64_t nw, int tile,
                    int path = TC3D_BP_AUTO, float damp = 0.0f);

// One iteration: b_out = BP(b_in) (messages in the form e^nu) where the
// incoming state is given by mode.
int launch_bp_iter(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu_in,
                   float* nu_out, int kclass);
// Posterior from the state (mode, nu); corr (edge plane) = [posterior < 0];
// post (may be null) = posterior floats.
int launch_bp_post(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu, Plane corr,
                   float* post);
// One more iteration from the state (mode, nu) and the posterior of its
// result, in one pass that stores no messages; bit-identical to
// launch_bp_iter followed by launch_bp_post. Needs bp_final_fits: undamped,
// per-edge priors folded into the state (as a whole decode keeps them).
bool bp_final_fits(Geo g, const BpArgs& a);
int launch_bp_final(const Ctx& c, Geo g, const BpArgs& a, int mode, const float* nu, Plane corr,
                    float* post);
// A whole decode (iters >= 1, scalar prior) with each shot's state in one
// workgroup's LDS; bit-identical to the streaming kernels. Possible when
// bp_resident_fits: L^3 <= 3072 and no per-edge prior; bp_resident_used adds
// the caller's choice of kernels (a.path).
bool bp_resident_fits(Geo g, const float* llr0, int64_t nw);
bool bp_resident_used(Geo g, const BpArgs& a);
// Allows the resident kernels their LDS size on the current device (once per
// device); called before a graph capture so that nothing of it runs inside one.
int bp_resident_prepare();
int launch_bp_resident(const Ctx& c, Geo g, const BpArgs& a, int32_t iters, Plane corr,
                       float* post);

// ------------------------------------------------ BP with meta-check factors
// FP64 state [W][N][21][64] (e^msg: 12 check->qubit, 3 check->measurement,
// 6 cube->measurement per site).
size_t bp_meta_state_bytes(Geo g, int64_t nw);
int launch_bp_meta_iter(const Ctx& c, Geo g, CPlane syn, int64_t nw, double p_dec, double q_dec,
                        const double* in, double* out);
int launch_bp_meta_post(const Ctx& c, Geo g, CPlane syn, int64_t nw, double p_dec,
                        double q_dec, const double* state, Plane corr, double* post);
int bp_meta_run(const Ctx& c, Geo g, CPlane syn, int64_t nw, double p_dec, double q_dec,
                int32_t iters, double* buf0, double* buf1, Plane corr, double* post);

// ----------------------------------------------------------------- CNN prior
int64_t cnn_param_count();
size_t cnn_packed_bytes();
size_t cnn_workspace_bytes(int64_t rows, int training);
int cnn_pack(const Ctx& c, const float* params, float beta, float l0, void* packed);
// llr [W][3N][64] = -CNN(syn, prev) for R = 64 W N rows; prev may be null.
int cnn_forward(const Ctx& c, Geo g, const uint64_t* syn, const uint64_t* prev, int64_t ld,
                int64_t rows, const void* packed, float* llr, void* ws);
int cnn_loss_grad(const Ctx& c, Geo g, const uint64_t* syn, const uint64_t* prev,
                  const uint64_t* target, int64_t ld, int64_t rows, const void* packed,
                  float* llr, float* grad, float* loss, void* ws);
int cnn_adam(const Ctx& c, float* params, const float* grad, float* m, float* v, int step,
             float lr, float b1, float b2, float eps, void* packed);
int copy_plane(const Ctx& c, Plane dst, CPlane src, int64_t rows, int64_t nw);

// Wrappers around hipGetLastError / timers for the launchers.
int after_launch(const Ctx& c);
int before_launch(const Ctx& c, int kclass);

// Blocks over (work items) rounded so that a workgroup index maps onto the 8
// XCDs in contiguous chunks: logical block of hardware block b.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
    const int64_t j = b & 7, i = b >> 3;
    const int64_t q = G >> 3, r = G & 7;
    return j < r ? j * (q + 1) + i : r * (q + 1) + (j - r) * q + i;
}

}  // namespace tc3d
