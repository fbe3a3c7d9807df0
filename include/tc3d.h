/*
 * tc3d.h -- C ABI of a shot-parallel Monte Carlo decoder for X errors on the
 * L x L x L periodic 3D toric code under phenomenological noise, running on
 * AMD Instinct MI355X (gfx950). The method is the p-BP decoder of
 * T. R. Scruby and K. Nemoto, "Local Probabilistic Decoding of a Quantum
 * Code", Quantum (2023): belief propagation followed by a schedule of flip and
 * p-flip sweeps, applied every code cycle, with a majority-vote readout.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Geometry (Section 2 of the paper): qubits on the 3L^3 edges, Z checks on
 * the 3L^3 faces of the periodic cubic lattice.
 *   site  v = x + L*y + L*L*z, coordinates taken mod L
 *   edge  e(v,a) = a*L^3 + v        the edge from v to v + unit(a)
 *   face  f(v,n) = n*L^3 + v        the unit square at corner v with normal n;
 *         with a < b its two spanning axes, its member edges are, in order,
 *         k=0: e(v,a)   k=1: e(v+unit(b),a)   k=2: e(v,b)   k=3: e(v+unit(a),b)
 * Shots are bit-sliced: a bit plane is a row-major uint64 array [rows][W]
 * with rows = 3L^3 (edges or faces) and W = ceil(n_shots/64) words per row;
 * bit i of word w belongs to shot 64*w + i. Bits of padding shots (64*W >
 * n_shots) are computed like any other shot and ignored by the readout.
 * Per-shot float arrays are blocked by word, [W][rows][64]: element
 * (w*rows + r)*64 + i belongs to row r and shot 64*w + i.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
 * 64-bit seed (key word 0 = low half, word 1 = high half).
 *   qubit noise of edge i, cycle t, shot s: word (s mod 4) of the block at
 *     counter (i, t, s div 4, 0); it fires when that word < floor(p * 2^32);
 *   check-outcome noise of face f: the same with counter word 3 = 1;
 *   p-flip coin of edge i, cycle t, sweep k, shot s: bit (s mod 64) of
 *     (r0 | r1 << 32) where r is the block at counter (i, t, s div 64, 2 + k).
 * Shot indices must stay below 2^34.
 *
 * Memory: every pointer is caller-owned device memory (for example a torch
 * tensor's data pointer). The library never allocates or frees device memory;
 * entry points that need scratch space take a workspace pointer and its size,
 * which must be at least what the matching *_workspace_bytes call returns.
 * Device pointers must be 8-byte aligned (EALIGN otherwise), workspaces
 * 256-byte aligned.
 *
 * Execution: every call is asynchronous on `stream` (a hipStream_t; NULL is
 * the default stream) except tc3d_run_cycles_timed, tc3d_run_jobs,
 * tc3d_autotune and runs with the TC3D_RUN_GRAPH flag, which block. Calls return TC3D_OK, or a negative TC3D_E*
 * code for invalid arguments or a failed launch; faults during execution
 * surface at the caller's next synchronisation. No exception crosses the ABI.
 *
 * State: results depend only on the arguments. The library caches, per
 * device, two facts it queries once (the LDS size of a compute unit, and
 * that the LDS-resident BP kernels were granted their LDS size) and the
 * address of its scratch array for tc3d_run_cycles_noalloc; none of them
 * changes a result. Concurrent calls on different buffers are safe, except
 * tc3d_run_cycles_noalloc calls that overlap on one device (they share its
 * scratch array).
 */
#ifndef TC3D_H
#define TC3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TC3D_OK = 0,
    TC3D_EINVAL = -1,     /* bad size, probability, flag or lattice          */
    TC3D_EALIGN = -2,     /* misaligned pointer                              */
    TC3D_EHIP = -3,       /* a HIP launch or runtime call failed             */
    TC3D_EWORKSPACE = -4  /* workspace missing or smaller than required      */
};

/* Lattice sizes. A plain value; build it with tc3d_make_lattice. */
typedef struct {
    int32_t L;
    int32_t reserved;   /* zero */
    int64_t n_sites;    /* L^3   */
    int64_t n_edges;    /* 3 L^3 */
    int64_t n_faces;    /* 3 L^3 */
} tc3d_lattice;

/* Section 2: the [[3L^3, 3, L]] code on the L^3 torus. 3 <= L <= 512. */
int tc3d_make_lattice(int32_t L, tc3d_lattice* out);

/* Phenomenological noise (Sections 3.1 and 4.1): XOR an independent
 * Bernoulli(prob) bit into every entry of a plane. kind 0: edge plane (qubit
 * X errors, counter word 3 = 0); kind 1: face plane (check-outcome errors,
 * counter word 3 = 1). The plane covers shots shot0 .. shot0 + 64*W - 1 with
 * W = ceil(n_shots/64); shot0 must be a multiple of 64. 0 <= prob <= 1. */
int tc3d_sample_noise(const tc3d_lattice* lat, uint64_t* plane, int32_t kind, double prob,
                      uint64_t seed, uint32_t cycle, uint64_t shot0, int64_t n_shots,
                      void* stream);

/* Section 2: the Z-check syndrome. syn[f] = XOR of err over the four member
 * edges of face f, for every word. xor_into != 0 XORs the result into syn
 * instead of overwriting it (used to update a working syndrome with the
 * parity of a correction). err and syn are [3L^3][n_words]; they must not
 * overlap. */
int tc3d_syndrome(const tc3d_lattice* lat, const uint64_t* err, uint64_t* syn,
                  int64_t n_words, int32_t xor_into, void* stream);

/* Apply a correction and carry the residual (Section 3.2: the accumulated
 * correction is applied at the end of the cycle; Section 1: residual errors
 * carry over): err ^= corr over two edge planes [3L^3][n_words]. */
int tc3d_apply_correction(const tc3d_lattice* lat, uint64_t* err, const uint64_t* corr,
                          int64_t n_words, void* stream);

/* Scratch needed by one flip, p-flip or subset p-flip sweep: one edge plane. */
size_t tc3d_sweep_workspace_bytes(const tc3d_lattice* lat, int64_t n_words);

/* flip (Section 3.1) in its parallel form (Section 3.2): every qubit with
 * more unsatisfied than satisfied checks (3 or 4 of its 4) is flipped, all
 * decided against the same syndrome. corr ^= F and syn ^= H F, in place. */
int tc3d_flip_sweep(const tc3d_lattice* lat, uint64_t* syn, uint64_t* corr, int64_t n_words,
                    void* ws, size_t ws_bytes, void* stream);

/* p-flip (Section 3.2): as flip, and a qubit with exactly 2 of 4 checks
 * unsatisfied flips when its coin (see Randomness; cycle and sweep index
 * select the counter) is 1, i.e. with probability 1/2. shot0: shot of bit 0
 * of word 0, a multiple of 64. */
int tc3d_pflip_sweep(const tc3d_lattice* lat, uint64_t* syn, uint64_t* corr, int64_t n_words,
                     uint64_t seed, uint32_t cycle, uint32_t sweep, uint64_t shot0, void* ws,
                     size_t ws_bytes, void* stream);

/* Subset p-flip: the recovery rule of Dennis et al. for the 4D toric code,
 * which the footnote of Section 3.2 contrasts with p-flip; it acts only on a
 * set of qubits no two of which share a check. Here the p-flip rule is
 * applied to the edges of one class (0 <= edge_class < 12): edge e(v,a) has
 * class 4a + 2 (v_b mod 2) + (v_c mod 2), b < c the two other axes. With L
 * even (required, else EINVAL) two edges of a class never share a face, so
 * the sweep equals the rule applied to the class one edge at a time. Coins
 * as in tc3d_pflip_sweep. */
int tc3d_subset_pflip_sweep(const tc3d_lattice* lat, uint64_t* syn, uint64_t* corr,
                            int64_t n_words, uint64_t seed, uint32_t cycle, uint32_t sweep,
                            uint64_t shot0, int32_t edge_class, void* ws, size_t ws_bytes,
                            void* stream);

/* Scratch of tc3d_bp_decode: two message buffers of 12 L^3 S_pad floats. */
size_t tc3d_bp_workspace_bytes(const tc3d_lattice* lat, int64_t n_shots);

/* Local belief propagation (Section 4.1, equations for the LLR, the factor
 * and variable messages and the posterior), flooding schedule, with one
 * measurement-error variable per check whose constant message contributes the
 * factor meas_factor = tanh(ln((1-q)/q)/2) = 1 - 2q to every check product.
 * Runs exactly `iters` >= 1 iterations in FP32, then corr_out (an edge plane,
 * overwritten) gets bit 1 where the posterior LLR is < 0.
 *   syn       face plane [3L^3][W], W = ceil(n_shots/64)
 *   llr0      per-edge priors [W][3L^3][64] in nats, or NULL to use
 *             llr0_scalar = ln((1-p)/p) on every edge
 *   post_out  posterior LLRs [W][3L^3][64], or NULL
 * 0 <= meas_factor < 1; |llr0_scalar| <= 40 (per-edge priors are clamped to
 * +-40 nats).
 * bp_path picks the kernels; it never changes a result:
 *   TC3D_BP_AUTO       the resident kernel where it applies, else streaming;
 *   TC3D_BP_STREAMING  one launch per iteration over messages in HBM; with
 *                      the scalar prior the last iteration and the posterior
 *                      (E4) share one launch that stores no messages;
 *   TC3D_BP_RESIDENT   the whole decode of each shot inside one workgroup,
 *                      its messages in LDS: scalar prior and at most 3072
 *                      sites (L <= 14), else EINVAL;
 *   TC3D_BP_STREAMING_SPLIT  as STREAMING, with the last iteration and the
 *                      posterior launched separately.
 * All four are bit-identical. */
enum {
    TC3D_BP_AUTO = 0,
    TC3D_BP_STREAMING = 1,
    TC3D_BP_RESIDENT = 2,
    TC3D_BP_STREAMING_SPLIT = 3
};
int tc3d_bp_decode(const tc3d_lattice* lat, const uint64_t* syn, int64_t n_shots,
                   const float* llr0, float llr0_scalar, float meas_factor, int32_t iters,
                   int32_t bp_path, uint64_t* corr_out, float* post_out, void* ws,
                   size_t ws_bytes, void* stream);

/* One flooding BP iteration, for inspection and parity checks. The state is
 * the factor-to-variable messages in multiplicative form, e^nu (the form the
 * decoder iterates in: sums of messages become products and the check rule
 * needs no exp or log). Arrays are FP32 [W][L^3][12][64]: row
 * (w L^3 + v) 12 + 4n + k holds e^nu of the message from face f(v,n) to its
 * member edge k for the 64 shots of word w. nu_in == NULL means the first
 * iteration (every variable-to-check message equals its prior). post_out
 * (NULL ok) receives the posterior LLR (nats) computed from nu_out,
 * [W][3L^3][64]. damp (0 <= damp < 1; scalar prior only) damps the new
 * messages: nu = (1 - damp) nu_new + damp nu_in, nu_in NULL counting as 0
 * (a reading of BP the paper leaves open; 0 is the paper's BP). */
int tc3d_bp_step(const tc3d_lattice* lat, const uint64_t* syn, int64_t n_shots,
                 const float* llr0, float llr0_scalar, float meas_factor, float damp,
                 const float* nu_in, float* nu_out, float* post_out, void* stream);

/* BP with meta-check factors: the extension of the factor graph that Section
 * 4.1 describes and leaves out, and that the closing discussion names as a
 * likely improvement. Each check has a measurement-error variable (prior
 * ln((1-q_dec)/q_dec)), a member of its check and of the meta-checks of the
 * two cubes that contain the check's face; a meta-check requires the six
 * measurement variables of a cube to have the parity of its six measured
 * outcomes. Flooding schedule, FP64, variable-to-factor messages clamped to
 * +-30 nats (the cube loops feed back and the messages grow without bound).
 *   syn       face plane [3L^3][W]
 *   corr_out  edge plane [3L^3][W], [posterior < 0] after `iters` iterations
 *   post_out  FP64 [W][3L^3][64] posterior LLRs, or NULL
 * 0 < p_dec, q_dec < 0.5. Workspace: tc3d_bp_meta_workspace_bytes. */
size_t tc3d_bp_meta_workspace_bytes(const tc3d_lattice* lat, int64_t n_shots);
int tc3d_bp_meta_decode(const tc3d_lattice* lat, const uint64_t* syn, int64_t n_shots,
                        double p_dec, double q_dec, int32_t iters, uint64_t* corr_out,
                        double* post_out, void* ws, size_t ws_bytes, void* stream);
/* One iteration of it, for inspection. State: FP64 [W][L^3][21][64] of e^msg
 * per site v: slots 0..11 the check -> qubit messages of faces f(v,0..2) (slot
 * 4n+k: face f(v,n) to its member k, the order of tc3d_bp_step), 12..14 the
 * check -> measurement messages of those faces, 15..20 the messages of cube
 * v to its faces (slot 15 + 2n: f(v,n); 15 + 2n + 1: f(v + unit(n), n)).
 * state_in NULL = first iteration. post_out as in tc3d_bp_meta_decode. */
int tc3d_bp_meta_step(const tc3d_lattice* lat, const uint64_t* syn, int64_t n_shots,
                      double p_dec, double q_dec, const double* state_in, double* state_out,
                      double* post_out, void* stream);

/* Majority-vote readout (Section 3.1 and Fig. 2 caption): for each axis d,
 * count the L^2 disjoint logical Z strings along d (the L d-edges through
 * fixed other coordinates) whose error parity is odd; the shot has a logical
 * X error on qubit d when that count is at least L^2/2 (a tie counts as a
 * failure). mask_out[s] bit d records it; odd_out (NULL ok) is
 * [n_shots][3] int32 counts. err is an edge plane [3L^3][ceil(n_shots/64)].
 * Scratch: the string parities, tc3d_logical_check_workspace_bytes. */
size_t tc3d_logical_check_workspace_bytes(const tc3d_lattice* lat, int64_t n_shots);
int tc3d_logical_check(const tc3d_lattice* lat, const uint64_t* err, int64_t n_shots,
                       uint8_t* mask_out, int32_t* odd_out, void* ws, size_t ws_bytes,
                       void* stream);

/* One Monte Carlo experiment. */
typedef struct {
    double p;                  /* qubit X-error probability per cycle           */
    double q;                  /* check-outcome error probability per cycle      */
    double p_dec;              /* BP prior: llr0 = ln((1-p_dec)/p_dec)           */
    double q_dec;              /* BP measurement prior: factor 1 - 2 q_dec      */
    int32_t noisy_cycles;      /* cycles with check-outcome noise                */
    int32_t perfect_final;     /* 1: one more cycle with perfect measurements   */
    int32_t final_qubit_noise; /* 1: that cycle still adds qubit noise          */
    int32_t bp_iters;          /* BP iterations per cycle; 0 disables BP         */
    int32_t n_sweeps;          /* flip / p-flip sweeps per cycle (0..32)        */
    uint32_t pflip_mask;       /* bit k set: sweep k is p-flip, else flip       */
    uint64_t seed;             /* Philox key                                     */
    uint64_t shot0;            /* first shot index, a multiple of 64            */
    int64_t n_shots;           /* shots in this call                             */
    int64_t batch_shots;       /* shots decoded together (multiple of 64);
                                  0 picks a size that keeps the workspace near
                                  24 GiB                                         */
    int32_t bp_tile;           /* BP traversal (a tuning knob that never changes
                                  results): 0 = the library's choice (whole
                                  x-y planes in memory order up to L = 64,
                                  bands of 8 rows above); T > 0: T x T site
                                  columns; T < 0: bands of whole x rows, -T
                                  rows high (-L: whole planes)                */
    uint32_t subset_mask;      /* bit k set: sweep k is a subset p-flip sweep
                                  (see tc3d_subset_pflip_sweep); the j-th of the
                                  m such sweeps of cycle t acts on edge class
                                  (j + t m) mod 12. Needs L even; 0 = none      */
    int32_t bp_meta;           /* 1: BP with meta-check factors
                                  (tc3d_bp_meta_decode) instead of the paper's */
    uint32_t cycle0;           /* index of this call's first cycle (0 for a
                                  fresh run): its cycle t draws the noise and
                                  coins of cycle cycle0 + t, so a run split
                                  after cycle k and resumed from its residual
                                  err_state with cycle0 = k equals the unsplit
                                  run bit for bit                             */
    int32_t bp_path;           /* TC3D_BP_AUTO / _STREAMING / _RESIDENT /
                                  _STREAMING_SPLIT (see tc3d_bp_decode);
                                  never changes a result                      */
    int32_t bp_warm;           /* 1: BP of every cycle but the call's first
                                  starts from the messages the previous
                                  cycle's BP ended with, 0: from the priors
                                  (the paper's BP); a reading the paper leaves
                                  open. A resumed call starts cold.            */
    double bp_damp;            /* damping 0 <= g < 1 of the BP messages:
                                  nu = (1 - g) nu_new + g nu_old, nu_old = 0
                                  before a cold start (0: the paper's BP);
                                  streaming kernels, scalar prior            */
    uint32_t flags;            /* TC3D_RUN_GRAPH: tc3d_run_cycles captures all
                                  its launches into one HIP graph, launches it
                                  and waits for it (for runs of many short
                                  launches); never changes a result          */
    int32_t bp_occupancy;      /* workgroups per compute unit of the streaming
                                  BP passes that read stored messages (the
                                  iterations and the fused last pass): 0 = the
                                  library's choice (4), 1..8 = that many (8: no
                                  cap); a tuning knob that never changes a
                                  result                                      */
} tc3d_run_params;

enum { TC3D_RUN_GRAPH = 1 };

size_t tc3d_run_workspace_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm);

/* The whole decoding experiment of Sections 3-4 for shots shot0 ..
 * shot0 + n_shots - 1. For each cycle t = 0 .. cycles-1 (cycles =
 * noisy_cycles + perfect_final): qubit noise (probability p; 0 in the perfect
 * cycle unless final_qubit_noise), syndrome measurement with check-outcome
 * noise (q; 0 in the perfect cycle), BP if bp_iters > 0 whose correction also
 * updates the working syndrome, then the flip / p-flip sweeps on the working
 * syndrome, then the accumulated correction is applied and the residual error
 * carries over. Finally the majority-vote readout of the residual.
 *   err_state  edge plane [3L^3][ceil(n_shots/64)], in/out (zero to start, or
 *              the residual of an earlier call to continue it: checkpoint =
 *              err_state + the next cycle index, passed as cycle0)
 *   mask_out   [n_shots] uint8, odd_out [n_shots][3] int32 or NULL
 * bp_iters > 0 needs 0 < p_dec < 0.5 and 0 < q_dec < 0.5. */
int tc3d_run_cycles(const tc3d_lattice* lat, const tc3d_run_params* prm, uint64_t* err_state,
                    uint8_t* mask_out, int32_t* odd_out, void* ws, size_t ws_bytes,
                    void* stream);

/* tc3d_run_cycles for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the scratch comes from a fixed array of 128 MiB that the library keeps on
 * each device it runs on until the process ends, and the call allocates
 * nothing. The caller passes only the inputs and outputs of tc3d_run_cycles.
 * With batch_shots = 0 the largest batch whose scratch fits is chosen (one
 * 64-shot word of the streaming BP state fits up to L = 24); a run whose
 * smallest batch, or whose given batch_shots, needs more than 128 MiB is
 * refused with TC3D_EWORKSPACE. Every call on a device shares that device's
 * array, which keeps the last call's contents (nothing in it has to start at
 * zero): calls that overlap on one device race, so order them on one stream
 * or synchronise between them. Results equal tc3d_run_cycles bit for bit. */
int tc3d_run_cycles_noalloc(const tc3d_lattice* lat, const tc3d_run_params* prm,
                            uint64_t* err_state, uint8_t* mask_out, int32_t* odd_out,
                            void* stream);

/* Kernel classes reported by tc3d_run_cycles_timed. */
enum {
    TC3D_K_BP_ITER = 0,   /* one BP iteration that reads and writes messages */
    TC3D_K_BP_FIRST = 1,  /* a BP iteration whose inputs are implied by the syndrome */
    TC3D_K_BP_POST = 2,   /* posterior + hard decision                      */
    TC3D_K_NOISE = 3,     /* qubit noise                                     */
    TC3D_K_SYNDROME = 4,  /* syndrome measurement / working-syndrome update */
    TC3D_K_SWEEP = 5,     /* flip / p-flip decision pass                    */
    TC3D_K_APPLY = 6,     /* plane XOR / clear                               */
    TC3D_K_READOUT = 7,   /* majority vote                                   */
    TC3D_K_CNN = 8,       /* CNN prior (input packing, convolutions)         */
    TC3D_K_COUNT = 9
};

typedef struct {
    double ms[TC3D_K_COUNT];        /* summed HIP-event durations per class */
    int64_t launches[TC3D_K_COUNT]; /* launches per class                   */
    double total_ms;                /* first to last event of the call      */
    int64_t bp_decisions;           /* BP hard decisions made (edges x
                                       padded shots x decoded cycles)      */
    int64_t bp_near_ties;           /* of those, posteriors |l| < 1e-3 nats:
                                       where FP32 and FP64 may decide apart */
} tc3d_timing;

/* tc3d_run_cycles with HIP events recorded on `stream` around every run of
 * consecutive launches of one kernel class (ms[k] then includes the short
 * gaps between the launches of a run; launches[k] counts every launch) and
 * with the near-tie count of the paper's BP (FP32 kernels; 0 for BP with
 * meta-checks); blocks until the work is done and fills *timing. */
int tc3d_run_cycles_timed(const tc3d_lattice* lat, const tc3d_run_params* prm,
                          uint64_t* err_state, uint8_t* mask_out, int32_t* odd_out, void* ws,
                          size_t ws_bytes, void* stream, tc3d_timing* timing);

/* ------------------------------------------------------------- CNN prior
 * A learned per-edge prior for BP (an addition to the paper's method, whose
 * BP starts from the channel prior ln((1-p)/p)): a translation-invariant
 * periodic 3D CNN of four 3x3x3 convolutions, channels 8 -> 32 -> 32 -> 32 ->
 * 3, ReLU between them, BF16 weights and activations, FP32 accumulation.
 *   input of site v: the measured syndrome bits of faces f(v,0..2) this
 *     cycle and the working-syndrome bits those faces kept at the end of the
 *     previous cycle (zero in the first cycle);
 *   layer: y[v][co] = b[co] + sum_{d, ci} W[d][ci][co] x[v + off(d)][ci] with
 *     off(d) = (d%3 - 1, d/3%3 - 1, d/9 - 1), coordinates mod L;
 *   output: z[v][c] = logit of an error on edge e(v,c); llr0 = -z.
 * Parameters are an FP32 vector of tc3d_cnn_param_count() floats: for each
 * layer W [27][cin][cout] then b [cout]. The kernels read a packed BF16 copy
 * (tc3d_cnn_packed_bytes(), made by tc3d_cnn_pack). */
int64_t tc3d_cnn_param_count(void);
size_t tc3d_cnn_packed_bytes(void);
/* Packs params for the kernels with the prior blended with the channel prior
 * l0 = ln((1-p)/p) at strength 0 <= beta <= 1: the packed network's prior is
 * llr0 = l0 + beta (llr_cnn - l0) (its last layer's weights scale by beta,
 * its biases become beta b - (1 - beta) l0). beta = 1 packs the network as
 * it is (training uses that); beta = 0 gives the paper's prior. |l0| <= 40. */
int tc3d_cnn_pack(const float* params, float beta, float l0, void* packed, void* stream);
/* Scratch of one pass over n_shots shots (training != 0: forward + backward). */
size_t tc3d_cnn_workspace_bytes(const tc3d_lattice* lat, int64_t n_shots, int32_t training);
/* llr_out [W][3L^3][64] = -z for the shots of the face planes syn and prev
 * ([3L^3][W], prev NULL = zeros). */
int tc3d_cnn_forward(const tc3d_lattice* lat, const uint64_t* syn, const uint64_t* prev,
                     int64_t n_shots, const void* packed, float* llr_out, void* ws,
                     size_t ws_bytes, void* stream);
/* Mean binary cross-entropy of the logits against the error bits of the
 * edge plane `target`, its gradient grad [param_count] (FP32) and the mean
 * loss (*loss, one device float). Every shot of the 64 W covered counts. */
int tc3d_cnn_loss_grad(const tc3d_lattice* lat, const uint64_t* syn, const uint64_t* prev,
                       const uint64_t* target, int64_t n_shots, const void* packed,
                       float* llr_out, float* grad, float* loss, void* ws, size_t ws_bytes,
                       void* stream);
/* One Adam step (step >= 1) on params with moment buffers m, v, then repack. */
int tc3d_cnn_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                  float beta1, float beta2, float eps, void* packed, void* stream);
/* tc3d_run_cycles with the BP prior of every cycle taken from the CNN
 * (llr0 = -z of that cycle's syndromes) instead of ln((1-p_dec)/p_dec). */
size_t tc3d_run_cnn_workspace_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm);
int tc3d_run_cycles_cnn(const tc3d_lattice* lat, const tc3d_run_params* prm, const void* packed,
                        uint64_t* err_state, uint8_t* mask_out, int32_t* odd_out, void* ws,
                        size_t ws_bytes, void* stream);
int tc3d_run_cycles_cnn_timed(const tc3d_lattice* lat, const tc3d_run_params* prm,
                              const void* packed, uint64_t* err_state, uint8_t* mask_out,
                              int32_t* odd_out, void* ws, size_t ws_bytes, void* stream,
                              tc3d_timing* timing);

/* -------------------------------------------------------- batched jobs
 * Many experiments of Sections 3-4 at once: any mix of lattice sizes, error
 * rates, cycle counts, decoders and seeds (the sweeps behind Figs. 2, 6, 7
 * and Table 1 are such mixes). Every job is exactly tc3d_run_cycles on its
 * own buffers, so its results do not depend on the other jobs or the flags. */
typedef struct {
    int32_t L;               /* lattice size of this job                     */
    int32_t reserved;        /* zero                                          */
    tc3d_run_params prm;     /* its experiment                                */
    uint64_t* err_state;     /* [3L^3][ceil(n_shots/64)], in/out              */
    uint8_t* mask_out;       /* [n_shots]                                     */
    int32_t* odd_out;        /* [n_shots][3] or NULL                          */
} tc3d_job;

enum {
    TC3D_JOBS_CONCURRENT = 1, /* each job on its own stream branch, so the
                                 kernels of small jobs overlap               */
    TC3D_JOBS_GRAPH = 2       /* capture every launch of every job into one
                                 HIP graph and launch that graph once        */
};

/* Workspace of tc3d_run_jobs: the sum of the jobs' run workspaces (each
 * rounded up to 256 bytes), 0 for invalid input. */
size_t tc3d_run_jobs_workspace_bytes(const tc3d_job* jobs, int32_t n_jobs);
/* Runs n_jobs (1 .. 4096) jobs, all validated before anything is enqueued.
 * Ordered after prior work on `stream`; blocks until every job is done (the
 * graph and the job streams are released before returning). */
int tc3d_run_jobs(const tc3d_job* jobs, int32_t n_jobs, void* ws, size_t ws_bytes,
                  int32_t flags, void* stream);

/* Autotuning of the knobs that never change results, one after the other
 * (each stage keeps the best of the previous ones):
 *   1. the BP iteration schedule, bp_path: one launch per iteration over
 *      messages in HBM, or (L <= 14) the whole decode in one launch per batch
 *      with the messages in LDS;
 *   2. the streaming traversal, bp_tile: planes, square columns or x-row
 *      bands;
 *   3. the streaming iterations' occupancy, bp_occupancy: 3 to 8 workgroups
 *      per compute unit (how many sites' loads are in flight per CU);
 *   4. the shots decoded together, batch_shots: the automatic size, 1/2, 1/4.
 * Each candidate decodes the first probe_cycles noisy cycles of *prm's shots
 * (timed with HIP events, after one untimed warm-up run) and the fastest is
 * written back into *prm. The candidates tried (at most max_out are
 * reported; *n_out = their number) are returned with their time. Workspace:
 * tc3d_autotune_workspace_bytes. Blocks until done. */
typedef struct {
    int32_t bp_tile;
    int32_t bp_path;
    int64_t batch_shots;
    double ms;
    int32_t bp_occupancy;
    int32_t reserved;
} tc3d_tune_choice;
size_t tc3d_autotune_workspace_bytes(const tc3d_lattice* lat, const tc3d_run_params* prm);
int tc3d_autotune(const tc3d_lattice* lat, tc3d_run_params* prm, int32_t probe_cycles,
                  void* ws, size_t ws_bytes, tc3d_tune_choice* out, int32_t max_out,
                  int32_t* n_out, void* stream);

/* -------------------------------------------------- measurement utility
 * Not part of the paper's method: a plain device copy of n_bytes (a multiple
 * of 16; 16-byte aligned, non-overlapping buffers), 16 bytes per lane, with
 * non-temporal stores if asked. Its rocprofv3 byte counters calibrate the
 * counters of the other kernels, and its rate is the read + write streaming
 * ceiling the BP iteration is compared with. */
int tc3d_stream_copy(void* dst, const void* src, int64_t n_bytes, int32_t nontemporal,
                     void* stream);

/* Human-readable text of a return code. */
const char* tc3d_strerror(int code);

/* SHA-256 (hex) of the sources the library was built from, so that a caller
 * can refuse a library older than its sources. */
const char* tc3d_build_id(void);

#ifdef __cplusplus
}
#endif
#endif
