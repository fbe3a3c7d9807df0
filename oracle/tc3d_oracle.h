/*
 * tc3d_oracle.h -- plain CPU oracle for shot-parallel Monte Carlo decoding of
 * X errors on the L x L x L periodic 3D toric code (Scruby & Nemoto, "Local
 * Probabilistic Decoding of a Quantum Code", Quantum 2023).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this library. It shares no code, header,
 * table or constant with the GPU library; the two meet only through the
 * published definitions (the paper's equations and algorithms, and the
 * Philox4x32-10 generator of Salmon, Moraes, Dror and Shaw, SC'11).
 *
 * Representation: one shot at a time, one uint8 (0 or 1) per qubit or check,
 * FP64 belief propagation. Arrays of several shots are [shot][site].
 *
 * Geometry (Section 2): qubits on the 3L^3 edges, Z checks on the 3L^3 faces.
 *   site  v = x + L*y + L*L*z                        (coordinates mod L)
 *   edge  e(v,a) = a*L^3 + v      edge from v to v + unit(a)
 *   face  f(v,n) = n*L^3 + v      unit square at corner v with normal n;
 *         its spanning axes a < b (both != n) give the members, in order
 *         k=0: e(v,a)   k=1: e(v+unit(b),a)   k=2: e(v,b)   k=3: e(v+unit(a),b)
 */
#ifndef TC3D_ORACLE_H
#define TC3D_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tco_lattice tco_lattice;

/* Run parameters of one Monte Carlo experiment (Sections 3-4). */
typedef struct {
    double p;                 /* qubit X-error probability per cycle           */
    double q;                 /* check-outcome error probability per cycle      */
    double p_dec;             /* BP prior: l0 = ln((1-p_dec)/p_dec)             */
    double q_dec;             /* BP measurement-error prior                     */
    int32_t noisy_cycles;     /* cycles with measurement noise                  */
    int32_t perfect_final;    /* 1: one more cycle with q = 0                   */
    int32_t final_qubit_noise;/* 1: that final cycle still adds qubit noise     */
    int32_t bp_iters;         /* 0: no BP                                       */
    int32_t n_sweeps;         /* number of flip / p-flip sweeps after BP        */
    uint32_t pflip_mask;      /* bit k set: sweep k is p-flip, else flip        */
    uint64_t seed;            /* Philox key                                     */
    uint32_t subset_mask;     /* bit k set: sweep k is a subset p-flip sweep on
                                 the edge class tco_subset_class(j, m, t)        */
    int32_t bp_meta;          /* 1: BP with meta-check factors (tco_bp_meta_*)   */
    uint32_t cycle0;          /* index of this call's first cycle: noise and
                                 coins of its cycle t are those of cycle
                                 cycle0 + t, so a run split at cycle k and
                                 resumed from its residual with cycle0 = k
                                 equals the unsplit run                         */
    int32_t bp_warm;          /* 1: BP of every cycle but a call's first starts
                                 from the factor-to-variable messages the
                                 previous cycle's BP ended with (0: from the
                                 priors, the paper's BP)                       */
    double bp_damp;           /* damping g in [0, 1): each iteration's new
                                 messages become (1 - g) nu_new + g nu_old,
                                 nu_old = 0 before a cold start's first
                                 iteration (0: the paper's BP)                 */
} tco_params;

tco_lattice* tco_lattice_new(int32_t L);
void tco_lattice_free(tco_lattice* lat);
int64_t tco_n_edges(const tco_lattice* lat);
/* face_edge: [n_faces][4] member edges; edge_face/edge_slot: [n_edges][4] */
void tco_incidence(const tco_lattice* lat, int32_t* face_edge, int32_t* edge_face,
                   int32_t* edge_slot);

/* Philox4x32-10 block function. */
void tco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* floor(prob * 2^32) clamped to [0, 2^32-1]; a trial fires iff U < threshold. */
uint64_t tco_threshold(double prob);
/* Uniform 32-bit word of (site, cycle, shot, tag). */
uint32_t tco_uniform(uint64_t seed, uint32_t site, uint32_t cycle, uint64_t shot, uint32_t tag);
/* Coin of p-flip sweep `sweep` at (edge, cycle, shot). */
int tco_coin(uint64_t seed, uint32_t edge, uint32_t cycle, uint32_t sweep, uint64_t shot);

/* bits[s][i] ^= Bernoulli(prob); kind 0 = edges (qubits), 1 = faces (checks). */
void tco_sample_noise(const tco_lattice* lat, uint8_t* bits, int32_t kind, double prob,
                      uint64_t seed, uint32_t cycle, uint64_t shot0, int64_t n_shots);
/* syn[s][f] = parity of the member edges of f (xor_into: syn ^= instead). */
void tco_syndrome(const tco_lattice* lat, const uint8_t* err, uint8_t* syn, int64_t n_shots,
                  int32_t xor_into);
/* One parallel sweep of the flip rule; corr ^= F, syn ^= H F. */
void tco_flip_sweep(const tco_lattice* lat, uint8_t* syn, uint8_t* corr, int64_t n_shots);
/* One parallel sweep of p-flip with coins drawn from Philox. */
void tco_pflip_sweep(const tco_lattice* lat, uint8_t* syn, uint8_t* corr, uint64_t seed,
                     uint32_t cycle, uint32_t sweep, uint64_t shot0, int64_t n_shots);
/* One parallel p-flip sweep of a single shot with explicit coins[n_edges]. */
void tco_pflip_sweep_coins(const tco_lattice* lat, uint8_t* syn, uint8_t* corr,
                           const uint8_t* coins);
/* Subset p-flip (the recovery of Dennis et al. that the footnote of Section
 * 3.2 contrasts with p-flip): the p-flip rule on one class of qubits no two of
 * which share a check. Classes (L even): edge e(v,a) is in class
 * 4a + 2 (v_b mod 2) + (v_c mod 2), b < c the two axes other than a. */
int32_t tco_edge_class(const tco_lattice* lat, int64_t edge);
/* Class of the j-th subset sweep (of m per cycle) in cycle t. */
int32_t tco_subset_class(int32_t j, int32_t m, uint32_t cycle);
void tco_subset_pflip_sweep(const tco_lattice* lat, uint8_t* syn, uint8_t* corr, uint64_t seed,
                            uint32_t cycle, uint32_t sweep, uint64_t shot0, int64_t n_shots,
                            int32_t edge_class);
/* Sequential flip: flip the lowest-index bit with more unsatisfied than
 * satisfied checks until none is left or max_flips is reached. One shot.
 * Returns the number of flips made. */
int64_t tco_sequential_flip(const tco_lattice* lat, uint8_t* syn, uint8_t* corr,
                            int64_t max_flips);

/* One flooding BP iteration of one shot (E2-E4 with measurement nodes).
 * nu_in, nu_out: factor-to-variable messages [n_faces][4] (member order);
 * nu_in == NULL means the first iteration (variable messages = priors).
 * llr0: per-edge priors [n_edges] or NULL (then ln((1-p_dec)/p_dec)).
 * post: posterior LLRs [n_edges] (may be NULL). */
void tco_bp_step(const tco_lattice* lat, const uint8_t* syn, const double* llr0,
                 double p_dec, double q_dec, const double* nu_in, double* nu_out,
                 double* post);
/* tco_bp_step followed by damping: nu_out = (1 - damp) nu_out + damp nu_in
 * (nu_in NULL counts as 0), and post from the damped messages. */
void tco_bp_step_damped(const tco_lattice* lat, const uint8_t* syn, const double* llr0,
                        double p_dec, double q_dec, double damp, const double* nu_in,
                        double* nu_out, double* post);
/* iters >= 1 BP iterations per shot; corr[s][i] = [posterior < 0]. post is
 * [n_shots][n_edges] or NULL; llr0 is [n_shots][n_edges] or NULL. */
void tco_bp_decode(const tco_lattice* lat, const uint8_t* syn, int64_t n_shots,
                   const double* llr0, double p_dec, double q_dec, int32_t iters,
                   uint8_t* corr, double* post);

/* BP with meta-check factors (see tco_bp_meta_step in the source for the
 * messages): one measurement-error variable per check and one parity factor
 * per cube over the six measurement variables of its faces. Variable-to-
 * factor messages are clamped to +-TCO_META_CLAMP nats: the cube loops feed
 * back and the messages grow without bound, which would reach atanh(1).
 * nu: [n_faces][4], lambda: [n_faces], kappa: [n_sites][6] with cube slot j =
 * 2n the face f(c,n), j = 2n+1 the face f(c+unit(n),n). */
#define TCO_META_CLAMP 30.0
void tco_bp_meta_step(const tco_lattice* lat, const uint8_t* syn, double p_dec, double q_dec,
                      const double* nu_in, const double* lam_in, const double* kap_in,
                      double* nu_out, double* lam_out, double* kap_out, double* post);
void tco_bp_meta_decode(const tco_lattice* lat, const uint8_t* syn, int64_t n_shots,
                        double p_dec, double q_dec, int32_t iters, uint8_t* corr,
                        double* post);

/* Majority-vote readout over the L^2 logical Z strings of each axis.
 * mask[s] bit d = logical X error on qubit d; odd[s][d] = odd strings. */
void tco_logical_check(const tco_lattice* lat, const uint8_t* err, int64_t n_shots,
                       uint8_t* mask, int32_t* odd);

/* Whole experiment for shots shot0 .. shot0+n_shots-1. err: [n_shots][n_edges]
 * residual error, in/out (zero for a fresh start; the residual of an earlier
 * call to resume it, with cycle0 set). trace (NULL ok):
 * [cycles][n_shots][n_edges] residual after each cycle of this call. */
void tco_run_cycles(const tco_lattice* lat, const tco_params* prm, uint64_t shot0,
                    int64_t n_shots, uint8_t* err, uint8_t* mask, int32_t* odd,
                    uint8_t* trace);

/* ------------------------------------------------------------------ CNN prior
 * A learned per-edge prior for BP (not part of the paper's method): a
 * translation-invariant periodic 3D CNN, four 3x3x3 convolutions with
 * channels 8 -> 32 -> 32 -> 32 -> 3 and ReLU between them.
 *   input  x0[s][v][8]: channels 0-2 the measured syndrome bits of faces
 *          f(v,0..2) this cycle, 3-5 the working-syndrome bits those faces
 *          kept at the end of the previous cycle, 6-7 zero;
 *   layer  y[v][co] = b[co] + sum over offsets d in {-1,0,1}^3 and ci of
 *          W[d][ci][co] x[v + d][ci] (coordinates mod L), offset index
 *          d = (dz+1)*9 + (dy+1)*3 + (dx+1);
 *   output z[s][v][c] = logit of an error on edge e(v,c); the BP prior is
 *          llr0 = -z;
 *   loss   mean over all edges of softplus(z) - t z (binary cross-entropy
 *          with the true error bit t).
 * Parameters (FP64 here): for l = 1..4, W_l [27][cin][cout] then b_l [cout]. */
#define TCO_CNN_LAYERS 4
int64_t tco_cnn_param_count(void);
/* x0 from syndrome bit arrays [S][3N] of this cycle and of the previous one. */
void tco_cnn_input(const tco_lattice* lat, int64_t n_shots, const uint8_t* syn,
                   const uint8_t* prev, double* x0);
/* z [S][N][3]; acts (NULL ok) receives the post-ReLU activations of layers
 * 1-3, each [S][N][32], concatenated. */
void tco_cnn_forward(const tco_lattice* lat, int64_t n_shots, const double* x0,
                     const double* params, double* z, double* acts);
/* Loss and its gradient with respect to every parameter; target [S][3N]
 * (edge bits, edge index c*N + v). */
double tco_cnn_loss_grad(const tco_lattice* lat, int64_t n_shots, const double* x0,
                         const double* params, const uint8_t* target, double* grad);

#ifdef __cplusplus
}
#endif
#endif
