/*
 * tc3d_oracle.c -- plain CPU oracle (see tc3d_oracle.h).
 *
 * TEST INFRASTRUCTURE: only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this file's library. It is deliberately slow
 * and literal: every step follows the paper's definitions in the paper's order,
 * one shot at a time, with uint8 bits and FP64 arithmetic. No blocking, fusion
 * or reordering beyond what the definitions state.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - noise per cycle: every qubit flips with probability p, then every check
 *     outcome flips with probability q (phenomenological model, Sections 3.1
 *     and 4.1, p = q in all experiments);
 *   - the syndrome is measured once per cycle; BP, flip and p-flip all act on
 *     a working copy that is updated with the parity of every correction they
 *     make; the accumulated correction is applied at the end of the cycle
 *     (the schedule listed in Section 3.2);
 *   - BP restarts from the priors every cycle and always runs the requested
 *     number of iterations, then flips every bit with posterior < 0
 *     (Section 4.1, "local" BP); a posterior of exactly 0 is not flipped;
 *   - after the noisy cycles one more cycle may run with perfect measurements
 *     (qubit noise still on unless disabled), decoded the same way;
 *   - majority vote: a logical error on axis d is declared when at least half
 *     of the L^2 parallel logical Z strings along d have odd parity (a tie
 *     counts as a failure).
 */
#include "tc3d_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct tco_lattice {
    int32_t L;
    int64_t n_sites, n_edges, n_faces;
    int32_t* face_edge; /* [n_faces][4]                               */
    int32_t* edge_face; /* [n_edges][4]: the faces containing the edge  */
    int32_t* edge_slot; /* [n_edges][4]: member index k inside that face */
};

/* ---------------------------------------------------------------- geometry */

static int64_t site_of(int32_t L, int64_t x, int64_t y, int64_t z) {
    x = ((x % L) + L) % L;
    y = ((y % L) + L) % L;
    z = ((z % L) + L) % L;
    return x + (int64_t)L * (y + (int64_t)L * z);
}

/* Section 2: one qubit per edge of the cubic lattice, one Z check per face;
 * a face check acts on the four edges of its boundary. */
tco_lattice* tco_lattice_new(int32_t L) {
    if (L < 2) return NULL;
    tco_lattice* lat = (tco_lattice*)calloc(1, sizeof(tco_lattice));
    lat->L = L;
    lat->n_sites = (int64_t)L * L * L;
    lat->n_edges = 3 * lat->n_sites;
    lat->n_faces = 3 * lat->n_sites;
    lat->face_edge = (int32_t*)malloc(sizeof(int32_t) * 4 * lat->n_faces);
    lat->edge_face = (int32_t*)malloc(sizeof(int32_t) * 4 * lat->n_edges);
    lat->edge_slot = (int32_t*)malloc(sizeof(int32_t) * 4 * lat->n_edges);
    int32_t* fill = (int32_t*)calloc(lat->n_edges, sizeof(int32_t));
    const int64_t N = lat->n_sites;
    for (int32_t n = 0; n < 3; ++n) {
        /* the two axes spanning a face with normal n, in increasing order */
        int32_t a = (n == 0) ? 1 : 0;
        int32_t b = (n == 2) ? 1 : 2;
        for (int64_t z = 0; z < L; ++z)
            for (int64_t y = 0; y < L; ++y)
                for (int64_t x = 0; x < L; ++x) {
                    int64_t c[3] = {x, y, z};
                    int64_t v = site_of(L, x, y, z);
                    int64_t f = n * N + v;
                    int64_t ca[3] = {c[0], c[1], c[2]};
                    int64_t cb[3] = {c[0], c[1], c[2]};
                    ca[a] += 1; /* v + unit(a) */
                    cb[b] += 1; /* v + unit(b) */
                    int64_t m[4];
                    m[0] = a * N + v;
                    m[1] = a * N + site_of(L, cb[0], cb[1], cb[2]);
                    m[2] = b * N + v;
                    m[3] = b * N + site_of(L, ca[0], ca[1], ca[2]);
                    for (int k = 0; k < 4; ++k) {
                        lat->face_edge[4 * f + k] = (int32_t)m[k];
                        int32_t j = fill[m[k]]++;
                        if (j < 4) {
                            lat->edge_face[4 * m[k] + j] = (int32_t)f;
                            lat->edge_slot[4 * m[k] + j] = k;
                        }
                    }
                }
    }
    free(fill);
    return lat;
}

void tco_lattice_free(tco_lattice* lat) {
    if (!lat) return;
    free(lat->face_edge);
    free(lat->edge_face);
    free(lat->edge_slot);
    free(lat);
}

int64_t tco_n_edges(const tco_lattice* lat) { return lat->n_edges; }

void tco_incidence(const tco_lattice* lat, int32_t* face_edge, int32_t* edge_face,
                   int32_t* edge_slot) {
    if (face_edge) memcpy(face_edge, lat->face_edge, sizeof(int32_t) * 4 * lat->n_faces);
    if (edge_face) memcpy(edge_face, lat->edge_face, sizeof(int32_t) * 4 * lat->n_edges);
    if (edge_slot) memcpy(edge_slot, lat->edge_slot, sizeof(int32_t) * 4 * lat->n_edges);
}

/* ------------------------------------------------------------- randomness */

/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 Philox
 * S-box; each round multiplies words 0 and 2 by the two round multipliers,
 * the high halves are mixed with the other two words and the key, and the
 * key is advanced by the two Weyl increments between rounds. */
void tco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

uint64_t tco_threshold(double prob) {
    if (!(prob > 0.0)) return 0;
    double t = floor(prob * 4294967296.0);
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint64_t)t;
}

/* The uniform word of shot s is word (s mod 4) of the block at counter
 * (site, cycle, s div 4, tag); key = (low, high) 32-bit halves of the seed. */
uint32_t tco_uniform(uint64_t seed, uint32_t site, uint32_t cycle, uint64_t shot, uint32_t tag) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {site, cycle, (uint32_t)(shot / 4), tag};
    uint32_t out[4];
    tco_philox4x32_10(ctr, key, out);
    return out[shot % 4];
}

/* A p-flip coin is one bit of the 64-bit word (r0 | r1 << 32) of the block at
 * counter (edge, cycle, s div 64, 2 + sweep): bit s mod 64. It is 1 with
 * probability exactly 1/2, matching "x < 0.5" for x uniform on (0,1) in the
 * p-flip algorithm (Section 3.2). */
int tco_coin(uint64_t seed, uint32_t edge, uint32_t cycle, uint32_t sweep, uint64_t shot) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {edge, cycle, (uint32_t)(shot / 64), 2u + sweep};
    uint32_t out[4];
    tco_philox4x32_10(ctr, key, out);
    uint64_t w = (uint64_t)out[0] | ((uint64_t)out[1] << 32);
    return (int)((w >> (shot % 64)) & 1u);
}

/* ------------------------------------------------------------------ noise */

/* Phenomenological noise (Sections 3.1, 4.1): independent bit flips with
 * probability prob on every qubit (kind 0) or check outcome (kind 1). */
void tco_sample_noise(const tco_lattice* lat, uint8_t* bits, int32_t kind, double prob,
                      uint64_t seed, uint32_t cycle, uint64_t shot0, int64_t n_shots) {
    int64_t n = (kind == 0) ? lat->n_edges : lat->n_faces;
    uint64_t th = tco_threshold(prob);
    for (int64_t s = 0; s < n_shots; ++s)
        for (int64_t i = 0; i < n; ++i)
            if ((uint64_t)tco_uniform(seed, (uint32_t)i, cycle, shot0 + (uint64_t)s,
                                      (uint32_t)kind) < th)
                bits[s * n + i] ^= 1u;
}

/* --------------------------------------------------------------- syndrome */

/* Section 2: a Z check on a face reports the parity of X errors on its four
 * boundary edges. */
void tco_syndrome(const tco_lattice* lat, const uint8_t* err, uint8_t* syn, int64_t n_shots,
                  int32_t xor_into) {
    const int64_t n = lat->n_edges, m = lat->n_faces;
    for (int64_t s = 0; s < n_shots; ++s) {
        const uint8_t* e = err + s * n;
        uint8_t* o = syn + s * m;
        for (int64_t f = 0; f < m; ++f) {
            uint8_t par = 0;
            for (int k = 0; k < 4; ++k) par ^= e[lat->face_edge[4 * f + k]];
            o[f] = xor_into ? (uint8_t)(o[f] ^ par) : par;
        }
    }
}

/* ---------------------------------------------------------- flip / p-flip */

/* |UNSAT(b)|: unsatisfied checks among the four containing bit b. */
static int unsat_count(const tco_lattice* lat, const uint8_t* syn, int64_t b) {
    int u = 0;
    for (int j = 0; j < 4; ++j) u += syn[lat->edge_face[4 * b + j]];
    return u;
}

/* Apply a set of flips found in one parallel sweep: every flipped bit toggles
 * the correction and the four checks containing it. */
static void apply_flips(const tco_lattice* lat, const uint8_t* flips, uint8_t* syn,
                        uint8_t* corr) {
    for (int64_t b = 0; b < lat->n_edges; ++b) {
        if (!flips[b]) continue;
        corr[b] ^= 1u;
        for (int j = 0; j < 4; ++j) syn[lat->edge_face[4 * b + j]] ^= 1u;
    }
}

/* flip (Section 3.1), parallel version (Section 3.2): the rule "flip b when
 * |SAT(b)| < |UNSAT(b)|" is evaluated on every bit against the same syndrome,
 * then all selected bits are flipped at once. */
void tco_flip_sweep(const tco_lattice* lat, uint8_t* syn, uint8_t* corr, int64_t n_shots) {
    const int64_t n = lat->n_edges, m = lat->n_faces;
    uint8_t* F = (uint8_t*)malloc(n);
    for (int64_t s = 0; s < n_shots; ++s) {
        uint8_t* sy = syn + s * m;
        for (int64_t b = 0; b < n; ++b) {
            int unsat = unsat_count(lat, sy, b);
            int sat = 4 - unsat;
            F[b] = (uint8_t)(sat < unsat);
        }
        apply_flips(lat, F, sy, corr + s * n);
    }
    free(F);
}

/* p-flip (Section 3.2): as flip, and a bit with |SAT| = |UNSAT| flips when its
 * coin is 1. All bits are evaluated against the same syndrome. */
void tco_pflip_sweep_coins(const tco_lattice* lat, uint8_t* syn, uint8_t* corr,
                           const uint8_t* coins) {
    const int64_t n = lat->n_edges;
    uint8_t* F = (uint8_t*)malloc(n);
    for (int64_t b = 0; b < n; ++b) {
        int unsat = unsat_count(lat, syn, b);
        int sat = 4 - unsat;
        if (sat < unsat)
            F[b] = 1;
        else if (sat == unsat)
            F[b] = (uint8_t)(coins[b] != 0);
        else
            F[b] = 0;
    }
    apply_flips(lat, F, syn, corr);
    free(F);
}

void tco_pflip_sweep(const tco_lattice* lat, uint8_t* syn, uint8_t* corr, uint64_t seed,
                     uint32_t cycle, uint32_t sweep, uint64_t shot0, int64_t n_shots) {
    const int64_t n = lat->n_edges, m = lat->n_faces;
    uint8_t* coins = (uint8_t*)malloc(n);
    for (int64_t s = 0; s < n_shots; ++s) {
        for (int64_t b = 0; b < n; ++b)
            coins[b] = (uint8_t)tco_coin(seed, (uint32_t)b, cycle, sweep, shot0 + (uint64_t)s);
        tco_pflip_sweep_coins(lat, syn + s * m, corr + s * n, coins);
    }
    free(coins);
}

/* Subset p-flip. Two edges of one class never share a face: a face spanned by
 * axes a < b holds two a-edges whose b coordinates differ by one and two
 * b-edges whose a coordinates differ by one, so with L even each pair differs
 * in the parity that the class records. */
int32_t tco_edge_class(const tco_lattice* lat, int64_t edge) {
    const int64_t N = lat->n_sites;
    const int a = (int)(edge / N);
    const int64_t v = edge % N;
    const int L = lat->L;
    const int c[3] = {(int)(v % L), (int)((v / L) % L), (int)(v / ((int64_t)L * L))};
    const int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;
    return 4 * a + 2 * (c[b0] & 1) + (c[b1] & 1);
}

int32_t tco_subset_class(int32_t j, int32_t m, uint32_t cycle) {
    return (int32_t)(((uint64_t)j + (uint64_t)cycle * (uint64_t)m) % 12u);
}

void tco_subset_pflip_sweep(const tco_lattice* lat, uint8_t* syn, uint8_t* corr, uint64_t seed,
                            uint32_t cycle, uint32_t sweep, uint64_t shot0, int64_t n_shots,
                            int32_t edge_class) {
    const int64_t n = lat->n_edges, m = lat->n_faces;
    uint8_t* F = (uint8_t*)malloc(n);
    for (int64_t s = 0; s < n_shots; ++s) {
        uint8_t* sy = syn + s * m;
        for (int64_t b = 0; b < n; ++b) {
            F[b] = 0;
            if (tco_edge_class(lat, b) != edge_class) continue;
            const int unsat = unsat_count(lat, sy, b), sat = 4 - unsat;
            if (sat < unsat)
                F[b] = 1;
            else if (sat == unsat)
                F[b] = (uint8_t)(tco_coin(seed, (uint32_t)b, cycle, sweep, shot0 + (uint64_t)s) != 0);
        }
        apply_flips(lat, F, sy, corr + s * n);
    }
    free(F);
}

/* flip as first stated (Section 3.1): one bit at a time. */
int64_t tco_sequential_flip(const tco_lattice* lat, uint8_t* syn, uint8_t* corr,
                            int64_t max_flips) {
    int64_t flips = 0;
    while (flips < max_flips) {
        int64_t pick = -1;
        for (int64_t b = 0; b < lat->n_edges && pick < 0; ++b) {
            int unsat = unsat_count(lat, syn, b);
            if (4 - unsat < unsat) pick = b;
        }
        if (pick < 0) break;
        corr[pick] ^= 1u;
        for (int j = 0; j < 4; ++j) syn[lat->edge_face[4 * pick + j]] ^= 1u;
        ++flips;
    }
    return flips;
}

/* ---------------------------------------------------------------------- BP */

/* One flooding iteration of sum-product BP in LLR form (Section 4.1).
 *   E1  l0_i = ln(P(v_i=0)/P(v_i=1)); for the binary symmetric channel
 *       l0 = ln((1-p)/p).
 *   E3  variable-to-factor: M(i->f) = l0_i + sum over the other factors f'
 *       of bit i of M(f'->i). At the first iteration there are no factor
 *       messages yet and M(i->f) = l0_i.
 *   E2  factor-to-variable: M(f->i) = (-1)^{s_f} 2 atanh(prod over the other
 *       neighbours i' of f of tanh(M(i'->f)/2)).
 *       Each check also has one measurement-error variable of degree 1
 *       (Section 4.1, measurement errors); its message to f is always its
 *       prior ln((1-q)/q), so its factor in the product is tanh of half that.
 *   E4  posterior: l_i = l0_i + sum over all factors f of i of M(f->i). */
void tco_bp_step(const tco_lattice* lat, const uint8_t* syn, const double* llr0,
                 double p_dec, double q_dec, const double* nu_in, double* nu_out,
                 double* post) {
    const int64_t n = lat->n_edges, m = lat->n_faces;
    const double l0s = log((1.0 - p_dec) / p_dec);
    const double lm = log((1.0 - q_dec) / q_dec); /* measurement variable prior */
    double* mu = (double*)malloc(sizeof(double) * 4 * m);
    /* E3 */
    for (int64_t f = 0; f < m; ++f)
        for (int k = 0; k < 4; ++k) {
            int64_t i = lat->face_edge[4 * f + k];
            double msg = llr0 ? llr0[i] : l0s;
            if (nu_in)
                for (int j = 0; j < 4; ++j) {
                    int64_t g = lat->edge_face[4 * i + j];
                    if (g == f) continue;
                    msg += nu_in[4 * g + lat->edge_slot[4 * i + j]];
                }
            mu[4 * f + k] = msg;
        }
    /* E2 */
    for (int64_t f = 0; f < m; ++f)
        for (int k = 0; k < 4; ++k) {
            double prod = tanh(lm / 2.0);
            for (int kk = 0; kk < 4; ++kk)
                if (kk != k) prod *= tanh(mu[4 * f + kk] / 2.0);
            double sign = syn[f] ? -1.0 : 1.0;
            nu_out[4 * f + k] = sign * 2.0 * atanh(prod);
        }
    /* E4 */
    if (post)
        for (int64_t i = 0; i < n; ++i) {
            double l = llr0 ? llr0[i] : l0s;
            for (int j = 0; j < 4; ++j)
                l += nu_out[4 * lat->edge_face[4 * i + j] + lat->edge_slot[4 * i + j]];
            post[i] = l;
        }
    free(mu);
}

/* Damped flooding BP: the new factor-to-variable messages are mixed with the
 * previous ones in the log domain, nu = (1 - g) nu_new + g nu_old. Section
 * 4.1 runs BP undamped; damping is one of the things its implementation
 * leaves open, tried here as a reading. */
void tco_bp_step_damped(const tco_lattice* lat, const uint8_t* syn, const double* llr0,
                        double p_dec, double q_dec, double damp, const double* nu_in,
                        double* nu_out, double* post) {
    const int64_t n = lat->n_edges, m = lat->n_faces;
    tco_bp_step(lat, syn, llr0, p_dec, q_dec, nu_in, nu_out, NULL);
    for (int64_t j = 0; j < 4 * m; ++j)
        nu_out[j] = (1.0 - damp) * nu_out[j] + damp * (nu_in ? nu_in[j] : 0.0);
    if (post) {
        const double l0s = log((1.0 - p_dec) / p_dec);
        for (int64_t i = 0; i < n; ++i) {
            double l = llr0 ? llr0[i] : l0s;
            for (int j = 0; j < 4; ++j)
                l += nu_out[4 * lat->edge_face[4 * i + j] + lat->edge_slot[4 * i + j]];
            post[i] = l;
        }
    }
}

/* ------------------------------------------------- BP with meta-checks */

/* Face slot j (0..5) of cube c (the unit cube at corner site c): the lower
 * face f(c,n) for j = 2n, the upper face f(c+unit(n), n) for j = 2n+1. */
static int64_t cube_face(const tco_lattice* lat, int64_t c, int j) {
    const int32_t L = lat->L;
    const int n = j / 2;
    int64_t x = c % L, y = (c / L) % L, z = c / ((int64_t)L * L);
    if (j & 1) {
        if (n == 0) x += 1;
        if (n == 1) y += 1;
        if (n == 2) z += 1;
    }
    return (int64_t)n * lat->n_sites + site_of(L, x, y, z);
}

/* The two cubes of face f(w,n): the one it is the lower face of (cube w,
 * slot 2n) and the one it is the upper face of (cube w - unit(n), slot 2n+1). */
static void face_cubes(const tco_lattice* lat, int64_t f, int64_t cube[2], int slot[2]) {
    const int32_t L = lat->L;
    const int n = (int)(f / lat->n_sites);
    const int64_t w = f % lat->n_sites;
    int64_t x = w % L, y = (w / L) % L, z = w / ((int64_t)L * L);
    cube[0] = w;
    slot[0] = 2 * n;
    if (n == 0) x -= 1;
    if (n == 1) y -= 1;
    if (n == 2) z -= 1;
    cube[1] = site_of(L, x, y, z);
    slot[1] = 2 * n + 1;
}

static double clamp_msg(double x) {
    return x > TCO_META_CLAMP ? TCO_META_CLAMP : (x < -TCO_META_CLAMP ? -TCO_META_CLAMP : x);
}

/* One flooding iteration of BP on the factor graph with meta-checks, the
 * extension Section 4.1 describes and leaves out: besides the qubits and the
 * checks, one measurement-error variable m_f per check (prior ln((1-q)/q))
 * and one meta-check per cube, whose six measurement variables must have the
 * parity of the six measured outcomes (valid syndromes are closed, so the
 * measured parity of a cube is the parity of its measurement errors).
 * Messages (LLRs; variable-to-factor ones clamped to +-TCO_META_CLAMP):
 *   qubit e -> check f     Q  = l0 + sum of the other checks' nu
 *   meas m_f -> check f    M  = lm + kappa from both cubes of f
 *   meas m_f -> cube c     R  = lm + lambda_f + kappa from the other cube
 *   check f -> qubit e     nu = (-1)^{s_f} 2 atanh(tanh(M/2) prod_{e' != e} tanh(Q/2))
 *   check f -> meas m_f    lambda = (-1)^{s_f} 2 atanh(prod_{e} tanh(Q/2))
 *   cube c -> meas m_f     kappa = (-1)^{mu_c} 2 atanh(prod_{f' != f} tanh(R/2))
 *   posterior              l_e = l0 + sum of nu
 * State: nu [n_faces][4] (member order), lambda [n_faces], kappa [n_sites][6]
 * (cube slot order); *_in NULL = first iteration (all factor messages 0). */
void tco_bp_meta_step(const tco_lattice* lat, const uint8_t* syn, double p_dec, double q_dec,
                      const double* nu_in, const double* lam_in, const double* kap_in,
                      double* nu_out, double* lam_out, double* kap_out, double* post) {
    const int64_t n = lat->n_edges, m = lat->n_faces, N = lat->n_sites;
    const double l0 = log((1.0 - p_dec) / p_dec);
    const double lm = log((1.0 - q_dec) / q_dec);
    double* Q = (double*)malloc(sizeof(double) * 4 * m);
    double* M = (double*)malloc(sizeof(double) * m);
    double* R = (double*)malloc(sizeof(double) * 6 * N);
    for (int64_t f = 0; f < m; ++f)
        for (int k = 0; k < 4; ++k) {
            const int64_t i = lat->face_edge[4 * f + k];
            double msg = l0;
            if (nu_in)
                for (int j = 0; j < 4; ++j) {
                    const int64_t g = lat->edge_face[4 * i + j];
                    if (g != f) msg += nu_in[4 * g + lat->edge_slot[4 * i + j]];
                }
            Q[4 * f + k] = clamp_msg(msg);
        }
    for (int64_t f = 0; f < m; ++f) {
        int64_t cb[2];
        int sl[2];
        face_cubes(lat, f, cb, sl);
        double msg = lm;
        if (kap_in) msg += kap_in[6 * cb[0] + sl[0]] + kap_in[6 * cb[1] + sl[1]];
        M[f] = clamp_msg(msg);
    }
    for (int64_t c = 0; c < N; ++c)
        for (int j = 0; j < 6; ++j) {
            const int64_t f = cube_face(lat, c, j);
            int64_t cb[2];
            int sl[2];
            face_cubes(lat, f, cb, sl);
            const int other = (cb[0] == c && sl[0] == j) ? 1 : 0;
            double msg = lm;
            if (lam_in) msg += lam_in[f] + kap_in[6 * cb[other] + sl[other]];
            R[6 * c + j] = clamp_msg(msg);
        }
    for (int64_t f = 0; f < m; ++f) {
        const double sign = syn[f] ? -1.0 : 1.0;
        double all = 1.0;
        for (int k = 0; k < 4; ++k) all *= tanh(Q[4 * f + k] / 2.0);
        lam_out[f] = sign * 2.0 * atanh(all);
        for (int k = 0; k < 4; ++k) {
            double prod = tanh(M[f] / 2.0);
            for (int kk = 0; kk < 4; ++kk)
                if (kk != k) prod *= tanh(Q[4 * f + kk] / 2.0);
            nu_out[4 * f + k] = sign * 2.0 * atanh(prod);
        }
    }
    for (int64_t c = 0; c < N; ++c) {
        int par = 0;
        for (int j = 0; j < 6; ++j) par ^= syn[cube_face(lat, c, j)];
        const double sign = par ? -1.0 : 1.0;
        for (int j = 0; j < 6; ++j) {
            double prod = 1.0;
            for (int jj = 0; jj < 6; ++jj)
                if (jj != j) prod *= tanh(R[6 * c + jj] / 2.0);
            kap_out[6 * c + j] = sign * 2.0 * atanh(prod);
        }
    }
    if (post)
        for (int64_t i = 0; i < n; ++i) {
            double l = l0;
            for (int j = 0; j < 4; ++j)
                l += nu_out[4 * lat->edge_face[4 * i + j] + lat->edge_slot[4 * i + j]];
            post[i] = l;
        }
    free(Q);
    free(M);
    free(R);
}

void tco_bp_meta_decode(const tco_lattice* lat, const uint8_t* syn, int64_t n_shots,
                        double p_dec, double q_dec, int32_t iters, uint8_t* corr,
                        double* post) {
    const int64_t n = lat->n_edges, m = lat->n_faces, N = lat->n_sites;
    double* buf = (double*)malloc(sizeof(double) * 2 * (4 * m + m + 6 * N));
    double* l = (double*)malloc(sizeof(double) * n);
    const double l0 = log((1.0 - p_dec) / p_dec);
    for (int64_t s = 0; s < n_shots; ++s) {
        const uint8_t* sy = syn + s * m;
        int cur = -1;
        for (int32_t it = 0; it < iters; ++it) {
            const int nxt = cur == 0 ? 1 : 0;
            double* o = buf + (size_t)nxt * (4 * m + m + 6 * N);
            double* i_ = cur < 0 ? NULL : buf + (size_t)cur * (4 * m + m + 6 * N);
            tco_bp_meta_step(lat, sy, p_dec, q_dec, i_, i_ ? i_ + 4 * m : NULL,
                             i_ ? i_ + 5 * m : NULL, o, o + 4 * m, o + 5 * m, l);
            cur = nxt;
        }
        for (int64_t i = 0; i < n; ++i) {
            const double li = iters > 0 ? l[i] : l0;
            corr[s * n + i] = (uint8_t)(li < 0.0);
            if (post) post[s * n + i] = li;
        }
    }
    free(buf);
    free(l);
}

/* Local BP (Section 4.1): a fixed number of iterations, then every bit whose
 * posterior LLR is negative is flipped. */
void tco_bp_decode(const tco_lattice* lat, const uint8_t* syn, int64_t n_shots,
                   const double* llr0, double p_dec, double q_dec, int32_t iters,
                   uint8_t* corr, double* post) {
    const int64_t n = lat->n_edges, m = lat->n_faces;
    double* nu_a = (double*)malloc(sizeof(double) * 4 * m);
    double* nu_b = (double*)malloc(sizeof(double) * 4 * m);
    double* l = (double*)malloc(sizeof(double) * n);
    for (int64_t s = 0; s < n_shots; ++s) {
        const uint8_t* sy = syn + s * m;
        const double* pr = llr0 ? llr0 + s * n : NULL;
        double* cur = NULL;
        for (int32_t it = 0; it < iters; ++it) {
            double* next = (cur == nu_a) ? nu_b : nu_a;
            tco_bp_step(lat, sy, pr, p_dec, q_dec, cur, next, l);
            cur = next;
        }
        for (int64_t i = 0; i < n; ++i) {
            double li = l[i];
            if (iters <= 0) li = pr ? pr[i] : log((1.0 - p_dec) / p_dec);
            corr[s * n + i] = (uint8_t)(li < 0.0);
            if (post) post[s * n + i] = li;
        }
    }
    free(nu_a);
    free(nu_b);
    free(l);
}

/* ------------------------------------------------------------------ readout */

/* Section 2: a logical Z operator of qubit d is a string of the L edges along
 * axis d through fixed values of the other two coordinates; the L^2 such
 * strings are disjoint. A logical X error flips all of them. The readout is a
 * majority vote over the strings' parities (Section 3.1, Fig. 2 caption). */
void tco_logical_check(const tco_lattice* lat, const uint8_t* err, int64_t n_shots,
                       uint8_t* mask, int32_t* odd) {
    const int32_t L = lat->L;
    const int64_t n = lat->n_edges, N = lat->n_sites;
    for (int64_t s = 0; s < n_shots; ++s) {
        const uint8_t* e = err + s * n;
        uint8_t msk = 0;
        for (int d = 0; d < 3; ++d) {
            int32_t count = 0;
            for (int64_t i = 0; i < L; ++i)
                for (int64_t j = 0; j < L; ++j) {
                    uint8_t par = 0;
                    for (int64_t t = 0; t < L; ++t) {
                        int64_t c[3];
                        c[d] = t;
                        c[(d + 1) % 3] = i;
                        c[(d + 2) % 3] = j;
                        par ^= e[d * N + site_of(L, c[0], c[1], c[2])];
                    }
                    count += par;
                }
            if (odd) odd[3 * s + d] = count;
            if (2 * (int64_t)count >= (int64_t)L * L) msk |= (uint8_t)(1u << d);
        }
        mask[s] = msk;
    }
}

/* --------------------------------------------------------------- experiment */

/* Multi-cycle Monte Carlo (Sections 3.1, 3.2, 4.2): per cycle, noise, one
 * syndrome measurement, BP (if enabled) whose correction also updates the
 * working syndrome, the flip / p-flip schedule on that working syndrome, then
 * the accumulated correction is applied and the residual carries over. */
void tco_run_cycles(const tco_lattice* lat, const tco_params* prm, uint64_t shot0,
                    int64_t n_shots, uint8_t* err, uint8_t* mask, int32_t* odd,
                    uint8_t* trace) {
    const int64_t n = lat->n_edges, m = lat->n_faces;
    const int32_t cycles = prm->noisy_cycles + (prm->perfect_final ? 1 : 0);
    uint8_t* syn = (uint8_t*)malloc(m);
    uint8_t* corr = (uint8_t*)malloc(n);
    uint8_t* cbp = (uint8_t*)malloc(n);
    /* BP read as damped or warm-started: messages kept between iterations
       and, warm, between cycles */
    const int bp_ext = prm->bp_iters > 0 && !prm->bp_meta && (prm->bp_warm || prm->bp_damp > 0.0);
    double* nu_a = bp_ext ? (double*)malloc(sizeof(double) * 4 * m) : NULL;
    double* nu_b = bp_ext ? (double*)malloc(sizeof(double) * 4 * m) : NULL;
    double* post = bp_ext ? (double*)malloc(sizeof(double) * n) : NULL;
    for (int64_t s = 0; s < n_shots; ++s) {
        const uint64_t shot = shot0 + (uint64_t)s;
        uint8_t* e = err + s * n;
        for (int32_t t = 0; t < cycles; ++t) {
            const int noisy = t < prm->noisy_cycles;
            /* counters are keyed by the cycle of the whole experiment */
            const uint32_t c = prm->cycle0 + (uint32_t)t;
            const double pt = (noisy || prm->final_qubit_noise) ? prm->p : 0.0;
            const double qt = noisy ? prm->q : 0.0;
            tco_sample_noise(lat, e, 0, pt, prm->seed, c, shot, 1);
            tco_syndrome(lat, e, syn, 1, 0);
            tco_sample_noise(lat, syn, 1, qt, prm->seed, c, shot, 1);
            memset(corr, 0, n);
            if (bp_ext) {
                /* start: the previous cycle's final messages (warm), else the
                   priors (nu_in NULL) */
                const int warm = prm->bp_warm && t > 0;
                for (int32_t it = 0; it < prm->bp_iters; ++it) {
                    const double* in = (it == 0 && !warm) ? NULL : nu_a;
                    tco_bp_step_damped(lat, syn, NULL, prm->p_dec, prm->q_dec, prm->bp_damp,
                                       in, nu_b, it == prm->bp_iters - 1 ? post : NULL);
                    double* tmp = nu_a;
                    nu_a = nu_b;
                    nu_b = tmp;
                }
                for (int64_t i = 0; i < n; ++i) cbp[i] = post[i] < 0.0;
                for (int64_t i = 0; i < n; ++i) corr[i] = cbp[i];
                tco_syndrome(lat, cbp, syn, 1, 1);
            } else if (prm->bp_iters > 0) {
                if (prm->bp_meta)
                    tco_bp_meta_decode(lat, syn, 1, prm->p_dec, prm->q_dec, prm->bp_iters, cbp,
                                       NULL);
                else
                    tco_bp_decode(lat, syn, 1, NULL, prm->p_dec, prm->q_dec, prm->bp_iters,
                                  cbp, NULL);
                for (int64_t i = 0; i < n; ++i) corr[i] = cbp[i];
                tco_syndrome(lat, cbp, syn, 1, 1);
            }
            int32_t n_subset = 0;
            for (int32_t k = 0; k < prm->n_sweeps; ++k) n_subset += (prm->subset_mask >> k) & 1u;
            for (int32_t k = 0, j = 0; k < prm->n_sweeps; ++k) {
                if ((prm->subset_mask >> k) & 1u)
                    tco_subset_pflip_sweep(lat, syn, corr, prm->seed, c, (uint32_t)k, shot, 1,
                                           tco_subset_class(j++, n_subset, c));
                else if ((prm->pflip_mask >> k) & 1u)
                    tco_pflip_sweep(lat, syn, corr, prm->seed, c, (uint32_t)k, shot, 1);
                else
                    tco_flip_sweep(lat, syn, corr, 1);
            }
            for (int64_t i = 0; i < n; ++i) e[i] ^= corr[i];
            if (trace) memcpy(trace + ((int64_t)t * n_shots + s) * n, e, n);
        }
        tco_logical_check(lat, e, 1, mask + s, odd ? odd + 3 * s : NULL);
    }
    free(syn);
    free(corr);
    free(cbp);
    free(nu_a);
    free(nu_b);
    free(post);
}

/* ---------------------------------------------------------------- CNN prior */

static const int kCnnCh[TCO_CNN_LAYERS + 1] = {8, 32, 32, 32, 3};

int64_t tco_cnn_param_count(void) {
    int64_t n = 0;
    for (int l = 0; l < TCO_CNN_LAYERS; ++l) n += 27 * kCnnCh[l] * kCnnCh[l + 1] + kCnnCh[l + 1];
    return n;
}

/* neighbour of site v at offset index d (d = (dz+1)*9 + (dy+1)*3 + (dx+1)) */
static int64_t cnn_nbr(int32_t L, int64_t v, int d) {
    int64_t x = v % L, y = (v / L) % L, z = v / ((int64_t)L * L);
    int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    return site_of(L, x + dx, y + dy, z + dz);
}

void tco_cnn_input(const tco_lattice* lat, int64_t n_shots, const uint8_t* syn,
                   const uint8_t* prev, double* x0) {
    const int64_t N = lat->n_sites, m = lat->n_faces;
    for (int64_t s = 0; s < n_shots; ++s)
        for (int64_t v = 0; v < N; ++v) {
            double* o = x0 + (s * N + v) * 8;
            for (int n = 0; n < 3; ++n) {
                o[n] = syn[s * m + n * N + v];
                o[3 + n] = prev ? prev[s * m + n * N + v] : 0.0;
            }
            o[6] = o[7] = 0.0;
        }
}

/* one periodic 3x3x3 convolution of one shot: y[v][co] = b + sum W x[v+d] */
static void cnn_conv(int32_t L, int64_t N, const double* x, int cin, const double* W,
                     const double* b, int cout, double* y) {
    for (int64_t v = 0; v < N; ++v)
        for (int co = 0; co < cout; ++co) {
            double acc = b[co];
            for (int d = 0; d < 27; ++d) {
                const double* xn = x + cnn_nbr(L, v, d) * cin;
                for (int ci = 0; ci < cin; ++ci) acc += W[(d * cin + ci) * cout + co] * xn[ci];
            }
            y[v * cout + co] = acc;
        }
}

/* Layer buffers of one shot: h[0] = input, h[l] = post-activation of layer l
 * (layers 1-3), h[4] = logits. */
static void cnn_forward_shot(int32_t L, int64_t N, const double* x0, const double* params,
                             double* h[TCO_CNN_LAYERS + 1]) {
    const double* p = params;
    for (int64_t i = 0; i < N * 8; ++i) h[0][i] = x0[i];
    for (int l = 0; l < TCO_CNN_LAYERS; ++l) {
        const int cin = kCnnCh[l], cout = kCnnCh[l + 1];
        const double* W = p;
        const double* b = p + 27 * cin * cout;
        cnn_conv(L, N, h[l], cin, W, b, cout, h[l + 1]);
        if (l + 1 < TCO_CNN_LAYERS)
            for (int64_t i = 0; i < N * cout; ++i)
                if (h[l + 1][i] < 0.0) h[l + 1][i] = 0.0;
        p = b + cout;
    }
}

void tco_cnn_forward(const tco_lattice* lat, int64_t n_shots, const double* x0,
                     const double* params, double* z, double* acts) {
    const int32_t L = lat->L;
    const int64_t N = lat->n_sites;
    double* h[TCO_CNN_LAYERS + 1];
    for (int l = 0; l <= TCO_CNN_LAYERS; ++l) h[l] = (double*)malloc(sizeof(double) * N * 32);
    for (int64_t s = 0; s < n_shots; ++s) {
        cnn_forward_shot(L, N, x0 + s * N * 8, params, h);
        memcpy(z + s * N * 3, h[TCO_CNN_LAYERS], sizeof(double) * N * 3);
        if (acts)
            for (int l = 1; l < TCO_CNN_LAYERS; ++l)
                memcpy(acts + ((int64_t)(l - 1) * n_shots + s) * N * 32, h[l],
                       sizeof(double) * N * 32);
    }
    for (int l = 0; l <= TCO_CNN_LAYERS; ++l) free(h[l]);
}

/* Binary cross-entropy with logits averaged over every edge of every shot,
 * and its gradient by the chain rule through the four layers. */
double tco_cnn_loss_grad(const tco_lattice* lat, int64_t n_shots, const double* x0,
                         const double* params, const uint8_t* target, double* grad) {
    const int32_t L = lat->L;
    const int64_t N = lat->n_sites, n_edges = lat->n_edges;
    const double count = (double)n_shots * (double)n_edges;
    double* h[TCO_CNN_LAYERS + 1];
    for (int l = 0; l <= TCO_CNN_LAYERS; ++l) h[l] = (double*)malloc(sizeof(double) * N * 32);
    double* dy = (double*)malloc(sizeof(double) * N * 32);  /* d loss / d pre-activation */
    double* dx = (double*)malloc(sizeof(double) * N * 32);  /* d loss / d layer input    */
    const int64_t P = tco_cnn_param_count();
    for (int64_t i = 0; i < P; ++i) grad[i] = 0.0;
    /* parameter offsets of each layer */
    int64_t off[TCO_CNN_LAYERS];
    {
        int64_t o = 0;
        for (int l = 0; l < TCO_CNN_LAYERS; ++l) {
            off[l] = o;
            o += 27 * kCnnCh[l] * kCnnCh[l + 1] + kCnnCh[l + 1];
        }
    }
    double loss = 0.0;
    for (int64_t s = 0; s < n_shots; ++s) {
        cnn_forward_shot(L, N, x0 + s * N * 8, params, h);
        const uint8_t* t = target + s * n_edges;
        for (int64_t v = 0; v < N; ++v)
            for (int c = 0; c < 3; ++c) {
                const double zz = h[TCO_CNN_LAYERS][v * 3 + c];
                const double tt = t[(int64_t)c * N + v];
                const double softplus = (zz > 0 ? zz : 0.0) + log1p(exp(-fabs(zz)));
                loss += softplus - tt * zz;
                dy[v * 3 + c] = (1.0 / (1.0 + exp(-zz)) - tt) / count;
            }
        for (int l = TCO_CNN_LAYERS - 1; l >= 0; --l) {
            const int cin = kCnnCh[l], cout = kCnnCh[l + 1];
            const double* W = params + off[l];
            double* gW = grad + off[l];
            double* gb = gW + 27 * cin * cout;
            /* weights and bias */
            for (int64_t v = 0; v < N; ++v)
                for (int co = 0; co < cout; ++co) {
                    const double g = dy[v * cout + co];
                    if (g == 0.0) continue;
                    gb[co] += g;
                    for (int d = 0; d < 27; ++d) {
                        const double* xn = h[l] + cnn_nbr(L, v, d) * cin;
                        for (int ci = 0; ci < cin; ++ci) gW[(d * cin + ci) * cout + co] += g * xn[ci];
                    }
                }
            if (l == 0) break;
            /* input of this layer: x[u] feeds y[v] for u = v + d */
            for (int64_t i = 0; i < N * cin; ++i) dx[i] = 0.0;
            for (int64_t v = 0; v < N; ++v)
                for (int d = 0; d < 27; ++d) {
                    const int64_t u = cnn_nbr(L, v, d);
                    for (int ci = 0; ci < cin; ++ci) {
                        double acc = 0.0;
                        for (int co = 0; co < cout; ++co)
                            acc += W[(d * cin + ci) * cout + co] * dy[v * cout + co];
                        dx[u * cin + ci] += acc;
                    }
                }
            /* through the ReLU of the previous layer */
            for (int64_t i = 0; i < N * cin; ++i) dy[i] = h[l][i] > 0.0 ? dx[i] : 0.0;
        }
    }
    for (int l = 0; l <= TCO_CNN_LAYERS; ++l) free(h[l]);
    free(dy);
    free(dx);
    return loss / count;
}
