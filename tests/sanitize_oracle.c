/* Test driver: runs every stage of the CPU oracle on small inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py compiles and runs it). Exits 0 when every
 * call returns; the sanitizers abort on the first invalid access or
 * undefined operation. Test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tc3d_oracle.h"

static void* xcalloc(size_t n, size_t sz) {
    void* p = calloc(n, sz);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static void run_lattice(int32_t L) {
    tco_lattice* lat = tco_lattice_new(L);
    const int64_t n = tco_n_edges(lat), S = 3;
    uint8_t* err = xcalloc((size_t)(S * n), 1);
    uint8_t* syn = xcalloc((size_t)(S * n), 1);
    uint8_t* corr = xcalloc((size_t)(S * n), 1);
    uint8_t* coins = xcalloc((size_t)n, 1);
    int32_t* fe = xcalloc((size_t)(4 * n), sizeof(int32_t));
    int32_t* ef = xcalloc((size_t)(4 * n), sizeof(int32_t));
    int32_t* es = xcalloc((size_t)(4 * n), sizeof(int32_t));
    tco_incidence(lat, fe, ef, es);
    tco_sample_noise(lat, err, 0, 0.1, 7, 0, 64, S);
    tco_syndrome(lat, err, syn, S, 0);
    tco_sample_noise(lat, syn, 1, 0.05, 7, 0, 64, S);
    tco_flip_sweep(lat, syn, corr, S);
    tco_pflip_sweep(lat, syn, corr, 7, 0, 1, 64, S);
    for (int64_t i = 0; i < n; ++i) coins[i] = (uint8_t)(i & 1);
    tco_pflip_sweep_coins(lat, syn, corr, coins);
    if (L % 2 == 0)
        for (int32_t c = 0; c < 12; ++c) tco_subset_pflip_sweep(lat, syn, corr, 7, 0, 2, 64, S, c);
    (void)tco_sequential_flip(lat, syn, corr, 1000);
    double* nu0 = xcalloc((size_t)(4 * n), sizeof(double));
    double* nu1 = xcalloc((size_t)(4 * n), sizeof(double));
    double* post = xcalloc((size_t)(S * n), sizeof(double));
    double* llr = xcalloc((size_t)(S * n), sizeof(double));
    for (int64_t i = 0; i < S * n; ++i) llr[i] = (double)(i % 11) - 3.0;
    tco_bp_step(lat, syn, NULL, 0.05, 0.05, NULL, nu0, post);
    tco_bp_step(lat, syn, llr, 0.05, 0.05, nu0, nu1, post);
    tco_bp_step_damped(lat, syn, NULL, 0.05, 0.05, 0.4, nu1, nu0, post);
    tco_bp_decode(lat, syn, S, NULL, 0.05, 0.05, 5, corr, post);
    tco_bp_decode(lat, syn, S, llr, 0.05, 0.05, 5, corr, post);
    tco_bp_meta_decode(lat, syn, S, 0.05, 0.05, 4, corr, post);
    uint8_t mask[3];
    int32_t odd[9];
    tco_logical_check(lat, err, S, mask, odd);
    for (int variant = 0; variant < 4; ++variant) {
        tco_params prm;
        memset(&prm, 0, sizeof(prm));
        prm.p = prm.q = prm.p_dec = prm.q_dec = 0.05;
        prm.noisy_cycles = 3;
        prm.perfect_final = 1;
        prm.final_qubit_noise = 1;
        prm.bp_iters = variant == 0 ? 0 : 4;
        prm.n_sweeps = 6;
        prm.pflip_mask = 9;
        prm.seed = 11;
        prm.bp_meta = variant == 2;
        prm.bp_warm = variant == 3;
        prm.bp_damp = variant == 3 ? 0.3 : 0.0;
        prm.cycle0 = (uint32_t)variant;
        if (L % 2 == 0 && variant == 1) prm.subset_mask = 2;
        uint8_t* trace = xcalloc((size_t)(4 * S * n), 1);
        memset(err, 0, (size_t)(S * n));
        tco_run_cycles(lat, &prm, 0, S, err, mask, odd, trace);
        free(trace);
    }
    const int64_t N = n / 3, P = tco_cnn_param_count();
    double* x0 = xcalloc((size_t)(S * N * 8), sizeof(double));
    double* params = xcalloc((size_t)P, sizeof(double));
    double* grad = xcalloc((size_t)P, sizeof(double));
    double* z = xcalloc((size_t)(S * N * 3), sizeof(double));
    double* acts = xcalloc((size_t)(3 * S * N * 32), sizeof(double));
    for (int64_t i = 0; i < P; ++i) params[i] = 0.01 * (double)((i * 37) % 19 - 9);
    tco_cnn_input(lat, S, syn, syn, x0);
    tco_cnn_forward(lat, S, x0, params, z, acts);
    (void)tco_cnn_loss_grad(lat, S, x0, params, err, grad);
    free(x0);
    free(params);
    free(grad);
    free(z);
    free(acts);
    free(nu0);
    free(nu1);
    free(post);
    free(llr);
    free(fe);
    free(ef);
    free(es);
    free(err);
    free(syn);
    free(corr);
    free(coins);
    tco_lattice_free(lat);
}

int main(void) {
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    tco_philox4x32_10(ctr, key, out);
    (void)tco_threshold(0.3);
    (void)tco_uniform(1, 2, 3, 4, 0);
    (void)tco_coin(1, 2, 3, 4, 5);
    (void)tco_subset_class(1, 2, 3);
    run_lattice(3);
    run_lattice(4);
    printf("sanitized oracle run ok\n");
    return 0;
}
