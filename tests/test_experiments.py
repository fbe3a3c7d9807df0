"""Host logic of experiments.py: the flip / p-flip schedules of
Sections 3.2 and 4.2 and the threshold fit of Section 3.2 (no GPU needed)."""
import numpy as np

from paper_2212_06985_amd import experiments as ex


def test_schedules():
    # n_A = 5, lambda_p = 3: F F P F F, the worked schedule of Section 3.2
    assert ex.flip_mask(5, 3) == 0b00100
    # lambda_p > n_A: only flip sweeps (the shaded cells of Table 1)
    assert ex.flip_mask(5, 6) == 0
    assert ex.flip_mask(9, 2) == 0b010101010
    assert ex.flip_mask(3, 1) == 0b111
    assert ex.decoder_params("flip", 1, 0) == (0, 1, 0)
    assert ex.decoder_params("bp") == (30, 0, 0)
    # p-BP: 20 BP iterations, then p-flip on the first and fourth of six sweeps
    assert ex.decoder_params("pbp") == (20, 6, 0b001001)


def test_table2_counts():
    assert sum(ex.TABLE2_COUNTS.values()) == 1000
    assert set(ex.TABLE2_COUNTS) == {format(k, "03b") for k in range(8)}


def test_threshold_fit_recovers_a_known_crossing():
    """Data drawn from the ansatz itself (with binomial noise) give back its
    crossing point and exponent within their fitted errors."""
    rng = np.random.default_rng(3)
    p_th, inv_nu, a = 0.0546, 0.8, (0.15, 4.0, 20.0)
    Ls, ps = [14, 18, 24, 32], np.linspace(0.0536, 0.0556, 6)
    rows = []
    for L in Ls:
        for p in ps:
            f = ex.threshold_ansatz((p, L), p_th, inv_nu, *a)
            n = 20000
            k = rng.binomial(n, f)
            rows.append((L, p, k / n, np.sqrt(f * (1 - f) / n)))
    L, p, f, s = map(np.array, zip(*rows))
    fit = ex.fit_threshold(L, p, f, s, p_th0=0.055)
    assert abs(fit["p_th"] - p_th) < 4 * fit["p_th_err"] + 1e-6
    assert fit["p_th_err"] < 2e-4
    assert abs(fit["inv_nu"] - inv_nu) < 4 * fit["inv_nu_err"] + 1e-3
    assert fit["chi2"] < 3 * fit["dof"]


def test_pfail_sigma():
    r = {"fails": [128, 129, 143], "shots": 1000}
    f, s = ex.pfail(r)
    assert f == 0.128 and abs(s - np.sqrt(0.128 * 0.872 / 1000)) < 1e-15
    f3, s3 = ex.pfail_pooled(r)
    assert abs(f3 - 0.4 / 3) < 1e-15 and s3 < s


def test_schedule_strings():
    assert ex.parse_schedule("PFFPFF") == (6, 0b001001, 0)
    assert ex.parse_schedule("cffcff") == (6, 0, 0b001001)
    assert ex.parse_schedule("FFPFF") == (5, ex.flip_mask(5, 3), 0)
    for bad in ("", "PFX", "F" * 33):
        try:
            ex.parse_schedule(bad)
        except ValueError:
            continue
        raise AssertionError(bad)
