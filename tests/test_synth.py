"""Seeded input generators: determinism and the stated distributions."""

import numpy as np

import synth


def test_determinism_and_streams():
    a = synth.gaussian_matrix(64, seed=3)
    b = synth.gaussian_matrix(64, seed=3)
    c = synth.gaussian_matrix(64, seed=4)
    d = synth.gaussian_matrix(64, seed=3, view=1)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)
    U1, V1 = synth.update_factors(64, 2, 5, seed=3)
    U2, V2 = synth.update_factors(64, 2, 5, seed=3)
    np.testing.assert_array_equal(U1, U2)
    np.testing.assert_array_equal(V1, V2)


def test_spectral_norm_exact_branch():
    A = synth.gaussian_matrix(300, seed=0)
    assert abs(np.linalg.norm(A, 2) - 0.9) < 1e-12


def test_spectral_norm_estimate_branch():
    A = synth.gaussian_matrix(1280, seed=0)   # above the exact-SVD threshold
    s = np.linalg.norm(A, 2)
    assert abs(s - 0.9) / 0.9 < 1e-10


def test_update_factor_scale():
    n = 4096
    U, V = synth.update_factors(n, 1, 4, seed=1)
    sd = np.std(U)
    assert abs(sd - 1e-2 / np.sqrt(n)) / (1e-2 / np.sqrt(n)) < 0.02


def test_zipf_rows_and_row_updates():
    rows = synth.zipf_rows(1000, 5000, 2.0, seed=2)
    assert rows.min() >= 0 and rows.max() < 1000
    top = np.bincount(rows).max()
    assert top > 2500                      # s = 2 concentrates on one row
    uni = synth.zipf_rows(1000, 5000, 0.0, seed=2)
    assert np.bincount(uni).max() < 30
    U, V = synth.row_updates(50, 7, 1.0, seed=2)
    assert U.shape == (7, 50, 1) and np.all(U.sum(axis=1) == 1.0)


def test_dag_is_strictly_upper():
    M = synth.random_dag(20, 0.3, seed=1)
    assert np.all(np.tril(M) == 0) and set(np.unique(M)) <= {0.0, 1.0}
