"""Generator recipe checks and the paper's printed storage example (CPU only)."""

import json
import os

import numpy as np

from paper_1304_2272_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_storage_example_fixes_eight_byte_elements():
    g = json.load(open(os.path.join(GOLDEN, "storage_example.json")))
    n, m, p = g["n"], g["m"], g["p"]

    def sizes(elem):
        inp = elem * n * n + elem * n * m
        out = elem * p * m
        return round(inp / (1000 * 2**30), 2), round(out / 2**20)

    assert sizes(8) == (1.49, 305)
    assert sizes(8) == (float(g["printed_input"].split()[0]), int(g["printed_output"].split()[0]))
    assert sizes(4) != (1.49, 305)           # single precision does not reproduce it


def test_background_genotypes_standardised():
    Z = synth.background_genotypes(500, seed=3, k=300)
    assert Z.shape == (500, 300)
    assert np.allclose(Z.mean(axis=0), 0.0, atol=1e-12)
    assert np.allclose(Z.std(axis=0), 1.0, atol=1e-12)


def test_covariance_spd_and_recipe():
    Z = synth.background_genotypes(400, seed=4, k=200)
    M = synth.covariance(Z, h2=0.3, sigma2=2.0)
    assert np.allclose(M, M.T)
    w = np.linalg.eigvalsh(M)
    assert w.min() > 2.0 * 0.7 * (1 - 1e-9)                 # sigma^2 (1 - h^2) floor
    # standardised columns: trace(Phi) = n, so the mean diagonal of M is sigma^2
    assert abs(np.mean(np.diag(M)) - 2.0) < 1e-12
    # standardised columns: Phi 1 = 0, so M 1 = sigma^2 (1 - h^2) 1
    assert np.allclose(M @ np.ones(400), 2.0 * 0.7, atol=1e-9)


def test_snp_blocks_partition_independent_and_binomial():
    a = synth.snp_block(300, 5, 0, 3000, dtype=np.int8)
    b = np.vstack([synth.snp_block(300, 5, s, c, dtype=np.int8)
                   for s, c in [(0, 700), (700, 1500), (2200, 800)]])
    assert np.array_equal(a, b)
    assert set(np.unique(a)) <= {0, 1, 2}
    # mean dosage of Binomial(2, f) with f ~ U(0.05, 0.5) is 2 * 0.275
    assert abs(a.mean() - 0.55) < 0.02


def test_problem_noise_covariance():
    # y - X_L beta ~ N(0, M): check E[e e^T] on a small problem by averaging traits
    prob = synth.make_problem(60, 3, seed=6, t=4000, k=100)
    E = prob["Y"] - prob["XL"] @ prob["beta"]
    C = E @ E.T / E.shape[1]
    assert np.max(np.abs(C - prob["M"])) < 0.15


def test_banded_problem_structure():
    # Phi of local markers: symmetric, zero past the half-bandwidth, diagonal
    # near 1, and M = sigma^2 (h^2 Phi + (1 - h^2) I) >= sigma^2 (1 - h^2) I
    n, w, h2, s2 = 500, 40, 0.6, 1.3
    pr = synth.banded_problem(n, 4, 9, w, h2=h2, sigma2=s2)
    M = synth.band_to_dense(pr["M_band"])
    assert np.array_equal(M, M.T)
    i, j = np.nonzero(M)
    assert np.max(np.abs(i - j)) == w
    ev = np.linalg.eigvalsh(M)
    assert ev[0] >= s2 * (1 - h2) * (1 - 1e-12)
    phi_diag = (np.diag(M) - s2 * (1 - h2)) / (s2 * h2)
    assert abs(phi_diag.mean() - 1.0) < 0.1
    # the band storage convention: M_band[j, d] = M(j + d, j)
    assert pr["M_band"][10, 3] == M[13, 10]
    # y = X_L beta when noise is off
    pr0 = synth.banded_problem(n, 4, 9, w, noise=False)
    assert np.allclose(pr0["Y"], pr0["XL"] @ pr0["beta"])
