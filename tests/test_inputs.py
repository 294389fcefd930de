"""The seeded generators reproduce the matrix classes they name: the
prescribed singular values of the Haar-factor classes (App. C), the noise
level of Type-2, the Kappa formula, Toeplitz structure, and seeding."""
import numpy as np

from paper_2504_19308_amd import inputs


def test_type1_type3_singular_values():
    n = 96
    s1 = np.linalg.svd(inputs.type1_matrix(n, np.random.default_rng(1)), compute_uv=False)
    assert np.allclose(s1, np.exp(-np.arange(n) / 10.0), rtol=1e-10, atol=1e-14)
    s3 = np.linalg.svd(inputs.type3_matrix(n, np.random.default_rng(2)), compute_uv=False)
    assert np.allclose(s3, (n - np.arange(n)) / n, rtol=1e-10)


def test_type2_noise_level():
    n = 64
    rng = np.random.default_rng(3)
    A = inputs.type2_matrix(n, rng)
    T = inputs.type1_matrix(n, np.random.default_rng(3))   # the same draw of T
    noise = A - T
    assert np.all(noise >= 0)                                # a positive multiple of U(0,1) entries
    assert np.isclose(np.linalg.norm(noise), 0.5 * np.linalg.norm(T), rtol=1e-12)


def test_kappa_entries():
    K = inputs.kappa_matrix(7)
    assert np.array_equal(K, K.T)
    for i in range(7):
        for j in range(i + 1):
            assert np.isclose(K[i, j], np.exp(-0.5 * (i - j)) * np.sin(i + 1))


def test_toeplitz_structure_and_seeding():
    T = inputs.toeplitz_uniform(9, np.random.default_rng(4))
    assert np.allclose(T[1:, 1:], T[:-1, :-1])
    assert T.min() >= 0 and T.max() < 1
    a = inputs.type1_matrix(16, inputs.rng_of(11, 0, 11))
    b = inputs.type1_matrix(16, inputs.rng_of(11, 0, 11))
    assert np.array_equal(a, b)


def test_symmetric_and_hankel():
    S = inputs.symmetric_uniform(8, np.random.default_rng(5))
    assert np.array_equal(S, S.T) and S.min() >= 0 and S.max() < 1
    H = inputs.hankel_uniform(8, np.random.default_rng(6))
    assert np.allclose(H[1:, :-1], H[:-1, 1:])
