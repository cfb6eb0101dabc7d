"""The seeded input generator: determinism and the known-spectrum construction."""
import numpy as np
import pytest

import jjgen


def test_deterministic_across_thread_counts():
    a = jjgen.make(96, True, 40, 1e-6, 1.0, seed=5, threads=1)
    b = jjgen.make(96, True, 40, 1e-6, 1.0, seed=5, threads=7)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    c = jjgen.make(96, True, 40, 1e-6, 1.0, seed=6)
    assert not np.array_equal(a[0], c[0])


@pytest.mark.parametrize("cplx", [False, True])
def test_construction(cplx):
    n, p = 50, 21
    G, J, lam = jjgen.make(n, cplx, p, 1e-2, 1e2, seed=3)
    assert np.sum(J == 1) == p and np.sum(J == -1) == n - p
    assert np.all(np.sign(lam) == J)
    assert np.all((np.abs(lam) >= 1e-2 * (1 - 1e-15)) & (np.abs(lam) <= 1e2 * (1 + 1e-15)))
    # H = G J G^* = Q diag(lam) Q^*: LAPACK's eigvalsh is accurate to eps ||H|| here
    H = G @ np.diag(J.astype(float)) @ G.conj().T
    ev = np.sort(np.linalg.eigvalsh(H))[::-1]
    assert np.max(np.abs(ev - np.sort(lam)[::-1])) <= 1e-12 * np.max(np.abs(lam))


def test_without_haar_is_diag_times_rotations():
    # haar=False gives B = diag(sqrt|lam|) W with W J-unitary: B^* ... W^* J W = J
    n = 12
    B, J, lam = jjgen.make(n, False, 5, 0.5, 2.0, seed=8, haar=False)
    W = np.diag(1.0 / np.sqrt(np.abs(lam))) @ B
    Jd = np.diag(J.astype(float))
    assert np.max(np.abs(W.T @ Jd @ W - Jd)) <= 1e-12 * np.max(np.abs(W)) ** 2


def test_configs_shapes():
    G, J, lam = jjgen.config(1)
    assert G.shape == (64, 64) and G.dtype == np.float64 and np.sum(J == 1) == 32
    G, J, lam = jjgen.config(2, n=128)
    assert G.shape == (128, 128) and G.dtype == np.complex128 and np.sum(J == 1) == 64
    specs = jjgen.batch_recipe(64)
    assert all(16 <= s["n"] <= 512 and 0 <= s["p"] <= s["n"] for s in specs)
    assert sum(s["cplx"] for s in specs) == 32
