"""Pins of the regularisers: finite differences, special cases, transposes."""
import numpy as np
import pytest

from oracle import prior
from oracle.minimiser import dense_matrix


@pytest.mark.parametrize("kind,param", [("tv", 1e-1), ("tv", 1e-3), ("huber", 0.3), ("huber", 100.0)])
@pytest.mark.parametrize("bc", ["neumann", "circular"])
def test_gradient_matches_finite_differences(kind, param, bc):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((7, 9))
    g = prior.gradient(x, kind, param, bc)
    h = 1e-6
    num = np.zeros_like(x)
    for i in range(x.shape[0]):
        for j in range(x.shape[1]):
            e = np.zeros_like(x)
            e[i, j] = h
            num[i, j] = (prior.value(x + e, kind, param, bc) - prior.value(x - e, kind, param, bc)) / (2 * h)
    assert np.max(np.abs(g - num)) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_tv_of_constant_is_zero_and_matches_definition():
    x = np.full((5, 6), 3.7)
    assert prior.value(x, "tv", 1e-3) == 0.0
    assert np.all(prior.gradient(x, "tv", 1e-3) == 0.0)
    # isotropic TV with Neumann differences, written out with np.diff
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 6))
    gh = np.zeros_like(x)
    gv = np.zeros_like(x)
    gh[:, :-1] = np.diff(x, axis=1)
    gv[:-1, :] = np.diff(x, axis=0)
    eps = 0.01
    ref = np.sum(np.sqrt(gh ** 2 + gv ** 2 + eps ** 2) - eps)
    assert abs(prior.value(x, "tv", eps) - ref) <= 1e-13


def test_huber_limits():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 6))
    quad = 0.5 * (np.sum(np.diff(x, axis=0) ** 2) + np.sum(np.diff(x, axis=1) ** 2))
    assert abs(prior.value(x, "huber", 1e9) - quad) <= 1e-12
    # tiny delta: delta * (|g| - delta/2) ~ delta * TV(eps=0)
    d = 1e-9
    gh = np.zeros_like(x)
    gv = np.zeros_like(x)
    gh[:, :-1] = np.diff(x, axis=1)
    gv[:-1, :] = np.diff(x, axis=0)
    tv0 = np.sum(np.sqrt(gh ** 2 + gv ** 2))
    assert abs(prior.value(x, "huber", d) / d - tv0) <= 1e-6 * tv0


@pytest.mark.parametrize("bc", ["neumann", "circular"])
def test_difference_adjoint_and_norm(bc):
    shape = (5, 7)
    Dh = dense_matrix(lambda z: prior.forward_diff(z, bc)[0], shape)
    Dv = dense_matrix(lambda z: prior.forward_diff(z, bc)[1], shape)
    D = np.vstack([Dh, Dv])
    n = int(np.prod(shape))
    DT = dense_matrix(lambda z: prior.forward_diff_adjoint(z[:n].reshape(shape), z[n:].reshape(shape), bc),
                      (2 * n,))
    assert np.max(np.abs(DT - D.T)) <= 1e-15
    assert np.linalg.norm(D, 2) ** 2 <= 8.0 + 1e-12
