"""Pins of the oracle's APE update with unit circle projection (Sec. II.C,
Eqs. V, W), the survey's f3 row.

* The projection is the polar factor of V divided by the principal cube root of
  its determinant: checked against scipy.linalg.polar.
* It is gauge equivariant: P{G V G'^dag} = G P{V} G'^dag.
* The paper's key result: on a centre-vortex field (V = r e^{i theta} G G'^dag)
  it can only return a centre element, e^{-2 pi i k/3} G G'^dag with k such
  that theta + 2 pi k/3 lies in (-pi/3, pi/3].
"""
import numpy as np
import pytest
import scipy.linalg

import fieldgen

SMALL = (4, 4, 4, 4)


def _rand(rng, n=3):
    return rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))


def test_projection_is_normalised_polar_factor(ora):
    rng = np.random.default_rng(11)
    for _ in range(20):
        V = _rand(rng)
        W = ora.unit_circle_projection(V)
        u, _ = scipy.linalg.polar(V)
        d = np.linalg.det(u)
        want = u / (np.abs(d) ** (1 / 3) * np.exp(1j * np.angle(d) / 3))
        assert np.abs(W - want).max() < 1e-13
        assert np.abs(W.conj().T @ W - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(W) - 1) < 1e-14


def test_projection_is_gauge_equivariant(ora):
    rng = np.random.default_rng(12)
    G = fieldgen.haar_su3(2, 13)
    for _ in range(10):
        V = _rand(rng)
        lhs = ora.unit_circle_projection(G[0] @ V @ G[1].conj().T)
        rhs = G[0] @ ora.unit_circle_projection(V) @ G[1].conj().T
        assert np.abs(lhs - rhs).max() < 1e-13


@pytest.mark.parametrize("theta", np.linspace(-3.1, 3.1, 13))
def test_centre_element_in_centre_element_out(ora, theta):
    G = fieldgen.haar_su3(2, 14)
    V = 0.7 * np.exp(1j * theta) * G[0] @ G[1].conj().T
    W = ora.unit_circle_projection(V)
    k = [kk for kk in (-1, 0, 1) if -np.pi / 3 < theta + 2 * np.pi * kk / 3 <= np.pi / 3][0]
    want = np.exp(-2j * np.pi * k / 3) * G[0] @ G[1].conj().T
    assert np.abs(W - want).max() < 1e-13


@pytest.mark.parametrize("gauge", [False, True])
def test_ape_sweep_maps_a_vortex_field_to_centre_elements(ora, gauge):
    """One smearing sweep of APE on a Z(3) field (alpha = 0.7, over-improved
    staples): every link comes out as a centre element (times G G^dag in a random
    gauge), namely the one nearest in phase to the scalar blocked matrix."""
    dims = SMALL
    V = fieldgen.volume(dims)
    n = fieldgen.z3_vortex_charges(dims, 0.3, 15)
    U = ora.z3_field(dims, n)
    G = fieldgen.haar_su3(V, 16) if gauge else np.broadcast_to(np.eye(3), (V, 3, 3)).astype(complex)
    if gauge:
        U = ora.gauge_transform(dims, U, G)
    alpha, eps = 0.7, -0.25
    W = U.copy()
    ora.smooth(dims, W, n, 1, order="jacobi", update="ape", alpha=alpha, eps=eps, measure_every=0)
    for mu in range(4):
        fwd = fieldgen.neighbour(dims, mu, 1)
        for s in range(0, V, 5):
            sp = fwd[s]
            Vb = (1 - alpha) * U[mu, s] + alpha / 6 * ora.staple(dims, U, mu, s, eps=eps)
            v = np.trace(G[s].conj().T @ Vb @ G[sp]) / 3  # the scalar of V in the gauge frame
            k = [kk for kk in (-1, 0, 1) if -np.pi / 3 < np.angle(v) + 2 * np.pi * kk / 3 <= np.pi / 3][0]
            want = np.exp(-2j * np.pi * k / 3) * G[s] @ G[sp].conj().T
            assert np.abs(W[mu, s] - want).max() < 1e-12
