"""Pins of the oracle's field-strength measurements (Sec. V, Eqs. 1LFST and
1LTopQ; the reconstructed action of Sec. V.A; the correlations of Sec. VII).

A constant abelian field in the T = diag(1, -1, 0) direction with plaquette
angle B in the (0,1) planes and B' in the (2,3) planes has, at every site,
  clover C_01 = exp(-i B T), F_01 = -sin(B) T, F_23 = -sin(B') T,
  S(x)/beta   = (2/72) [2(1 - cos B) + 2(1 - cos B')],
  S_R(x)/beta = (1/72) [2 sin^2 B + 2 sin^2 B'],
  q(x)        = 8 Tr[F_01 F_23] / (32 pi^2) = sin B sin B' / (2 pi^2),
so S_R/S = cos^2(B/2) -> 1 as the field becomes smooth (the paper's
smoothness condition).
"""
import numpy as np
import pytest

import fieldgen

DIMS = (4, 6, 4, 8)


def _abelian_field(dims, n1, n3):
    """U_0(x) = exp(i B x_1 T), U_2(x) = exp(i B' x_3 T), U_1 = U_3 = 1 with
    B = 2 pi n1 / L_1, B' = 2 pi n3 / L_3 (periodic: the flux is quantised)."""
    L0, L1, L2, L3 = dims
    V = fieldgen.volume(dims)
    B, Bp = 2 * np.pi * n1 / L1, 2 * np.pi * n3 / L3
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    s = np.arange(V)
    x1 = (s // L0) % L1
    x3 = s // (L0 * L1 * L2)
    t = np.array([1.0, -1.0, 0.0])
    for mu in range(4):
        U[mu][:, [0, 1, 2], [0, 1, 2]] = 1.0
    U[0][:, [0, 1, 2], [0, 1, 2]] = np.exp(1j * B * x1[:, None] * t[None, :])
    U[2][:, [0, 1, 2], [0, 1, 2]] = np.exp(1j * Bp * x3[:, None] * t[None, :])
    return U, B, Bp


@pytest.mark.parametrize("n1,n3", [(1, 1), (1, -2), (2, 3), (0, 1), (-1, 1)])
def test_constant_abelian_field_closed_forms(ora, n1, n3):
    U, B, Bp = _abelian_field(DIMS, n1, n3)
    sr, q, s, sd, qd = ora.clover(DIMS, U, densities=True)
    s_site = 2.0 / 72 * (2 * (1 - np.cos(B)) + 2 * (1 - np.cos(Bp)))
    sr_site = 1.0 / 72 * (2 * np.sin(B) ** 2 + 2 * np.sin(Bp) ** 2)
    q_site = np.sin(B) * np.sin(Bp) / (2 * np.pi ** 2)
    np.testing.assert_allclose(sd, s_site, atol=1e-15)
    np.testing.assert_allclose(qd, q_site, atol=1e-15)
    assert abs(s - s_site) < 1e-15 and abs(sr - sr_site) < 1e-15
    assert abs(q - q_site * fieldgen.volume(DIMS)) < 1e-12
    # the ordinary measurement agrees on <S>/beta
    assert abs(ora.measure(DIMS, U, np.zeros((4, fieldgen.volume(DIMS)), np.int8)).action - s) < 1e-15


def test_reconstructed_action_approaches_wilson_action_when_smooth(ora):
    dims = (4, 64, 4, 64)
    ratios = []
    for n in (8, 4, 2, 1):
        U, B, Bp = _abelian_field(dims, n, n)
        sr, q, s = ora.clover(dims, U)
        ratios.append(sr / s)
        # sin^2 B / (2 (1 - cos B)) = cos^2(B/2)
        assert abs(sr / s - np.cos(B / 2) ** 2) < 1e-13
    assert all(a < b < 1 for a, b in zip(ratios, ratios[1:]))


def test_clover_quantities_are_gauge_invariant(ora):
    """F -> G F G^dagger under a gauge transform, so Tr[F F] and q(x) are
    invariant site by site; so is S(x)."""
    V = fieldgen.volume(DIMS)
    U = fieldgen.haar_su3(4 * V, 71).reshape(4, V, 3, 3).copy()
    G = fieldgen.haar_su3(V, 72)
    W = ora.gauge_transform(DIMS, U, G)
    a = ora.clover(DIMS, U, densities=True)
    b = ora.clover(DIMS, W, densities=True)
    np.testing.assert_allclose(a[3], b[3], atol=1e-13)
    np.testing.assert_allclose(a[4], b[4], atol=1e-13)
    assert abs(a[0] - b[0]) < 1e-13 and abs(a[1] - b[1]) < 1e-11


def test_charge_is_odd_under_reflection(ora):
    """Reversing the flux in one plane (B -> -B) reverses q; a field with flux in
    only one plane has q = 0."""
    U1, _, _ = _abelian_field(DIMS, 1, 2)
    U2, _, _ = _abelian_field(DIMS, -1, 2)
    U3, _, _ = _abelian_field(DIMS, 1, 0)
    q1, q2, q3 = ora.clover(DIMS, U1)[1], ora.clover(DIMS, U2)[1], ora.clover(DIMS, U3)[1]
    assert q1 > 0 and abs(q1 + q2) < 1e-12 and abs(q3) < 1e-13


def test_correlation(ora):
    rng = np.random.default_rng(5)
    a = rng.normal(size=1000)
    b = rng.normal(size=1000)
    assert abs(ora.correlation(a, a) - 1) < 1e-15
    assert abs(ora.correlation(a, -a) + 1) < 1e-15
    assert abs(ora.correlation(a, 3.5 * a) - 1) < 1e-15
    c = ora.correlation(a, b)
    assert abs(c - np.dot(a, b) / np.sqrt(np.dot(a, a) * np.dot(b, b))) < 1e-14
    assert abs(c) < 0.15
