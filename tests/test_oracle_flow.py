"""Pins of the oracle's Wilson flow (Sec. II.B, V.B; the survey's f4 row):
the Euler step is the simultaneous stout step (rho = eps), the third-order
Runge-Kutta scheme converges at third order while Euler converges at first,
a centre field does not flow, the flow is gauge equivariant and lowers the
Wilson action."""
import numpy as np
import pytest

import fieldgen

DIMS = (4, 4, 4, 4)


def _smooth_random_field(dims, seed, amp=0.3):
    """exp(amp X) for random traceless anti-Hermitian X, X = i H with H from the
    Gell-Mann basis (a field near the identity, where the flow is smooth)."""
    from tests._loops import gell_mann_generators

    rng = np.random.default_rng(seed)
    V = fieldgen.volume(dims)
    T = gell_mann_generators()  # anti-Hermitian, Tr T^a T^b = -delta/2
    c = rng.normal(size=(4, V, 8))
    X = np.einsum("dsa,aij->dsij", c, T) * amp
    from scipy.linalg import expm

    return np.array([[expm(X[d, s]) for s in range(V)] for d in range(4)])


def test_euler_step_is_the_simultaneous_stout_step(ora):
    U = _smooth_random_field(DIMS, 1)
    n = np.zeros((4, fieldgen.volume(DIMS)), np.int8)
    A = U.copy()
    ora.flow(DIMS, A, 1, 0.05, eps_oi=-0.25, integrator="euler")
    B = U.copy()
    ora.smooth(DIMS, B, n, 1, order="jacobi", rho=0.05, eps=-0.25, measure_every=0)
    np.testing.assert_array_equal(A, B)


@pytest.mark.parametrize("integrator,order", [("euler", 1), ("rk3", 3)])
def test_convergence_order(ora, integrator, order):
    U = _smooth_random_field(DIMS, 2)
    tau = 0.12
    ref = U.copy()
    ora.flow(DIMS, ref, 48, tau / 48, integrator="rk3")
    errs = []
    for nst in (3, 6, 12):
        W = U.copy()
        ora.flow(DIMS, W, nst, tau / nst, integrator=integrator)
        errs.append(np.abs(W - ref).max())
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(abs(r - order) < 0.35 for r in rates), (errs, rates)


@pytest.mark.parametrize("integrator", ["euler", "rk3"])
def test_centre_field_does_not_flow(ora, integrator):
    """Sec. II.B: Q = 0 on a centre field, in any gauge."""
    V = fieldgen.volume(DIMS)
    n = fieldgen.z3_vortex_charges(DIMS, 0.3, 3)
    G = fieldgen.haar_su3(V, 4)
    U = ora.gauge_transform(DIMS, ora.z3_field(DIMS, n), G)
    W = U.copy()
    ora.flow(DIMS, W, 3, 0.05, eps_oi=-0.25, integrator=integrator)
    assert np.abs(W - U).max() < 1e-14


def test_flow_is_gauge_equivariant(ora):
    V = fieldgen.volume(DIMS)
    U = _smooth_random_field(DIMS, 5)
    G = fieldgen.haar_su3(V, 6)
    A = ora.gauge_transform(DIMS, U, G)
    ora.flow(DIMS, A, 2, 0.05, integrator="rk3")
    B = U.copy()
    ora.flow(DIMS, B, 2, 0.05, integrator="rk3")
    B = ora.gauge_transform(DIMS, B, G)
    assert np.abs(A - B).max() < 1e-13


def test_flow_lowers_the_wilson_action(ora):
    V = fieldgen.volume(DIMS)
    U = fieldgen.haar_su3(4 * V, 7).reshape(4, V, 3, 3).copy()
    n = np.zeros((4, V), np.int8)
    s = [ora.measure(DIMS, U, n).action]
    for _ in range(5):
        ora.flow(DIMS, U, 1, 0.02, integrator="rk3")
        s.append(ora.measure(DIMS, U, n).action)
    assert all(b < a for a, b in zip(s, s[1:]))
