"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types an oracle
formula: the checks go through closed forms, invariants, library routines
(scipy), hand-derived fixtures under tests/golden/ and brute force on small
lattices, built with code that shares nothing with the oracle.
"""
import os

import numpy as np
import pytest
import scipy.linalg

import fieldgen
from tests import _loops

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SMALL = (4, 4, 4, 4)
TINY = (2, 2, 2, 2)  # every wrap-around as short as it can be


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _site(dims, x, y, z, t):
    L = dims
    return (x % L[0]) + L[0] * ((y % L[1]) + L[1] * ((z % L[2]) + L[2] * (t % L[3])))


def _centrifuged(ora, dims, p=0.1, seed=7, omega=0.02):
    n = fieldgen.z3_vortex_charges(dims, p, seed)
    pairs = fieldgen.centrifuge_pairs(dims, seed + 1)
    return n, ora.centrifuge(dims, n, pairs, omega)


def _haar_field(dims, seed):
    V = fieldgen.volume(dims)
    return fieldgen.haar_su3(4 * V, seed).reshape(4, V, 3, 3).copy()


# ----------------------------------------------------------- centre projection


def test_sector_hand_points(ora):
    """Eq. (centre_element): hand-picked traces, boundaries undefined."""
    for re, im, exp in _rows("sector_points.txt"):
        want = ora.UNDEF if exp == "U" else int(exp)
        assert ora.sector(complex(float(re), float(im))) == want, (re, im)


def test_sector_of_centre_elements(ora):
    """A centre element e^{2 pi i n/3} 1 projects to n (Eq. centre_project)."""
    for n in (-1, 0, 1):
        z = np.exp(2j * np.pi * n / 3.0)
        assert ora.sector(3 * z) == n
        # small rotations inside the sector keep it
        for d in (-0.9, -0.3, 0.3, 0.9):
            assert ora.sector(3 * z * np.exp(1j * d * np.pi / 3)) == n


# ------------------------------------------------------------- field ingest


def test_z3_field_plaquettes_exact(ora):
    """Sec. I: projected plaquettes are e^{2 pi i p/3} 1, so Re Tr P/3 = cos(2 pi p/3)
    is 1 or -1/2, and the flux equals the lattice curl of the vortex seed s (the
    random gauge part g cancels).  <P> = 1 - (3/2) N_pierced / (6V) exactly."""
    dims = (4, 4, 4, 8)
    n, g, s = fieldgen.z3_vortex_charges(dims, 0.15, 11, return_parts=True)
    U = ora.z3_field(dims, n)
    V = fieldgen.volume(dims)
    st, flux = ora.measure(dims, U, n, with_flux=True)
    plaqs = _loops.plaquettes(dims, U)
    pierced = 0
    plane = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            curl = (s[mu] + _loops.shift(dims, s[nu], mu, 1) - _loops.shift(dims, s[mu], nu, 1)
                    - s[nu]) % 3
            want_flux = np.where(curl == 2, -1, curl)
            np.testing.assert_array_equal(flux[plane], want_flux)
            tr = np.trace(plaqs[plane], axis1=1, axis2=2) / 3.0
            np.testing.assert_allclose(tr.real, np.cos(2 * np.pi * curl / 3.0), atol=2e-15)
            np.testing.assert_allclose(tr.imag, np.sin(2 * np.pi * curl / 3.0), atol=2e-15)
            pierced += int(np.count_nonzero(curl))
            plane += 1
    assert pierced > 0
    assert abs(st.plaq - (1.0 - 1.5 * pierced / (6.0 * V))) < 1e-14
    assert abs(st.action - 0.5 * (1.0 - st.plaq)) < 1e-14
    assert st.flux_mismatch == 0 and st.undefined_sector == 0 and st.nonfinite == 0
    np.testing.assert_array_equal(ora.sectors(dims, U), n)


def test_zero_density_field_is_cold(ora):
    """p = 0 gives a pure gauge Z(3) field: every plaquette is 1."""
    dims = SMALL
    n = fieldgen.z3_vortex_charges(dims, 0.0, 3)
    st = ora.measure(dims, ora.z3_field(dims, n), n)
    assert abs(st.plaq - 1.0) < 1e-15 and abs(st.action) < 1e-15


# -------------------------------------------------------------- centrifuge


def test_centrifuge_single_defect_fixture(ora):
    """Sec. IV staple phase: hand-derived m for a single non-zero charge."""
    dims = SMALL
    V = fieldgen.volume(dims)
    n = np.zeros((4, V), dtype=np.int8)
    n[0, 0] = 1
    pairs = np.zeros((4, V), dtype=np.int8)
    _, m = ora.centrifuge(dims, n, pairs, 0.02, return_m=True)
    want = np.zeros((4, V), dtype=np.int32)
    for mu, dx, dy, dz, dt, val in _rows("centrifuge_single_defect.txt"):
        want[int(mu), _site(dims, int(dx), int(dy), int(dz), int(dt))] = int(val)
    np.testing.assert_array_equal(m, want)


def test_centrifuge_phases_and_trace(ora):
    """Sec. IV/IV.A: det Z' = 1 (phase sum kept), Tr Z' = (2 cos L- + 1) e^{2 pi i n/3}
    with L- = (lambda^j - lambda^k)/2 = omega (sigma - lambda), sector of n kept,
    links diagonal, and the rotated phases are lambda -+ omega (lambda - sigma)."""
    dims = (4, 4, 4, 8)
    n = fieldgen.z3_vortex_charges(dims, 0.12, 5)
    pairs = fieldgen.centrifuge_pairs(dims, 6)
    omega = 0.02
    U, m = ora.centrifuge(dims, n, pairs, omega, return_m=True)
    V = fieldgen.volume(dims)
    off = U.copy()
    for i in range(3):
        off[..., i, i] = 0
    assert np.count_nonzero(off) == 0
    det = np.linalg.det(U.reshape(-1, 3, 3))
    np.testing.assert_allclose(det, 1.0, atol=1e-15)
    lam = 2 * np.pi * n.astype(float) / 3.0
    sig = 2 * np.pi * m.astype(float) / 18.0
    lminus = omega * (sig - lam)
    tr = np.trace(U, axis1=2, axis2=3)
    np.testing.assert_allclose(tr, (2 * np.cos(lminus) + 1) * np.exp(1j * lam), atol=1e-14)
    np.testing.assert_array_equal(ora.sectors(dims, U), n)
    assert np.abs(m).max() <= 18
    # per-link phase placement: pair (j, k) = (1,2), (2,3), (3,1)
    diag = np.stack([U[..., i, i] for i in range(3)], axis=-1)
    for mu in range(4):
        for s in range(0, V, 37):
            j = int(pairs[mu, s])
            k = (j + 1) % 3
            third = 3 - j - k
            ph = np.angle(diag[mu, s] / np.exp(1j * lam[mu, s]))
            assert abs(ph[j] - lminus[mu, s]) < 1e-14
            assert abs(ph[k] + lminus[mu, s]) < 1e-14
            assert abs(ph[third]) < 1e-15


def test_centrifuge_m_mod3_matches_staple_matrices(ora):
    """6 sigma is the sum of the six staple phases, so e^{2 pi i m/3} 1 must equal the
    product of the six plain staples of the Z(3) field (independent matrix route)."""
    dims = SMALL
    n = fieldgen.z3_vortex_charges(dims, 0.3, 9)
    pairs = fieldgen.centrifuge_pairs(dims, 10)
    _, m = ora.centrifuge(dims, n, pairs, 0.01, return_m=True)
    U = ora.z3_field(dims, n)
    for mu in range(4):
        prod = np.broadcast_to(np.eye(3), (fieldgen.volume(dims), 3, 3)).astype(complex)
        for nu in range(4):
            if nu == mu:
                continue
            up = U[nu] @ _loops.shift(dims, U[mu], nu, 1) @ _loops.dag(_loops.shift(dims, U[nu], mu, 1))
            bm = _loops.shift(dims, U[nu], nu, -1)
            dn = _loops.dag(bm) @ _loops.shift(dims, U[mu], nu, -1) @ _loops.shift(dims, bm, mu, 1)
            prod = prod @ up @ dn
        want = np.exp(2j * np.pi * m[mu] / 3.0)
        np.testing.assert_allclose(prod[:, 0, 0], want, atol=1e-13)


def test_centrifuge_zero_omega_is_identity(ora):
    dims = SMALL
    n = fieldgen.z3_vortex_charges(dims, 0.2, 12)
    pairs = fieldgen.centrifuge_pairs(dims, 13)
    np.testing.assert_array_equal(ora.centrifuge(dims, n, pairs, 0.0), ora.z3_field(dims, n))


def test_centrifuge_preservation_bound(ora):
    """Sec. IV.A: with m = 18 and n = -1 the condition omega |m - 6n| < 6 needs
    omega < 1/4; just above, the oracle refuses, just below it accepts."""
    dims = SMALL
    V = fieldgen.volume(dims)
    n = np.zeros((4, V), dtype=np.int8)
    o = _site(dims, 1, 1, 1, 1)
    n[0, o] = -1
    e0 = (1, 0, 0, 0)
    for nu in (1, 2, 3):
        e = [0, 0, 0, 0]
        e[nu] = 1

        def at(mu, dx, val):
            c = [1 + dx[0], 1 + dx[1], 1 + dx[2], 1 + dx[3]]
            n[mu, _site(dims, *c)] = val

        at(nu, (0, 0, 0, 0), 1)                                      # lambda_nu(x)
        at(0, tuple(e), 1)                                           # lambda_mu(x+nu)
        at(nu, e0, -1)                                               # -lambda_nu(x+mu)
        at(nu, tuple(-v for v in e), -1)                             # -lambda_nu(x-nu)
        at(0, tuple(-v for v in e), 1)                               # lambda_mu(x-nu)
        at(nu, tuple(a - b for a, b in zip(e0, e)), 1)               # lambda_nu(x-nu+mu)
    pairs = np.zeros((4, V), dtype=np.int8)
    _, m = ora.centrifuge(dims, n, pairs, 0.1, return_m=True)
    assert m[0, o] == 18
    ora.centrifuge(dims, n, pairs, 0.2499)
    with pytest.raises(ValueError):
        ora.centrifuge(dims, n, pairs, 0.2501)


# --------------------------------------------------------- staples and Q


@pytest.mark.parametrize("dims,eps", [(SMALL, 1.0), (SMALL, -0.25), (TINY, 1.0), (TINY, -0.25)])
def test_staple_is_action_gradient(ora, dims, eps):
    """Sec. II.B: the generator of the Wilson flow is the gradient of the action,
    d/ds A(e^{s T^a} U)|_0 for the loop-sum action A = sum c_p Re Tr P + sum c_r Re Tr R
    (Eq. over-improvement weights).  sum_a T^a dA_a equals half the traceless
    anti-Hermitian part of Omega = Sigma U^dagger (Eq. generator).  Brute force by
    central differences on Haar-random 4^4 and 2^4 fields.  On 2^4 a 1x2
    rectangle runs through the updated link twice (once each way); the staple
    sum holds one path per occurrence, which is the product rule, so it is
    still the gradient."""
    U = _haar_field(dims, 21)
    T = _loops.gell_mann_generators()
    h = 1e-5
    rng = np.random.default_rng(3)
    for _ in range(3):
        mu = int(rng.integers(0, 4))
        s = int(rng.integers(0, fieldgen.volume(dims)))
        Sigma = ora.staple(dims, U, mu, s, eps=eps)
        Q = ora.generator(Sigma @ U[mu, s].conj().T)
        grad = np.zeros((3, 3), dtype=complex)
        for a in range(8):
            vals = []
            for sg in (+1, -1):
                W = U.copy()
                W[mu, s] = scipy.linalg.expm(sg * h * T[a]) @ U[mu, s]
                vals.append(_loops.improved_action(dims, W, eps))
            grad += T[a] * (vals[0] - vals[1]) / (2 * h)
        np.testing.assert_allclose(grad, 0.5 * Q, atol=2e-8)


@pytest.mark.parametrize("dims", [SMALL, TINY])
def test_staple_gauge_covariance(ora, dims):
    """Sec. II.A: Sigma -> G(x) Sigma G^dagger(x + mu) under a gauge transform,
    also on 2^4 where x + 2 nu = x."""
    U = _haar_field(dims, 31)
    V = fieldgen.volume(dims)
    G = fieldgen.haar_su3(V, 32)
    UG = ora.gauge_transform(dims, U, G)
    for eps in (1.0, -0.25):
        for mu, s in ((0, 0), (3, 77 % V), (1, 200 % V)):
            a = ora.staple(dims, UG, mu, s, eps=eps)
            sp = fieldgen.neighbour(dims, mu, 1)[s]
            b = G[s] @ ora.staple(dims, U, mu, s, eps=eps) @ G[sp].conj().T
            np.testing.assert_allclose(a, b, atol=1e-13)


def test_gauge_transform_keeps_plaquette_traces(ora):
    dims = SMALL
    U = _haar_field(dims, 41)
    G = fieldgen.haar_su3(fieldgen.volume(dims), 42)
    UG = ora.gauge_transform(dims, U, G)
    for a, b in zip(_loops.plaquettes(dims, U), _loops.plaquettes(dims, UG)):
        np.testing.assert_allclose(np.trace(a, axis1=1, axis2=2), np.trace(b, axis1=1, axis2=2),
                                   atol=1e-13)
    I = np.broadcast_to(np.eye(3), (fieldgen.volume(dims), 3, 3)).astype(complex)
    np.testing.assert_array_equal(ora.gauge_transform(dims, U, I), U)


def test_centre_field_staple_is_identity_proportional(ora):
    """Sec. II.A: every path sum of a (gauge-rotated) centre field is r e^{i theta} 1,
    so Omega is proportional to 1 and Q vanishes."""
    dims = SMALL
    n = fieldgen.z3_vortex_charges(dims, 0.3, 51)
    U = ora.z3_field(dims, n)
    for eps in (1.0, -0.25):
        for mu, s in ((0, 5), (2, 100)):
            Sig = ora.staple(dims, U, mu, s, eps=eps)
            om = Sig @ U[mu, s].conj().T
            assert np.allclose(om, om[0, 0] * np.eye(3), atol=1e-14)
            np.testing.assert_allclose(ora.generator(om), 0, atol=1e-15)


def test_generator_projection(ora):
    """Eq. (generator): Q is traceless and anti-Hermitian; it returns a traceless
    anti-Hermitian input unchanged and drops Hermitian and identity parts."""
    rng = np.random.default_rng(8)
    for _ in range(5):
        A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        Q = ora.generator(A)
        np.testing.assert_allclose(Q, -Q.conj().T, atol=1e-15)
        assert abs(np.trace(Q)) < 1e-15
        np.testing.assert_allclose(ora.generator(Q), Q, atol=1e-15)
        H = A + A.conj().T
        np.testing.assert_allclose(ora.generator(A + H + (2 - 3j) * np.eye(3)), Q, atol=1e-14)


# --------------------------------------------------------------- exponential


def test_expm_against_scipy_and_closed_forms(ora):
    rng = np.random.default_rng(17)
    for scale in (1e-8, 0.05, 0.7, 3.0):
        A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        X = scale * 0.5 * (A - A.conj().T)
        X -= np.trace(X) / 3 * np.eye(3)
        E = ora.expm(X)
        np.testing.assert_allclose(E, scipy.linalg.expm(X), atol=2e-15 * max(1, scale))
        np.testing.assert_allclose(E @ E.conj().T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(E) - 1) < 1e-14
    th = np.array([0.3, -1.1, 0.8])
    np.testing.assert_allclose(ora.expm(np.diag(1j * th)), np.diag(np.exp(1j * th)), atol=1e-15)
    # SU(2) embedded in (1,3): exp(i a sigma_y) = cos a + i sin a sigma_y
    a = 0.9
    X = np.zeros((3, 3), complex)
    X[0, 2], X[2, 0] = a, -a
    want = np.eye(3, dtype=complex)
    want[0, 0] = want[2, 2] = np.cos(a)
    want[0, 2], want[2, 0] = np.sin(a), -np.sin(a)
    np.testing.assert_allclose(ora.expm(X), want, atol=1e-15)
    np.testing.assert_array_equal(ora.expm(np.zeros((3, 3))), np.eye(3))


# -------------------------------------------------------- stout smoothing


@pytest.mark.parametrize("order,eps", [("jacobi", 1.0), ("annealed", 1.0), ("annealed", -0.25)])
def test_centre_field_invariant_under_stout(ora, order, eps):
    """Sec. II.A, II.B: stout smearing and the Wilson flow leave a centre field,
    and a gauge-rotated one, unchanged."""
    dims = SMALL
    n = fieldgen.z3_vortex_charges(dims, 0.25, 61)
    U = ora.z3_field(dims, n)
    W = U.copy()
    ora.smooth(dims, W, n, 4, order=order, rho=0.1, eps=eps, measure_every=0)
    np.testing.assert_allclose(W, U, atol=1e-15, rtol=0)
    G = fieldgen.haar_su3(fieldgen.volume(dims), 62)
    UG = ora.gauge_transform(dims, U, G)
    WG = UG.copy()
    ora.smooth(dims, WG, n, 3, order=order, rho=0.1, eps=eps, measure_every=0)
    np.testing.assert_allclose(WG, UG, atol=1e-13)


@pytest.mark.parametrize("order,eps", [("jacobi", 1.0), ("annealed", -0.25)])
def test_stout_gauge_equivariance(ora, order, eps):
    """Sec. V.C: S{U^G} = G S{U} G^dagger for stout / Wilson flow."""
    dims = SMALL
    n, U = _centrifuged(ora, dims, p=0.2, seed=71, omega=0.05)
    U = _haar_field(dims, 72) if order == "jacobi" else U
    G = fieldgen.haar_su3(fieldgen.volume(dims), 73)
    A = U.copy()
    ora.smooth(dims, A, n, 2, order=order, rho=0.08, eps=eps, measure_every=0)
    B = ora.gauge_transform(dims, U, G)
    ora.smooth(dims, B, n, 2, order=order, rho=0.08, eps=eps, measure_every=0)
    np.testing.assert_allclose(B, ora.gauge_transform(dims, A, G), atol=1e-12)


def test_diagonal_field_stays_diagonal(ora):
    """Sec. V.B: smoothing a preconditioned field in MCG keeps it diagonal."""
    dims = SMALL
    n, U = _centrifuged(ora, dims, p=0.2, seed=81)
    ora.smooth(dims, U, n, 3, order="annealed", rho=0.06, eps=-0.25, vp=True, measure_every=0)
    for i in range(3):
        for j in range(3):
            if i != j:
                assert np.count_nonzero(U[..., i, j]) == 0


def test_stout_single_link_closed_form(ora):
    """Eq. (stout) for a diagonal link: with Omega = diag(w), Q = i diag(q) where
    q_i = Im w_i - mean(Im w), so U' = diag(e^{i rho q}) U."""
    dims = SMALL
    n, U = _centrifuged(ora, dims, p=0.3, seed=91, omega=0.1)
    for mu, s in ((0, 3), (1, 50), (3, 200)):
        Sig = ora.staple(dims, U, mu, s, eps=-0.25)
        w = np.diag(Sig @ U[mu, s].conj().T)
        q = w.imag - w.imag.mean()
        want = np.diag(np.exp(1j * 0.06 * q)) @ U[mu, s]
        got, acc = ora.update_link(dims, U, n, mu, s, rho=0.06, eps=-0.25)
        assert acc
        np.testing.assert_allclose(got, want, atol=1e-15)


def test_annealed_subset_is_independent(ora):
    """Sec. III.A masking: an in-place subset step equals updating every link of the
    subset from the field before the step (no link of a subset is in another's
    over-improved staple), and leaves every other link untouched."""
    dims = (4, 4, 4, 8)
    U = _haar_field(dims, 101)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 102)
    V = fieldgen.volume(dims)
    for mu, c in ((0, 0), (2, 3)):
        before = U.copy()
        after = U.copy()
        ora.anneal_pass(dims, after, n, mu, c, rho=0.07, eps=-0.25)
        for s in range(V):
            if ora.colour(dims, mu, s) == c:
                want, _ = ora.update_link(dims, before, n, mu, s, rho=0.07, eps=-0.25)
                np.testing.assert_array_equal(after[mu, s], want)
        mask = np.array([ora.colour(dims, mu, s) != c for s in range(V)])
        np.testing.assert_array_equal(after[mu][mask], before[mu][mask])
        for nu in range(4):
            if nu != mu:
                np.testing.assert_array_equal(after[nu], before[nu])


def test_colouring_conflict_free_by_enumeration():
    """The annealing subsets c = (2 x_mu + sum_{nu != mu} x_nu) mod 4 never put a link
    and another link of its own staple paths (same direction) in the same subset.
    The stencil is enumerated by walking the over-improvement diagrams."""
    offs = set()
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            for sg in (1, -1):
                n, m = sg * (nu + 1), mu + 1
                for path in ([n, m, -n], [n, n, m, -n, -n], [n, m, m, -n, -m], [-m, n, m, m, -n]):
                    pos = [0, 0, 0, 0]
                    for st in path:
                        d = abs(st) - 1
                        if st < 0:
                            pos[d] -= 1
                        if d == mu and tuple(pos) != (0, 0, 0, 0):
                            offs.add((mu, tuple(pos)))
                        if st > 0:
                            pos[d] += 1
    assert len(offs) > 0
    for mu, off in offs:
        dc = sum((2 if d == mu else 1) * off[d] for d in range(4)) % 4
        assert dc != 0, (mu, off)


def test_plain_staples_even_subsets_commute(ora):
    """With plain staples (eps = 1) the subsets 0 and 2 do not touch each other, so
    the two annealing steps equal one simultaneous update of their union."""
    dims = SMALL
    U = _haar_field(dims, 111)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 112)
    a = U.copy()
    ora.anneal_pass(dims, a, n, 1, 0, rho=0.1, eps=1.0)
    ora.anneal_pass(dims, a, n, 1, 2, rho=0.1, eps=1.0)
    for s in range(fieldgen.volume(dims)):
        if ora.colour(dims, 1, s) in (0, 2):
            want, _ = ora.update_link(dims, U, n, 1, s, rho=0.1, eps=1.0)
            np.testing.assert_array_equal(a[1, s], want)


def _np_plain_stout(dims, U, mu, sites, rho):
    """Plain-staple stout updates (Eq. plaq_staples, Eq. generator, Eq. stout) of
    the links (mu, s) for s in sites, all from the field U, in numpy with
    scipy's matrix exponential (no oracle code)."""
    V = fieldgen.volume(dims)
    S = np.zeros((V, 3, 3), dtype=complex)
    up = fieldgen.neighbour(dims, mu, 1)
    for nu in range(4):
        if nu == mu:
            continue
        vp, vm = fieldgen.neighbour(dims, nu, 1), fieldgen.neighbour(dims, nu, -1)
        S += U[nu] @ U[mu][vp] @ _loops.dag(U[nu][up])
        S += _loops.dag(U[nu][vm]) @ U[mu][vm] @ U[nu][vm][up]
    om = S[sites] @ _loops.dag(U[mu][sites])
    A = 0.5 * (om - _loops.dag(om))
    Q = A - np.trace(A, axis1=1, axis2=2)[:, None, None] / 3 * np.eye(3)
    return scipy.linalg.expm(rho * Q) @ U[mu][sites]


def test_annealed_sweep_is_direction_then_parity(ora):
    """Sec. III.A and the direction/parity subset order: with plain staples an
    annealed sweep takes, for mu = 0..3, first every link whose coordinates
    off the mu axis sum to an even number, all from the current field, then the
    odd ones from the field that includes the even updates.  Built in numpy from
    the definitions; a different subset or direction order fails."""
    dims = SMALL
    U = _haar_field(dims, 141)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 142)
    V = fieldgen.volume(dims)
    coords = np.stack([np.arange(V) // int(np.prod(dims[:d])) % dims[d] for d in range(4)])
    want = U.copy()
    for mu in range(4):
        par = (coords.sum(axis=0) - coords[mu]) % 2
        for p in (0, 1):
            sites = np.nonzero(par == p)[0]
            want[mu][sites] = _np_plain_stout(dims, want, mu, sites, 0.2)
    got = U.copy()
    ora.smooth(dims, got, n, 1, order="annealed", rho=0.2, eps=1.0, measure_every=0)
    np.testing.assert_allclose(got, want, atol=1e-13)
    # the same sweep with the parities the other way round is a different map
    other = U.copy()
    for mu in range(4):
        par = (coords.sum(axis=0) - coords[mu]) % 2
        for p in (1, 0):
            sites = np.nonzero(par == p)[0]
            other[mu][sites] = _np_plain_stout(dims, other, mu, sites, 0.2)
    assert np.abs(other - want).max() > 1e-3


def test_annealed_flow_decreases_wilson_action(ora):
    """Sec. II.B / V.B: annealed stout with plain staples and a small step is an
    Euler step of the Wilson flow, which lowers the Wilson action monotonically."""
    dims = SMALL
    n, U = _centrifuged(ora, dims, p=0.2, seed=121, omega=0.05)
    G = fieldgen.haar_su3(fieldgen.volume(dims), 122)
    U = ora.gauge_transform(dims, U, G)
    st0 = ora.measure(dims, U, n)
    st = ora.smooth(dims, U, n, 6, order="annealed", rho=0.01, eps=1.0)
    acts = np.concatenate([[st0.action], st["action"]])
    assert np.all(np.diff(acts) < 0), acts


def test_flow_time_scaling(ora):
    """Sec. V.B: flow time tau = n rho; halving the step and doubling the sweeps
    reaches the same field up to O(rho)."""
    dims = SMALL
    n, U = _centrifuged(ora, dims, p=0.2, seed=131, omega=0.05)
    a, b, c = U.copy(), U.copy(), U.copy()
    sa = ora.smooth(dims, a, n, 4, order="annealed", rho=0.02, eps=1.0)[-1]
    sb = ora.smooth(dims, b, n, 8, order="annealed", rho=0.01, eps=1.0)[-1]
    sc = ora.smooth(dims, c, n, 16, order="annealed", rho=0.005, eps=1.0)[-1]
    s0 = ora.measure(dims, U, n)
    assert abs(sb.action - sc.action) < 0.6 * abs(sa.action - sc.action)
    assert abs(sa.action - sc.action) < 0.05 * abs(s0.action - sc.action)


def test_small_rho_first_order(ora):
    """Eq. (stout) to first order: U' = U + rho Q U + O(rho^2)."""
    dims = SMALL
    U = _haar_field(dims, 141)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 142)
    mu, s = 2, 99
    Q = ora.generator(ora.staple(dims, U, mu, s, eps=-0.25) @ U[mu, s].conj().T)
    for rho in (1e-3, 1e-4):
        got, _ = ora.update_link(dims, U, n, mu, s, rho=rho, eps=-0.25)
        np.testing.assert_allclose((got - U[mu, s]) / rho, Q @ U[mu, s], atol=5 * rho * 40)


# ---------------------------------------------------- vortex preservation


def test_vp_keeps_flux_and_rejects_consistently(ora):
    """Sec. VI: with the accept/reject step every link keeps its centre sector, so
    every plaquette keeps its vortex flux; without it, a rough field loses flux."""
    dims = (4, 4, 4, 8)
    n, U = _centrifuged(ora, dims, p=0.15, seed=151, omega=0.02)
    W = U.copy()
    st = ora.smooth(dims, W, n, 4, order="annealed", rho=0.3, eps=-0.25, vp=True)
    assert np.all(st["flux_mismatch"] == 0) and np.all(st["undefined_sector"] == 0)
    np.testing.assert_array_equal(ora.sectors(dims, W), n)
    X = U.copy()
    st2 = ora.smooth(dims, X, n, 4, order="annealed", rho=0.3, eps=-0.25, vp=False)
    assert st2["flux_mismatch"][-1] > 0
    assert st["rejected"].sum() > 0
    Y = U.copy()
    st3 = ora.smooth(dims, Y, n, 2, order="annealed", rho=1e-4, eps=-0.25, vp=True)
    assert np.all(st3["rejected"] == 0)


def test_vp_in_random_gauge(ora):
    """Sec. VI: in a random gauge the test undoes the transform first, so the whole
    vortex-preserved smoothing commutes with the gauge transform."""
    dims = SMALL
    n, U = _centrifuged(ora, dims, p=0.2, seed=161, omega=0.05)
    G = fieldgen.haar_su3(fieldgen.volume(dims), 162)
    A = U.copy()
    sa = ora.smooth(dims, A, n, 3, order="annealed", rho=0.4, eps=-0.25, vp=True)
    B = ora.gauge_transform(dims, U, G)
    sb = ora.smooth(dims, B, n, 3, order="annealed", rho=0.4, eps=-0.25, vp=True, gauge=G,
                    measure_every=0)
    assert sa["rejected"].sum() > 0
    np.testing.assert_allclose(B, ora.gauge_transform(dims, A, G), atol=1e-12)
    # the vortex content measured in the random gauge (centre projections of
    # G^dag(x) U G(x+mu)) is the MCG field's: no plaquette changed its flux
    ma, fa = ora.measure(dims, A, n, with_flux=True)
    mb, fb = ora.measure(dims, B, n, with_flux=True, gauge=G)
    np.testing.assert_array_equal(fa, fb)
    assert ma.flux_mismatch == 0 and mb.flux_mismatch == 0
    assert abs(ma.plaq - mb.plaq) < 1e-13
    sc = ora.smooth(dims, B.copy(), n, 2, order="annealed", rho=0.4, eps=-0.25, vp=True, gauge=G)
    assert np.all(sc["flux_mismatch"] == 0) and np.all(sc["undefined_sector"] == 0)


def test_measure_undoes_a_random_gauge(ora):
    """Sec. I, V.C: the vortex flux of a Z(3) field is the lattice curl of its
    seed s; after a random gauge transform the links are no longer centre
    elements, and the flux is recovered only by projecting G^dag(x) U G(x+mu)."""
    dims = SMALL
    n, g, sd = fieldgen.z3_vortex_charges(dims, 0.2, 165, return_parts=True)
    U = ora.z3_field(dims, n)
    G = fieldgen.haar_su3(fieldgen.volume(dims), 166)
    W = ora.gauge_transform(dims, U, G)
    st0, f0 = ora.measure(dims, U, n, with_flux=True)
    st1, f1 = ora.measure(dims, W, n, with_flux=True, gauge=G)
    np.testing.assert_array_equal(f0, f1)
    assert st1.flux_mismatch == 0 and st1.undefined_sector == 0
    assert abs(st1.plaq - st0.plaq) < 1e-14
    st2 = ora.measure(dims, W, n)  # sectors of the transformed links themselves
    assert st2.flux_mismatch > 0


# ------------------------------------------------------------- MaxReTr


def test_maxretr_converges_to_polar_factor(ora):
    """Eq. (maxReTr): the maximiser of Re Tr[W V^dagger] over SU(3) for V = P W0
    (P Hermitian positive, W0 in SU(3)) is W0, the unitary polar factor."""
    rng = np.random.default_rng(171)
    for k in range(3):
        W0 = fieldgen.haar_su3(1, 172 + k)[0]
        A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        P = A @ A.conj().T + 0.5 * np.eye(3)
        V = P @ W0
        Wp, _ = scipy.linalg.polar(V, side="left")
        np.testing.assert_allclose(Wp, W0, atol=1e-12)
        start = fieldgen.haar_su3(1, 180 + k)[0]
        out = ora.maxretr(start, V, loops=400)
        np.testing.assert_allclose(out, W0, atol=1e-9)


def test_maxretr_centre_closed_form(ora):
    """Sec. III: on a centre field L^1 = r e^{i phi} 1 and T^c_1 = sgn(r cos phi):
    for r cos phi > 0 the link is unchanged; for r cos phi < 0 it moves and
    Re Tr[U V^dagger] increases."""
    for n in (-1, 0, 1):
        Z = np.exp(2j * np.pi * n / 3) * np.eye(3)
        for r, th in ((2.0, 0.3), (0.7, -1.0), (3.0, 2.0), (1.5, -2.6)):
            V = r * np.exp(1j * th) * np.eye(3)
            phi = 2 * np.pi * n / 3 - th
            out = ora.maxretr(Z, V, loops=3)
            if r * np.cos(phi) > 0:
                np.testing.assert_array_equal(out, Z)
            else:
                assert np.abs(out - Z).max() > 0.1
                assert np.trace(out @ V.conj().T).real > np.trace(Z @ V.conj().T).real
                np.testing.assert_allclose(out @ out.conj().T, np.eye(3), atol=1e-14)


def test_maxretr_centre_one_loop_fixture(ora):
    """Sec. III, Eqs. (def_L1), (def_T1) and the T_2, T_3 matrices: one loop over
    the subgroups (1,2), (2,3), (1,3) on a centre link with r cos(phi) < 0 and
    sin(phi) != 0, against the hand derivation in maxretr_centre_one_loop.txt
    (the subgroup order decides the result)."""
    rows = _rows("maxretr_centre_one_loop.txt")
    assert len(rows) == 4
    for n, r, th, p0, p1, p2 in rows:
        n, r, th = int(n), float(r), float(th) * np.pi
        U = np.exp(2j * np.pi * n / 3) * np.eye(3)
        V = r * np.exp(1j * th) * np.eye(3)
        want = np.diag(np.exp(1j * np.pi * np.array([float(p0), float(p1), float(p2)])))
        np.testing.assert_allclose(ora.maxretr(U, V, loops=1), want, atol=1e-14)


@pytest.mark.parametrize("block", [(0, 1), (1, 2), (0, 2)])
def test_maxretr_single_subgroup_hit(ora, block):
    """Sec. III: if L^1 = U V^dagger is r times an SU(2) matrix W embedded in the
    rows/columns of one subgroup (W's diagonal real, 1 on the remaining
    diagonal entry), every other hit sees an identity-proportional block and
    leaves U alone, while that subgroup's hit gives T = r W, k = r and
    U <- W^dagger U, after which L = r 1.  So one loop, and three, return
    W^dagger U exactly; an index or conjugation slip in any subgroup's T fails."""
    p, q = block
    U = fieldgen.haar_su3(1, 231 + p + 3 * q)[0]
    a, b = 0.6, 0.48 + 0.64j  # a^2 + |b|^2 = 1
    E = np.eye(3, dtype=complex)
    E[p, p], E[p, q], E[q, p], E[q, q] = a, b, -np.conj(b), a
    r = 1.7
    V = (r * E).conj().T @ U  # L = U V^dagger = r E
    want = E.conj().T @ U
    for loops in (1, 3):
        np.testing.assert_allclose(ora.maxretr(U, V, loops=loops), want, atol=1e-14)


def test_alpha_min_threshold(ora):
    """Sec. III / Appendix B: for Z = 1 the real part of L^1 is smallest when the six
    plaquette staples are non-trivial (S = -3) and the 18 rectangles trivial
    (R = 18); the MaxReTr update then moves the link exactly when alpha exceeds
    alpha_min(eps, u0), printed as 0.4486 for eps = -0.25, u0 = 1."""
    (eps, u0, amin_printed, tol), = [[float(v) for v in r] for r in _rows("alpha_min.txt")]
    cp = (5 - 2 * eps) / 3
    cr = (eps - 1) / (12 * u0 * u0)
    Sigma = (cp * (3 * np.exp(2j * np.pi / 3) + 3 * np.exp(-2j * np.pi / 3)) + cr * 18) * np.eye(3)
    lo, hi = 0.0, 1.0
    for _ in range(60):
        a = 0.5 * (lo + hi)
        V = (1 - a) * np.eye(3) + a / 6 * Sigma
        out = ora.maxretr(np.eye(3, dtype=complex), V, loops=1)
        if np.array_equal(out, np.eye(3)):
            lo = a
        else:
            hi = a
    assert abs(hi - amin_printed) < tol
    closed = -6.0 / (2 * eps - 11 + 1.5 * (eps - 1) / u0 ** 2)
    assert abs(hi - closed) < 1e-9


def test_cooling_pathology_is_skipped(ora):
    """Sec. III.A: Sigma = 2 + 4 e^{+-2 pi i/3} (cooling, alpha = 1) makes the SU(2)
    hit undefined; the oracle's reading skips it, so no NaN appears."""
    for n1, n2, sg, absim, tol in _rows("cooling_pathology.txt"):
        s = int(n1) + int(n2) * np.exp(int(sg) * 2j * np.pi / 3)
        assert abs(abs(s.imag) - float(absim)) < float(tol) and abs(s.real) < 1e-15
        V = s / 6 * np.eye(3)
        out = ora.maxretr(np.eye(3, dtype=complex), V, loops=3)
        assert np.all(np.isfinite(out))
        np.testing.assert_array_equal(out, np.eye(3))


def test_cooling_field_sweep_stays_unitary(ora):
    """Sec. III.A: cooling (alpha = 1) on a rough random-gauge field produces SU(3)
    links and lowers the Wilson action."""
    dims = SMALL
    n, U = _centrifuged(ora, dims, p=0.2, seed=191, omega=0.05)
    U = ora.gauge_transform(dims, U, fieldgen.haar_su3(fieldgen.volume(dims), 192))
    st0 = ora.measure(dims, U, n)
    st = ora.smooth(dims, U, n, 3, order="annealed", update="cooling", alpha=1.0, eps=1.0)
    assert st["max_unitarity"].max() < 1e-13
    assert st["action"][-1] < st0.action


# ------------------------------------------------------------- measurement


@pytest.mark.parametrize("dims", [SMALL, TINY])
def test_measure_normalisation_random_field(ora, dims):
    """Sec. V.A: S(x) with n_c = 3, n_d = 4; the mean over the lattice equals
    (1/2)(1 - <P>) because Re Tr[1 - P] = 3 - Re Tr P.  Checked against the
    independent numpy plaquettes, also by brute force on 2^4."""
    U = _haar_field(dims, 201)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 202)
    st = ora.measure(dims, U, n)
    V = fieldgen.volume(dims)
    tot = sum(np.trace(p, axis1=1, axis2=2).real.sum() for p in _loops.plaquettes(dims, U))
    assert abs(st.plaq - tot / (18 * V)) < 1e-14
    assert abs(st.action - 0.5 * (1 - st.plaq)) < 1e-14
    assert st.max_unitarity < 1e-14
    W = U.copy()
    W[2, 17 % V, 1, 1] = np.nan
    assert ora.measure(dims, W, n).nonfinite == 1


@pytest.mark.parametrize("order", ["jacobi", "annealed"])
def test_sweep_updates_every_link_once(ora, order):
    """A sweep applies Eq. (stout) once to every link: to first order in rho,
    U' - U = rho Q[U] U for every link, whatever the order of the updates (a link
    visited twice would move by 2 rho Q U, a skipped one not at all)."""
    dims = SMALL
    U = _haar_field(dims, 211)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 212)
    rho = 1e-6
    W = U.copy()
    ora.smooth(dims, W, n, 1, order=order, rho=rho, eps=-0.25, measure_every=0)
    for mu in range(4):
        for s in range(0, fieldgen.volume(dims), 7):
            Q = ora.generator(ora.staple(dims, U, mu, s, eps=-0.25) @ U[mu, s].conj().T)
            np.testing.assert_allclose((W[mu, s] - U[mu, s]) / rho, Q @ U[mu, s], atol=2e-3)


def test_batched_update_equals_the_pass(ora):
    """update_links on the field before a subset pass gives, link for link, what
    the pass stores (the links of one subset are independent, Sec. III.A)."""
    dims = SMALL
    U = _haar_field(dims, 311)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 312)
    V = fieldgen.volume(dims)
    mu, colour = 2, 1
    sites = np.array([s for s in range(V) if ora.colour(dims, mu, s) == colour][::3])
    out, acc = ora.update_links(dims, U, n, np.full(len(sites), mu), sites, rho=0.05, eps=-0.25, vp=True)
    W = U.copy()
    ora.anneal_pass(dims, W, n, mu, colour, rho=0.05, eps=-0.25, vp=True)
    np.testing.assert_array_equal(out, W[mu, sites])
    single, a1 = ora.update_link(dims, U, n, mu, int(sites[0]), rho=0.05, eps=-0.25, vp=True)
    np.testing.assert_array_equal(single, out[0])
    assert a1 == acc[0]
