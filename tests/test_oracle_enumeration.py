"""The beta -> 0 enumeration of Sec. III / VI (CPU, oracle only).

On a Z(3) field every staple path is a centre element, so for a link Z = 1 the
blocked matrix V = (1 - alpha) 1 + (alpha/6) Sigma^OI is v 1 with
v = (1 - alpha) + (alpha/6) (c_p S_p + c_r S_r), S_p the sum of the 6 plaquette
staple phases and S_r that of the 18 rectangle phases.  Each staple has a link
of its own, so with uniformly random centre links the staple phases are
independent and uniform: every class (counts of each phase among the 6 and
the 18 staples, 28 x 190 classes) carries a multinomial weight.  For each
class the oracle's MaxReTr update of Z = 1 gives
  * in:   |phi| > pi/2 for L^1 = r e^{i phi} = conj(v) (the condition for the
          update to move the link),
  * diff: the updated link differs from Z,
  * pass: its Z(3) projection still equals Z.
The paper finds p_pass = 0 for all alpha (every update that moves a vortex
link leaves its sector), p_in >= p_diff, and no combination with |phi| > pi/2
below alpha_min (0.4486 at eps = -0.25, u0 = 1; Fig. L1 shows none at
alpha = 0.4 and many at 0.7).
"""
from math import factorial

import numpy as np
import pytest

EPS, U0 = -0.25, 1.0
W = np.exp(2j * np.pi / 3)


def _classes(n):
    for a in range(n + 1):
        for b in range(n + 1 - a):
            c = n - a - b
            yield (a, b, c), factorial(n) // (factorial(a) * factorial(b) * factorial(c))


def _enumerate(ora, alpha, eps=EPS, u0=U0):
    cp = (5 - 2 * eps) / 3
    cr = (eps - 1) / (12 * u0 * u0)
    tot = p_in = p_diff = p_diff_pass = 0.0
    one = np.eye(3, dtype=complex)
    for (p0, p1, p2), wp in _classes(6):
        sp = p0 + p1 * W + p2 * W * W
        for (r0, r1, r2), wr in _classes(18):
            sr = r0 + r1 * W + r2 * W * W
            w = wp * wr / (3.0 ** 24)
            v = (1 - alpha) + alpha / 6 * (cp * sp + cr * sr)
            out = ora.maxretr(one, v * one, loops=3)
            moved = not np.array_equal(out, one)
            tot += w
            if v.real < 0:  # conj(v) = r e^{i phi} with cos(phi) < 0
                p_in += w
            if moved:
                p_diff += w
                if ora.sector(np.trace(out)) == 0:
                    p_diff_pass += w
    return tot, p_in, p_diff, (p_diff_pass / p_diff if p_diff > 0 else 0.0)


@pytest.mark.parametrize("alpha", [0.02, 0.2, 0.4, 0.44, 0.46, 0.5, 0.6, 0.7, 0.8, 0.9, 0.99])
def test_beta0_enumeration(ora, alpha):
    tot, p_in, p_diff, p_pass = _enumerate(ora, alpha)
    assert abs(tot - 1.0) < 1e-12  # the weights are a probability distribution
    assert p_in >= p_diff - 1e-15
    assert p_pass == 0.0  # a moved vortex link always leaves its sector
    amin = -6.0 / (2 * EPS - 11 + 1.5 * (EPS - 1) / U0 ** 2)
    if alpha < amin:
        assert p_in == 0.0 and p_diff == 0.0
    else:
        assert p_in > 0.0 and p_diff > 0.0


def test_beta0_enumeration_grows_with_alpha(ora):
    """More blocking weight on the staples moves more links (Fig. p_in)."""
    ps = [_enumerate(ora, a)[1] for a in (0.5, 0.6, 0.7, 0.8, 0.9)]
    assert all(x < y for x, y in zip(ps, ps[1:]))
