"""GPU parity of the field-strength measurements (vsm_measure_clover,
vsm_correlate) against the oracle: a constant abelian field with closed forms,
random SU(3) fields, a smoothed vortex field in both precisions, and the
density correlations of Sec. VII.  FP64 arithmetic on both sides: densities
within 1e-13, lattice sums within 1e-12 relative."""
import numpy as np
import pytest
import torch

import fieldgen
import oracle as ora
from paper_2203_09764_amd import api
from tests.test_oracle_clover import _abelian_field

pytestmark = pytest.mark.gpu


def _gpu(dims, U, precision="fp64"):
    f = api.Field(dims, precision, device=torch.device("cuda:0"))
    api.set_links(f, torch.from_numpy(U))
    return f


def _check(f, dims, tol_d=1e-13):
    out, sd, qd = api.measure_clover(f, densities=True)
    out = out.cpu().numpy()
    U = api.get_links(f).cpu().numpy()  # the links exactly as the GPU holds them
    sr, q, s, sd_o, qd_o = ora.clover(dims, U, densities=True)
    np.testing.assert_allclose(sd.cpu().numpy(), sd_o, rtol=0, atol=tol_d)
    np.testing.assert_allclose(qd.cpu().numpy(), qd_o, rtol=0, atol=tol_d)
    assert abs(out[0] - sr) <= 1e-12 * abs(sr) + 1e-15
    assert abs(out[2] - s) <= 1e-12 * abs(s) + 1e-15
    assert abs(out[1] - q) <= 1e-12 * np.abs(qd_o).sum() + 1e-13
    return out, sd, qd


@pytest.mark.parametrize("n1,n3", [(1, 1), (1, -2)])
def test_constant_abelian_field(n1, n3):
    dims = (4, 8, 4, 12)
    U, B, Bp = _abelian_field(dims, n1, n3)
    out, sd, qd = _check(_gpu(dims, U), dims)
    assert abs(out[1] - fieldgen.volume(dims) * np.sin(B) * np.sin(Bp) / (2 * np.pi ** 2)) < 1e-11


@pytest.mark.parametrize("dims", [(8, 8, 4, 8), (4, 12, 8, 16)])
def test_random_field(dims):
    V = fieldgen.volume(dims)
    U = fieldgen.haar_su3(4 * V, 81).reshape(4, V, 3, 3).copy()
    _check(_gpu(dims, U), dims)


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_smoothed_vortex_field_and_smoothness(precision):
    """On a preconditioned vortex field smoothing brings <S_R> towards <S>
    (the smoothness condition of Sec. V.A)."""
    dims = (16, 16, 16, 32)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 1001)
    f = api.Field(dims, precision, device=torch.device("cuda:0"), jacobi_workspace=False)
    f.set_charges(n)
    api.precondition(f, fieldgen.centrifuge_pairs(dims, 2001), 0.02)
    out0, _, _ = _check(f, dims)
    api.smooth(f, 40, 0.06, -0.25, order="annealed", vp=True)
    out1, _, _ = _check(f, dims)
    r0, r1 = out0[0] / out0[2], out1[0] / out1[2]
    assert abs(1 - r1) < abs(1 - r0)


def test_density_correlations():
    dims = (8, 8, 8, 16)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 5)
    f = api.Field(dims, "fp64", device=torch.device("cuda:0"), jacobi_workspace=False)
    f.set_charges(n)
    api.precondition(f, fieldgen.centrifuge_pairs(dims, 6), 0.02)
    _, s0, q0 = api.measure_clover(f, densities=True)
    api.smooth(f, 10, 0.06, -0.25, order="annealed", vp=True)
    _, s1, q1 = api.measure_clover(f, densities=True)
    for a, b in ((s0, s1), (q0, q1), (s0, s0)):
        got = api.correlate(a, b).cpu().numpy()
        want = ora.correlation(a.cpu().numpy(), b.cpu().numpy())
        assert abs(got[0] - want) < 1e-13
    assert abs(api.correlate(s0, s0).cpu().numpy()[0] - 1) < 1e-14
