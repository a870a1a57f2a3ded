"""GPU parity of the Wilson flow (vsm_flow: Euler and third-order Runge-Kutta,
every link at once) against the oracle's flow; FP64 links within 1e-12, the
FP32-bulk form within a stated bound; the Euler step agrees with the
simultaneous stout sweep of vsm_smooth."""
import numpy as np
import pytest
import torch

import fieldgen
import oracle as ora
from paper_2203_09764_amd import api
from tests.test_oracle_flow import _smooth_random_field

pytestmark = pytest.mark.gpu


def _field(dims, U, precision="fp64"):
    f = api.Field(dims, precision, device=torch.device("cuda:0"))
    api.set_links(f, torch.from_numpy(U))
    return f


def _links(f):
    return api.get_links(f).cpu().numpy()


@pytest.mark.parametrize("integrator", ["euler", "rk3"])
@pytest.mark.parametrize("eps_oi", [1.0, -0.25])
def test_flow_matches_oracle(integrator, eps_oi):
    dims = (8, 4, 8, 4)
    U = _smooth_random_field(dims, 21)
    f = _field(dims, U)
    U = _links(f)  # the links exactly as the GPU stores them
    api.flow(f, 3, 0.04, eps_oi=eps_oi, integrator=integrator)
    ora.flow(dims, U, 3, 0.04, eps_oi=eps_oi, integrator=integrator)
    assert np.abs(_links(f) - U).max() < 1e-12


def test_flow_of_a_preconditioned_vortex_field():
    dims = (8, 8, 8, 16)
    n = fieldgen.z3_vortex_charges(dims, 0.1, 22)
    U = ora.centrifuge(dims, n, fieldgen.centrifuge_pairs(dims, 23), 0.02)
    f = _field(dims, U)
    U = _links(f)
    api.flow(f, 4, 0.02, integrator="rk3")
    ora.flow(dims, U, 4, 0.02, integrator="rk3")
    assert np.abs(_links(f) - U).max() < 1e-12


def test_euler_flow_equals_the_simultaneous_stout_sweep():
    dims = (8, 4, 8, 4)
    U = _smooth_random_field(dims, 24)
    a = _field(dims, U)
    b = _field(dims, U)
    api.flow(a, 2, 0.05, eps_oi=-0.25, integrator="euler")
    api.smooth(b, 2, 0.05, -0.25, order="jacobi")
    assert np.abs(_links(a) - _links(b)).max() < 1e-15


def test_fp32_bulk_flow_error_bound():
    dims = (8, 4, 8, 4)
    U = _smooth_random_field(dims, 25)
    f = _field(dims, U, "fp32_bulk")
    U = _links(f)
    api.flow(f, 3, 0.04, integrator="rk3")
    ora.flow(dims, U, 3, 0.04, integrator="rk3")
    assert np.abs(_links(f) - U).max() < 2e-6
