"""Host checks of the FP32-against-FP64 study's field analysis: on
populations w_i (1 + delta + 3 c_i.u0) (density 1 + delta, momentum
(1 + delta) u0 exactly, by the weight moments of D3Q19), in both storages and
with solid nodes masked out, the analysis returns rho - 1 = delta and
u = u0.  CPU tensors stand in for the library's device views."""
import numpy as np
import pytest
import torch

from paper_0711_2665_amd import lbmd
from paper_0711_2665_amd.precision_study import _err, fluid_fields


class _FakeSim:
    def __init__(self, pops, flags, precision):
        self._p, self._f, self.precision = pops, flags, precision

    def pops(self):
        return self._p

    def flags(self):
        return self._f


@pytest.mark.parametrize("precision", [lbmd.LB_FP64, lbmd.LB_FP32_DEV])
def test_fluid_fields_recover_density_and_velocity(precision):
    rng = np.random.default_rng(4)
    nz, ny, nx = 3, 4, 5
    n = nx * ny * nz
    delta = 1e-3 * rng.standard_normal(n)
    u0 = 0.01 * rng.standard_normal((n, 3))
    c = np.asarray(lbmd.VELOCITIES, dtype=np.float64)
    w = np.asarray(lbmd.WEIGHTS)
    rho = 1.0 + delta
    f = w[:, None] * (rho[None, :] + 3.0 * rho[None, :] * (c @ u0.T))       # [19, n]
    flags = np.zeros(n, dtype=np.uint8)
    flags[::7] = 1                                                          # solid nodes
    f[:, flags == 1] = 123.0 if precision == lbmd.LB_FP64 else 77.0         # must be ignored
    stored = f - w[:, None] if precision == lbmd.LB_FP32_DEV else f
    dt = torch.float32 if precision == lbmd.LB_FP32_DEV else torch.float64
    sim = _FakeSim(torch.tensor(stored, dtype=dt).view(19, nz, ny, nx), torch.tensor(flags).view(nz, ny, nx),
                   precision)
    vel = torch.tensor(lbmd.VELOCITIES, dtype=torch.float64)
    drho, u = fluid_fields(sim, vel)
    fluid = flags == 0
    tol = 1e-7 if precision == lbmd.LB_FP32_DEV else 1e-14
    assert drho.shape == (int(fluid.sum()),) and u.shape == (3, int(fluid.sum()))
    assert np.abs(drho.numpy() - delta[fluid]).max() < tol
    assert np.abs(u.numpy().T - u0[fluid]).max() < 10 * tol


def test_err_reports_max_and_rms():
    a = torch.tensor([0.0, 3.0, -4.0], dtype=torch.float64)
    b = torch.zeros(3, dtype=torch.float64)
    mx, rms = _err(a, b, 2.0)
    assert mx == 2.0 and abs(rms - np.sqrt(25.0 / 3.0) / 2.0) < 1e-15
