"""Host-side pieces of the trajectory-learning loop (Sec. IV-B): the
quadratic B-spline basis, the radial start, the soft hardware limits and
their conversion to radians per voxel.  No GPU needed."""
import math

import numpy as np
import torch

from paper_2111_02912_amd import learn


def test_bspline_basis_is_a_partition_of_unity_and_reproduces_quadratics():
    B = learn.quadratic_bspline_basis(1280, 40)
    assert B.shape == (1280, 40)
    assert torch.allclose(B.sum(1), torch.ones(1280, dtype=torch.float64), atol=1e-12)
    assert (B >= 0).all() and (B <= 0.75 + 1e-15).all()
    s = torch.arange(1280, dtype=torch.float64)
    for f in (s, s * s / 1280.0):
        c = torch.linalg.lstsq(B, f[:, None]).solution
        assert torch.allclose(B @ c, f[:, None], atol=1e-8 * f.abs().max())
    # each sample sees at most three kernels
    assert int((B > 0).sum(1).max()) <= 3


def test_radial_start_and_its_spline_fit():
    om = learn.radial_init(16, 1280)
    assert om.shape == (16, 1280, 2)
    assert torch.allclose(om[:, 640], torch.zeros(16, 2, dtype=torch.float64))
    assert float(om.abs().max()) <= math.pi + 1e-12
    B = learn.quadratic_bspline_basis(1280, 40)
    c = torch.linalg.lstsq(B[None].expand(16, -1, -1), om).solution
    # a straight spoke is a linear function of the sample index: fitted exactly
    assert torch.allclose(B @ c, om, atol=1e-9)


def test_hardware_limits_and_penalty():
    dt = 5e-3 / 1280
    l1, l2 = learn.hardware_limits(dt, 22.0, 320, 5.0, 15.0)
    dx = 22.0 / 320
    assert math.isclose(l1, 2 * math.pi * dx * 4257.6 * 5.0 * dt, rel_tol=1e-12)
    assert math.isclose(l2, 2 * math.pi * dx * 4257.6 * 15e3 * dt * dt, rel_tol=1e-12)
    # the radial start (2 pi / 1280 rad per sample, no curvature) is feasible
    om = learn.radial_init(16, 1280)
    assert float(learn.hardware_penalty(om, l1, l2)) == 0.0
    # soft limit: sum of the excess over the limit
    v = torch.tensor([0.5, -2.0, 1.0, 3.0], dtype=torch.float64)
    assert float(learn.soft_limit(v, 1.0)) == 3.0
    # penalty gradient against central differences (away from the kinks)
    g = torch.Generator().manual_seed(3)
    w = (torch.rand((2, 30, 2), generator=g, dtype=torch.float64) * 0.4).cumsum(1).requires_grad_(True)
    p = learn.hardware_penalty(w, 0.05, 0.02, 10.0, 7.0)
    p.backward()
    d = torch.randn(w.shape, generator=g, dtype=torch.float64)
    h = 1e-7
    with torch.no_grad():
        fd = (learn.hardware_penalty(w + h * d, 0.05, 0.02, 10.0, 7.0)
              - learn.hardware_penalty(w - h * d, 0.05, 0.02, 10.0, 7.0)) / (2 * h)
    assert abs(float(fd) - float((w.grad * d).sum())) <= 1e-6 * max(1.0, abs(float(fd)))
    # first and second differences as in the definition
    x = torch.tensor([[[0.0], [1.0], [3.0], [6.0]]], dtype=torch.float64)
    assert float(learn.hardware_penalty(x, 0.0, 0.0, 1.0, 0.0)) == 6.0   # |1| + |2| + |3|
    assert float(learn.hardware_penalty(x, 10.0, 0.0, 1.0, 1.0)) == 2.0  # |1| + |1|
