"""Pins of the L2 error of Section 5.1 and of the vortex input (eq. VP_Solution)."""
import math

import numpy as np

import fr_inputs as fi
from oracle.problem import l2_error, make_euler, sample_state


def test_l2_error_of_constant_and_polynomial_difference():
    nodes = fi.perturbed_nodes(4, 3, -5, -5, 10, 10, 0.1, seed=1)
    op = make_euler(nodes, 3)
    x, y = op.geo.points()
    assert l2_error(op, np.full(x.shape, 2.5), np.zeros(x.shape)) == np.float64(2.5) or \
        abs(l2_error(op, np.full(x.shape, 2.5), np.zeros(x.shape)) - 2.5) < 1e-14
    # difference d = x: exact mean of x^2 over the box [-5,5]^2 is 25/3 (bilinear elements
    # tile the box exactly and the rule integrates x^2 |J| exactly at P = 3)
    e = l2_error(op, x, np.zeros(x.shape))
    assert abs(e - math.sqrt(25.0 / 3.0)) < 1e-12


def test_vortex_input_is_isentropic_and_translates():
    v = fi.Vortex()
    x, y = np.meshgrid(np.linspace(-5, 5, 41), np.linspace(-5, 5, 41))
    rho, u, w, p = v.primitive(x, y)
    assert np.allclose(p / rho ** 1.4, 1.0, rtol=1e-13)
    # velocity perturbation magnitude alpha/(2 pi) r exp(phi (1 - r^2)) at r = 1
    rho1, u1, w1, _ = v.primitive(np.array(1.0), np.array(0.0))
    assert abs(w1 - 1.0 - 5.0 / (2 * math.pi)) < 1e-14 and abs(u1 - 1.0) < 1e-14
    # translation by (u_inf, v_inf) t with periodic wrap
    a = v.conservative(x, y, 0.0)
    b = v.conservative(x + 3.0, y + 3.0, 3.0)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    c = v.conservative(x, y, 10.0)        # one period
    assert np.allclose(a, c, rtol=1e-12, atol=1e-12)
