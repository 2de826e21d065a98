"""Pins of the oracle's 1D FR basis against closed forms (Section 3)."""
import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6])
def test_radau_endpoint_values(P):
    # g_R(1) = 1, g_R(-1) = 0 and g_R'(1) = (P+1)^2 / 2 (Radau polynomial of degree P+1)
    assert basis.radau_right(P, 1.0) == pytest.approx(1.0, abs=1e-15)
    assert basis.radau_right(P, -1.0) == pytest.approx(0.0, abs=1e-15)
    assert basis.radau_right_deriv(P, 1.0) == pytest.approx((P + 1) ** 2 / 2.0, rel=1e-14)
    # Right Radau: vanishes at the P+1 right-Radau points, i.e. is orthogonal to degree P-1
    x, w = np.polynomial.legendre.leggauss(P + 3)
    for k in range(P):
        assert abs(np.sum(w * basis.radau_right(P, x) * x ** k)) < 1e-14


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 6])
def test_gauss_rule_and_lagrange(P):
    x, w = basis.gauss_points(P)
    assert np.sum(w) == pytest.approx(2.0, abs=1e-14)
    # exact for degree 2P+1
    for k in range(2 * P + 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.sum(w * x ** k) == pytest.approx(exact, abs=1e-14)
    L = basis.lagrange(x, x)
    assert np.allclose(L, np.eye(P + 1), atol=1e-14)


@pytest.mark.parametrize("P", [1, 2, 3, 4, 6])
def test_diff_matrix_exact_on_polynomials(P):
    x, _ = basis.gauss_points(P)
    D = basis.diff_matrix(x)
    for k in range(P + 1):
        assert np.allclose(D @ x ** k, k * x ** max(k - 1, 0) * (k > 0), atol=1e-12)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-13)


@pytest.mark.parametrize("P", [1, 2, 3, 4, 5])
def test_radau_correction_recovers_nodal_dg(P):
    # FR with g_DG on Gauss points equals collocated nodal DG: the lifting of a unit
    # jump at the right face is M^{-1} e_R, i.e. g_R'(x_a) = ell_a(1) / w_a, and
    # g_L'(x_a) = -ell_a(-1) / w_a at the left face.
    b = basis.Basis(P)
    assert np.allclose(b.gRp, b.lp / b.w, rtol=1e-12, atol=1e-12)
    assert np.allclose(b.gLp, -b.lm / b.w, rtol=1e-12, atol=1e-12)
