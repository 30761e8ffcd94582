"""Ensemble statistics (host side): kurtosis and the ageing overlap."""
import numpy as np
import pytest

from paper_0906_3611_amd import analysis


def test_kurtosis_reference_values():
    assert analysis.kurtosis([1, -1, 1, -1]) == pytest.approx(1.0)
    # two-point x in {0, a} with p(a) = p: <x^4>/<x^2>^2 = 1/p
    assert analysis.kurtosis([0, 0, 0, 2.0]) == pytest.approx(4.0)
    g = np.random.default_rng(0).standard_normal(400000)
    assert analysis.kurtosis(g) == pytest.approx(3.0, abs=0.03)
    with pytest.raises(ValueError):
        analysis.kurtosis([0.0, 0.0])


def test_overlap_definition():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((5, 8, 9))
    assert analysis.overlap(a, a) == pytest.approx(1.0)
    assert analysis.overlap(a, -a) == pytest.approx(-1.0)
    assert analysis.overlap(a, 0.5 * a) == pytest.approx(0.5)
    # ensemble brackets over numerator and denominator separately (Eq. (68))
    w = np.stack([np.ones((2, 2)), 2 * np.ones((2, 2))])
    t = np.stack([np.ones((2, 2)), np.zeros((2, 2))])
    assert analysis.overlap(w, t) == pytest.approx(4.0 / (4.0 + 16.0))
    with pytest.raises(ValueError):
        analysis.overlap(a, a[:4])


def test_order_parameter_and_response():
    rho = np.zeros((3, 2, 4, 5))
    rho[:, 0] = 1.5
    rho[:, 1] = 0.25
    assert np.all(analysis.order_parameter(rho) == 1.25)
    assert np.allclose(analysis.response([0.01, 0.02], 0.02), [0.5, 1.0])
