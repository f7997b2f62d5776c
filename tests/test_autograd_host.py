"""Host-side parts of the autograd wrapper (no GPU): the SE(3) exponential
used to apply the pose tangent (Eq. tangent)."""
import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

from paper_2110_06635_amd.autograd import se3_exp


@pytest.mark.parametrize("seed", range(6))
def test_se3_exp_matches_matrix_exponential(seed):
    rng = np.random.default_rng(seed)
    xi = rng.normal(size=6) * (10.0 ** rng.uniform(-9, 0.3))
    rho, w = xi[:3], xi[3:]
    twist = np.zeros((4, 4))
    twist[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    twist[:3, 3] = rho
    T = expm(twist)
    R, t = se3_exp(xi)
    np.testing.assert_allclose(R, T[:3, :3], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(t, T[:3, 3], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(R, Rotation.from_rotvec(w).as_matrix(), rtol=1e-10, atol=1e-12)


def test_se3_exp_zero_and_translation():
    R, t = se3_exp(np.zeros(6))
    assert np.array_equal(R, np.eye(3)) and np.array_equal(t, np.zeros(3))
    R, t = se3_exp(np.array([1.0, -2.0, 0.5, 0, 0, 0]))
    np.testing.assert_allclose(t, [1.0, -2.0, 0.5])
