"""The plaquette winding rounds circ / (2 pi) to an integer (Sec. VI); the vorticity kernels
multiply by the double 1 / (2 pi) instead of dividing.  The circulation is a sum of four
wrapped phase differences whose unwrapped sum is zero, so it lies within a few units in the
last place of a multiple of 2 pi and both forms round to the same integer.  Checked here on
phases as atan2 returns them, special values (0, -0, +-pi) included."""
import numpy as np

TWO_PI = 2.0 * np.pi


def _wrap(d):
    return np.where(d > np.pi, d - TWO_PI, np.where(d <= -np.pi, d + TWO_PI, d))


def _circ(s00, s10, s11, s01):
    return ((_wrap(s10 - s00) + _wrap(s11 - s10)) + _wrap(s01 - s11)) + _wrap(s00 - s01)


def test_divide_and_multiply_give_the_same_winding():
    rng = np.random.default_rng(1907)
    n = 1 << 20
    z = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
    s = np.arctan2(z.imag, z.real)
    # phases at and next to the branch cut, and signed zeros
    special = np.array([0.0, -0.0, np.pi, -np.pi, np.nextafter(np.pi, 0), -np.nextafter(np.pi, 0),
                        np.pi / 2, -np.pi / 2])
    idx = rng.integers(0, special.size, size=(4, n // 4))
    s[:, : n // 4] = special[idx]
    circ = _circ(*s)
    k_div = np.rint(circ / TWO_PI)
    k_mul = np.rint(circ * 0.15915494309189535)
    assert np.array_equal(k_div, k_mul)
    assert np.abs(circ / TWO_PI - k_div).max() < 1e-14
    assert set(np.unique(k_div)) <= {-1.0, 0.0, 1.0, 2.0}
    # every winding value is reached (2 only with all four differences exactly pi)
    assert {-1.0, 0.0, 1.0} <= set(np.unique(k_div))
