"""Host logic of the training-data generator: the closed-form labels of the
analytic families (a candidate is flagged iff a singular point lies strictly
inside its cells)."""
import numpy as np

from paper_2207_08500_amd import datagen


def test_step_at_interface_flags_the_straddling_candidates():
    N = 100
    dx = 2.0 / N
    i = 40
    x0 = -1.0 + (i + 1) * dx  # the interface x_{i+1/2}
    y = datagen.geometric_labels([i], [x0], N)[0]
    # S0 = {i-1,i,i+1}, S1 = {i,i+1,i+2}, S3 = {i..i+3} hold both sides; S2 = {i-2,i-1,i} does not
    assert y == 0b1011


def test_kink_inside_a_cell():
    N = 50
    dx = 2.0 / N
    i = 20
    xc = -1.0 + (i + 2 + 0.5) * dx  # centre of cell i+2
    y = datagen.geometric_labels([i], [xc], N)[0]
    # cell i+2 belongs to S1 and S3 only
    assert y == 0b1010


def test_far_singular_points_flag_nothing():
    assert datagen.geometric_labels([10, 11], [5.0, -7.0], 50).tolist() == [0, 0]


def test_family_singular_points_are_where_the_function_breaks():
    g = np.random.default_rng(3)
    for fam in (4, 5, 7, 8):
        for _ in range(5):
            f, sing = datagen._family(g, fam, 100)
            for x0 in sing:
                if abs(x0) > 0.95:
                    continue
                h = 1e-7
                # a jump or a change of slope at x0; smooth a little away from it
                left = (f(np.array([x0 - h])) - f(np.array([x0 - 2 * h]))) / h
                right = (f(np.array([x0 + 2 * h])) - f(np.array([x0 + h]))) / h
                jump = abs(f(np.array([x0 + h])) - f(np.array([x0 - h])))[0]
                assert jump > 1e-3 or abs(right - left)[0] > 1e-3 or fam == 5
