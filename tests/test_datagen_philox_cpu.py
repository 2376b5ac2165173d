"""The counter-based sample generator's host twin (the input module's
reference for the device generator): Philox4x32-10 against the published
known-answer vectors, and the sample distribution and labels against their
definition."""
import numpy as np

from paper_2207_08500_amd import inputs


def test_philox_known_answers():
    # known-answer vectors of Philox4x32 with 10 rounds (Salmon et al., SC 2011)
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF),
              (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        got = inputs.philox4x32_10(np.array([ctr], np.uint32), key)[0]
        assert [int(v) for v in got] == list(want)


def test_ranges_are_independent():
    s, y, _ = inputs.classifier_samples_philox(11, 0, 300)
    s2, y2, _ = inputs.classifier_samples_philox(11, 120, 180)
    assert np.array_equal(s[120:], s2) and np.array_equal(y[120:], y2)
    s3, _, _ = inputs.classifier_samples_philox(12, 120, 180)
    assert not np.array_equal(s2, s3)


def test_distribution_and_labels():
    n = 1 << 16
    s, y, s64 = inputs.classifier_samples_philox(inputs.BASE_SEED, 0, n)
    assert np.all(np.isfinite(s64)) and np.array_equal(s, s64.astype(np.float32))
    # about half the samples carry a jump, and a jump anywhere in
    # (x_0, x_5) crosses at least one candidate
    jump = y != 0
    assert abs(jump.mean() - 0.5) < 5 * 0.5 / np.sqrt(n)
    # by the jump's cell interval (x_m, x_m+1), the spans (1,3), (2,4), (0,2),
    # (2,5) give exactly these label sets: m = 0 {S2}, 1 {S0, S2},
    # 2 {S0, S1, S3}, 3 {S1, S3}, 4 {S3}; all five occur
    allowed = {0b0100, 0b0101, 0b1011, 0b1010, 0b1000}
    assert set(np.unique(y[jump]).tolist()) == allowed
    # smooth samples: constants and linear data among them are exactly
    # representable; amplitudes stay within the stated ranges
    assert np.abs(s64).max() < 2e3


def test_jump_samples_match_their_recipe():
    """Rebuild the jump samples from the uniforms by the stated recipe in
    plain Python (one sample at a time) and compare."""
    import math
    n = 64
    seed = 2207085000
    _, y, s64 = inputs.classifier_samples_philox(seed, 0, n)
    for i in range(n):
        ctr = np.array([[i, 0, b, inputs.C5_STREAM] for b in range(5)], np.uint32)
        w = inputs.philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
        u = (w.astype(np.float64) + 0.5) / 2.0 ** 32
        N = 50 if u[0, 0] < 0.4 else (100 if u[0, 0] < 0.8 else 200)
        dx = 2.0 / N
        xs = [(-1.0 + 2.0 * u[0, 1]) + (j - 2) * dx for j in range(6)]
        if u[0, 2] < 0.5:
            assert y[i] == 0
            continue
        xd = xs[0] + u[3, 2] * (xs[5] - xs[0])
        a = (0.1 + 0.9 * u[3, 3]) * (-1.0 if u[4, 0] < 0.5 else 1.0)
        r = math.exp(inputs.LN_1EM3 + u[4, 1] * (inputs.LN_1E3 - inputs.LN_1EM3))
        want = [(a * r if x > xd else a) * ((x - xd) if u[0, 3] >= 0.5 else 1.0) for x in xs]
        np.testing.assert_allclose(s64[i], want, rtol=1e-15, atol=0)
        lab = 0
        for k, (lo, hi) in enumerate(inputs.CANDIDATE_SPAN):
            lab |= (1 << k) if xs[lo] < xd < xs[hi] else 0
        assert y[i] == lab
