"""Host-side logic of the surrogate (CPU only): the monitor threshold rule."""
from paper_2112_03592_amd import surrogate as N


def test_calibrate_tau_rule():
    # largest monitor value below which every calibration case meets the target
    assert N.calibrate_tau([0.1, 0.2, 0.3], [0.01, 0.015, 0.03], 0.02) == 0.2
    # the smallest monitor already misses: always fall back
    assert N.calibrate_tau([0.1, 0.2], [0.03, 0.01], 0.02) == 0.0
    # ties: a failing case at a monitor value excludes that value
    assert N.calibrate_tau([0.2, 0.2, 0.1], [0.01, 0.03, 0.01], 0.02) == 0.1
    # every case meets the target: the largest monitor seen
    assert N.calibrate_tau([0.1, 0.3], [0.01, 0.01], 0.02) == 0.3
