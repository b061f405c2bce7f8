"""The oracle against its pins (CPU only)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


def test_invariants_rmat12():
    P.pin_invariants_rmat12()


def test_reservoir_sampler_matches_enumeration():
    """Algorithm 2 (sequential weighted reservoir sampling), implemented in
    the test, reaches the same one-step distribution as the enumeration the
    oracle is tested against (Appendix B's claim)."""
    import numpy as np
    from fractions import Fraction
    from scipy.stats import chisquare
    from helpers import reservoir_pick
    w = [3, 0, 5, 1, 7, 2]
    rng = np.random.default_rng(1)
    n = 200_000
    counts = np.bincount([reservoir_pick(w, rng) for _ in range(n)], minlength=len(w))
    assert counts[1] == 0
    nz = [i for i in range(len(w)) if w[i]]
    exp = [float(Fraction(w[i], sum(w))) * n for i in nz]
    assert chisquare(counts[nz], exp).pvalue > 1e-4
