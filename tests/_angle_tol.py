"""Tolerance of the crossing sweeps' angle term against the oracle.

The sweeps hold each line angle as an integer in units u = pi / 2^26 and
evaluate a crossing's deviation |ideal - a| exactly on those integers.
Against the oracle's double angles, a is off by at most u (the two angle
roundings, u/2 each) and pi/2 - ideal by at most u/2, so each deviation is
within 1.5 u.  A sum of n deviations divided by the ideal angle (the
deviation sum the library reports) is then within n * 1.5 u / ideal, and
E_ca = 1 - that sum / n within 1.5 u / ideal (5.7e-8 at 70 degrees); a
relative 1e-12 covers the double sums.  The oracle itself does not round.
"""
import math

import pytest

UNIT = math.pi / 2 ** 26


def eca_tol(ideal):
    return 1.5 * UNIT / ideal


def dev_tol(n, ideal):
    return n * 1.5 * UNIT / ideal


def approx_eca(want, ideal):
    return pytest.approx(want, rel=1e-12, abs=eca_tol(ideal) + 1e-15)


def approx_dev(want, n, ideal):
    return pytest.approx(want, rel=1e-12, abs=dev_tol(n, ideal) + 1e-12)
