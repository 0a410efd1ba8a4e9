"""The library's AAA (host code behind wl_aaa / wl_exp_poles, the pole construction of
Alg. 1) against the oracle's and against what the mathematics fixes.  Host only: no GPU.

AAA's last greedy steps near its tolerance pick among points whose errors differ only
by rounding, and the poles of an approximant to an entire function move with any such
difference.  The two implementations are therefore compared pole by pole where every
greedy step is decisive (tolerance 1e-8: each step's error is far above rounding).
Even there the poles are only as well determined as the weight vector, the singular
vector of a smallest singular value some 1e-9 of the largest: agreement to 1e-5 of the
poles' scale (measured 4e-7 at worst).  At the default 1e-13 both must reach the
tolerance with a similar number of poles."""

import numpy as np
import pytest

from oracle import rational


@pytest.fixture(scope="module")
def wl():
    import paper_2601_11338_amd as wl
    wl.load()
    return wl


def match(a, b):
    """Largest distance from a pole of a to the nearest pole of b, and vice versa."""
    d1 = np.abs(a[:, None] - b[None, :]).min(axis=1).max()
    d2 = np.abs(b[:, None] - a[None, :]).min(axis=1).max()
    return max(d1, d2)


def test_rational_function_poles(wl):
    Z = np.linspace(0.0, 10.0, 2000)
    F = 1.0 / (Z + 1.0) + 2.0 / ((Z - 3.0) ** 2 + 1.0)
    poles, err = wl.aaa(Z, F)
    assert err < 1e-13 and poles.size == 3
    assert match(poles, np.array([-1.0, 3 + 1j, 3 - 1j])) < 1e-9


def test_constant_has_no_poles(wl):
    Z = np.linspace(0.0, 1.0, 50)
    poles, err = wl.aaa(Z, np.full(50, 2.5))
    assert err < 1e-14 and poles.size == 0


@pytest.mark.parametrize("xmax", [10.0, 100.0, 1000.0, 7000.0])
def test_exp_poles_match_oracle_in_decisive_regime(wl, xmax):
    got, err = wl.exp_poles(xmax, tol=1e-8)
    want = rational.exp_poles(xmax, tol=1e-8)
    assert err <= 1e-8
    assert got.size == want.size
    assert match(got, want) < 1e-5 * np.abs(want).max()


@pytest.mark.parametrize("xmax", [10.0, 300.0, 1000.0, 1e5])
def test_exp_poles_default_tolerance(wl, xmax):
    got, err = wl.exp_poles(xmax)
    want = rational.exp_poles(xmax)
    assert err <= 1e-13
    assert abs(got.size - want.size) <= 2
    on = (np.abs(got.imag) <= 1e-8 * xmax) & (got.real >= 0) & (got.real <= xmax)
    assert not on.any()
    assert match(got, got.conj()) < 1e-6 * np.abs(got).max()   # closed under conjugation


def test_bad_arguments(wl):
    with pytest.raises(wl.WLError):
        wl.aaa(np.zeros(1), np.zeros(1))
    with pytest.raises(wl.WLError):
        wl.exp_poles(-1.0)
    with pytest.raises(wl.WLError):
        wl.aaa(np.array([0.0, 1.0, np.nan]), np.ones(3))
