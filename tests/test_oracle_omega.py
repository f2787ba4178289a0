"""Oracle pins: the counter-based Gaussian sketch (Sec. 2, Def. of a Gaussian
quaternion matrix).

- Philox4x32-10 against the published known-answer vectors
  (tests/golden/philox4x32_10_kat.txt).
- The series-based log, sqrt and sin/cos against the C library within a few
  ulp on the uniforms the generator can produce.
- The generated planes: mean 0, variance 1, kurtosis 3, uncorrelated planes
  and entries, and each entry depends only on (seed, row, col).
"""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def kat_rows():
    rows = []
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if line:
            rows.append([int(t, 16) for t in line.split()])
    return rows


@pytest.mark.parametrize("row", kat_rows())
def test_philox_known_answers(oracle, row):
    out = oracle.philox4x32_10(row[0:4], row[4:6])
    assert [int(x) for x in out] == row[6:10]


def grid_uniforms(step=613):
    x = np.arange(0, 1 << 23, step, dtype=np.int64)
    return (2 * x + 1) / float(1 << 24)


def test_log_against_libm(oracle):
    for u in grid_uniforms():
        ref = math.log(u)
        assert abs(oracle.log_unit(u) - ref) <= 4 * np.spacing(abs(ref)), u


def test_sqrt_against_libm(oracle):
    for x in np.concatenate([np.linspace(1e-7, 40.0, 5001), [2.0 ** -48, 1.0, 4.0, 33.27]]):
        ref = math.sqrt(x)
        assert abs(oracle.sqrt_pos(x) - ref) <= 2 * np.spacing(ref), x


def test_sincos_against_libm(oracle):
    # reference in x87 extended precision, so that the rounding of the angle
    # 2 pi u does not dominate the comparison
    two_pi = 2 * np.longdouble("3.14159265358979323846264338327950288")
    for u in np.concatenate([grid_uniforms(), [0.0, 0.125, 0.25, 0.375, 0.5, 0.75, 1 - 2.0 ** -24]]):
        s, c = oracle.sincos_2pi(u)
        th = two_pi * np.longdouble(u)
        assert abs(s - float(np.sin(th))) <= 3e-16, u
        assert abs(c - float(np.cos(th))) <= 3e-16, u


def test_omega_moments_and_independence(oracle):
    Om = oracle.omega(12345, 4096, 64).astype(np.float64)   # 1M draws
    x = Om.reshape(4, -1)
    n = x.shape[1]
    se = 1.0 / math.sqrt(n)
    for p in range(4):
        assert abs(x[p].mean()) < 5 * se
        assert abs(x[p].var() - 1.0) < 5 * math.sqrt(2.0) * se
        kurt = np.mean(x[p] ** 4) / np.mean(x[p] ** 2) ** 2
        assert abs(kurt - 3.0) < 5 * math.sqrt(24.0) * se
    c = np.corrcoef(x)
    assert np.abs(c - np.eye(4)).max() < 5 * se
    # neighbouring entries (consecutive counters) are uncorrelated
    assert abs(np.corrcoef(Om[0, :, :-1].ravel(), Om[0, :, 1:].ravel())[0, 1]) < 5 * se


def test_omega_normal_cdf(oracle):
    """Kolmogorov-Smirnov distance of one plane to the standard normal."""
    from scipy.stats import kstest
    x = oracle.omega(7, 2000, 50)[2].ravel().astype(np.float64)
    assert kstest(x, "norm").pvalue > 1e-4


def test_omega_prefix_and_seed(oracle):
    a = oracle.omega(99, 300, 40)
    b = oracle.omega(99, 200, 15)
    np.testing.assert_array_equal(a[:, :200, :15], b)
    c = oracle.omega(100, 200, 15)
    assert np.abs(c - b).max() > 0.1
    # the high seed word is part of the key
    d = oracle.omega(99 + (1 << 32), 200, 15)
    assert np.abs(d - b).max() > 0.1


def test_omega_single_entry_by_hand(oracle):
    """Entry (i, j) recomputed from Philox + Box-Muller with libm: equal up to
    the last FP32 rounding."""
    seed, i, j = 0xDEADBEEF12345678, 17, 5
    Om = oracle.omega(seed, 20, 8)
    x = oracle.philox4x32_10([i, j, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
    u = [(2 * (int(t) >> 9) + 1) / 2.0 ** 24 for t in x]
    r0 = math.sqrt(-2 * math.log(u[0]))
    r1 = math.sqrt(-2 * math.log(u[2]))
    ref = [r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
           r1 * math.cos(2 * math.pi * u[3]), r1 * math.sin(2 * math.pi * u[3])]
    for p in range(4):
        assert abs(float(Om[p, i, j]) - ref[p]) <= np.spacing(np.float32(abs(ref[p]))) * 1.0 + 1e-15
