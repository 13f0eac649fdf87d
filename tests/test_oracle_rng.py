"""Pins of the oracle's counter-based random streams (Philox4x32-10,
uniform conversion, Box-Muller) against published values and exact
distributional facts."""
import math
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert orc.philox_kat(ctr, key).tolist() == out


def test_philox_batch_matches_single(orc):
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, (50, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x1234_5678_9ABC_DEF0
    out = orc.philox(seed, ctr)
    for i in range(50):
        ref = orc.philox_kat(ctr[i], [seed & 0xFFFFFFFF, seed >> 32])
        assert out[i].tolist() == ref.tolist()


def test_philox_words_uniform(orc):
    # counter-mode output over consecutive counters: bytes uniform (chi^2)
    n = 1 << 16
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    w = orc.philox(7, ctr).ravel()
    hist = np.bincount((w >> 24).astype(np.int64), minlength=256)
    chi2 = ((hist - hist.mean()) ** 2 / hist.mean()).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    # a single flipped counter bit changes about half the output bits
    ctr2 = ctr.copy()
    ctr2[:, 2] ^= 1
    w2 = orc.philox(7, ctr2).ravel()
    flips = np.unpackbits((w ^ w2).view(np.uint8)).mean()
    assert abs(flips - 0.5) < 0.01


def test_uniform_exact_open_interval(orc):
    u = orc.uniform(np.array([0, 0x1FF, 0x200, 0xFFFFFFFF], dtype=np.uint32))
    assert u[0] == 2.0 ** -24
    assert u[1] == 2.0 ** -24                     # low 9 bits are dropped
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(0)
    w = rng.integers(0, 2**32, 2000, dtype=np.uint64).astype(np.uint32)
    uu = orc.uniform(w)
    assert np.all((uu > 0) & (uu < 1))
    assert np.all(uu.astype(np.float32).astype(np.float64) == uu)   # exact in binary32


def test_box_muller_closed_form(orc):
    # u1 = exp(-1/2) gives radius 1; u2 = 1/8 is an eighth of a turn
    z0, z1 = orc.box_muller(math.exp(-0.5), 0.125)
    assert z0 == pytest.approx(math.cos(math.pi / 4), abs=1e-15)
    assert z1 == pytest.approx(math.sin(math.pi / 4), abs=1e-15)
    z0, z1 = orc.box_muller(math.exp(-2.0), 0.5)     # radius 2, half a turn
    assert z0 == pytest.approx(-2.0, abs=1e-14)
    assert z1 == pytest.approx(0.0, abs=1e-14)


def test_mh_draws_are_standard_normal(orc):
    P = 5
    z = []
    u = []
    for v in range(200):
        for t in range(100):
            zz, uu = orc.mh_draws(11, v, 0, t, P)
            z.append(zz)
            u.append(uu)
    z = np.array(z)
    u = np.array(u)
    n = len(z)
    for p in range(P):
        assert abs(z[:, p].mean()) < 5 / math.sqrt(n)
        assert abs(z[:, p].var() - 1) < 5 * math.sqrt(2 / n)
        assert stats.kstest(z[:, p], "norm").pvalue > 1e-4
    # pairwise independence of the components (a cos/sin mix-up correlates them)
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(P))) < 5 / math.sqrt(n)
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    assert abs(np.corrcoef(u, z[:, 0])[0, 1]) < 5 / math.sqrt(n)


def test_mh_draws_depend_on_every_counter_field(orc):
    base = orc.mh_draws(3, 10, 1, 7, 2)
    for args in [(4, 10, 1, 7), (3, 11, 1, 7), (3, 10, 2, 7), (3, 10, 1, 8)]:
        other = orc.mh_draws(*args, 2)
        assert not np.allclose(base[0], other[0])
    again = orc.mh_draws(3, 10, 1, 7, 2)
    assert np.array_equal(base[0], again[0]) and base[1] == again[1]


def test_init_uniform_in_box(orc):
    lb = np.array([0.0, 1.0, -3.0])
    ub = np.array([3.0, 250.0, 3.0])
    th = np.array([orc.init_uniform(9, v, c, lb, ub) for v in range(500) for c in range(4)])
    assert np.all((th >= lb) & (th <= ub))
    for p in range(3):
        x = (th[:, p] - lb[p]) / (ub[p] - lb[p])
        assert stats.kstest(x, "uniform").pvalue > 1e-4
