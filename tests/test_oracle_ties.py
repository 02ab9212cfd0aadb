"""Pins of the oracle's near-tie outcomes (CPU).

An implementation that evaluates the Eq. 1 distance with rounding error can
take the other branch of a decision whose exact distance lies within that
error of the threshold.  The oracle enumerates the outcomes such near ties
admit; these tests pin the enumeration against what it must contain,
computed independently: the segmentation at a threshold moved by less than the
band flips exactly the near ties on one side, so it is one of the outcomes,
and so is the bisection whose every pass is evaluated at its midpoint moved by
the same amount.
"""
import numpy as np
import pytest

import oracle
from paper_2206_14503_amd import synth


def _random_stream(rng, n):
    """n touching unit elements (f, b, r, g, b, a) with a few transparent ones."""
    e = np.zeros((n, 6))
    e[:, 0] = np.arange(n)
    e[:, 1] = np.arange(n) + 1
    e[:, 2:5] = rng.uniform(0, 1, (n, 3))
    e[:, 5] = rng.uniform(0.02, 0.6, n) * (rng.uniform(size=n) > 0.1)
    return e


def _same(outcome, count, gamma, lst, N):
    c, g, l = outcome
    if c != count or (gamma is not None and g != gamma):
        return False
    k = min(count, N)
    return np.allclose(l[:k], lst[:k], rtol=0, atol=1e-6)   # alternatives are stored in fp32


def test_exact_tie_has_both_outcomes():
    """Two unit elements whose Eq. 1 distance is exactly 1/8: at gamma = 1/8
    the fp64 decision merges (gamma < d is false); with a band the close is an
    outcome too, and it equals the segmentation just below 1/8."""
    e = np.array([[0, 1, 0.5, 0, 0, 0.5], [1, 2, 0.25, 0, 0, 0.5]], float)
    outs, complete = oracle.seg_outcomes(e, oracle.FIXED, gamma=0.125, max_n=4, tie=1e-6)
    assert complete and len(outs) == 2
    assert outs[0][0] == 1 and outs[1][0] == 2
    below, c_below, _, _ = oracle.seg(e, oracle.FIXED, gamma=0.125 - 1e-9, cap=4)
    assert c_below == 2 and np.allclose(outs[1][2], below)
    outs0, _ = oracle.seg_outcomes(e, oracle.FIXED, gamma=0.125, max_n=4, tie=0.0)
    assert len(outs0) == 1 and outs0[0][0] == 1


@pytest.mark.parametrize("gaps", [False, True])
def test_fixed_outcomes_contain_moved_thresholds(gaps):
    """Seg(gamma +- delta) with delta below the band is an outcome of Seg(gamma)."""
    rng = np.random.default_rng(1)
    tie, N = 0.02, 64
    hits = 0
    for trial in range(300):
        e = _random_stream(rng, int(rng.integers(4, 24)))
        if gaps:
            e[:, 0] += np.cumsum(rng.uniform(0, 0.5, len(e)) * (rng.uniform(size=len(e)) < 0.3))
            e[:, 1] = e[:, 0] + 1
        g = float(rng.uniform(0.01, 0.4))
        outs, complete = oracle.seg_outcomes(e, oracle.FIXED, gamma=g, max_n=N, gaps=gaps, tie=tie)
        if not complete:
            continue
        hits += len(outs) > 1
        for delta in (0.4 * tie, -0.9 * tie):
            lst, c, _, _ = oracle.seg(e, oracle.FIXED, gamma=g + delta, cap=N, gaps=gaps)
            assert any(_same(o, c, None, lst, N) for o in outs), (trial, delta)
    assert hits > 50


def _moved_bisection(e, N, iters, delta, gaps):
    """The bisection of Sec. 2.4 with every pass evaluated at its midpoint plus delta."""
    lo, hi = 0.0, 2.0
    for _ in range(iters):
        m = 0.5 * (lo + hi)
        _, c, _, _ = oracle.seg(e, oracle.FIXED, gamma=m + delta, cap=0, gaps=gaps)
        if c <= N:
            hi = m
        else:
            lo = m
    lst, c, _, _ = oracle.seg(e, oracle.FIXED, gamma=hi + delta, cap=0, gaps=gaps, max_out=max(len(e), 1))
    return hi, c, lst


@pytest.mark.parametrize("gaps", [False, True])
def test_bisection_outcomes_contain_moved_bisections(gaps):
    rng = np.random.default_rng(2)
    tie, N, iters = 4e-3, 5, 10
    split = 0
    for trial in range(300):
        e = _random_stream(rng, int(rng.integers(6, 30)))
        outs, complete = oracle.seg_outcomes(e, oracle.BISECT, max_n=N, iters=iters, gaps=gaps, tie=tie)
        if not complete:
            continue
        lst0, c0, g0, _ = oracle.seg(e, oracle.BISECT, max_n=N, iters=iters, gaps=gaps, max_out=N)
        assert _same(outs[0], c0, g0, lst0, N)
        split += len({o[1] for o in outs}) > 1
        for delta in (0.5 * tie, -0.5 * tie):
            g, c, lst = _moved_bisection(e, N, iters, delta, gaps)
            assert any(_same(o, c, g, lst, N) for o in outs), (trial, delta)
    assert split > 5


def test_generation_outcomes_are_consistent():
    """Generation: without a band every list has one outcome and no
    alternatives, with it the fp64 outputs are unchanged; every alternative
    belongs to a list with several outcomes and differs from its fp64 one."""
    vol = synth.gaussian_volume(32, 6, 0)
    tf = synth.transfer_function()
    cam = synth.orbit_camera(10_000, 40, 30)
    bricks = synth.brick_grid((32, 32, 32), (1, 1, 2))
    a = oracle.generate(vol, bricks, cam, tf, 1 / 32, 1 / 32, oracle.BISECT, 0.0, 4, 10, tie=0.0)
    b = oracle.generate(vol, bricks, cam, tf, 1 / 32, 1 / 32, oracle.BISECT, 0.0, 4, 10, tie=2e-3)
    assert np.all(a["nout"] == 1) and len(a["alts"]["ray"]) == 0
    for k in ("color", "depth", "count", "gamma"):
        assert np.array_equal(a[k], b[k])
    no = b["nout"].ravel()
    assert (no >= 2).sum() > 10
    al = b["alts"]
    assert len(al["ray"]) == int(np.abs(no)[no != 1].sum() - (no != 1).sum())
    for i, ray in enumerate(al["ray"]):
        r, q = divmod(int(ray), cam.width * cam.height)
        assert no[ray] >= 2 or no[ray] < 0
        same = (al["count"][i] == b["count"][r, q] and al["gamma"][i] == b["gamma"][r, q]
                and np.array_equal(al["color"][i], b["color"][r, :, q]))
        assert not same


def test_composite_outcomes_are_consistent():
    k, n, P = 6, 5, 64
    col, dep, cnt = synth.dense_interleaved_lists(k, n, P, seed=5)
    c, d, m = col.numpy(), dep.numpy(), cnt.numpy()
    a = oracle.composite([c[r] for r in range(k)], [d[r] for r in range(k)], [m[r] for r in range(k)], 0.01,
                         oracle.BISECT, 0.0, 8, 10, tie=0.0)
    b = oracle.composite([c[r] for r in range(k)], [d[r] for r in range(k)], [m[r] for r in range(k)], 0.01,
                         oracle.BISECT, 0.0, 8, 10, tie=5e-3)
    assert np.all(a["nout"] == 1)
    for key in ("color", "depth", "count", "gamma"):
        assert np.array_equal(a[key], b[key])
    assert (b["nout"] >= 2).sum() > 0
