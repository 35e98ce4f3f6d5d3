"""CPU pins of the oracle's Estimate (Sec. III-A: repeated Raw Estimate
calls that tighten the probability bound): its rounding of trajectory
counts, its reduction to one Raw Estimate call, its schedule, and its error
guarantee against exact probabilities."""
import math

import numpy as np

import oracle
import workloads as W


def test_round_to_four_bits_is_the_smallest_such_count():
    allowed = sorted({m << e for m in range(1, 16) for e in range(0, 14)})
    for t in range(1, 5000):
        r = oracle.round_to_four_bits(t)
        assert r == next(a for a in allowed if a >= t), t
        assert r <= t * (1 + 1 / 8)


def test_loose_target_is_one_raw_estimate_call():
    """eps >= 1/2: one round at p_max = 1, every bitstring in one group, so
    the result is a plain Raw Estimate call with the rounded Eq. 6 count."""
    w = W.random_circuit(31, 7, 3, 4, n_rot=2, theta_scale=1.0)
    eps, delta = 0.6, 0.1
    p, tb, rounds = oracle.estimate(w.rot, w.pairs, w.layer, w.theta, w.input_bits, w.bits, eps, delta, seed=9)
    t = oracle.round_to_four_bits(oracle.trajectory_bound(eps, delta / 2, 1.0, oracle.extent(w.theta)))
    assert rounds == 1 and np.all(tb == t)
    ref = oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, w.bits, "approx", t=t, seed=9)
    np.testing.assert_array_equal(p, ref)


def test_schedule_and_tightened_counts():
    """The number of rounds is the first i with 2^-i <= eps; the last round's
    counts follow Eq. 6 at delta 2^-rounds and a bound below 1 for every
    bitstring, so they are below the count a single call at p_max = 1 needs."""
    w = W.random_circuit(32, 8, 4, 5, n_rot=2, theta_scale=0.8)
    eps, delta = 0.02, 0.05
    p, tb, rounds = oracle.estimate(w.rot, w.pairs, w.layer, w.theta, w.input_bits, w.bits, eps, delta, seed=1)
    assert rounds == math.ceil(math.log2(1 / eps))
    xi = oracle.extent(w.theta)
    one_shot = oracle.round_to_four_bits(oracle.trajectory_bound(eps, delta, 1.0, xi))
    assert np.all(tb < one_shot)
    # t_b is Eq. 6 at some p_max in [0, 1): the bound is increasing in p_max
    lo = oracle.round_to_four_bits(oracle.trajectory_bound(eps, delta * 2.0 ** -rounds, 0.0, xi))
    assert np.all(tb >= lo)


def test_error_within_eps_against_exact():
    """|p_hat - p| <= eps for every bitstring of a small circuit, over three
    seeds (the guarantee allows a failure rate delta per bitstring)."""
    w = W.random_circuit(33, 6, 3, 4, n_rot=3, theta_scale=1.2)
    exact = oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, w.bits, "exact")
    eps, delta = 0.03, 0.02
    fails = 0
    for seed in (1, 2, 3):
        p, tb, rounds = oracle.estimate(w.rot, w.pairs, w.layer, w.theta, w.input_bits, w.bits, eps, delta,
                                        seed=seed)
        fails += int(np.sum(np.abs(p - exact) > eps))
    assert fails <= 1, fails
