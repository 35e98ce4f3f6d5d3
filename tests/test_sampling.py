"""CPU pins of the oracle's weak simulation (gate-by-gate sampling, Sec.
II-A): with exact probabilities its samples follow the output distribution of
the brute-force qubit state vector; gates that cannot move a chain leave it
in place."""
import math

import numpy as np

import oracle
import workloads as W
from bruteforce import gate_list_amplitudes


def _ints(samples):
    return [int(a) | (int(b) << 64) for a, b in samples]


def test_gate_by_gate_samples_follow_the_output_distribution():
    n, eta = 5, 2
    gates, inp, bits = W.random_gate_circuit(91, n, eta, 2, 4, theta_scale=2.0)
    S = 6000
    xs = _ints(oracle.sample_gates(n, gates, inp, S, "exact", seed=11))
    psi = gate_list_amplitudes(n, gates, int(np.asarray(inp, dtype=np.uint64)[0]))
    probs = np.abs(psi) ** 2
    assert all(bin(v).count("1") == eta for v in xs)
    counts = np.bincount(xs, minlength=1 << n)
    # chi-square over the outcomes of weight eta with expected count >= 5
    outs = [v for v in range(1 << n) if bin(v).count("1") == eta and probs[v] * S >= 5]
    chi2 = sum((counts[v] - S * probs[v]) ** 2 / (S * probs[v]) for v in outs)
    dof = len(outs) - 1
    # well above the 0.999 quantile of chi-square with dof <= 9 degrees of freedom
    assert chi2 < dof + 6 * math.sqrt(2 * dof) + 10, (chi2, dof)
    # and the mass outside those outcomes matches
    rest = S - sum(counts[v] for v in outs)
    exp_rest = S * (1 - sum(probs[v] for v in outs))
    assert abs(rest - exp_rest) < 6 * math.sqrt(max(exp_rest, 1)) + 3


def test_chains_without_one_particle_on_the_pair_do_not_move():
    """A matchgate on a pair holding zero or two particles keeps every chain
    (particle-number conservation leaves one candidate)."""
    rng = np.random.default_rng(2)
    G = W.random_matchgate(rng)
    inp = W.bits_from_modes([0, 1])
    xs = oracle.sample_gates(4, [("mg", 0, G), ("mg", 2, G)], inp, 8, "exact", seed=3)
    assert all(int(a) == 0b0011 for a, _ in xs)
