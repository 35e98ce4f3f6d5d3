"""GPU parity of weak simulation (xf_sample_gates, gate-by-gate sampling,
Sec. II-A) against the oracle's sampler on the same gate list: the same
decision uniforms and the same candidate probabilities (Exact, and Raw
Estimate keyed by the candidates' batch positions) give the same samples."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_12416_amd as X
    X.lib()
    return X


CASES = [
    # seed, n, eta, CPhase gates, matchgates per layer, samples, mode, t
    (95, 6, 3, 2, 5, 200, "exact", 0),
    (96, 8, 4, 4, 7, 150, "exact", 0),
    (97, 8, 4, 3, 7, 120, "approx", 400),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[6]}_n{c[1]}_L{c[3]}" for c in CASES])
def test_samples_match_oracle(X, case):
    seed, n, eta, ncp, per, S, mode, t = case
    gates, inp, _ = W.random_gate_circuit(seed, n, eta, ncp, per, theta_scale=1.0)
    say(f"gate-by-gate sampling n={n} eta={eta}, {len(gates)} gates, {S} samples, {mode}")
    ref = oracle.sample_gates(n, gates, inp, S, mode, t=t, seed=seed)
    got = X.sample_gates(n, gates, inp, S, mode, t=t, seed=seed)
    same = np.all(got == ref, axis=1)
    say(f"  identical samples: {int(same.sum())} of {S}")
    assert same.all()
    w = [bin(int(a)).count("1") + bin(int(b)).count("1") for a, b in got]
    assert all(v == eta for v in w)
