"""GPU parity of Estimate (xf_estimate: repeated Raw Estimate calls that
tighten each bitstring's probability bound, Sec. III-A) against the oracle's
Estimate on the same inputs: the same rounds, the same trajectory counts and
the same estimates."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import make_plan, oracle_rot, rel_err, say

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
    # label, workload, bitstrings, eps, delta
    ("random n12 eta6 k8", lambda: W.random_circuit(41, 12, 6, 8, n_rot=2, theta_scale=0.6), 60, 0.01, 0.05),
    ("two layers n10 eta4 k6", lambda: W.random_circuit(42, 10, 4, 6, n_rot=3, theta_scale=0.9), 80, 0.02, 0.1),
    ("LUCJ n32 eta8a+8b", lambda: W.workload(2, B=48), 48, 0.005, 0.05),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_estimate_matches_oracle(X, case):
    label, make, count, eps, delta = case
    w = make()
    bits = w.bits[:count]
    say(f"Estimate {label}: {len(bits)} bitstrings, eps={eps} delta={delta}")
    ref, ref_t, ref_rounds = oracle.estimate(oracle_rot(w), w.pairs, w.layer, w.theta, w.input_bits, bits, eps,
                                             delta, seed=77)
    plan = make_plan(w, X)
    p, tb, rounds = plan.estimate(X.bits_tensor(bits, plan.device), eps, delta, seed=77)
    torch.cuda.synchronize()
    p = p.cpu().numpy()
    say(f"  rounds {rounds}, t in [{tb.min()}, {tb.max()}]")
    assert rounds == ref_rounds
    np.testing.assert_array_equal(tb, ref_t)
    e = rel_err(p, ref)
    say(f"  max rel err {e.max():.3e}")
    assert e.max() <= 1e-10


def test_estimate_rejects_bad_arguments(X):
    w = W.random_circuit(43, 6, 3, 2)
    plan = make_plan(w, X)
    b = X.bits_tensor(w.bits, plan.device)
    for eps, delta in ((0.0, 0.1), (1.0, 0.1), (0.1, 0.0), (0.1, 1.0)):
        with pytest.raises(X.XfError) as e:
            plan.estimate(b, eps, delta)
        assert e.value.status == 1
