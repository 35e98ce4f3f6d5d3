"""GPU parity of circuits with more than two CPhase layers (general
interleaved circuits, ingested gate by gate from nearest-neighbour
matchgates and CPhase gates, Sec. II-B / Sec. III-B) against the FP64
oracle, which composes every trajectory's mode matrix layer by layer.  The
library evaluates them with the determinant lemma over (layer, mode)
positions, det M_N = det M_0 det(I + 2 TT[N, N] - 2 K[N, N]), and with the
direct composition of each submatrix under XF_EVAL_LU (also its fallback
for singular bases)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_probs, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_MIXED = 1e-5


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_12416_amd as X
    X.lib()
    return X


# Outputs that the matchgate layers cannot reach have probability zero in
# exact arithmetic and come out as rounding noise (around 1e-36) on both
# sides: relative errors are taken against max(p, FLOOR).
FLOOR = 1e-20


def _check(p, ref, tol, label):
    assert np.count_nonzero(ref) > 0
    e = np.abs(np.asarray(p) - ref) / np.maximum(ref, FLOOR)
    say(f"  {label}: n={len(p)} max rel err {e.max():.3e} median {np.median(e):.3e}")
    assert np.all(np.isfinite(p))
    assert e.max() <= tol, (label, int(np.argmax(e)), p[np.argmax(e)], ref[np.argmax(e)])


CASES = [
    # seed, n, eta, CPhase gates (= layers), matchgates per layer, bitstrings, mode
    (81, 8, 4, 4, 7, 70, "exact"),
    (82, 10, 5, 6, 9, 120, "approx"),
    (83, 12, 6, 8, 11, 64, "exact"),
    (84, 14, 7, 10, 13, 48, "approx"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[6]}_n{c[1]}_eta{c[2]}_L{c[3]}" for c in CASES])
def test_many_layers_match_oracle(X, case):
    seed, n, eta, ncp, per, count, mode = case
    gates, inp, bits = W.random_gate_circuit(seed, n, eta, ncp, per, theta_scale=1.0)
    bits = bits[:count]
    rot, pairs, layer, theta = X.circuit_from_gates(n, gates)
    say(f"{ncp} CPhase layers, n={n} eta={eta}, {mode}: {len(bits)} bitstrings")
    t, smp = (2000, 29) if mode == "approx" else (0, 0)
    ref = oracle.probabilities(rot, pairs, layer, theta, inp, bits, mode, t=t, seed=smp)
    for prec, tol in (("fp64", TOL_FP64), ("mixed", TOL_MIXED)):
        plan = X.Plan(rot, pairs, layer, theta, inp, prec)
        p = gpu_probs(plan, X, bits, mode, t, smp)
        assert plan.last_work()["general"]
        _check(p, ref, tol, f"{prec} lemma")
        plan.set_evaluation("lu")
        q = gpu_probs(plan, X, bits, mode, t, smp)
        _check(q, ref, tol, f"{prec} composition")
        plan.close()


def test_random_benchmark_shape_exact(X):
    """The shape of the paper's random extended-matchgate benchmark: 16
    CPhase gates (2^16 trajectories), matchgates proportional to the size;
    exact probabilities of a few outcomes."""
    n, eta = 20, 10
    gates, inp, far = W.random_gate_circuit(85, n, eta, 16, n - 1, theta_scale=1.0, max_bits=4)
    # outcomes near the input (where the weight is) and, from the uniform
    # draw, far ones whose probability vanishes (every base singular: the
    # composition kernel, split over segments)
    bits = np.concatenate([W.nearby_outcomes(7, n, range(eta), 6, hops=4), far[:2]])
    rot, pairs, layer, theta = X.circuit_from_gates(n, gates)
    say(f"random benchmark shape: n={n} eta={eta} 16 CPhase layers, {len(bits)} outcomes, exact")
    ref = oracle.probabilities(rot, pairs, layer, theta, inp, bits, "exact")
    plan = X.Plan(rot, pairs, layer, theta, inp)
    p = gpu_probs(plan, X, bits, "exact")
    wk = plan.last_work()
    say(f"  {wk['determinants']} determinants, eval {wk['eval_ms']:.2f} ms")
    _check(p, ref, TOL_FP64, "fp64")


def test_singular_base_falls_back_to_composition(X):
    """Last rotation's row 0 orthogonal to the columns of the rest at the
    empty trajectory: M_0 is singular for every bitstring with mode 0
    occupied, which the composition kernel evaluates."""
    rng = W.rng_for(909)
    n, eta, L = 9, 4, 4
    Rs = [W.haar_unitary(rng, n) for _ in range(L)]
    pairs = W.random_pairs(rng, n, L)
    layer = np.arange(L, dtype=np.int32)
    theta = rng.uniform(-1.0, 1.0, L)
    C = list(range(1, eta + 1))
    Y = Rs[0][:, C]
    for l in range(L):
        d = np.ones(n, dtype=np.complex128)
        a, b = pairs[l]
        d[a] *= np.exp(0.5j * theta[l])
        d[b] *= np.exp(0.5j * theta[l])
        Y = d[:, None] * Y
        if l + 1 < L:
            Y = Rs[l + 1] @ Y
    _, _, vh = np.linalg.svd(Y.T)
    v = vh[eta:].conj().T[:, 0]
    Z = np.concatenate([v.conj()[:, None], rng.standard_normal((n, n - 1)) + 1j * rng.standard_normal((n, n - 1))],
                       axis=1)
    last = np.linalg.qr(Z)[0].conj().T
    rot = np.stack(Rs + [last])
    inp = W.bits_from_modes(C)
    bits = W.all_fixed_weight(n, eta)
    for mode, t, smp in (("exact", 0, 0), ("approx", 1500, 5)):
        say(f"singular bases, {L} layers, {mode}")
        ref = oracle.probabilities(rot, pairs, layer, theta, inp, bits, mode, t=t, seed=smp)
        plan = X.Plan(rot, pairs, layer, theta, inp)
        p = gpu_probs(plan, X, bits, mode, t, smp)
        _check(p, ref, TOL_FP64, f"{mode}")
