"""GPU parity of exact mode along the term list's prefix tree (every
pattern's det S a principal minor of one matrix per bitstring, anchors every
four positions as Schur complements of their parents) against the FP64
oracle, which builds each trajectory's mode matrix and factorises its
submatrix directly, and against the library's per-pattern evaluation of the
same bitstrings (XF_EVAL_PATTERNS).  Below 1024 bitstrings each
bitstring's walk is split into parts (runs of the depth-first order, each
after its first anchor's ancestors) whose exact partial sums are added
afterwards."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_probs, make_plan, oracle_probs, sample_indices, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_MIXED = 1e-5
# Outputs whose probability vanishes in exact arithmetic come out as rounding
# noise on every side: relative errors are taken against max(p, FLOOR).
FLOOR = 1e-20


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_12416_amd as X
    X.lib()
    return X


def _err(p, ref):
    return np.abs(np.asarray(p) - ref) / np.maximum(np.asarray(ref), FLOOR)


def _check(p, ref, tol, label):
    assert np.count_nonzero(ref) > 0, f"{label}: every reference probability is zero"
    e = _err(p, ref)
    say(f"  {label}: n={len(p)} max rel err {e.max():.3e} median {np.median(e):.3e}")
    assert np.all(np.isfinite(p))
    assert e.max() <= tol, (label, int(np.argmax(e)), p[np.argmax(e)], ref[np.argmax(e)])


def _tile(bits, B=1024):
    bits = np.asarray(bits)
    reps = -(-B // len(bits))
    return np.concatenate([bits] * reps)[:max(B, len(bits))]


def _tree_vs_patterns(X, plan, bits, ref_idx, ref, tol, label, expect_tree=0.9):
    p = gpu_probs(plan, X, bits, "exact")
    wk = plan.last_work()
    assert wk["general"]
    say(f"  {label}: {wk['tree_bitstrings']} of {len(bits)} bitstrings along the tree, eval {wk['eval_ms']:.2f} ms")
    assert wk["tree_bitstrings"] >= expect_tree * len(bits), wk
    _check(p[ref_idx], ref, tol, f"{label} tree vs oracle")
    plan.set_evaluation("patterns")
    q = gpu_probs(plan, X, bits, "exact")
    assert plan.last_work()["tree_bitstrings"] == 0
    _check(p, q, tol, f"{label} tree vs per-pattern")
    plan.set_evaluation("auto")
    p2 = gpu_probs(plan, X, bits, "exact")
    assert np.array_equal(p, p2), "the tree's sums are not bitwise reproducible"
    return p


CASES = [
    # seed, n, eta, k, spin, theta_scale
    (951, 14, 7, 10, False, 1.0),    # one block, 3432 outputs
    (952, 16, 8, 12, True, 0.8),     # two spin blocks
    (953, 40, 20, 14, False, 0.6),   # 16384 terms, up to 28 flipped positions
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[1]}_eta{c[2]}_k{c[3]}{'_spin' if c[4] else ''}" for c in CASES])
def test_tree_one_layer(X, case):
    seed, n, eta, k, spin, scale = case
    inp = None
    if spin:
        inp = list(range(eta // 2)) + list(range(n // 2, n // 2 + eta - eta // 2))
    w = W.random_circuit(seed, n, eta, k, n_rot=2, theta_scale=scale, spin=spin, input_modes=inp, max_bits=4096)
    if spin:
        bits = W.spin_bitstrings(np.random.default_rng(seed), n // 2, eta // 2, eta - eta // 2, 1024)
    else:
        bits = _tile(w.bits[:1024])
    idx = sample_indices(len(bits), 24 if n >= 40 else 64, seed=seed)
    say(f"prefix tree, one layer {case}: B={len(bits)}, oracle on {len(idx)}")
    ref = oracle_probs(w, bits[idx], mode="exact")
    for prec, tol in (("fp64", TOL_FP64), ("mixed", TOL_MIXED)):
        plan = make_plan(w, X, prec)
        _tree_vs_patterns(X, plan, bits, idx, ref, tol, prec)
        plan.close()


TWO_LAYER_CASES = [
    # seed, n, eta, k, spin
    (961, 12, 6, 10, False),   # one block, both layers' positions
    (962, 16, 8, 12, True),    # two spin blocks
]


@pytest.mark.parametrize("case", TWO_LAYER_CASES, ids=[f"n{c[1]}_eta{c[2]}_k{c[3]}{'_spin' if c[4] else ''}"
                                                        for c in TWO_LAYER_CASES])
def test_tree_two_layers(X, case):
    """Two CPhase layers: G = I + 2T - 2H with T = R'_1 from layer-0 to
    layer-1 positions (the two-layer form of the per-pattern evaluation)."""
    seed, n, eta, k, spin = case
    inp = None
    if spin:
        inp = list(range(eta // 2)) + list(range(n // 2, n // 2 + eta - eta // 2))
    w = W.random_circuit(seed, n, eta, k, n_rot=3, theta_scale=0.8, spin=spin, input_modes=inp, max_bits=4096)
    if spin:
        bits = W.spin_bitstrings(np.random.default_rng(seed), n // 2, eta // 2, eta - eta // 2, 1024)
    else:
        bits = _tile(w.bits[:1024])
    idx = sample_indices(len(bits), 48, seed=seed)
    say(f"prefix tree, two layers {case}: B={len(bits)}")
    ref = oracle_probs(w, bits[idx], mode="exact")
    for prec, tol in (("fp64", TOL_FP64), ("mixed", TOL_MIXED)):
        plan = make_plan(w, X, prec)
        _tree_vs_patterns(X, plan, bits, idx, ref, tol, f"{prec} two layers", expect_tree=0.5)
        plan.close()


def test_tree_many_layers(X):
    """Eight CPhase layers (keys are trajectories; positions are (layer,
    mode) pairs, at most 16): G = I + 2TT - 2K."""
    n, eta = 12, 6
    gates, inp, bits = W.random_gate_circuit(83, n, eta, 8, 11, theta_scale=1.0)
    rot, pairs, layer, theta = X.circuit_from_gates(n, gates)
    bits = _tile(bits[:256])
    idx = sample_indices(len(bits), 48, seed=83)
    say(f"prefix tree, 8 CPhase layers: n={n} eta={eta} B={len(bits)}")
    ref = oracle.probabilities(rot, pairs, layer, theta, inp, bits[idx], "exact")
    plan = X.Plan(rot, pairs, layer, theta, inp, "fp64")
    _tree_vs_patterns(X, plan, bits, idx, ref, TOL_FP64, "fp64 8 layers", expect_tree=0.25)
    plan.close()


def test_tree_config3(X):
    """The exact stress workload (n=52, eta=26, 12 gates sharing modes: 4096
    distinct patterns over 19 positions)."""
    w = W.workload(3)
    idx = sample_indices(w.B, 16, seed=34)
    say("prefix tree, config 3: n=52 eta=26 k=12 B=4096")
    ref = oracle.run_workload(w, index=idx)
    plan = make_plan(w, X)
    _tree_vs_patterns(X, plan, w.bits, idx, ref, TOL_FP64, "cfg3 fp64")
    plan.close()


@pytest.mark.parametrize("B", [300, 1000])
def test_tree_split_into_parts(X, B):
    """Batches under 1024 bitstrings: each walk split into parts, their
    partial sums added by a reduction; against the oracle and the
    per-pattern evaluation, bitwise repeatable."""
    w = W.workload(3)
    bits = w.bits[:B]
    idx = sample_indices(B, 12, seed=B)
    say(f"prefix tree split into parts: config 3, B={B}")
    ref = oracle.run_workload(w, index=idx)
    plan = make_plan(w, X)
    _tree_vs_patterns(X, plan, bits, idx, ref, TOL_FP64, f"cfg3 B={B}")
    plan.close()


@pytest.mark.parametrize("B", [1, 7, 100])
def test_tree_few_bitstrings(X, B):
    """A few bitstrings: each walk split into up to 16 parts (runs of the
    depth-first order after their first anchor's ancestors)."""
    w = W.workload(3)
    plan = make_plan(w, X)
    bits = w.bits[:B]
    p = gpu_probs(plan, X, bits, "exact")
    assert plan.last_work()["tree_bitstrings"] == B
    idx = sample_indices(B, 4, seed=B)
    _check(p[idx], oracle.run_workload(w, index=idx), TOL_FP64, f"cfg3 B={B} tree")
    plan.set_evaluation("patterns")
    q = gpu_probs(plan, X, bits, "exact")
    _check(p, q, TOL_FP64, f"cfg3 B={B} tree vs per-pattern")
    plan.close()


def test_tree_growth_limit_hands_bitstrings_to_the_pattern_pass(X):
    """With a growth limit below any bitstring's growth, every bitstring is
    left to the per-pattern pass: the results are bitwise those of the
    per-pattern evaluation; restoring the limit takes the tree again."""
    w = W.random_circuit(951, 14, 7, 10, n_rot=2, max_bits=4096)
    bits = _tile(w.bits[:1024])
    plan = make_plan(w, X)
    plan.set_evaluation("patterns")
    q = gpu_probs(plan, X, bits, "exact")
    plan.set_evaluation("auto")
    plan.set_tree_growth(1e-6)
    p = gpu_probs(plan, X, bits, "exact")
    assert plan.last_work()["tree_bitstrings"] == 0
    assert np.array_equal(p, q)
    plan.set_tree_growth(1e4)
    p2 = gpu_probs(plan, X, bits, "exact")
    assert plan.last_work()["tree_bitstrings"] == len(bits)
    _check(p2, q, TOL_FP64, "tree vs per-pattern after restoring the limit")
    with pytest.raises(X.XfError):
        plan.set_tree_growth(0.0)
    plan.close()


def test_tree_at_32_positions(X):
    """16 disjoint gates flip 32 positions (the largest tree: seven anchor
    levels, the largest LDS layout), 65536 terms: the tree against the
    oracle."""
    n, eta, k = 34, 6, 16
    rng = W.rng_for(956)
    u = W.haar_unitary(rng, n)
    v = W.haar_unitary(rng, n)
    pairs = np.array([(2 * j, 2 * j + 1) for j in range(k)], dtype=np.int32)
    theta = rng.uniform(-0.6, 0.6, k)
    modes = W.random_fixed_weight(rng, np.arange(n), eta, 1024)
    bits = np.array([W.bits_from_modes(s) for s in modes], dtype=np.uint64)
    w = W.Workload("disjoint gates n=34 eta=6 k=16", n, W.bits_from_modes(range(eta)), np.stack([u, v]), pairs,
                   np.zeros(k, np.int32), theta, bits, "exact")
    idx = sample_indices(len(bits), 4, seed=956)
    say("32 flipped positions: B=1024, 2^16 terms")
    ref = oracle_probs(w, bits[idx], mode="exact")
    plan = make_plan(w, X)
    p = gpu_probs(plan, X, bits, "exact")
    wk = plan.last_work()
    say(f"  {wk['tree_bitstrings']} of {len(bits)} along the tree, eval {wk['eval_ms']:.2f} ms")
    assert wk["tree_bitstrings"] >= 0.9 * len(bits), wk
    _check(p[idx], ref, TOL_FP64, "fp64 tree at 32 positions")
    p2 = gpu_probs(plan, X, bits, "exact")
    assert np.array_equal(p, p2)
    plan.close()


def test_tree_off_beyond_32_positions(X):
    """17 disjoint gates flip 34 positions: no tree; every bitstring takes the
    pattern pass or, past 32 positions in a pattern, the LU kernel."""
    n, eta, k = 36, 6, 17
    rng = W.rng_for(954)
    u = W.haar_unitary(rng, n)
    v = W.haar_unitary(rng, n)
    pairs = np.array([(2 * j, 2 * j + 1) for j in range(k)], dtype=np.int32)
    theta = rng.uniform(-0.6, 0.6, k)
    modes = W.random_fixed_weight(rng, np.arange(n), eta, 1024)
    bits = np.array([W.bits_from_modes(s) for s in modes], dtype=np.uint64)
    w = W.Workload("disjoint gates n=36 eta=6 k=17", n, W.bits_from_modes(range(eta)), np.stack([u, v]), pairs,
                   np.zeros(k, np.int32), theta, bits, "exact")
    idx = sample_indices(len(bits), 2, seed=954)
    say("34 flipped positions: B=1024, 2^17 terms")
    ref = oracle_probs(w, bits[idx], mode="exact")
    plan = make_plan(w, X)
    p = gpu_probs(plan, X, bits, "exact")
    wk = plan.last_work()
    assert wk["general"] and wk["tree_bitstrings"] == 0, wk
    _check(p[idx], ref, TOL_FP64, "fp64 per-pattern")
    plan.close()


def test_tree_leaves_shifted_bases_to_the_pattern_pass(X):
    """Row 0 of the second rotation orthogonal to the columns of D_0 R_0[:, C]
    (D_0 the empty trajectory's phases): outputs with mode 0 occupied have a
    singular empty-pattern base, take a shifted base and the per-pattern pass;
    the rest go along the tree."""
    rng = W.rng_for(955)
    n, eta, k = 14, 6, 9
    R0 = W.haar_unitary(rng, n)
    pairs = W.random_pairs(rng, n, k)
    theta = rng.uniform(-0.8, 0.8, k)
    C = list(range(1, eta + 1))
    d0 = np.ones(n, dtype=np.complex128)
    for (a, b), th in zip(pairs, theta):
        d0[a] *= np.exp(0.5j * th)
        d0[b] *= np.exp(0.5j * th)
    Q = d0[:, None] * R0[:, C]
    _, _, vh = np.linalg.svd(Q.T)
    v = vh[eta:].conj().T[:, 0]
    Z = np.concatenate([v.conj()[:, None], rng.standard_normal((n, n - 1)) + 1j * rng.standard_normal((n, n - 1))],
                       axis=1)
    R1 = np.linalg.qr(Z)[0].conj().T
    modes = W.random_fixed_weight(rng, np.arange(n), eta, 1024)
    bits = np.array([W.bits_from_modes(s) for s in modes], dtype=np.uint64)
    w = W.Workload("singular bases n=14 eta=6 k=9", n, W.bits_from_modes(C), np.stack([R0, R1]), pairs,
                   np.zeros(k, np.int32), theta, bits, "exact")
    zero_in = np.array([0 in list(s) for s in modes])
    assert 0.2 < zero_in.mean() < 0.8
    idx = np.concatenate([np.flatnonzero(zero_in)[:24], np.flatnonzero(~zero_in)[:24]])
    say("singular empty-pattern bases: B=1024")
    ref = oracle_probs(w, bits[idx], mode="exact")
    plan = make_plan(w, X)
    p = gpu_probs(plan, X, bits, "exact")
    wk = plan.last_work()
    say(f"  {wk['tree_bitstrings']} of {len(bits)} along the tree")
    assert wk["tree_bitstrings"] <= int((~zero_in).sum()), wk
    assert wk["tree_bitstrings"] >= 0.9 * int((~zero_in).sum()), wk
    _check(p[idx], ref, TOL_FP64, "fp64 tree + shifted bases")
    plan.close()
