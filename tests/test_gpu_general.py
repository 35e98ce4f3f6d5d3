"""GPU parity of the general determinant-lemma evaluation (exact mode, one or
two CPhase layers, bases of up to 32 rows, block-diagonal rotations split into
blocks) against the FP64 oracle, which always builds each trajectory's full
mode matrix and factorises its submatrix directly, and against the LU
evaluation of the same library."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import gpu_probs, make_plan, oracle_probs, rel_err, sample_indices, say

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


def _check(p, ref, tol, label):
    assert np.count_nonzero(ref) > 0, f"{label}: every reference probability is zero"
    e = rel_err(p, ref)
    say(f"  {label}: n={len(p)} max rel err {e.max():.3e} median {np.median(e):.3e}")
    assert np.all(np.isfinite(p))
    assert e.max() <= tol, (label, int(np.argmax(e)), p[np.argmax(e)], ref[np.argmax(e)])


CASES = [
    # seed, n, eta, k, n_rot, spin, theta_scale, mode
    (901, 8, 3, 5, 2, False, 1.0, "exact"),
    (902, 12, 6, 8, 2, True, 0.8, "exact"),      # two blocks
    (903, 10, 4, 6, 3, False, 1.0, "exact"),     # two CPhase layers
    (904, 16, 8, 10, 3, True, 0.7, "exact"),     # two layers, two blocks
    (905, 40, 24, 12, 2, False, 0.5, "exact"),   # eta = 24 in one block
    (906, 14, 6, 9, 3, True, 0.9, "approx"),     # two layers, two blocks
    (907, 44, 20, 16, 3, True, 0.6, "approx"),   # two layers, blocks of 10 rows
    (908, 48, 28, 10, 2, False, 0.6, "approx"),  # one layer, eta = 28
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[7]}_n{c[1]}_eta{c[2]}_k{c[3]}_L{c[4] - 1}" for c in CASES])
def test_general_lemma_matches_oracle_and_lu(X, case):
    seed, n, eta, k, n_rot, spin, scale, mode = case
    inp = None
    if spin:
        inp = list(range(eta // 2)) + list(range(n // 2, n // 2 + eta - eta // 2))
    w = W.random_circuit(seed, n, eta, k, n_rot=n_rot, theta_scale=scale, spin=spin, input_modes=inp,
                         max_bits=256)
    count = 256 if n < 40 else 32
    if spin:
        # outputs in the input's spin sector (others have p = 0)
        bits = W.spin_bitstrings(np.random.default_rng(seed), n // 2, eta // 2, eta - eta // 2, count)
    else:
        bits = w.bits[:count]
    t, smp = (1000, 41) if mode == "approx" else (0, 0)
    say(f"general lemma {case}: {len(bits)} bitstrings")
    ref = oracle_probs(w, bits, mode=mode, t=t, seed=smp)
    for prec, tol in (("fp64", TOL_FP64), ("mixed", TOL_MIXED)):
        plan = make_plan(w, X, prec)
        p = gpu_probs(plan, X, bits, mode, t, smp)
        wk = plan.last_work()
        assert wk["general"], "the general lemma kernel was expected"
        _check(p, ref, tol, f"{prec} general")
        plan.set_evaluation("lu")
        q = gpu_probs(plan, X, bits, mode, t, smp)
        assert not plan.last_work()["general"]
        _check(q, ref, tol, f"{prec} LU")


def test_config3_exact_general_vs_oracle(X):
    w = W.workload(3)
    say("config 3 (general lemma, exact): n=52 eta=26 k=12, all 4096 terms, B=4096")
    idx = sample_indices(w.B, 24, seed=33)
    ref = oracle.run_workload(w, index=idx)
    plan = make_plan(w, X)
    p = gpu_probs(plan, X, w.bits, "exact")
    wk = plan.last_work()
    assert wk["general"]
    _check(p[idx], ref, TOL_FP64, "cfg3 fp64")
    p2 = gpu_probs(plan, X, w.bits, "exact")
    assert np.array_equal(p, p2)


def _config5_golden():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config5_subset_oracle.json")
    with open(path) as f:
        return json.load(f)


def test_config5_general_vs_oracle(X):
    """The full batch in the launch configuration of the benchmark; 1000
    outputs spread over the batch against the stored FP64 oracle values
    (tests/golden/make_config5_subset.py), 8 more against the oracle live."""
    w = W.workload(5)
    gold = _config5_golden()
    assert gold["workload"] == w.name and gold["t"] == w.t and gold["seed"] == w.seed
    gidx = np.asarray(gold["index"], dtype=np.int64)
    gref = np.asarray(gold["prob"])
    gamp = np.asarray(gold["amp_re"]) + 1j * np.asarray(gold["amp_im"])
    say("config 5 (general lemma, two layers, two blocks): n=100 eta=25a+25b k=40 t=65536 B=1e5")
    idx = sample_indices(w.B, 8, seed=55)
    ref = oracle.run_workload(w, index=idx)
    for prec, tol in (("fp64", TOL_FP64), ("mixed", TOL_MIXED)):
        plan = make_plan(w, X, prec)
        bits = X.bits_tensor(w.bits, torch.device("cuda", 0))
        out = torch.empty(w.B, dtype=torch.float64, device=bits.device)
        amp = torch.empty((w.B, 2), dtype=torch.float64, device=bits.device)
        plan.probabilities(bits, "approx", w.t, w.seed, out=out, amp=amp)
        torch.cuda.synchronize()
        p = out.cpu().numpy()
        a = amp.cpu().numpy()
        a = a[:, 0] + 1j * a[:, 1]
        wk = plan.last_work()
        assert wk["general"] and wk["lemma"]
        say(f"  {prec}: {wk['fp32_bases']} of {2 * w.B} bases in FP32, {wk['determinants']} patterns")
        _check(p[idx], ref, tol, f"cfg5 {prec} live")
        _check(p[gidx], gref, tol, f"cfg5 {prec} stored")
        ea = np.abs(a[gidx] - gamp) / np.maximum(np.abs(gamp), 1e-300)
        say(f"  {prec} amplitudes: max rel err {ea.max():.3e}")
        assert ea.max() <= tol
        plan.close()


def test_exact_general_defers_ill_conditioned_bases(X):
    """Row 0 of the second rotation (nearly) orthogonal to the columns of
    D_0 R_0[:, C]: bases with mode 0 occupied are ill-conditioned, their
    bitstrings go to the LU kernel within the same exact-mode call."""
    say("exact mode, ill-conditioned bases")
    rng = W.rng_for(707)
    n, eta, k = 9, 4, 5
    R0 = W.haar_unitary(rng, n)
    pairs = W.random_pairs(rng, n, k)
    theta = rng.uniform(-1.0, 1.0, k)
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
    rot = np.stack([R0, R1])
    inp = W.bits_from_modes(C)
    bits = W.all_fixed_weight(n, eta)
    ref = oracle.probabilities(rot, pairs, np.zeros(k), theta, inp, bits, "exact")
    plan = X.Plan(rot, pairs, np.zeros(k), theta, inp)
    p = gpu_probs(plan, X, bits, "exact")
    assert plan.last_work()["general"]
    _check(p, ref, TOL_FP64, "deferred exact")


def _ill_conditioned_two_layer_circuit(seed):
    """Two CPhase layers (n_rot = 3) whose last rotation's row 0 is
    orthogonal to the columns of D_1(0) R_1 D_0(0) R_0[:, C]: every bitstring
    with mode 0 occupied has a singular M_0 (every D(0) the diagonal of the
    empty trajectory)."""
    rng = W.rng_for(seed)
    n, eta, k = 10, 4, 6
    R0, R1 = W.haar_unitary(rng, n), W.haar_unitary(rng, n)
    pairs = W.random_pairs(rng, n, k)
    layer = np.array([0, 0, 0, 1, 1, 1], dtype=np.int32)
    theta = rng.uniform(-1.0, 1.0, k)
    C = list(range(1, eta + 1))
    d = [np.ones(n, dtype=np.complex128), np.ones(n, dtype=np.complex128)]
    for (a, b), th, l in zip(pairs, theta, layer):
        d[l][a] *= np.exp(0.5j * th)
        d[l][b] *= np.exp(0.5j * th)
    Y = (d[1][:, None] * (R1 @ (d[0][:, None] * R0)))[:, C]
    _, _, vh = np.linalg.svd(Y.T)
    v = vh[eta:].conj().T[:, 0]
    Z = np.concatenate([v.conj()[:, None], rng.standard_normal((n, n - 1)) + 1j * rng.standard_normal((n, n - 1))],
                       axis=1)
    R2 = np.linalg.qr(Z)[0].conj().T
    return np.stack([R0, R1, R2]), pairs, layer, theta, W.bits_from_modes(C), n, eta


@pytest.mark.parametrize("mode", ["exact", "approx"])
def test_two_layer_bases_shift_past_singular_ones(X, mode):
    """Two CPhase layers, M_0 exactly singular for every bitstring with mode 0
    occupied: those bitstrings take a base shifted by a layer-0 gate (the
    layer-1 rows of S then carry the pattern's own layer-0 flips), and match
    the oracle like the others."""
    say(f"two-layer base shift, {mode}")
    rot, pairs, layer, theta, inp, n, eta = _ill_conditioned_two_layer_circuit(808)
    bits = W.all_fixed_weight(n, eta)
    t, smp = (3000, 17) if mode == "approx" else (0, 0)
    ref = oracle.probabilities(rot, pairs, layer, theta, inp, bits, mode, t=t, seed=smp)
    plan = X.Plan(rot, pairs, layer, theta, inp)
    p = gpu_probs(plan, X, bits, mode, t, smp)
    assert plan.last_work()["general"]
    zero0 = np.array([(int(b[0]) & 1) == 1 for b in bits])
    assert zero0.sum() > 10
    _check(p[zero0], ref[zero0], TOL_FP64, f"{mode} mode-0 occupied")
    _check(p, ref, TOL_FP64, f"{mode} all")


def test_wide_patterns_take_the_second_pass(X):
    """Raw Estimate with large angles on one block of 40 active modes:
    patterns flip up to 40 positions, those of 17..32 go to the evaluation
    with lane groups of 32, wider ones to the composition kernel; all match
    the oracle."""
    w = W.random_circuit(917, 44, 22, 20, n_rot=2, theta_scale=3.0, max_bits=64)
    bits = w.bits[:24]
    say("wide patterns: n=44 eta=22 k=20 theta~U[-3,3], t=600")
    ref = oracle_probs(w, bits, mode="approx", t=600, seed=3)
    plan = make_plan(w, X)
    p = gpu_probs(plan, X, bits, "approx", 600, 3)
    assert plan.last_work()["general"]
    _check(p, ref, TOL_FP64, "wide fp64")


def test_sampler_counts_the_philox_blocks_of_the_definition(X):
    """The sampler's count of Philox4x32-10 blocks equals the number the
    sampling definition draws, from the oracle's trajectories: one block per
    four samples' first draws, and per sample one per four further draws (a
    sample draws once more than it selects gates, unless it selects the last
    gate)."""
    w = W.random_circuit(919, 30, 14, 18, n_rot=3, theta_scale=1.5, max_bits=16)
    bits = w.bits[:12]
    t = 997
    plan = make_plan(w, X)
    gpu_probs(plan, X, bits, "approx", t, 5)
    wk = plan.last_work()
    assert wk["lemma"]
    expect = 0
    for b in range(len(bits)):
        xs = oracle.sample_trajectories(w.theta, seed=5, bidx=b, t=t)
        expect += (t + 3) // 4
        for x in xs:
            v = int(x[0]) | (int(x[1]) << 64)
            sel = bin(v).count("1")
            draws = sel + (0 if sel and (v >> (w.k - 1)) & 1 else 1)
            expect += (draws - 1 + 3) // 4
    say(f"  Philox blocks: {wk['philox_blocks']} (definition {expect})")
    assert wk["philox_blocks"] == expect


@pytest.mark.parametrize("mode", ["exact", "approx"])
def test_blocks_with_wrong_counts_interleaved(X, mode):
    """Bitstrings whose spin blocks hold the wrong particle counts (p = 0 by
    the block structure), of the wrong weight or with bits past n, interleaved
    with valid ones, on the general lemma with two blocks and two CPhase
    layers: the zero outcomes come out as exact zeros (amplitude 0, log p =
    -inf) and their neighbours still match the oracle."""
    n, eta, k = 16, 8, 10
    inp = list(range(eta // 2)) + list(range(n // 2, n // 2 + eta // 2))
    w = W.random_circuit(931, n, eta, k, n_rot=3, theta_scale=0.8, spin=True, input_modes=inp, max_bits=64)
    rng = np.random.default_rng(931)
    good = W.spin_bitstrings(rng, n // 2, eta // 2, eta // 2, 48)
    skew = W.spin_bitstrings(rng, n // 2, eta // 2 + 1, eta // 2 - 1, 16)   # right weight, wrong split
    heavy = np.array([W.bits_from_modes(list(range(eta + 1)))] * 4)           # wrong weight
    wide = np.array([W.bits_from_modes(list(range(eta - 1)) + [n + 3])] * 4)   # a bit past n
    bits = np.concatenate([good, skew, heavy, wide])
    order = rng.permutation(len(bits))
    bits = bits[order]
    zero = order >= len(good)
    t, smp = (2000, 17) if mode == "approx" else (0, 0)
    ref = oracle_probs(w, bits[~zero], mode=mode, t=t, seed=smp, batch_index=np.nonzero(~zero)[0])
    for prec, tol in (("fp64", TOL_FP64), ("mixed", TOL_MIXED)):
        plan = make_plan(w, X, prec)
        p, amp = gpu_probs(plan, X, bits, mode, t, smp, return_amp=True)
        assert plan.last_work()["general"]
        say(f"wrong block counts ({mode}, {prec}): {int(zero.sum())} zero of {len(bits)}")
        assert np.all(p[zero] == 0.0) and np.all(amp[zero] == 0.0)
        _check(p[~zero], ref, tol, f"{prec} valid neighbours")
        logp = torch.empty(len(bits), dtype=torch.float64, device=plan.device)
        plan.probabilities(X.bits_tensor(bits, plan.device), mode, t, smp, logp=logp)
        torch.cuda.synchronize()
        lp = logp.cpu().numpy()
        assert np.all(np.isneginf(lp[zero]))
        assert np.allclose(lp[~zero], np.log(ref), rtol=0, atol=2 * tol)
