"""GPU adjoint: gradients of sum_b g_b log p_b from the HIP backward pass
against the FP64 oracle's analytic gradient (same samples) and against
central finite differences of the HIP forward pass (h = 1e-6, samples held
fixed), through the rotation generators and the CPhase angles."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import make_plan, oracle_rot, sample_indices, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_12416_amd as X
    X.lib()
    return X


def _rel(a, b, floor=1e-6):
    """Largest per-element relative error, with an absolute floor of
    ``floor`` times the largest reference magnitude (so entries that are zero
    up to rounding do not dominate)."""
    a, b = np.asarray(a), np.asarray(b)
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor * scale)))


CASES = [
    # seed, n, eta, k, n_rot, spin, theta_scale
    (601, 6, 3, 4, 2, False, 1.0),     # G = 4
    (602, 10, 6, 6, 2, True, 0.8),     # G = 8
    (603, 20, 12, 8, 2, True, 0.5),    # G = 16
    (604, 8, 4, 0, 1, False, 0.0),     # single rotation, no CPhase
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[1]}_eta{c[2]}_k{c[3]}" for c in CASES])
@pytest.mark.parametrize("mode", ["exact", "approx"])
@pytest.mark.parametrize("evaluation", ["auto", "lu"])
def test_backward_matches_oracle(X, case, mode, evaluation):
    seed, n, eta, k, n_rot, spin, scale = case
    if mode == "approx" and k == 0:
        pytest.skip("no CPhase")
    if mode == "exact" and evaluation == "lu":
        pytest.skip("exact mode always uses the LU backward")
    inp = None
    if spin:
        inp = list(range(eta // 2)) + list(range(n // 2, n // 2 + eta - eta // 2))
    w = W.random_circuit(seed, n, eta, k, n_rot=n_rot, theta_scale=scale, spin=spin, input_modes=inp)
    bits = w.bits[:64]
    g = np.random.default_rng(seed).standard_normal(len(bits))
    t, smp = (1500, 21) if mode == "approx" else (0, 0)
    say(f"backward {mode} {evaluation} {case}")
    # mixed: the FP32 correction of the LU evaluation limits small entries, so
    # their error is measured against 1e-2 of the largest gradient entry
    for prec, tol, floor in (("fp64", 1e-9, 1e-6), ("mixed", 1e-5, 1e-2)):
        plan = make_plan(w, X, prec)
        plan.set_evaluation(evaluation)
        grot, gth = plan.log_prob_backward(X.bits_tensor(bits), torch.tensor(g, device="cuda"), mode, t, smp)
        used = plan.last_work()["backward_lemma"]
        orot, oth = oracle.log_prob_grad(w.rot, w.pairs, w.layer, w.theta, w.input_bits, bits, g, mode, t, smp)
        er, et = _rel(grot, orot, floor), (_rel(gth, oth, floor) if k else 0.0)
        say(f"  {prec}: rotation grad rel err {er:.2e}, angle grad rel err {et:.2e} (lemma backward: {used})")
        if mode == "approx" and evaluation == "auto" and n_rot == 2:
            assert used
        assert er < tol and et < tol


def _cfg4_plan(X, w, rot):
    return X.Plan(rot, w.pairs, w.layer, w.theta, w.input_bits, "fp64")


@pytest.mark.parametrize("evaluation", ["auto", "lu"])
def test_config4_gradient_vs_oracle_on_sampled_bitstrings(X, evaluation):
    """Full batch on the GPU, g_b non-zero only on a sample of bitstrings so the
    oracle can recompute exactly those terms."""
    w = W.workload(4)
    say(f"config 4 backward ({evaluation}) vs oracle: B=4096 t=16384, g nonzero on 12 bitstrings")
    rot = X.spin_rotations(w.gens)
    plan = _cfg4_plan(X, w, rot)
    plan.set_evaluation(evaluation)
    idx = sample_indices(w.B, 12, seed=44)
    g = np.zeros(w.B)
    g[idx] = 1.0 / w.B
    grot, gth = plan.log_prob_backward(X.bits_tensor(w.bits), torch.tensor(g, device="cuda"), "approx",
                                       w.t, w.seed)
    orot, oth = oracle.log_prob_grad(oracle_rot(w), w.pairs, w.layer, w.theta, w.input_bits, w.bits[idx],
                                     g[idx], "approx", w.t, w.seed, batch_index=idx)
    say(f"  rotation grad rel err {_rel(grot, orot):.2e}, angle grad rel err {_rel(gth, oth):.2e}")
    assert _rel(grot, orot) < 1e-9 and _rel(gth, oth) < 1e-9


def test_config4_backward_is_bitwise_reproducible(X):
    """Two full-batch backward calls (every bitstring contributing) give
    bitwise the same gradients; the determinant-lemma backward is used."""
    w = W.workload(4)
    say("config 4 full-batch backward twice (lemma path), bitwise comparison")
    plan = _cfg4_plan(X, w, X.spin_rotations(w.gens))
    bits = X.bits_tensor(w.bits)
    g = torch.full((w.B,), 1.0 / w.B, dtype=torch.float64, device="cuda")
    r1 = plan.log_prob_backward(bits, g, "approx", w.t, w.seed)
    assert plan.last_work()["backward_lemma"]
    r2 = plan.log_prob_backward(bits, g, "approx", w.t, w.seed)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])
    assert np.all(np.isfinite(r1[0])) and np.all(np.isfinite(r1[1]))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_config4_backward_reusing_forward_samples(X, prec):
    """With reuse on, a backward call after a forward call on the same bitstring
    tensor, t and seed takes the forward call's patterns and gives bitwise the
    gradients of a backward that draws them again; a forward call with another
    seed, a parameter change or a setting change in between ends the reuse."""
    w = W.workload(4)
    say(f"config 4 backward reusing the forward call's samples ({prec})")
    rot = X.spin_rotations(w.gens)
    bits = X.bits_tensor(w.bits)
    g = torch.full((w.B,), 1.0 / w.B, dtype=torch.float64, device="cuda")
    logp = torch.empty(w.B, dtype=torch.float64, device="cuda")
    ref_plan = X.Plan(rot, w.pairs, w.layer, w.theta, w.input_bits, prec)
    ref = ref_plan.log_prob_backward(bits, g, "approx", w.t, w.seed)
    assert not ref_plan.last_work()["backward_reused"]
    ref_plan.close()
    plan = X.Plan(rot, w.pairs, w.layer, w.theta, w.input_bits, prec)
    plan.set_reuse_samples(True)

    def check(expect_reuse):
        r = plan.log_prob_backward(bits, g, "approx", w.t, w.seed)
        assert plan.last_work()["backward_reused"] == expect_reuse
        assert np.array_equal(r[0], ref[0]) and np.array_equal(r[1], ref[1])

    plan.probabilities(bits, "approx", w.t, w.seed, logp=logp)
    check(True)
    check(True)            # the workspace still holds the forward call's patterns
    plan.probabilities(bits, "approx", w.t, w.seed + 1, logp=logp)
    check(False)           # another seed: drawn again
    check(False)           # ... and the workspace now holds the backward's own draws
    plan.probabilities(bits, "approx", w.t, w.seed, logp=logp)
    plan.set_params(rot, w.theta)
    check(False)
    plan.probabilities(bits, "approx", w.t, w.seed, logp=logp)
    plan.set_workspace_limit(1 << 34)
    check(False)
    plan.probabilities(bits[: w.B // 2], "approx", w.t, w.seed, logp=logp[: w.B // 2])
    check(False)           # another batch
    plan.set_reuse_samples(False)
    plan.probabilities(bits, "approx", w.t, w.seed, logp=logp)
    check(False)
    plan.close()


def test_config4_gradient_vs_finite_differences(X):
    """Mean log-probability over all 4096 bitstrings (t = 2^14, samples frozen):
    analytic gradients for every generator real and every angle vs central
    differences with h = 1e-6 of the GPU forward pass."""
    w = W.workload(4)
    say("config 4 backward vs central FD over all 2 x 256 generator reals and 24 angles")
    bits = X.bits_tensor(w.bits)
    K = w.gens.copy()
    th0 = w.theta.copy()
    plan = _cfg4_plan(X, w, X.spin_rotations(K))
    logp = torch.empty(w.B, dtype=torch.float64, device="cuda")

    def loss(Kx, thx):
        plan.set_params(X.spin_rotations(Kx), thx)
        plan.probabilities(bits, "approx", w.t, w.seed, logp=logp)
        return float(logp.mean().item())

    L0 = loss(K, th0)
    assert np.isfinite(L0)
    plan.set_params(X.spin_rotations(K), th0)
    grot, gth = plan.log_prob_backward(bits, torch.full((w.B,), 1.0 / w.B, dtype=torch.float64, device="cuda"),
                                       "approx", w.t, w.seed)
    assert plan.last_work()["backward_lemma"]
    d = K.shape[1]
    h = 1e-6
    worst = 0.0
    for l in range(K.shape[0]):
        GK = X.expm_adjoint(K[l], grot[l][:d, :d] + grot[l][d:, d:])
        an = X.autograd.generator_reals_grad(GK)
        iu = np.triu_indices(d, 1)
        params = [("re", i, j) for i, j in zip(*iu)] + [("im", i, j) for i, j in zip(*iu)] + \
                 [("diag", i, i) for i in range(d)]
        fd = np.zeros(len(params))
        for q, (kind, i, j) in enumerate(params):
            Kp, Km = K.copy(), K.copy()
            if kind == "re":
                Kp[l, i, j] += h; Kp[l, j, i] -= h; Km[l, i, j] -= h; Km[l, j, i] += h
            elif kind == "im":
                Kp[l, i, j] += 1j * h; Kp[l, j, i] += 1j * h; Km[l, i, j] -= 1j * h; Km[l, j, i] -= 1j * h
            else:
                Kp[l, i, i] += 1j * h; Km[l, i, i] -= 1j * h
            fd[q] = (loss(Kp, th0) - loss(Km, th0)) / (2 * h)
        err = np.max(np.abs(fd - an))
        say(f"  layer {l}: {len(params)} generator reals, max |FD - adjoint| = {err:.2e} (max |grad| {np.abs(an).max():.2e})")
        worst = max(worst, err)
    fdt = np.zeros(len(th0))
    for j in range(len(th0)):
        tp, tm = th0.copy(), th0.copy()
        tp[j] += h
        tm[j] -= h
        fdt[j] = (loss(K, tp) - loss(K, tm)) / (2 * h)
    errt = np.max(np.abs(fdt - gth))
    say(f"  angles: max |FD - adjoint| = {errt:.2e} (max |grad| {np.abs(gth).max():.2e})")
    assert worst < 1e-4 and errt < 1e-4


def test_autograd_function_matches_direct_call(X):
    say("torch.autograd path: generators -> rotations -> log p -> mean")
    w = W.workload(4, B=256)
    plan = _cfg4_plan(X, w, X.spin_rotations(w.gens))
    bits = X.bits_tensor(w.bits)
    gens = torch.tensor(w.gens, dtype=torch.complex128, requires_grad=True)
    theta = torch.tensor(w.theta, dtype=torch.float64, requires_grad=True)
    rot = X.autograd.spin_rotations(gens)
    lp = X.autograd.log_prob(plan, bits, rot, theta, "approx", 4096, w.seed)
    lp.mean().backward()
    plan.set_params(X.spin_rotations(w.gens), w.theta)
    grot, gth = plan.log_prob_backward(bits, torch.full((w.B,), 1.0 / w.B, dtype=torch.float64, device="cuda"),
                                       "approx", 4096, w.seed)
    d = w.gens.shape[1]
    for l in range(w.gens.shape[0]):
        GK = X.expm_adjoint(w.gens[l], grot[l][:d, :d] + grot[l][d:, d:])
        np.testing.assert_allclose(gens.grad[l].numpy(), GK, rtol=0, atol=1e-12)
    np.testing.assert_allclose(theta.grad.numpy(), gth, rtol=0, atol=1e-12)
