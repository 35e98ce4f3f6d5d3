"""xf_probabilities_noalloc (fixed per-device scratch, no allocation) against
xf_probabilities through the C ABI: bitwise equal results on two calls in a
row, the second with a smaller batch of another circuit; a clear error when
bitstrings whose patterns overflow their workspace region."""
import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_helpers import make_plan, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_12416_amd as X
    X.lib()
    return X


def _both(X, plan, bits, t, seed, mode=None):
    mode = X._abi.XF_RAW_ESTIMATE if mode is None else mode
    lib = X.lib()
    B = bits.shape[0]
    stream = torch.cuda.current_stream().cuda_stream
    outs = []
    for fn in (lib.xf_probabilities, lib.xf_probabilities_noalloc):
        p = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
        a = torch.full((B, 2), -1.0, dtype=torch.float64, device="cuda")
        lp = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
        X._abi.check(fn(plan._h, bits.data_ptr(), B, mode, t, seed, p.data_ptr(),
                        a.data_ptr(), lp.data_ptr(), ctypes.c_void_p(stream)))
        torch.cuda.synchronize()
        outs.append((p.cpu().numpy(), a.cpu().numpy(), lp.cpu().numpy()))
    return outs


def test_noalloc_matches_allocating_call_twice(X):
    # 1: the LUCJ workload at full batch (several scratch chunks of about 1000
    # bitstrings each), determinant-lemma path
    w = W.workload(2)
    say(f"no-allocation call 1: {w.name}")
    plan = make_plan(w, X)
    (p1, a1, l1), (q1, b1, m1) = _both(X, plan, X.bits_tensor(w.bits), w.t, w.seed)
    assert plan.last_work()["lemma"]
    assert np.array_equal(p1, q1) and np.array_equal(a1, b1) and np.array_equal(l1, m1)
    assert np.count_nonzero(p1) == w.B
    # 2: a smaller batch of the generator workload (one chunk)
    w2 = W.workload(4, B=1500)
    say(f"no-allocation call 2: {w2.name} B={w2.B} t=4096")
    plan2 = make_plan(w2, X)
    (p2, a2, l2), (q2, b2, m2) = _both(X, plan2, X.bits_tensor(w2.bits), 4096, 77)
    assert np.array_equal(p2, q2) and np.array_equal(a2, b2) and np.array_equal(l2, m2)
    assert np.count_nonzero(p2) == w2.B


def test_noalloc_general_lemma_two_calls(X):
    """The general lemma (two CPhase layers, two spin blocks), whose setup
    keeps H and the base records in the scratch beside the entry regions:
    Raw Estimate twice in a row (the second batch smaller, of another
    circuit), then exact mode, each bitwise equal to the allocating call."""
    for seed, n, eta, k, B in ((911, 44, 20, 16, 600), (912, 14, 6, 9, 100)):
        inp = list(range(eta // 2)) + list(range(n // 2, n // 2 + eta // 2))
        w = W.random_circuit(seed, n, eta, k, n_rot=3, theta_scale=0.6, spin=True, input_modes=inp, max_bits=16)
        bits = W.spin_bitstrings(np.random.default_rng(seed), n // 2, eta // 2, eta // 2, B)
        plan = make_plan(w, X)
        say(f"no-allocation general lemma: n={n} eta={eta} k={k} two layers B={B} t=4096")
        (p1, a1, l1), (q1, b1, m1) = _both(X, plan, X.bits_tensor(bits), 4096, 31)
        assert plan.last_work()["general"]
        assert np.array_equal(p1, q1) and np.array_equal(a1, b1) and np.array_equal(l1, m1)
        assert np.count_nonzero(p1) == B
    # exact mode on the last plan (its term list built by the allocating call)
    say(f"no-allocation general lemma, exact mode: B={B}")
    (p2, a2, l2), (q2, b2, m2) = _both(X, plan, X.bits_tensor(bits), 0, 0, X._abi.XF_EXACT)
    assert plan.last_work()["general"]
    assert np.array_equal(p2, q2) and np.array_equal(a2, b2) and np.array_equal(l2, m2)


def test_noalloc_exact_prefix_tree_two_calls(X):
    """Exact mode along the term list's prefix tree (batches of at least 1024
    bitstrings), the setup records and segment partials in the scratch: the
    exact stress workload, then a smaller batch of another circuit, each
    bitwise equal to the allocating call."""
    w = W.workload(3)
    w2 = W.random_circuit(951, 14, 7, 10, n_rot=2, max_bits=4096)
    for ww, bits in ((w, w.bits), (w2, w2.bits[:1024])):
        plan = make_plan(ww, X)
        say(f"no-allocation prefix tree: {ww.name} B={len(bits)}")
        (p1, a1, l1), (q1, b1, m1) = _both(X, plan, X.bits_tensor(bits), 0, 0, X._abi.XF_EXACT)
        wk = plan.last_work()
        assert wk["general"] and wk["tree_bitstrings"] > 0, wk
        assert np.array_equal(p1, q1) and np.array_equal(a1, b1) and np.array_equal(l1, m1)
        assert np.count_nonzero(p1) == len(bits)
        plan.close()


def test_noalloc_overflowing_regions_match(X):
    """Large angles: every sample is a distinct pattern, more than a
    workspace region holds, so the bitstrings are left to the LU kernel; the
    no-allocation call agrees bitwise with the allocating one."""
    rng = W.rng_for(404)
    n = 16
    rot = np.stack([W.haar_unitary(rng, n) for _ in range(2)])
    pairs = W.random_pairs(rng, n, 40)
    theta = rng.uniform(-3.0, 3.0, 40)
    inp = W.bits_from_modes(range(6))
    bits = W.all_fixed_weight(n, 6)[::997][:8]
    plan = X.Plan(rot, pairs, np.zeros(40), theta, inp)
    say("no-allocation call with overflowing regions: n=16 eta=6 k=40 theta~U[-3,3] t=12000")
    (p1, a1, l1), (q1, b1, m1) = _both(X, plan, X.bits_tensor(bits), 12000, 5)
    assert np.array_equal(p1, q1) and np.array_equal(a1, b1) and np.array_equal(l1, m1)
    assert np.count_nonzero(p1) == len(bits)


def test_noalloc_exact_needs_a_built_term_list(X):
    w = W.workload(1)
    plan = make_plan(w, X)
    bits = X.bits_tensor(w.bits)
    out = torch.empty(w.B, dtype=torch.float64, device="cuda")
    with pytest.raises(X.XfError) as e:
        plan.probabilities_noalloc(bits, out, "exact")
    assert e.value.status == 2
    ref = plan.probabilities(bits, "exact").cpu().numpy()
    plan.probabilities_noalloc(bits, out, "exact")
    assert np.array_equal(out.cpu().numpy(), ref)
