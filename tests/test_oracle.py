"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None compares the oracle with itself: the
references are a brute-force state vector (second quantisation, no
determinants), closed forms, special cases reducing to a library routine
(numpy's det / inv, scipy's expm_frechet, rocRAND's Philox), values printed in
the paper, exact rational arithmetic and sampling statistics.
"""
import json
import math
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

import oracle
import workloads as W
from bruteforce import bits_to_int, statevector_amplitudes

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _exact(w, bits=None, **kw):
    return oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits,
                                w.bits if bits is None else bits, "exact", **kw)


# ----------------------------------------------------------------------------
# exact sum vs brute force (Sec. II-B Eq. 2-3, Sec. III-B Eq. 7-9)
# ----------------------------------------------------------------------------

CASES = [
    # seed, n, eta, k, n_rot, spin
    (11, 4, 2, 2, 2, False),
    (12, 5, 2, 3, 2, False),
    (13, 6, 3, 4, 3, False),
    (14, 7, 3, 5, 2, False),
    (15, 8, 4, 6, 3, False),
    (16, 8, 4, 5, 2, True),
    (17, 10, 4, 4, 3, True),
]


@pytest.mark.parametrize("seed,n,eta,k,n_rot,spin", CASES)
def test_exact_matches_state_vector(seed, n, eta, k, n_rot, spin):
    w = W.random_circuit(seed, n, eta, k, n_rot=n_rot, theta_scale=2.0, spin=spin,
                         input_modes=(list(range(eta // 2)) + list(range(n // 2, n // 2 + eta - eta // 2)))
                         if spin else None)
    p, a = oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, w.bits,
                                "exact", return_amp=True)
    states, psi = statevector_amplitudes(w.rot, w.pairs, w.layer, w.theta,
                                         W.modes_from_bits(w.input_bits), n)
    idx = {s: i for i, s in enumerate(states)}
    ref = np.array([psi[idx[bits_to_int(b)]] for b in w.bits])
    # the oracle drops the global phase e^{-i theta_j / 4} of every gate
    glob = np.exp(-1j * np.sum(w.theta) / 4)
    np.testing.assert_allclose(a * glob, ref, atol=1e-12, rtol=0)
    np.testing.assert_allclose(p, np.abs(ref) ** 2, atol=1e-12, rtol=0)


def test_config1_sums_to_one_and_matches_state_vector():
    w = W.workload(1)
    p = _exact(w)
    assert len(p) == math.comb(8, 4) == 70
    assert abs(p.sum() - 1.0) < 1e-12
    states, psi = statevector_amplitudes(w.rot, w.pairs, w.layer, w.theta, list(range(4)), 8)
    idx = {s: i for i, s in enumerate(states)}
    ref = np.array([abs(psi[idx[bits_to_int(b)]]) ** 2 for b in w.bits])
    np.testing.assert_allclose(p, ref, atol=1e-13)


def test_spin_sector_sums_to_one():
    # spin-restricted rotations conserve (n_alpha, n_beta): the sector sums to 1
    rng = W.rng_for(101)
    norb = 5
    rot = np.stack([W.block_diag2(W.haar_unitary(rng, norb)) for _ in range(3)])
    pairs = np.array([[0, 1], [5, 6], [2, 7], [3, 4], [8, 9], [1, 6]], np.int32)
    layer = np.array([0, 0, 0, 1, 1, 1], np.int32)
    theta = rng.uniform(-1, 1, 6)
    inp = W.bits_from_modes([0, 1, 5, 6])
    bits = np.array([W.bits_from_modes(list(a) + [5 + x for x in b])
                     for a in combinations(range(5), 2) for b in combinations(range(5), 2)])
    p = oracle.probabilities(rot, pairs, layer, theta, inp, bits, "exact")
    assert abs(p.sum() - 1.0) < 1e-12


# ----------------------------------------------------------------------------
# special cases with closed forms
# ----------------------------------------------------------------------------

def test_no_cphase_is_single_slater_overlap():
    w = W.random_circuit(21, 9, 4, 0, n_rot=3)
    V = w.rot[2] @ w.rot[1] @ w.rot[0]
    C = W.modes_from_bits(w.input_bits)
    ref = np.array([abs(np.linalg.det(V[np.ix_(W.modes_from_bits(b), C)])) ** 2 for b in w.bits])
    np.testing.assert_allclose(_exact(w), ref, atol=1e-14)


def test_term_magnitude_sum():
    """sum_i |w_i det M_i| (the cancellation measure reported beside the
    errors): the single term's |det| = sqrt(p) without CPhase gates, |A| when
    every sampled term is the same (all angles zero), never below |A|."""
    w = W.random_circuit(21, 9, 4, 0, n_rot=3)
    p, a, s = oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, w.bits, "exact",
                                   return_amp=True, return_abs_sum=True)
    np.testing.assert_allclose(s, np.sqrt(p), rtol=1e-13, atol=1e-15)
    w = W.random_circuit(25, 8, 4, 5, n_rot=2, theta_scale=1.0)
    p, a, s = oracle.probabilities(w.rot, w.pairs, w.layer, np.zeros(5), w.input_bits, w.bits, "approx",
                                   t=64, seed=3, return_amp=True, return_abs_sum=True)
    np.testing.assert_allclose(s, np.abs(a), rtol=1e-12, atol=1e-15)
    for mode, t in (("exact", 0), ("approx", 200)):
        p, a, s = oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, w.bits, mode,
                                       t=t, seed=4, return_amp=True, return_abs_sum=True)
        assert np.all(s >= np.abs(a) * (1 - 1e-12))
        assert np.any(s > np.abs(a) * 1.01)


def test_zero_angle_gate_is_identity():
    w = W.random_circuit(22, 7, 3, 4, n_rot=2, theta_scale=1.0)
    th = w.theta.copy()
    th[2] = 0.0
    p_with = oracle.probabilities(w.rot, w.pairs, w.layer, th, w.input_bits, w.bits, "exact")
    keep = [0, 1, 3]
    p_without = oracle.probabilities(w.rot, w.pairs[keep], w.layer[keep], th[keep], w.input_bits,
                                     w.bits, "exact")
    np.testing.assert_allclose(p_with, p_without, atol=1e-14)


def test_single_particle_ignores_cphase():
    w = W.random_circuit(23, 6, 1, 5, n_rot=3, theta_scale=3.0)
    p1 = _exact(w)
    p0 = oracle.probabilities(w.rot, w.pairs, w.layer, np.zeros(5), w.input_bits, w.bits, "exact")
    np.testing.assert_allclose(p1, p0, atol=1e-14)


def test_full_occupation_has_probability_one():
    w = W.random_circuit(24, 6, 6, 4, n_rot=2, theta_scale=3.0)
    assert w.bits.shape[0] == 1
    np.testing.assert_allclose(_exact(w), [1.0], atol=1e-13)


def test_identity_rotations_give_delta():
    n, eta = 7, 3
    rot = np.stack([np.eye(n, dtype=np.complex128)] * 3)
    rng = np.random.default_rng(5)
    pairs = np.array([[0, 1], [2, 5], [1, 6], [3, 4]], np.int32)
    layer = np.array([0, 1, 1, 0], np.int32)
    theta = rng.uniform(-2, 2, 4)
    inp = W.bits_from_modes([1, 2, 5])
    bits = W.all_fixed_weight(n, eta)
    p = oracle.probabilities(rot, pairs, layer, theta, inp, bits, "exact")
    ref = np.array([1.0 if (b == inp).all() else 0.0 for b in bits])
    np.testing.assert_allclose(p, ref, atol=1e-14)


def test_weight_mismatch_gives_zero():
    w = W.random_circuit(25, 6, 3, 2)
    bad = np.array([W.bits_from_modes([0, 1]), W.bits_from_modes([0, 1, 2, 3])])
    np.testing.assert_array_equal(_exact(w, bad), [0.0, 0.0])


# ----------------------------------------------------------------------------
# determinant (textbook partial-pivot LU) vs numpy
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 3, 7, 16, 26])
def test_det_matches_numpy(m):
    rng = np.random.default_rng(m)
    a = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    ref = np.linalg.det(a)
    assert abs(oracle.det(a) - ref) <= 1e-12 * max(1.0, abs(ref))


def test_det_of_singular_matrix_is_zero():
    a = np.ones((4, 4), dtype=np.complex128)
    assert oracle.det(a) == 0
    b = np.zeros((3, 3), dtype=np.complex128)
    b[0, 1] = b[1, 2] = 1.0
    assert oracle.det(b) == 0


# ----------------------------------------------------------------------------
# extent (Eq. 5) and trajectory bound (Eq. 6)
# ----------------------------------------------------------------------------

def test_extent_closed_forms():
    assert oracle.extent(np.zeros(7)) == 1.0
    assert oracle.extent(np.full(43, math.pi)) == pytest.approx(2.0 ** 43, rel=1e-14)
    assert oracle.extent(np.full(3, -math.pi)) == pytest.approx(8.0, rel=1e-14)
    th = np.random.default_rng(3).normal(0, 0.3, 20)
    c_xi = oracle.lib().xfo_extent(20, oracle._ptr(np.ascontiguousarray(th)))
    assert c_xi == pytest.approx(oracle.extent(th), rel=1e-14)


def _extent_samples(k, mean, var, n=20000, seed=0):
    th = np.random.default_rng(seed).normal(mean, math.sqrt(var), size=(n, k))
    return np.array([oracle.extent(r) for r in th])


@pytest.mark.parametrize("key", ["extent_43_gates_near_zero", "extent_111_gates_near_zero",
                                 "extent_43_gates", "extent_12_gates"])
def test_extent_reproduces_printed_values(key):
    e = GOLDEN[key]
    means = e.get("means", [e.get("mean")])
    printed = e["printed"] if isinstance(e["printed"], list) else [e["printed"]]
    for mu, val in zip(means, printed):
        xs = _extent_samples(e["k"], mu, e["variance"], n=4000)
        q = (xs < val).mean()
        assert 0.001 < q < 0.999, (key, mu, val, np.median(xs))
    if key == "extent_43_gates":
        # near theta = pi the spread is tiny: the printed 8.77e12 fixes the formula tightly
        xs = _extent_samples(43, math.pi, 1e-3, n=4000, seed=1)
        assert abs(np.median(xs) / 8.77e12 - 1) < 1e-3


def test_trajectory_bound_shape():
    t0 = oracle.trajectory_bound(0.01, 0.05, 0.1, 2.0)
    assert t0 > 0
    assert oracle.trajectory_bound(0.02, 0.05, 0.1, 2.0) < t0          # looser eps
    assert oracle.trajectory_bound(0.01, 0.10, 0.1, 2.0) < t0          # looser delta
    assert oracle.trajectory_bound(0.01, 0.05, 0.1, 4.0) > t0          # larger extent
    assert oracle.trajectory_bound(0.01, 0.05, 0.2, 2.0) > t0          # larger p_max
    # eps -> 0 scaling: (sqrt(p+eps)-sqrt(p))^2 ~ eps^2 / (4p)
    r = oracle.trajectory_bound(1e-4, 0.05, 0.1, 2.0) / oracle.trajectory_bound(2e-4, 0.05, 0.1, 2.0)
    assert 3.9 < r < 4.1


# ----------------------------------------------------------------------------
# trajectory sampling (Eq. 10-12) and the RNG
# ----------------------------------------------------------------------------

def test_philox_matches_rocrand():
    """Oracle Philox4x32-10 vs rocRAND's implementation of the same published
    generator (a library routine, compiled here for the host)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    rng = np.random.default_rng(7)
    vals = rng.integers(0, 2 ** 32, size=(64, 6), dtype=np.uint64)
    vals[0] = 0
    vals[1] = 2 ** 32 - 1
    src = r'''
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
int main() {
  struct open_engine : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
  };
  unsigned a,b,c,d,e,f;
  open_engine eng;
  while (scanf("%u %u %u %u %u %u", &a,&b,&c,&d,&e,&f) == 6) {
    uint4 r = eng.ten_rounds(uint4{a,b,c,d}, uint2{e,f});
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
}
'''
    with tempfile.TemporaryDirectory() as td:
        cpp = os.path.join(td, "ref.cpp")
        exe = os.path.join(td, "ref")
        open(cpp, "w").write(src)
        subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", cpp, "-o", exe],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        inp = "\n".join(" ".join(str(int(v)) for v in row) for row in vals)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()], np.uint64)
    mine = np.array([oracle.philox4x32_10(r[:4], r[4:]) for r in vals], np.uint64)
    np.testing.assert_array_equal(mine, ref)


def test_sampling_probability_worked_example():
    ex = GOLDEN["trajectory_example"]
    np.testing.assert_allclose(oracle.sampling_probability(ex["theta"]), ex["p_one"], atol=1e-15)
    # theta = 0 is never sampled as d_1; theta = pi is a fair coin
    xs = oracle.sample_trajectories([0.0, math.pi, 0.0], seed=3, bidx=0, t=20000)
    bits = np.stack([(xs[:, 0] >> j) & 1 for j in range(3)], axis=1)
    assert bits[:, 0].sum() == 0 and bits[:, 2].sum() == 0
    assert abs(bits[:, 1].mean() - 0.5) < 5 * math.sqrt(0.25 / 20000)


def test_sampler_table_exact_rationals():
    """T[a, j] = floor(2^32 (1 - prod_{i=a..j} (1 - p_i))) checked in exact
    rational arithmetic on the same FP64 p_i (one unit of slack for the FP64
    rounding of the running product)."""
    theta = np.array([0.3, -0.05, 0.0, 1.2, -2.5, 0.7, 3.1])
    p = [Fraction(float(v)) for v in oracle.sampling_probability(theta)]
    T = oracle.sampler_table(theta)
    k = len(theta)
    for a in range(k):
        surv = Fraction(1)
        for j in range(k):
            if j < a:
                assert T[a, j] == 0
                continue
            surv *= (1 - p[j])
            exact = math.floor((1 - surv) * 2 ** 32)
            exact = min(exact, 2 ** 32 - 1)
            assert abs(int(T[a, j]) - exact) <= 1, (a, j)


def test_sampler_induced_distribution_is_the_product_distribution():
    """Enumerate every trajectory and compute the exact probability with which
    the next-selected-gate sampler emits it, from the integer table alone."""
    theta = np.array([0.4, -1.1, 0.0, 2.2, 0.05, -0.6])
    k = len(theta)
    T = oracle.sampler_table(theta).astype(np.int64)
    p = oracle.sampling_probability(theta)
    for x in range(1 << k):
        ones = [j for j in range(k) if (x >> j) & 1]
        prob = 1.0
        a = 0
        for j in ones:
            lo = T[a, j - 1] if j - 1 >= a else 0
            prob *= (T[a, j] - lo) / 2 ** 32
            a = j + 1
        if a < k:
            prob *= (2 ** 32 - T[a, k - 1]) / 2 ** 32
        ref = np.prod([p[j] if (x >> j) & 1 else 1 - p[j] for j in range(k)])
        assert abs(prob - ref) < 1e-8, (x, prob, ref)


def test_sampler_draw_layout():
    """The counter layout of the uniform draws: u_0 of sample s is word s mod 4
    of the Philox block (s div 4, 2^32 - 1, i), u_d (d >= 1) word (d-1) mod 4
    of block (s, (d-1) div 4, i).  Two gates at theta = pi (p = 1/2), walked
    by hand from the table with draws taken from the rocRAND-pinned Philox."""
    theta = [math.pi, math.pi]
    T = oracle.sampler_table(theta).astype(np.int64)
    seed, bidx, t = 0x1234_5678_9ABC_DEF0, (5 << 32) | 17, 64
    key = [seed & 0xFFFFFFFF, seed >> 32]
    xs = oracle.sample_trajectories(theta, seed=seed, bidx=bidx, t=t)

    def u(smp, d):
        if d == 0:
            return int(oracle.philox4x32_10([smp >> 2, 0xFFFFFFFF, bidx & 0xFFFFFFFF, bidx >> 32], key)[smp & 3])
        return int(oracle.philox4x32_10([smp, (d - 1) >> 2, bidx & 0xFFFFFFFF, bidx >> 32], key)[(d - 1) & 3])

    for smp in range(t):
        x, a, d = 0, 0, 0
        while a < 2:
            v = u(smp, d)
            d += 1
            js = [j for j in range(a, 2) if v < T[a, j]]
            if not js:
                break
            x |= 1 << js[0]
            a = js[0] + 1
        assert int(xs[smp, 0]) == x, smp


def test_sampler_statistics():
    theta = np.array([0.2, -0.9, 1.5, 3.0, -0.4, 0.05, 2.0, -1.3])
    t = 200_000
    xs = oracle.sample_trajectories(theta, seed=12345, bidx=77, t=t)
    bits = np.stack([(xs[:, 0] >> j) & 1 for j in range(8)], axis=1).astype(np.float64)
    p = oracle.sampling_probability(theta)
    z = (bits.mean(0) - p) / np.sqrt(p * (1 - p) / t)
    assert np.all(np.abs(z) < 5), z
    # pairwise independence
    for i in range(8):
        for j in range(i + 1, 8):
            pij = p[i] * p[j]
            zz = ((bits[:, i] * bits[:, j]).mean() - pij) / math.sqrt(pij * (1 - pij) / t)
            assert abs(zz) < 5.5, (i, j, zz)
    # different bitstring indices give different streams
    xs2 = oracle.sample_trajectories(theta, seed=12345, bidx=78, t=1000)
    assert not np.array_equal(xs[:1000], xs2)


# ----------------------------------------------------------------------------
# Raw Estimate (Sec. III-A): exactness at theta = 0, unbiasedness, convergence
# ----------------------------------------------------------------------------

def test_estimate_is_exact_without_phases():
    w = W.random_circuit(31, 7, 3, 5, n_rot=3, theta_scale=1.0)
    th0 = np.zeros(5)
    pe = oracle.probabilities(w.rot, w.pairs, w.layer, th0, w.input_bits, w.bits, "exact")
    pa = oracle.probabilities(w.rot, w.pairs, w.layer, th0, w.input_bits, w.bits, "approx", t=17, seed=4)
    np.testing.assert_allclose(pa, pe, rtol=1e-13, atol=1e-16)


def test_estimator_is_unbiased():
    w = W.random_circuit(32, 6, 3, 4, n_rot=2, theta_scale=1.5)
    bits = w.bits[[0, 3, 7, 11]]
    _, a_ex = oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, bits, "exact",
                                   return_amp=True)
    est = np.array([oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, bits,
                                         "approx", t=16, seed=s, return_amp=True)[1]
                    for s in range(1500)])
    mean = est.mean(0)
    se = np.sqrt(est.real.var(0) / len(est)) + 1j * np.sqrt(est.imag.var(0) / len(est))
    assert np.all(np.abs((mean - a_ex).real) < 5 * se.real + 1e-12)
    assert np.all(np.abs((mean - a_ex).imag) < 5 * se.imag + 1e-12)


def test_estimator_error_falls_like_inverse_sqrt_t():
    """Stand-in for the paper's error study on a 12-qubit LUCJ circuit
    (6 orbitals, 3 alpha + 3 beta, 12 CPhase; all 400 outcomes)."""
    g = GOLDEN["support_12_qubit_lucj"]
    rng = W.rng_for(112)
    norb = g["norb"]
    rot = np.stack([W.block_diag2(W.haar_unitary(rng, norb)) for _ in range(2)])
    pairs = W.lucj_pairs(norb)[:12]
    theta = rng.normal(math.pi / 3, math.sqrt(0.1), 12)
    inp = W.bits_from_modes([0, 1, 2, 6, 7, 8])
    bits = W.spin_bitstrings(rng, norb, 3, 3, 1)  # shape only
    bits = np.array([W.bits_from_modes(list(a) + [norb + x for x in b])
                     for a in combinations(range(norb), 3) for b in combinations(range(norb), 3)])
    assert len(bits) == g["support"]
    layer = np.zeros(12, np.int32)
    pe = oracle.probabilities(rot, pairs, layer, theta, inp, bits, "exact")
    assert abs(pe.sum() - 1) < 1e-12
    errs = []
    for t in (1000, 100_000):
        e = [np.abs(oracle.probabilities(rot, pairs, layer, theta, inp, bits, "approx", t=t, seed=s)
                    - pe).mean() for s in range(3)]
        errs.append(np.mean(e))
    ratio = errs[0] / errs[1]
    assert 5.0 < ratio < 20.0, errs   # sqrt(100) = 10


def test_hoeffding_failure_rate_within_delta():
    w = W.random_circuit(33, 6, 3, 3, n_rot=2, theta_scale=0.6)
    bits = w.bits[:3]
    pe = oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, bits, "exact")
    eps, delta = 0.03, 0.2
    t = oracle.trajectory_bound(eps, delta, 1.0, oracle.extent(w.theta))
    fails = 0
    trials = 40
    for s in range(trials):
        pa = oracle.probabilities(w.rot, w.pairs, w.layer, w.theta, w.input_bits, bits, "approx",
                                  t=t, seed=1000 + s)
        fails += int(np.any(np.abs(pa - pe) > eps))
    assert fails / trials <= delta


# ----------------------------------------------------------------------------
# gradients
# ----------------------------------------------------------------------------

def _fd_check(w, bits, g, mode, t=0, seed=0, h=1e-6, entries=None):
    def L(rot, th):
        p = oracle.probabilities(rot, w.pairs, w.layer, th, w.input_bits, bits, mode, t, seed,
                                 theta_sample=w.theta)
        return float(np.sum(g * np.log(p)))
    grot, gth = oracle.log_prob_grad(w.rot, w.pairs, w.layer, w.theta, w.input_bits, bits, g,
                                     mode, t, seed)
    for j in range(len(w.theta)):
        tp, tm = w.theta.copy(), w.theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (L(w.rot, tp) - L(w.rot, tm)) / (2 * h)
        assert abs(fd - gth[j]) < 1e-6 * max(1, abs(fd)), (j, fd, gth[j])
    for (l, p, q) in entries:
        for comp in (1.0, 1j):
            rp, rm = w.rot.copy(), w.rot.copy()
            rp[l, p, q] += h * comp
            rm[l, p, q] -= h * comp
            fd = (L(rp, w.theta) - L(rm, w.theta)) / (2 * h)
            an = grot[l, p, q].real if comp == 1.0 else grot[l, p, q].imag
            assert abs(fd - an) < 1e-6 * max(1, abs(fd)), (l, p, q, comp, fd, an)


@pytest.mark.parametrize("mode,t", [("exact", 0), ("approx", 64)])
def test_gradient_matches_finite_differences(mode, t):
    w = W.random_circuit(41, 6, 3, 4, n_rot=3, theta_scale=1.0)
    bits = w.bits[:10]
    g = np.random.default_rng(2).standard_normal(10)
    _fd_check(w, bits, g, mode, t, seed=5,
              entries=[(0, 1, 2), (0, 4, 0), (1, 0, 5), (1, 3, 3), (2, 2, 1), (2, 5, 4)])


def test_gradient_without_cphase_closed_form():
    """k = 0, one layer: log p = log |det U[R, C]|^2, whose gradient with
    respect to U[R_i, C_j] is 2 conj((M^{-1})_{ji}) (Jacobi's formula)."""
    w = W.random_circuit(42, 6, 3, 0, n_rot=1)
    bits = w.bits[:5]
    g = np.array([1.0, -0.5, 2.0, 0.25, 1.5])
    grot, _ = oracle.log_prob_grad(w.rot, w.pairs, w.layer, w.theta, w.input_bits, bits, g, "exact")
    C = W.modes_from_bits(w.input_bits)
    ref = np.zeros((6, 6), np.complex128)
    for gb, b in zip(g, bits):
        R = W.modes_from_bits(b)
        Mi = np.linalg.inv(w.rot[0][np.ix_(R, C)])
        for i, r in enumerate(R):
            for j, c in enumerate(C):
                ref[r, c] += gb * 2 * np.conj(Mi[j, i])
    np.testing.assert_allclose(grot[0], ref, atol=1e-12)


def test_expm_adjoint_matches_finite_differences():
    rng = np.random.default_rng(9)
    K = W.anti_hermitian(rng, 5, 0.3)
    G = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    # loss L(K) = Re sum conj(G) * expm(K)  =>  dL/dU = G (dL/dRe + i dL/dIm convention)
    def L(Kp):
        return float(np.real(np.sum(np.conj(G) * oracle.expm(Kp))))
    GK = oracle.expm_adjoint(K, G)
    h = 1e-6
    for (p, q) in [(0, 1), (2, 2), (4, 3)]:
        for comp in (1.0, 1j):
            Kp, Km = K.copy(), K.copy()
            Kp[p, q] += h * comp
            Km[p, q] -= h * comp
            fd = (L(Kp) - L(Km)) / (2 * h)
            an = GK[p, q].real if comp == 1.0 else GK[p, q].imag
            assert abs(fd - an) < 1e-7, (p, q, comp, fd, an)


# ----------------------------------------------------------------------------
# Eq. 6 derived independently (Raw Estimate, Sec. III-A)
#
# The estimator averages t i.i.d. complex samples Z_s = sqrt(xi*) phase(x_s)
# det V(x_s)[R, C] with mean A (|A|^2 = p <= p_max).  Every determinant is that
# of a submatrix of a unitary matrix, so |det| <= 1 and |Z_s| <= sqrt(xi*);
# the centred steps (Z_s - A) / t are bounded by c / t with
# c = sqrt(xi*) + sqrt(p_max).  Their partial sums form a martingale in the
# plane, so the large-deviation bound for vector-valued martingales with
# steps of norm <= 1 (T. P. Hayes, "A large-deviation inequality for
# vector-valued martingales", 2005): P(|X_n| >= a) < 2 e^2 exp(-a^2 / (2 n)),
# applied to X_t = (t / c) sum_s (Z_s - A) / t, gives
#     P(|A_hat - A| >= r) < 2 e^2 exp(-t r^2 / (2 c^2)).
# An amplitude within r of A gives |p_hat - p| <= (2 sqrt(p_max) + r) r,
# which equals eps for the root r of that quadratic.  The trajectory count of
# Eq. 6 must be the smallest t for which the tail is at most delta.  The test
# finds r by bisection and t by an integer search on the tail itself, so it
# does not restate the closed form.
# ----------------------------------------------------------------------------

def _hayes_tail(a: float, steps: int) -> float:
    return 2.0 * math.e ** 2 * math.exp(-a * a / (2.0 * steps))


def _amplitude_radius(eps: float, p_max: float) -> float:
    """Largest r with (2 sqrt(p_max) + r) r <= eps, by bisection."""
    lo, hi = 0.0, math.sqrt(eps) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (2.0 * math.sqrt(p_max) + mid) * mid <= eps:
            lo = mid
        else:
            hi = mid
    return lo


def _derived_count(eps, delta, p_max, xi):
    c = math.sqrt(xi) + math.sqrt(p_max)
    r = _amplitude_radius(eps, p_max)

    def tail(t):
        return _hayes_tail(r * t / c, t)

    hi = 1
    while tail(hi) > delta:
        hi *= 2
    lo = hi // 2 if hi > 1 else 0      # tail(lo) > delta (or lo = 0)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if tail(mid) > delta:
            lo = mid
        else:
            hi = mid
    return hi, tail


_EQ6_GRID = [(eps, delta, p_max, xi)
             for eps in (1e-3, 7.3e-3, 0.05)
             for delta in (1e-6, 0.013, 0.2)
             for p_max in (0.0, 0.011, 0.37, 1.0)
             for xi in (1.0, 1.732, 5.281, 228.091)]


def test_trajectory_bound_is_the_smallest_count_the_tail_bound_allows():
    for eps, delta, p_max, xi in _EQ6_GRID:
        t = oracle.trajectory_bound(eps, delta, p_max, xi)
        want, tail = _derived_count(eps, delta, p_max, xi)
        assert t == want, (eps, delta, p_max, xi, t, want)
        assert tail(t) <= delta < tail(t - 1)


def test_trajectory_bound_pin_catches_a_wrong_log_or_constant():
    """The derivation above separates Eq. 6 from plausible misreadings: a
    base-10 logarithm, or e^2 in place of 2 e^2 inside the logarithm."""
    def variant(eps, delta, p_max, xi, log, const):
        num = (math.sqrt(xi) + math.sqrt(p_max)) ** 2
        den = (math.sqrt(p_max + eps) - math.sqrt(p_max)) ** 2
        return math.ceil(2.0 * num / den * log(const / delta))

    for log, const in ((math.log10, 2 * math.e ** 2), (math.log, math.e ** 2), (math.log, 2.0)):
        wrong = sum(variant(*g, log, const) != _derived_count(*g)[0] for g in _EQ6_GRID)
        assert wrong == len(_EQ6_GRID), (log, const, wrong)


def test_amplitude_radius_bounds_the_probability_error():
    """Brute force over amplitudes |A|^2 <= p_max and estimates within r of A:
    the worst |p_hat - p| approaches eps and never exceeds it."""
    rng = np.random.default_rng(61)
    for eps, p_max in ((1e-3, 0.3), (0.05, 1.0), (0.02, 0.0)):
        r = _amplitude_radius(eps, p_max)
        a = np.sqrt(p_max) * np.sqrt(rng.uniform(0, 1, 20000)) * np.exp(2j * np.pi * rng.uniform(0, 1, 20000))
        a[:100] = math.sqrt(p_max)           # the extreme modulus
        d = r * np.sqrt(rng.uniform(0, 1, 20000)) * np.exp(2j * np.pi * rng.uniform(0, 1, 20000))
        d[:100] = r                          # aligned with the extreme amplitude
        err = np.abs(np.abs(a + d) ** 2 - np.abs(a) ** 2)
        assert err.max() <= eps * (1 + 1e-12)
        assert err.max() >= eps * (1 - 1e-9)


def test_sampled_determinants_are_bounded_by_one():
    """The step bound uses |det V(x)[R, C]| <= 1 (V(x) unitary): checked on
    the oracle's own determinant for submatrices of Haar unitaries."""
    rng = np.random.default_rng(62)
    worst = 0.0
    for _ in range(200):
        n = int(rng.integers(2, 12))
        m = int(rng.integers(1, n + 1))
        U = W.haar_unitary(rng, n)
        R = np.sort(rng.choice(n, m, replace=False))
        C = np.sort(rng.choice(n, m, replace=False))
        worst = max(worst, abs(oracle.det(U[np.ix_(R, C)])))
    assert worst <= 1.0 + 1e-12


def test_hayes_bound_holds_for_bounded_planar_walks():
    """Monte Carlo of worst-case-like planar martingales (steps of norm exactly
    1 in random directions, and +-1 along one axis): the empirical tail stays
    below the bound used above."""
    rng = np.random.default_rng(63)
    n, trials = 200, 20000
    ang = rng.uniform(0, 2 * np.pi, (trials, n))
    walks = [np.abs(np.exp(1j * ang).sum(1)), np.abs(rng.choice([-1.0, 1.0], (trials, n)).sum(1))]
    for x in walks:
        for a in (20.0, 30.0, 40.0):
            assert (x >= a).mean() <= _hayes_tail(a, n)
