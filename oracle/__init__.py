"""FP64 CPU oracle for the Born-rule probability path (ExtraFerm, arXiv 2511.12416).

TEST INFRASTRUCTURE ONLY: this package may be imported by the test-suite, by
the smoke check and by the benchmark's CPU-baseline leg, nothing else.  It
shares no code with the HIP library.  The heavy part (``xfo.c``) is plain C:
explicit mode-matrix products, a textbook partial-pivot LU, the exact sum over
all 2^k trajectories (Sec. III-B, Eq. 8) or the Raw Estimate average over
sampled trajectories (Sec. III-A, Eq. 10-12).  The small closed forms (extent,
Eq. 5; trajectory bound, Eq. 6) and the matrix exponential of rotation
generators with its adjoint are written here in NumPy/SciPy.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xfo.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle.  No FMA contraction, baseline x86-64 ISA, so the
    FP64 sampler thresholds are computed operation by operation as written."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11",
                               "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.xfo_philox4x32_10.argtypes = [P, P, P]
        L.xfo_sampler_table.argtypes = [ctypes.c_int, P, P]
        L.xfo_sample_trajectories.argtypes = [ctypes.c_int, P, ctypes.c_uint64, ctypes.c_uint64,
                                              ctypes.c_int64, P]
        L.xfo_det.argtypes = [ctypes.c_int, P, P]
        L.xfo_extent.argtypes = [ctypes.c_int, P]
        L.xfo_extent.restype = ctypes.c_double
        sig = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P, P, P, ctypes.c_int64, P, P,
               ctypes.c_int, ctypes.c_int64, ctypes.c_uint64]
        L.xfo_probabilities.argtypes = sig + [P, P, P]
        L.xfo_probabilities.restype = ctypes.c_int
        L.xfo_log_prob_grad.argtypes = sig + [P, P, P]
        L.xfo_log_prob_grad.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ----------------------------------------------------------------------------
# closed forms
# ----------------------------------------------------------------------------

def extent(theta) -> float:
    """Eq. 5: xi* = prod_j (cos(|theta_j|/4) + sin(|theta_j|/4))^2."""
    th = np.abs(np.asarray(theta, dtype=np.float64))
    return float(np.prod((np.cos(th / 4) + np.sin(th / 4)) ** 2))


def trajectory_bound(eps: float, delta: float, p_max: float, xi: float) -> int:
    """Eq. 6 (natural logarithm):
    t = ceil( 2 (sqrt(xi) + sqrt(p_max))^2 / (sqrt(p_max + eps) - sqrt(p_max))^2
              * log(2 e^2 / delta) )."""
    num = (math.sqrt(xi) + math.sqrt(p_max)) ** 2
    den = (math.sqrt(p_max + eps) - math.sqrt(p_max)) ** 2
    return int(math.ceil(2.0 * num / den * math.log(2.0 * math.e ** 2 / delta)))


def sampling_probability(theta) -> np.ndarray:
    """Eq. 11: p(x_j = 1) = sin(|theta|/4) / (sin(|theta|/4) + cos(|theta|/4))."""
    th = np.abs(np.asarray(theta, dtype=np.float64))
    s, c = np.sin(th / 4), np.cos(th / 4)
    return s / (s + c)


def expm(K: np.ndarray) -> np.ndarray:
    import scipy.linalg
    return scipy.linalg.expm(np.asarray(K, dtype=np.complex128))


def expm_adjoint(K: np.ndarray, G_U: np.ndarray) -> np.ndarray:
    """Gradient with respect to K (dL/dRe K + i dL/dIm K) of a real loss whose
    gradient with respect to U = exp(K) is G_U, via the adjoint of the
    Frechet derivative: L(K, .)^* = L(K^H, .)."""
    import scipy.linalg
    K = np.asarray(K, dtype=np.complex128)
    _, L = scipy.linalg.expm_frechet(K.conj().T, np.asarray(G_U, dtype=np.complex128))
    return L


def rotations_from_generators(gens: np.ndarray) -> np.ndarray:
    """Spin-restricted layers exp(K_l) (+) exp(K_l)."""
    out = []
    for K in gens:
        U = expm(K)
        d = U.shape[0]
        R = np.zeros((2 * d, 2 * d), dtype=np.complex128)
        R[:d, :d] = U
        R[d:, d:] = U
        out.append(R)
    return np.stack(out)


# ----------------------------------------------------------------------------
# wrappers of the C oracle
# ----------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().xfo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sampler_table(theta) -> np.ndarray:
    th = _c(theta, np.float64)
    k = th.shape[0]
    T = np.zeros((max(k, 1), max(k, 1)), np.uint32)
    lib().xfo_sampler_table(k, _ptr(th), _ptr(T))
    return T[:k, :k]


def sample_trajectories(theta, seed: int, bidx: int, t: int) -> np.ndarray:
    """[t, 2] uint64 trajectory bitmasks (bit j <=> x_j = 1)."""
    th = _c(theta, np.float64)
    out = np.zeros((t, 2), np.uint64)
    lib().xfo_sample_trajectories(th.shape[0], _ptr(th), seed, bidx, t, _ptr(out))
    return out


def det(a: np.ndarray) -> complex:
    a = _c(a, np.complex128)
    m = a.shape[0]
    out = np.zeros(2)
    lib().xfo_det(m, _ptr(a), _ptr(out))
    return complex(out[0], out[1])


def _circuit_args(rot, pairs, layer, theta, input_bits):
    rot = _c(rot, np.complex128)
    n_rot, n, _ = rot.shape
    pairs = _c(pairs, np.int32).reshape(-1, 2)
    layer = _c(layer, np.int32)
    theta = _c(theta, np.float64)
    inp = _c(input_bits, np.uint64)
    return rot, n, n_rot, pairs, layer, theta, inp


def _theta_sample(theta_sample):
    if theta_sample is None:
        return None, None
    ts = _c(theta_sample, np.float64)
    return ts, _ptr(ts)


def _batch_index(batch_index, B):
    if batch_index is None:
        return None, None
    bi = np.ascontiguousarray(np.asarray(batch_index, dtype=np.uint64).reshape(-1))
    assert bi.shape[0] == B
    return bi, _ptr(bi)


def probabilities(rot, pairs, layer, theta, input_bits, bits, mode="exact", t=0, seed=0,
                  return_amp=False, theta_sample=None, batch_index=None, return_abs_sum=False):
    """Born-rule probabilities p_b (exact, Eq. 8) or Raw Estimate p_hat_b.
    ``theta_sample`` freezes the sampling table at other angles;
    ``batch_index[b]`` is the index keying bitstring b's samples (default b);
    ``return_abs_sum`` appends sum_i |w_i det M_i| over the bitstring's terms."""
    rot, n, n_rot, pairs, layer, theta, inp = _circuit_args(rot, pairs, layer, theta, input_bits)
    ts_keep, ts_ptr = _theta_sample(theta_sample)
    bits = _c(bits, np.uint64).reshape(-1, 2)
    B = bits.shape[0]
    bi_keep, bi_ptr = _batch_index(batch_index, B)
    prob = np.zeros(B)
    amp = np.zeros((B, 2))
    abss = np.zeros(B)
    md = 0 if mode == "exact" else 1
    rc = lib().xfo_probabilities(n, n_rot, _ptr(rot), theta.shape[0], _ptr(pairs), _ptr(layer),
                                 _ptr(theta), ts_ptr, _ptr(inp), B, _ptr(bits), bi_ptr, md, int(t), int(seed),
                                 _ptr(prob), _ptr(amp), _ptr(abss))
    if rc != 0:
        raise ValueError("oracle: unsupported sizes")
    out = (prob,)
    if return_amp:
        out += (amp[:, 0] + 1j * amp[:, 1],)
    if return_abs_sum:
        out += (abss,)
    return out[0] if len(out) == 1 else out


def log_prob_grad(rot, pairs, layer, theta, input_bits, bits, g, mode="exact", t=0, seed=0,
                  theta_sample=None, batch_index=None):
    """(dL/drot, dL/dtheta) for L = sum_b g_b log p_b; rotation gradients in
    the dL/dRe + i dL/dIm convention.  Raw Estimate samples are held fixed."""
    rot, n, n_rot, pairs, layer, theta, inp = _circuit_args(rot, pairs, layer, theta, input_bits)
    ts_keep, ts_ptr = _theta_sample(theta_sample)
    bits = _c(bits, np.uint64).reshape(-1, 2)
    g = _c(g, np.float64)
    B = bits.shape[0]
    bi_keep, bi_ptr = _batch_index(batch_index, B)
    grot = np.zeros((n_rot, n, n, 2))
    gth = np.zeros(max(theta.shape[0], 1))
    md = 0 if mode == "exact" else 1
    rc = lib().xfo_log_prob_grad(n, n_rot, _ptr(rot), theta.shape[0], _ptr(pairs), _ptr(layer),
                                 _ptr(theta), ts_ptr, _ptr(inp), B, _ptr(bits), bi_ptr, md, int(t), int(seed),
                                 _ptr(g), _ptr(grot), _ptr(gth))
    if rc != 0:
        raise ValueError("oracle: unsupported sizes")
    return grot[..., 0] + 1j * grot[..., 1], gth[:theta.shape[0]]


def circuit_from_gates(n: int, gates):
    """Layered circuit (rot [n_rot, n, n], pairs, layer, theta) of a gate list
    in time order (Sec. II-B): a matchgate ("mg", q, G) on qubits (q, q + 1)
    maps the one-particle state a_c^dag|0> (c in {q, q + 1}; |10> and |01> in
    the basis |x_q x_{q+1}>) to sum_r U[r, c] a_r^dag|0>, U[r, c] being the
    matrix element of G between those states divided by the vacuum phase
    G[00, 00]; the layer's mode matrix is the product of its gates' embedded
    2 x 2 blocks, later gates on the left.  CPhase gates ("cp", q0, q1, theta)
    between two runs of matchgates form one CPhase layer."""
    one = {0: 2, 1: 1}   # basis index of a_q^dag|0> (offset 0) and a_{q+1}^dag|0> (offset 1)
    layers = [np.eye(n, dtype=np.complex128)]
    pairs, layer, theta = [], [], []
    prev_cp = False
    for g in gates:
        if g[0] == "cp":
            if not prev_cp:
                layers.append(np.eye(n, dtype=np.complex128))
            pairs.append((g[1], g[2]))
            layer.append(len(layers) - 2)
            theta.append(g[3])
            prev_cp = True
        else:
            q, G = g[1], np.asarray(g[2], dtype=np.complex128)
            E = np.eye(n, dtype=np.complex128)
            for dr in (0, 1):
                for dc in (0, 1):
                    E[q + dr, q + dc] = G[one[dr], one[dc]] / G[0, 0]
            layers[-1] = E @ layers[-1]
            prev_cp = False
    return (np.stack(layers), np.array(pairs, dtype=np.int32).reshape(-1, 2), np.array(layer, dtype=np.int32),
            np.array(theta, dtype=np.float64))


def sample_gates(n: int, gates, input_bits, S: int, mode: str = "exact", t: int = 0, seed: int = 0):
    """Weak simulation by the gate-by-gate algorithm (Bravyi, Gosset and Liu,
    2022; Sec. II-A names it): S chains start at the input; at matchgate gi
    on (q, q + 1) every chain with one particle on the pair moves to c10 or
    c01 with the probabilities of the circuit of gates 0..gi (Exact or Raw
    Estimate with t samples and seed + gi; candidates of the moving chains in
    chain order, c10 first), taking c10 when u (p10 + p01) < p10 with
    u = word 0 of Philox4x32-10 at (lo32(s), gi, 2^32 - 2, hi32(s)) times
    2^-32; CPhase gates change nothing.  Returns [S, 2] uint64."""
    inp = np.asarray(input_bits, dtype=np.uint64).reshape(2)
    x = [(int(inp[0]) | (int(inp[1]) << 64)) for _ in range(S)]
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    for gi, g in enumerate(gates):
        if g[0] != "mg":
            continue
        q = g[1]
        movers = [s for s in range(S) if ((x[s] >> q) & 1) + ((x[s] >> (q + 1)) & 1) == 1]
        if not movers:
            continue
        cands = []
        for s in movers:
            base = x[s] & ~((1 << q) | (1 << (q + 1)))
            cands += [base | (1 << q), base | (1 << (q + 1))]
        rot, pairs, layer, theta = circuit_from_gates(n, gates[:gi + 1])
        cb = np.array([[c & 0xFFFFFFFFFFFFFFFF, c >> 64] for c in cands], dtype=np.uint64)
        pr = probabilities(rot, pairs, layer, theta, inp, cb, mode, t=t, seed=(seed + gi) % (1 << 64))
        for a, s in enumerate(movers):
            p10, p01 = float(pr[2 * a]), float(pr[2 * a + 1])
            if not p10 + p01 > 0.0:
                continue
            w = int(philox4x32_10([s & 0xFFFFFFFF, gi, 0xFFFFFFFE, s >> 32], key)[0])
            u = w * 2.0 ** -32
            x[s] = cands[2 * a] if u * (p10 + p01) < p10 else cands[2 * a + 1]
    return np.array([[v & 0xFFFFFFFFFFFFFFFF, v >> 64] for v in x], dtype=np.uint64).reshape(-1, 2)


def round_to_four_bits(t: int) -> int:
    """The smallest integer >= t of the form m * 2^e with m < 16."""
    e = max(0, t.bit_length() - 4)
    return -(-t // (1 << e)) << e


def estimate(rot, pairs, layer, theta, input_bits, bits, eps, delta, seed=0):
    """Estimate (Sec. III-A): repeated Raw Estimate calls that tighten each
    bitstring's probability bound.  The paper names the algorithm without a
    schedule; this one halves the error target each round
    (eps_i = max(eps, 2^-i)), spends delta_i = delta 2^-i of the failure
    budget, takes t_b from Eq. 6 at the current bound p_max_b (rounded up to
    four significant bits), runs Raw Estimate once per distinct t_b over the
    bitstrings with that t_b (ascending batch index, seed + i - 1, samples
    keyed by the position in that group), and lowers p_max_b to
    p_hat_b + eps_i until eps_i = eps.  Returns (p_hat, last t_b, rounds)."""
    bits = np.ascontiguousarray(np.asarray(bits, dtype=np.uint64).reshape(-1, 2))
    B = bits.shape[0]
    xi = extent(theta)
    p_max = np.ones(B)
    p_hat = np.zeros(B)
    t_b = np.zeros(B, dtype=np.int64)
    i = 0
    while True:
        i += 1
        eps_i = max(eps, 2.0 ** -i)
        delta_i = delta * 2.0 ** -i
        t_b = np.array([round_to_four_bits(trajectory_bound(eps_i, delta_i, float(pm), xi)) for pm in p_max],
                       dtype=np.int64)
        for tv in sorted(set(t_b.tolist())):
            members = np.nonzero(t_b == tv)[0]   # ascending batch index
            p_hat[members] = probabilities(rot, pairs, layer, theta, input_bits, bits[members], "approx",
                                           t=int(tv), seed=(seed + i - 1) % (1 << 64),
                                           batch_index=np.arange(len(members)))
        if eps_i == eps:
            return p_hat, t_b, i
        p_max = np.minimum(p_max, np.minimum(1.0, p_hat + eps_i))


def run_workload(w, index=None, mode=None, return_amp=False, return_abs_sum=False):
    """Oracle probabilities for a ``workloads.Workload``, optionally for the
    batch positions ``index`` only (their samples keyed by those positions)."""
    rot = w.rot if w.rot is not None else rotations_from_generators(w.gens)
    bits = w.bits if index is None else w.bits[np.asarray(index)]
    return probabilities(rot, w.pairs, w.layer, w.theta, w.input_bits, bits,
                         mode or w.mode, w.t, w.seed, return_amp=return_amp,
                         batch_index=None if index is None else np.asarray(index),
                         return_abs_sum=return_abs_sum)
