"""Seeded synthetic inputs for the Born-rule probability path.

This module only draws inputs: rotation matrices (or their anti-Hermitian
generators), controlled-phase pairs and angles, the input occupation and the
output bitstrings.  It holds none of the simulation arithmetic, so both the
FP64 oracle and the HIP path can consume exactly the same inputs.

Conventions (shared by every consumer):
  * ``n`` modes; Jordan-Wigner qubit p <-> fermionic mode p.  For spinful
    workloads modes ``0..n/2-1`` are alpha orbitals and ``n/2..n-1`` beta.
  * ``rot``: complex128 array ``[n_rot, n, n]``; rotation layer 0 acts first.
    Column convention: the layer maps a_c^dagger to sum_r U[r, c] a_r^dagger.
  * ``pairs``: int32 ``[k, 2]``; ``layer``: int32 ``[k]`` (gate j sits after
    rotation layer ``layer[j]`` and before ``layer[j] + 1``); ``theta``: f64 ``[k]``.
  * bitstrings: uint64 ``[B, 2]`` (low word, high word); bit p <=> mode p.

Recipes follow the five named workloads: a tiny exact case, an LUCJ-shaped
approximate case, an exact stress case, a differentiation case with
generator-parametrised rotations, and a large-batch two-layer case.  Random
draws use NumPy's PCG64 seeded with ``2511124160 + workload number``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 2511124160


@dataclass
class Workload:
    name: str
    n: int
    input_bits: np.ndarray          # uint64 [2]
    rot: Optional[np.ndarray]       # complex128 [n_rot, n, n] (None if gens given)
    pairs: np.ndarray               # int32 [k, 2]
    layer: np.ndarray               # int32 [k]
    theta: np.ndarray               # float64 [k]
    bits: np.ndarray                # uint64 [B, 2]
    mode: str                       # "exact" | "approx"
    t: int = 0                      # samples per bitstring (approx mode)
    seed: int = 0                   # sampler seed (approx mode)
    gens: Optional[np.ndarray] = None   # complex128 [n_rot, n/2, n/2] anti-Hermitian
    n_rot: int = 2
    extra: dict = field(default_factory=dict)

    @property
    def k(self) -> int:
        return int(self.theta.shape[0])

    @property
    def B(self) -> int:
        return int(self.bits.shape[0])

    @property
    def eta(self) -> int:
        return popcount128(self.input_bits)


# ----------------------------------------------------------------------------
# elementary draws
# ----------------------------------------------------------------------------

def rng_for(cfg: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + cfg))


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-distributed d x d unitary: QR of a complex Gaussian matrix with the
    phases of R's diagonal moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diagonal(r) / np.abs(np.diagonal(r))
    return q * ph[None, :]


def anti_hermitian(rng: np.random.Generator, d: int, sigma: float) -> np.ndarray:
    """Anti-Hermitian generator: Re and Im of each upper off-diagonal entry and
    Im of each diagonal entry are N(0, sigma^2)."""
    k = np.zeros((d, d), dtype=np.complex128)
    iu = np.triu_indices(d, 1)
    re = rng.standard_normal(len(iu[0])) * sigma
    im = rng.standard_normal(len(iu[0])) * sigma
    k[iu] = re + 1j * im
    k = k - k.conj().T
    k[np.diag_indices(d)] = 1j * rng.standard_normal(d) * sigma
    return k


def block_diag2(u: np.ndarray) -> np.ndarray:
    d = u.shape[0]
    out = np.zeros((2 * d, 2 * d), dtype=np.complex128)
    out[:d, :d] = u
    out[d:, d:] = u
    return out


def bits_from_modes(modes) -> np.ndarray:
    lo = 0
    hi = 0
    for p in modes:
        p = int(p)
        if p < 64:
            lo |= 1 << p
        else:
            hi |= 1 << (p - 64)
    return np.array([lo, hi], dtype=np.uint64)


def modes_from_bits(b) -> list:
    lo, hi = int(b[0]), int(b[1])
    out = [p for p in range(64) if (lo >> p) & 1]
    out += [64 + p for p in range(64) if (hi >> p) & 1]
    return out


def popcount128(b) -> int:
    return bin(int(b[0])).count("1") + bin(int(b[1])).count("1")


def random_fixed_weight(rng: np.random.Generator, modes: np.ndarray, w: int, count: int) -> list:
    """``count`` draws (with replacement across draws) of a uniformly random
    ``w``-subset of ``modes``."""
    out = []
    for _ in range(count):
        out.append(np.sort(rng.choice(modes, size=w, replace=False)))
    return out


def spin_bitstrings(rng: np.random.Generator, norb: int, na: int, nb: int, count: int) -> np.ndarray:
    """Bitstrings uniform at fixed (alpha, beta) occupation (alpha modes
    0..norb-1, beta modes norb..2norb-1)."""
    a = np.arange(norb)
    bits = np.zeros((count, 2), dtype=np.uint64)
    for i in range(count):
        sa = rng.choice(a, size=na, replace=False)
        sb = rng.choice(a, size=nb, replace=False) + norb
        bits[i] = bits_from_modes(np.concatenate([sa, sb]))
    return bits


def all_fixed_weight(n: int, w: int) -> np.ndarray:
    from itertools import combinations
    rows = [bits_from_modes(c) for c in combinations(range(n), w)]
    return np.array(rows, dtype=np.uint64).reshape(-1, 2)


def lucj_pairs(norb: int) -> np.ndarray:
    """Controlled-phase pair pattern of an LUCJ layer: same-spin nearest
    neighbours (i, i+1) in each spin sector, then alpha-beta pairs on the same
    orbital (i, norb + i)."""
    pairs = [(i, i + 1) for i in range(norb - 1)]
    pairs += [(norb + i, norb + i + 1) for i in range(norb - 1)]
    pairs += [(i, norb + i) for i in range(norb)]
    return np.array(pairs, dtype=np.int32)


def random_pairs(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """``k`` distinct unordered mode pairs, uniform over all C(n, 2)."""
    chosen = set()
    out = []
    while len(out) < k:
        q = rng.choice(n, size=2, replace=False)
        key = (int(min(q)), int(max(q)))
        if key in chosen:
            continue
        chosen.add(key)
        out.append(key)
    return np.array(out, dtype=np.int32)


# ----------------------------------------------------------------------------
# the five named workloads
# ----------------------------------------------------------------------------

def workload(cfg: int, B: Optional[int] = None) -> Workload:
    """Workload ``cfg`` (1..5).  ``B`` truncates the bitstring batch (the
    draws are made for the full batch first so a prefix is stable)."""
    rng = rng_for(cfg)
    if cfg == 1:
        n = 8
        u1 = haar_unitary(rng, n)
        u2 = haar_unitary(rng, n)
        pairs = random_pairs(rng, n, 2)
        theta = rng.uniform(-0.3, 0.3, size=2)
        w = Workload("exact n=8 eta=4 k=2", n, bits_from_modes(range(4)),
                     np.stack([u1, u2]), pairs, np.zeros(2, np.int32), theta,
                     all_fixed_weight(n, 4), "exact")
    elif cfg == 2:
        norb = 16
        n = 2 * norb
        u0 = haar_unitary(rng, norb)
        u1 = haar_unitary(rng, norb)
        pairs = lucj_pairs(norb)
        theta = rng.normal(0.0, 0.05, size=pairs.shape[0])
        bits = spin_bitstrings(rng, norb, 8, 8, 10_000)
        w = Workload("LUCJ n=32 eta=8a+8b k=46 t=2^14 B=1e4", n,
                     bits_from_modes(list(range(8)) + list(range(16, 24))),
                     np.stack([block_diag2(u0), block_diag2(u1)]), pairs,
                     np.zeros(pairs.shape[0], np.int32), theta, bits, "approx",
                     t=1 << 14, seed=0x5EED0002)
    elif cfg == 3:
        norb = 26
        n = 2 * norb
        u0 = haar_unitary(rng, n)
        u1 = haar_unitary(rng, n)
        pairs = random_pairs(rng, n, 12)
        theta = rng.uniform(-0.5, 0.5, size=12)
        modes = np.arange(n)
        sel = random_fixed_weight(rng, modes, 26, 4096)
        bits = np.array([bits_from_modes(s) for s in sel], dtype=np.uint64)
        w = Workload("exact stress n=52 eta=26 k=12 B=4096", n,
                     bits_from_modes(list(range(13)) + list(range(26, 39))),
                     np.stack([u0, u1]), pairs, np.zeros(12, np.int32), theta,
                     bits, "exact")
    elif cfg == 4:
        norb = 16
        n = 2 * norb
        g0 = anti_hermitian(rng, norb, 0.1)
        g1 = anti_hermitian(rng, norb, 0.1)
        allp = lucj_pairs(norb)
        idx = np.sort(rng.choice(allp.shape[0], size=24, replace=False))
        pairs = allp[idx].copy()
        theta = rng.normal(0.0, 0.1, size=24)
        bits = spin_bitstrings(rng, norb, 8, 8, 4096)
        w = Workload("differentiation n=32 eta=8a+8b k=24 t=2^14 B=4096", n,
                     bits_from_modes(list(range(8)) + list(range(16, 24))),
                     None, pairs, np.zeros(24, np.int32), theta, bits, "approx",
                     t=1 << 14, seed=0x5EED0004, gens=np.stack([g0, g1]))
    elif cfg == 5:
        norb = 50
        n = 2 * norb
        us = [haar_unitary(rng, norb) for _ in range(3)]
        p1 = random_pairs(rng, n, 20)
        p2 = random_pairs(rng, n, 20)
        pairs = np.concatenate([p1, p2]).astype(np.int32)
        layer = np.array([0] * 20 + [1] * 20, dtype=np.int32)
        theta = rng.uniform(-0.05, 0.05, size=40)
        bits = spin_bitstrings(rng, norb, 25, 25, 100_000 if B is None else max(B, 1000))
        w = Workload("large batch n=100 eta=25a+25b k=40 L=2 t=2^16 B=1e5", n,
                     bits_from_modes(list(range(25)) + list(range(50, 75))),
                     np.stack([block_diag2(u) for u in us]), pairs, layer, theta,
                     bits, "approx", t=1 << 16, seed=0x5EED0005, n_rot=3)
    else:
        raise ValueError(f"unknown workload {cfg}")
    if w.rot is not None:
        w.n_rot = w.rot.shape[0]
    if B is not None:
        w.bits = w.bits[:B].copy()
    return w


def random_circuit(seed: int, n: int, eta: int, k: int, n_rot: int = 2,
                   theta_scale: float = 1.0, spin: bool = False,
                   input_modes=None, max_bits: int = 4096) -> Workload:
    """Small random circuit for tests: Haar rotation layers, ``k`` CPhase gates
    on random distinct pairs spread over the ``n_rot - 1`` CPhase layers,
    angles uniform in [-theta_scale, theta_scale]; all weight-``eta`` outputs
    when there are at most ``max_bits`` of them, else ``max_bits`` uniform
    draws of weight-``eta`` outputs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if spin:
        norb = n // 2
        rot = np.stack([block_diag2(haar_unitary(rng, norb)) for _ in range(n_rot)])
    else:
        rot = np.stack([haar_unitary(rng, n) for _ in range(n_rot)])
    pairs = random_pairs(rng, n, k) if k <= n * (n - 1) // 2 else \
        np.array([rng.choice(n, 2, replace=False) for _ in range(k)], dtype=np.int32)
    layer = (rng.integers(0, n_rot - 1, size=k) if n_rot > 1 else np.zeros(k)).astype(np.int32)
    theta = rng.uniform(-theta_scale, theta_scale, size=k)
    if input_modes is None:
        input_modes = list(range(eta))
    from math import comb
    if comb(n, eta) <= max_bits:
        bits = all_fixed_weight(n, eta)
    else:
        sel = random_fixed_weight(rng, np.arange(n), eta, max_bits)
        bits = np.array([bits_from_modes(x) for x in sel], dtype=np.uint64).reshape(-1, 2)
    return Workload(f"random n={n} eta={eta} k={k}", n, bits_from_modes(input_modes),
                    rot, pairs, layer, theta, bits, "exact", n_rot=n_rot)


def random_matchgate(rng: np.random.Generator) -> np.ndarray:
    """A random particle-number-conserving matchgate G(A, B) (4 x 4, basis
    |x_q x_{q+1}> = 00, 01, 10, 11): A = diag(e^{i a}, e^{i b}) and B a Haar
    2 x 2 unitary rescaled so that det B = det A."""
    a, b = rng.uniform(-np.pi, np.pi, size=2)
    B = haar_unitary(rng, 2)
    B = B * np.sqrt(np.exp(1j * (a + b)) / np.linalg.det(B))
    G = np.zeros((4, 4), dtype=np.complex128)
    G[0, 0], G[3, 3] = np.exp(1j * a), np.exp(1j * b)
    G[1:3, 1:3] = B
    return G


def random_gate_circuit(seed: int, n: int, eta: int, n_cphase: int, mg_per_layer: Optional[int] = None,
                        theta_scale: float = 1.0, max_bits: int = 4096):
    """A random interleaved circuit given gate by gate, shaped like the
    paper's random extended-matchgate benchmark: layers of nearest-neighbour
    matchgates (``mg_per_layer``, default n - 1, on random neighbour pairs)
    each followed by one CPhase gate on a random distinct pair, angles uniform
    in [-theta_scale, theta_scale], with a closing matchgate layer.  Returns
    (gates, input_bits, output bitstrings): gates as ("mg", q, G) and
    ("cp", q0, q1, theta) in time order, the input the first eta modes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per = n - 1 if mg_per_layer is None else mg_per_layer
    gates = []
    for layer in range(n_cphase + 1):
        for _ in range(per):
            q = int(rng.integers(0, n - 1))
            gates.append(("mg", q, random_matchgate(rng)))
        if layer < n_cphase:
            q0, q1 = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append(("cp", q0, q1, float(rng.uniform(-theta_scale, theta_scale))))
    from itertools import combinations
    from math import comb
    if comb(n, eta) <= max_bits:
        bits = np.array([bits_from_modes(c) for c in combinations(range(n), eta)], dtype=np.uint64)
    else:
        sel = random_fixed_weight(rng, np.arange(n), eta, max_bits)
        bits = np.array([bits_from_modes(c) for c in sel], dtype=np.uint64)
    return gates, bits_from_modes(range(eta)), bits


def nearby_outcomes(seed: int, n: int, input_modes, count: int, hops: int = 3) -> np.ndarray:
    """``count`` outcomes reached from the input occupation by ``hops``
    random moves of one particle to a free neighbouring mode: the outcomes a
    circuit of nearest-neighbour matchgates puts most of its weight on (an
    outcome far from the input has a negligible probability).  Distinct,
    seeded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    start = sorted(int(q) for q in input_modes)
    seen, out = set(), []
    for _ in range(count * 200):
        occ = set(start)
        for _ in range(hops):
            q = int(rng.choice(sorted(occ)))
            d = int(rng.choice([-1, 1]))
            if 0 <= q + d < n and q + d not in occ:
                occ.remove(q)
                occ.add(q + d)
        key = tuple(sorted(occ))
        if key not in seen:
            seen.add(key)
            out.append(bits_from_modes(key))
        if len(out) == count:
            break
    return np.array(out, dtype=np.uint64)
