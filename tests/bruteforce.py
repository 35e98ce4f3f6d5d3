"""Brute-force Jordan-Wigner state-vector simulation (tests only, n <= 14).

Independent of the determinant identity (Sec. II-B, Eq. 3) and of the
controlled-phase decomposition (Sec. III-B, Eq. 7): each rotation layer U is
applied as the many-body operator exp(sum_pq K_pq a_p^dag a_q) with K = log U
(second quantisation, via scipy's expm_multiply on the fixed-particle-number
sector), and each controlled-phase gate as the diagonal phase e^{i theta} on
basis states with both qubits set, exactly as the gate is defined.

Jordan-Wigner: a_p^dag |s> = (-1)^{sum_{i<p} s_i} |s + e_p> for s_p = 0, so the
ascending product a_{c1}^dag ... a_{cm}^dag |0> equals +|s>.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


def sector_basis(n: int, eta: int):
    states = [sum(1 << p for p in c) for c in combinations(range(n), eta)]
    index = {s: i for i, s in enumerate(states)}
    return states, index


def _parity_below(s: int, p: int) -> int:
    return bin(s & ((1 << p) - 1)).count("1") & 1


def one_body_operator(K: np.ndarray, states, index) -> scipy.sparse.csr_matrix:
    """Matrix of sum_pq K[p, q] a_p^dag a_q on the sector."""
    n = K.shape[0]
    rows, cols, vals = [], [], []
    for col, s in enumerate(states):
        for q in range(n):
            if not (s >> q) & 1:
                continue
            sq = s ^ (1 << q)
            sign_q = -1 if _parity_below(s, q) else 1
            for p in range(n):
                if (sq >> p) & 1:
                    continue
                if K[p, q] == 0:
                    continue
                sp = sq | (1 << p)
                sign_p = -1 if _parity_below(sq, p) else 1
                rows.append(index[sp])
                cols.append(col)
                vals.append(K[p, q] * sign_q * sign_p)
    d = len(states)
    return scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(d, d), dtype=np.complex128)


def statevector_amplitudes(rot, pairs, layer, theta, input_modes, n: int):
    """Amplitudes <b|circuit|a> for every b of the input's weight.

    Circuit (time order): rotation 0, the controlled-phase gates with
    layer == 0, rotation 1, ..., rotation n_rot-1.  Returns (states, amps)."""
    eta = len(input_modes)
    states, index = sector_basis(n, eta)
    psi = np.zeros(len(states), dtype=np.complex128)
    psi[index[sum(1 << p for p in input_modes)]] = 1.0
    n_rot = len(rot)
    for l in range(n_rot):
        K = scipy.linalg.logm(np.asarray(rot[l], dtype=np.complex128))
        G = one_body_operator(K, states, index)
        psi = scipy.sparse.linalg.expm_multiply(G, psi)
        if l + 1 < n_rot:
            for j in range(len(theta)):
                if layer[j] != l:
                    continue
                q1, q2 = int(pairs[j][0]), int(pairs[j][1])
                for i, s in enumerate(states):
                    if (s >> q1) & 1 and (s >> q2) & 1:
                        psi[i] *= np.exp(1j * theta[j])
    return states, psi


def bits_to_int(b) -> int:
    return int(b[0]) | (int(b[1]) << 64)


def gate_list_amplitudes(n: int, gates, input_bits: int) -> np.ndarray:
    """Full 2^n qubit state vector of a gate list applied to the basis state
    `input_bits` (bit p = qubit p): each gate's 4 x 4 matrix acts on its two
    qubits as written (basis |x_q0 x_q1> = 00, 01, 10, 11), a CPhase gate as
    diag(1, 1, 1, e^{i theta}).  No fermionic formalism."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[int(input_bits)] = 1.0
    idx = np.arange(1 << n)
    for g in gates:
        if g[0] == "mg":
            q0, q1, M = g[1], g[1] + 1, np.asarray(g[2], dtype=np.complex128)
        else:
            q0, q1 = g[1], g[2]
            M = np.diag([1.0, 1.0, 1.0, np.exp(1j * g[3])]).astype(np.complex128)
        sub = 2 * ((idx >> q0) & 1) + ((idx >> q1) & 1)
        base = idx & ~((1 << q0) | (1 << q1))
        new = np.zeros_like(psi)
        for out in range(4):
            tgt = base | (((out >> 1) & 1) << q0) | ((out & 1) << q1)
            np.add.at(new, tgt, M[out, sub] * psi)
        psi = new
    return psi
