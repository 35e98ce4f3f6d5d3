"""CPU pins of gate-list ingestion (Sec. II-B: nearest-neighbour passive
matchgates G(A, B) and controlled-phase gates, grouped into rotation layers
and CPhase layers): the oracle's layered circuit against a brute-force qubit
state vector that applies every 4 x 4 gate as written, and the library's
ingestion (host code, no GPU) against the oracle's."""
import numpy as np
import pytest

import oracle
import workloads as W
from bruteforce import gate_list_amplitudes


def _int_bits(b) -> int:
    b = np.asarray(b, dtype=np.uint64).reshape(2)
    return int(b[0]) | (int(b[1]) << 64)


@pytest.mark.parametrize("seed,n,eta,ncp,per", [(61, 4, 2, 2, 3), (62, 6, 3, 3, 5), (63, 7, 3, 4, 4),
                                                (64, 8, 4, 3, None)])
def test_layered_circuit_matches_qubit_state_vector(seed, n, eta, ncp, per):
    gates, inp, bits = W.random_gate_circuit(seed, n, eta, ncp, per, theta_scale=2.0)
    rot, pairs, layer, theta = oracle.circuit_from_gates(n, gates)
    assert rot.shape[0] == ncp + 1 and len(theta) == ncp
    for R in rot:
        np.testing.assert_allclose(R.conj().T @ R, np.eye(n), atol=1e-12)
    psi = gate_list_amplitudes(n, gates, _int_bits(inp))
    ref = np.array([abs(psi[_int_bits(b)]) ** 2 for b in bits])
    p = oracle.probabilities(rot, pairs, layer, theta, inp, bits, "exact")
    np.testing.assert_allclose(p, ref, atol=1e-12)
    # the dropped vacuum phases are global: amplitudes agree up to one phase
    _, a = oracle.probabilities(rot, pairs, layer, theta, inp, bits, "exact", return_amp=True)
    ref_a = np.array([psi[_int_bits(b)] for b in bits])
    big = np.argmax(np.abs(ref_a))
    ph = ref_a[big] / a[big]
    assert abs(abs(ph) - 1) < 1e-10
    np.testing.assert_allclose(a * ph, ref_a, atol=1e-12)


def test_consecutive_cphase_gates_share_a_layer_and_edges_are_identity():
    rng = np.random.default_rng(5)
    G = W.random_matchgate(rng)
    gates = [("cp", 0, 2, 0.3), ("cp", 1, 3, -0.2), ("mg", 1, G), ("cp", 0, 1, 0.5)]
    rot, pairs, layer, theta = oracle.circuit_from_gates(4, gates)
    assert rot.shape[0] == 3
    np.testing.assert_array_equal(layer, [0, 0, 1])
    np.testing.assert_allclose(rot[0], np.eye(4))
    np.testing.assert_allclose(rot[2], np.eye(4))


def test_library_ingestion_matches_oracle():
    import paper_2511_12416_amd as X
    for seed, n, ncp in ((71, 6, 3), (72, 10, 5), (73, 12, 8)):
        gates, _, _ = W.random_gate_circuit(seed, n, n // 2, ncp, None, theta_scale=1.0)
        mine = X.circuit_from_gates(n, gates)
        ref = oracle.circuit_from_gates(n, gates)
        np.testing.assert_allclose(mine[0], ref[0], atol=1e-14)
        for a, b in zip(mine[1:], ref[1:]):
            np.testing.assert_array_equal(a, b)


def test_library_ingestion_rejects_non_passive_gates():
    import paper_2511_12416_amd as X
    G = np.eye(4, dtype=np.complex128)
    G[0, 0], G[0, 3], G[3, 0], G[3, 3] = 0, 1, 1, 0   # swaps |00> and |11>: not passive
    with pytest.raises(X.XfError) as e:
        X.circuit_from_gates(4, [("mg", 0, G)])
    assert e.value.status == 1
    with pytest.raises(X.XfError):
        X.circuit_from_gates(4, [("mg", 3, np.eye(4))])   # no neighbour q + 1
