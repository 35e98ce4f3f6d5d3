"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and its host-only helpers and argument validation behave
as documented (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def xf():
    import paper_2511_12416_amd as X
    return X


def header_functions():
    src = open(os.path.join(ROOT, "include", "xf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function(xf):
    names = header_functions()
    assert len(names) >= 12
    lib = xf.lib()
    for name in names:
        assert hasattr(lib, name), name
    from paper_2511_12416_amd import _abi
    assert sorted(_abi.EXPORTS) == names


def test_trajectory_bound_matches_oracle(xf):
    for args in [(0.01, 0.05, 0.1, 2.0), (1e-3, 1e-4, 1.0, 1.732), (0.05, 0.5, 0.0, 5.281)]:
        assert xf.trajectory_bound(*args) == oracle.trajectory_bound(*args)


@pytest.mark.parametrize("args", [(0.0, 0.1, 0.1, 1.0), (0.1, 0.0, 0.1, 1.0), (0.1, 1.0, 0.1, 1.0),
                                  (0.1, 0.1, 1.5, 1.0), (0.1, 0.1, 0.1, 0.5), (float("nan"), 0.1, 0.1, 1.0)])
def test_trajectory_bound_rejects_bad_arguments(xf, args):
    with pytest.raises(xf.XfError) as e:
        xf.trajectory_bound(*args)
    assert e.value.status == 1


def test_expm_and_adjoint(xf):
    rng = np.random.default_rng(4)
    for d, sigma in [(3, 0.1), (16, 0.1), (8, 3.0)]:
        K = W.anti_hermitian(rng, d, sigma)
        U = xf.expm_antihermitian(K)
        np.testing.assert_allclose(U, oracle.expm(K), atol=1e-13)
        np.testing.assert_allclose(U.conj().T @ U, np.eye(d), atol=1e-13)
        G = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        np.testing.assert_allclose(xf.expm_adjoint(K, G), oracle.expm_adjoint(K, G), atol=1e-12)


def test_spin_rotations_and_their_adjoint(xf):
    """exp(K) (+) exp(K) per layer, and its adjoint against central finite
    differences of L = Re sum conj(G) * R(K) along every anti-Hermitian
    direction E of every layer (dL = Re sum conj(G_K) * E)."""
    rng = np.random.default_rng(6)
    d, nl = 3, 2
    K = np.stack([W.anti_hermitian(rng, d, 0.4) for _ in range(nl)])
    R = xf.spin_rotations(K)
    for l in range(nl):
        np.testing.assert_allclose(R[l], W.block_diag2(oracle.expm(K[l])), atol=1e-13)
    G = rng.standard_normal((nl, 2 * d, 2 * d)) + 1j * rng.standard_normal((nl, 2 * d, 2 * d))
    GK = xf.spin_rotations_adjoint(K, G)
    loss = lambda KK: float(np.sum((np.conj(G) * xf.spin_rotations(KK)).real))
    h = 1e-6
    for l in range(nl):
        for i in range(d):
            for j in range(i, d):
                for unit in ((1.0, 1j) if i < j else (1j,)):
                    E = np.zeros_like(K)
                    E[l, i, j] += unit
                    E[l, j, i] -= np.conj(unit)
                    fd = (loss(K + h * E) - loss(K - h * E)) / (2 * h)
                    ref = float(np.sum((np.conj(GK) * E).real))
                    assert abs(fd - ref) < 1e-7, (l, i, j, unit, fd, ref)


def test_antihermitian_reals_grad(xf):
    """d/d(real parameters) of L = Re sum conj(G) * K(params) by central
    finite differences, K built from (Re K_ij, Im K_ij) for i < j and Im K_ii."""
    rng = np.random.default_rng(7)
    d = 4
    G = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    iu = np.triu_indices(d, 1)
    npair = len(iu[0])

    def build(x):
        K = np.zeros((d, d), np.complex128)
        K[iu] = x[:npair] + 1j * x[npair:2 * npair]
        K = K - K.conj().T
        K[np.diag_indices(d)] = 1j * x[2 * npair:]
        return K

    x0 = rng.standard_normal(d * d)
    g = xf.antihermitian_reals_grad(G)
    loss = lambda x: float(np.sum((np.conj(G) * build(x)).real))
    for q in range(d * d):
        e = np.zeros(d * d)
        e[q] = 1e-6
        fd = (loss(x0 + e) - loss(x0 - e)) / 2e-6
        assert abs(fd - g[q]) < 1e-8, (q, fd, g[q])


def test_expm_rejects_non_antihermitian(xf):
    with pytest.raises(xf.XfError) as e:
        xf.expm_antihermitian(np.array([[1.0, 0.0], [0.0, 0.0]]))
    assert e.value.status == 1


def _create(xf, rot, pairs, layer, theta, inp, precision=0):
    from paper_2511_12416_amd import _abi
    rot = np.ascontiguousarray(np.asarray(rot, np.complex128)).view(np.float64)
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    layer = np.ascontiguousarray(np.asarray(layer, np.int32).reshape(-1))
    theta = np.ascontiguousarray(np.asarray(theta, np.float64).reshape(-1))
    n_rot, n = rot.shape[0], rot.shape[1]
    circ = _abi.Circuit(n, n_rot, rot.ctypes.data, theta.shape[0], pairs.ctypes.data, layer.ctypes.data,
                        theta.ctypes.data)
    bits = _abi.Bits128()
    bits.w[0], bits.w[1] = int(inp[0]), int(inp[1])
    h = ctypes.c_void_p()
    st = xf.lib().xf_plan_create(ctypes.byref(circ), bits, precision, 0, ctypes.byref(h))
    return st, h


def test_plan_create_validation(xf):
    """Validation happens before any device call, so every error below is
    reported on a machine without a GPU too."""
    rng = W.rng_for(500)
    n = 6
    U = np.stack([W.haar_unitary(rng, n), W.haar_unitary(rng, n)])
    pairs = np.array([[0, 1], [2, 3]])
    layer = np.array([0, 0])
    theta = np.array([0.1, -0.2])
    inp = W.bits_from_modes([0, 1, 2])
    cases = [
        (dict(pairs=np.array([[0, 0], [2, 3]])), 1),          # q1 == q2
        (dict(pairs=np.array([[0, 6], [2, 3]])), 1),          # out of range
        (dict(layer=np.array([0, 1])), 1),                    # no CPhase layer 1 with 2 rotations
        (dict(theta=np.array([np.nan, 0.1])), 1),
        (dict(theta=np.array([7.0, 0.1])), 1),                # |theta| >= 2 pi
        (dict(rot=U * 1.01), 1),                              # not unitary
        (dict(inp=W.bits_from_modes([0, 7])), 1),             # input bit >= n
    ]
    for change, status in cases:
        args = dict(rot=U, pairs=pairs, layer=layer, theta=theta, inp=inp)
        args.update(change)
        st, h = _create(xf, **args)
        assert st == status, change
        assert not h.value
        assert len(xf.lib().xf_last_error()) > 0
    # n > 128, more than 65 rotation layers, and more than three with k > 63
    # are unsupported, not invalid
    big = np.stack([np.eye(130, dtype=np.complex128)] * 2)
    st, _ = _create(xf, big, pairs, layer, theta, inp)
    assert st == 2
    many = np.stack([np.eye(n, dtype=np.complex128)] * 66)
    st, _ = _create(xf, many, pairs, layer, theta, inp)
    assert st == 2
    k64 = 64
    four = np.stack([np.eye(n, dtype=np.complex128)] * 4)
    st, _ = _create(xf, four, np.array([[0, 1]] * k64), np.zeros(k64, np.int32), np.full(k64, 0.1), inp)
    assert st == 2


def test_null_arguments(xf):
    L = xf.lib()
    h = ctypes.c_void_p()
    from paper_2511_12416_amd import _abi
    assert L.xf_plan_create(None, _abi.Bits128(), 0, 0, ctypes.byref(h)) == 1
    assert L.xf_probabilities(None, None, 0, 0, 0, 0, None, None, None, None) == 1
    assert L.xf_extent(None, None) == 1
    assert L.xf_plan_destroy(None) == 0
