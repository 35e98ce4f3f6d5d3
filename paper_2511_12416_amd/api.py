"""Python view of the C ABI: plans, probabilities and gradients.

Only argument marshalling happens here: host arrays are packed into the
interleaved (re, im) layout the ABI expects, device tensors are passed by
pointer together with torch's current HIP stream.  Every step of the
computation runs in libxf.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _abi
from ._abi import check, lib

_MODES = {"exact": _abi.XF_EXACT, "approx": _abi.XF_RAW_ESTIMATE, "raw_estimate": _abi.XF_RAW_ESTIMATE}
_PREC = {"fp64": _abi.XF_FP64, "mixed": _abi.XF_MIXED}
_EVAL = {"auto": 0, "lu": 1, "patterns": 2}


def _f64(a) -> np.ndarray:
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a)


def _complex_host(a) -> np.ndarray:
    """complex array -> contiguous float64 [..., 2]."""
    a = _f64(a)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a.astype(np.complex128)).view(np.float64).reshape(*a.shape, 2)
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def bits_tensor(bits, device="cuda") -> torch.Tensor:
    """[B, 2] uint64 bit patterns as an int64 tensor on ``device``."""
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint64).reshape(-1, 2))
    return torch.from_numpy(b.view(np.int64)).to(device)


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A circuit (rotation layers, CPhase pairs / layers / angles) bound to an
    input occupation, a precision and a HIP device."""

    def __init__(self, rot, pairs, layer, theta, input_bits, precision: str = "fp64", device: int = 0):
        L = lib()
        self._rot = _complex_host(rot)
        n_rot, n = self._rot.shape[0], self._rot.shape[1]
        self._pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        self._layer = np.ascontiguousarray(np.asarray(layer, dtype=np.int32).reshape(-1))
        self._theta = np.ascontiguousarray(_f64(theta), dtype=np.float64).reshape(-1)
        k = self._theta.shape[0]
        circ = _abi.Circuit(n, n_rot, self._rot.ctypes.data, k, self._pairs.ctypes.data,
                            self._layer.ctypes.data, self._theta.ctypes.data)
        ib = np.asarray(input_bits, dtype=np.uint64).reshape(2)
        bits = _abi.Bits128()
        bits.w[0], bits.w[1] = int(ib[0]), int(ib[1])
        h = ctypes.c_void_p()
        check(L.xf_plan_create(ctypes.byref(circ), bits, _PREC[precision], int(device), ctypes.byref(h)))
        self._h = h
        self.n, self.n_rot, self.k = n, n_rot, k
        self.eta = int(bin(int(ib[0])).count("1") + bin(int(ib[1])).count("1"))
        self.device = torch.device("cuda", int(device))
        self.precision = precision

    # -- lifetime -----------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().xf_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- parameters ---------------------------------------------------------
    def set_params(self, rot=None, theta=None) -> None:
        r = _complex_host(rot) if rot is not None else None
        th = np.ascontiguousarray(_f64(theta), dtype=np.float64).reshape(-1) if theta is not None else None
        check(lib().xf_plan_set_params(self._h, _ptr(r) if r is not None else None,
                                       _ptr(th) if th is not None else None))

    def refreeze(self) -> None:
        check(lib().xf_plan_refreeze(self._h))

    def extent(self) -> float:
        xi = ctypes.c_double()
        check(lib().xf_extent(self._h, ctypes.byref(xi)))
        return xi.value

    def last_term_count(self, with_rank: bool = False):
        """Determinants evaluated by the last probabilities() call (and, with
        ``with_rank``, the summed rank of their low-rank corrections)."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        check(lib().xf_plan_last_term_count(self._h, ctypes.byref(c), ctypes.byref(r)))
        return (c.value, r.value) if with_rank else c.value

    def last_work(self) -> dict:
        """Work of the last probabilities() call: determinants, summed rank of
        their corrections, FP64-equivalent FLOPs executed, kernel times in ms
        (sampling and evaluation kernels under the determinant lemma), and
        whether the lemma was used."""
        w = _abi.Work()
        check(lib().xf_plan_last_work(self._h, ctypes.byref(w)))
        return {"determinants": w.determinants, "rank_sum": w.rank_sum, "flops": w.flops,
                "sample_ms": w.sample_ms, "eval_ms": w.eval_ms, "lemma": bool(w.lemma),
                "backward_lemma": bool(w.backward_lemma), "general": bool(w.general),
                "backward_reused": bool(w.backward_reused),
                "fp32_bases": w.fp32_bases, "philox_blocks": w.philox_blocks,
                "tree_bitstrings": w.tree_bitstrings}

    def set_evaluation(self, evaluation: str) -> None:
        """"auto" (determinant lemma where it applies; exact mode along the
        term list's prefix tree where it applies), "patterns" (the lemma, each
        pattern's determinant on its own) or "lu" (LU of every distinct
        submatrix)."""
        if evaluation not in _EVAL:
            raise ValueError(f"evaluation must be one of {sorted(_EVAL)}")
        check(lib().xf_plan_set_evaluation(self._h, _EVAL[evaluation]))

    def set_mixed_condition(self, kappa_max: float) -> None:
        """Mixed precision: bases with kappa_1 <= kappa_max form H on the FP32
        matrix cores, others in FP64."""
        check(lib().xf_plan_set_mixed_condition(self._h, float(kappa_max)))

    def set_tree_growth(self, growth: float) -> None:
        """Exact mode along the prefix tree: the largest entry growth accepted
        before a bitstring takes the per-pattern evaluation."""
        check(lib().xf_plan_set_tree_growth(self._h, float(growth)))

    def set_reuse_samples(self, on: bool) -> None:
        """Raw Estimate backward calls on the same bitstring tensor, t and seed
        as the last forward call take its sampled patterns instead of drawing
        them again (the bitstrings must not change in between)."""
        check(lib().xf_plan_set_reuse_samples(self._h, 1 if on else 0))

    def set_workspace_limit(self, nbytes: int) -> None:
        """Device memory the determinant-lemma workspace may use (bitstrings
        are processed in chunks that fit, at least one at a time)."""
        check(lib().xf_plan_set_workspace_limit(self._h, int(nbytes)))

    # -- the hot path ---------------------------------------------------------
    def probabilities(self, bits: torch.Tensor, mode: str = "exact", t: int = 0, seed: int = 0,
                      out: Optional[torch.Tensor] = None, amp: Optional[torch.Tensor] = None,
                      return_amp: bool = False, logp: Optional[torch.Tensor] = None):
        """p_b for a [B, 2] int64 device tensor of bit patterns (optionally the
        amplitudes A_b and, into ``logp``, log p_b)."""
        bits = bits.contiguous()
        if bits.device != self.device or bits.dtype != torch.int64:
            raise ValueError("bits must be an int64 tensor on the plan's device")
        B = bits.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=self.device)
        if return_amp and amp is None:
            amp = torch.empty(B, 2, dtype=torch.float64, device=self.device)
        check(lib().xf_probabilities(self._h, bits.data_ptr(), B, _MODES[mode], int(t),
                                     int(seed) & 0xFFFFFFFFFFFFFFFF, out.data_ptr(),
                                     amp.data_ptr() if amp is not None else None,
                                     logp.data_ptr() if logp is not None else None,
                                     _stream_handle(self.device)))
        if return_amp:
            return out, torch.view_as_complex(amp)
        return out

    def probabilities_noalloc(self, bits: torch.Tensor, out: torch.Tensor, mode: str = "approx", t: int = 0,
                              seed: int = 0, amp: Optional[torch.Tensor] = None,
                              logp: Optional[torch.Tensor] = None) -> torch.Tensor:
        """probabilities() through xf_probabilities_noalloc: the library
        allocates nothing (its workspace is a fixed per-device array), so the
        caller passes every output tensor."""
        bits = bits.contiguous()
        if bits.device != self.device or bits.dtype != torch.int64:
            raise ValueError("bits must be an int64 tensor on the plan's device")
        check(lib().xf_probabilities_noalloc(self._h, bits.data_ptr(), bits.shape[0], _MODES[mode], int(t),
                                             int(seed) & 0xFFFFFFFFFFFFFFFF, out.data_ptr(),
                                             amp.data_ptr() if amp is not None else None,
                                             logp.data_ptr() if logp is not None else None,
                                             _stream_handle(self.device)))
        return out

    def estimate(self, bits: torch.Tensor, eps: float, delta: float, seed: int = 0,
                 out: Optional[torch.Tensor] = None):
        """Estimate (xf_estimate): p_hat_b within eps of p_b with probability
        >= 1 - delta each, by Raw Estimate calls that tighten p_max.  Returns
        (p_hat device tensor, last t per bitstring as a numpy array, number of
        iterations)."""
        bits = bits.contiguous()
        if bits.device != self.device or bits.dtype != torch.int64:
            raise ValueError("bits must be an int64 tensor on the plan's device")
        B = bits.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=self.device)
        tb = np.zeros(max(B, 1), dtype=np.int64)
        it = ctypes.c_int32()
        check(lib().xf_estimate(self._h, bits.data_ptr(), B, float(eps), float(delta),
                                int(seed) & 0xFFFFFFFFFFFFFFFF, out.data_ptr(), _ptr(tb), ctypes.byref(it),
                                _stream_handle(self.device)))
        return out, tb[:B], it.value

    def log_prob_backward(self, bits: torch.Tensor, grad_logp: torch.Tensor, mode: str = "exact",
                          t: int = 0, seed: int = 0):
        """(dL/drot as complex [n_rot, n, n], dL/dtheta [k]) for L = sum_b g_b log p_b."""
        bits = bits.contiguous()
        g = grad_logp.to(device=self.device, dtype=torch.float64).contiguous()
        grot = np.zeros((self.n_rot, self.n, self.n, 2))
        gth = np.zeros(max(self.k, 1))
        check(lib().xf_log_prob_backward(self._h, bits.data_ptr(), bits.shape[0], _MODES[mode], int(t),
                                         int(seed) & 0xFFFFFFFFFFFFFFFF, g.data_ptr(), _ptr(grot),
                                         _ptr(gth), _stream_handle(self.device)))
        return grot[..., 0] + 1j * grot[..., 1], gth[: self.k]


def trajectory_bound(eps: float, delta: float, p_max: float, xi: float) -> int:
    t = ctypes.c_int64()
    check(lib().xf_trajectory_bound(eps, delta, p_max, xi, ctypes.byref(t)))
    return t.value


def expm_antihermitian(K) -> np.ndarray:
    Kh = _complex_host(K)
    n = Kh.shape[0]
    U = np.zeros((n, n, 2))
    check(lib().xf_expm_antihermitian(n, _ptr(Kh), _ptr(U)))
    return U[..., 0] + 1j * U[..., 1]


def expm_adjoint(K, G_U) -> np.ndarray:
    Kh = _complex_host(K)
    Gh = _complex_host(G_U)
    n = Kh.shape[0]
    GK = np.zeros((n, n, 2))
    check(lib().xf_expm_adjoint(n, _ptr(Kh), _ptr(Gh), _ptr(GK)))
    return GK[..., 0] + 1j * GK[..., 1]


def spin_rotations(gens) -> np.ndarray:
    """Layers exp(K_l) (+) exp(K_l) for anti-Hermitian generators K_l
    ([n_layers, d, d] complex), through xf_spin_rotations."""
    Kh = _complex_host(gens)
    nl, d = Kh.shape[0], Kh.shape[1]
    R = np.zeros((nl, 2 * d, 2 * d, 2))
    check(lib().xf_spin_rotations(nl, d, _ptr(Kh), _ptr(R)))
    return R[..., 0] + 1j * R[..., 1]


def spin_rotations_adjoint(gens, G_rot) -> np.ndarray:
    """dL/dRe K_l + i dL/dIm K_l of every generator from the gradient of the
    layers exp(K_l) (+) exp(K_l), through xf_spin_rotations_adjoint."""
    Kh = _complex_host(gens)
    Gh = _complex_host(G_rot)
    nl, d = Kh.shape[0], Kh.shape[1]
    GK = np.zeros((nl, d, d, 2))
    check(lib().xf_spin_rotations_adjoint(nl, d, _ptr(Kh), _ptr(Gh), _ptr(GK)))
    return GK[..., 0] + 1j * GK[..., 1]


def antihermitian_reals_grad(G_K) -> np.ndarray:
    """Gradient with respect to the d^2 real parameters of an anti-Hermitian
    K ((Re K_ij, Im K_ij) for i < j, then Im K_ii), through
    xf_antihermitian_reals_grad."""
    Gh = _complex_host(G_K)
    d = Gh.shape[0]
    g = np.zeros(d * d)
    check(lib().xf_antihermitian_reals_grad(d, _ptr(Gh), _ptr(g)))
    return g


def _gate_array(gates):
    arr = (_abi.Gate * max(len(gates), 1))()
    for i, gt in enumerate(gates):
        if gt[0] == "mg":
            arr[i].kind, arr[i].q0, arr[i].q1 = _abi.XF_GATE_MATCHGATE, int(gt[1]), int(gt[1]) + 1
            G = np.asarray(gt[2], dtype=np.complex128).reshape(16)
            for e in range(16):
                arr[i].g[e][0], arr[i].g[e][1] = float(G[e].real), float(G[e].imag)
        elif gt[0] == "cp":
            arr[i].kind, arr[i].q0, arr[i].q1 = _abi.XF_GATE_CPHASE, int(gt[1]), int(gt[2])
            arr[i].theta = float(gt[3])
        else:
            raise ValueError(f"unknown gate kind {gt[0]!r}")
    return arr


def sample_gates(n: int, gates, input_bits, S: int, mode: str = "exact", t: int = 0, seed: int = 0,
                 precision: str = "fp64", device: int = 0) -> np.ndarray:
    """S output samples ([S, 2] uint64 bit patterns) of a gate list by
    gate-by-gate sampling (xf_sample_gates)."""
    arr = _gate_array(gates)
    ib = np.asarray(input_bits, dtype=np.uint64).reshape(2)
    b = _abi.Bits128()
    b.w[0], b.w[1] = int(ib[0]), int(ib[1])
    out = np.zeros((max(S, 1), 2), dtype=np.uint64)
    check(lib().xf_sample_gates(int(n), len(gates), arr, b, int(S), _MODES[mode], int(t),
                                int(seed) & 0xFFFFFFFFFFFFFFFF, _PREC[precision], int(device), _ptr(out),
                                _stream_handle(torch.device("cuda", int(device)))))
    return out[:S]


def circuit_from_gates(n: int, gates):
    """Layered circuit (rot [n_rot, n, n] complex, pairs [k, 2], layer [k],
    theta [k]) of a gate list in time order, through xf_circuit_from_gates.
    Gates: ("mg", q, G) for a matchgate G(A, B) (4 x 4 complex, basis
    |x_q x_{q+1}> = 00, 01, 10, 11) on qubits (q, q + 1), ("cp", q0, q1, theta)
    for a controlled-phase gate."""
    arr = _gate_array(gates)
    nr, k = ctypes.c_int32(), ctypes.c_int32()
    L = lib()
    check(L.xf_circuit_from_gates(int(n), len(gates), arr, 0, 0, None, None, None, None, ctypes.byref(nr),
                                  ctypes.byref(k)))
    rot = np.zeros((nr.value, n, n, 2))
    pairs = np.zeros((max(k.value, 1), 2), dtype=np.int32)
    layer = np.zeros(max(k.value, 1), dtype=np.int32)
    theta = np.zeros(max(k.value, 1))
    check(L.xf_circuit_from_gates(int(n), len(gates), arr, nr.value, k.value, _ptr(rot), _ptr(pairs), _ptr(layer),
                                  _ptr(theta), ctypes.byref(nr), ctypes.byref(k)))
    kk = k.value
    return rot[..., 0] + 1j * rot[..., 1], pairs[:kk], layer[:kk], theta[:kk]
