"""Shared helpers of the GPU parity tests (inputs from ``workloads``, expected
values from ``oracle``, results from the HIP library through its C ABI)."""
import sys

import numpy as np

import oracle


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_rot(w, X):
    return w.rot if w.rot is not None else X.spin_rotations(w.gens)


def oracle_rot(w):
    return w.rot if w.rot is not None else oracle.rotations_from_generators(w.gens)


def make_plan(w, X, precision="fp64"):
    return X.Plan(gpu_rot(w, X), w.pairs, w.layer, w.theta, w.input_bits, precision)


def gpu_probs(plan, X, bits, mode, t=0, seed=0, return_amp=False):
    import torch
    tb = X.bits_tensor(bits, plan.device)
    r = plan.probabilities(tb, mode, t, seed, return_amp=return_amp)
    torch.cuda.synchronize()
    if return_amp:
        return r[0].cpu().numpy(), r[1].cpu().numpy()
    return r.cpu().numpy()


def oracle_probs(w, bits, mode=None, t=None, seed=None, return_amp=False, batch_index=None):
    return oracle.probabilities(oracle_rot(w), w.pairs, w.layer, w.theta, w.input_bits, bits,
                                mode or w.mode, w.t if t is None else t, w.seed if seed is None else seed,
                                return_amp=return_amp, batch_index=batch_index)


def rel_err(p, ref):
    p = np.asarray(p)
    ref = np.asarray(ref)
    scale = np.where(ref > 0, ref, 1.0)
    return np.abs(p - ref) / scale


def sample_indices(B: int, count: int, seed: int = 0) -> np.ndarray:
    """``count`` distinct batch indices spread over [0, B), always with the
    first and the last."""
    rng = np.random.default_rng(seed)
    idx = set([0, B - 1])
    while len(idx) < min(count, B):
        idx.add(int(rng.integers(0, B)))
    return np.array(sorted(idx))
