"""Seeded synthetic inputs.

Random draws only: this module holds none of the method's arithmetic, so that
both the GPU path and the CPU oracle can take their inputs from it.
"""
import numpy as np


def random_phase_state(n, seed=0, amplitude=0.9):
    """psi_i = amplitude * exp(i theta_i), theta_i ~ U[0, 2 pi) in node order."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * np.pi, n)
    return amplitude * np.exp(1j * theta)


def random_complex(n, seed=0):
    """Standard normal real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def constant_state(n, value=1.0):
    return np.full(n, value, dtype=np.complex128)


def batch_grid_sizes(count=64, seed=0, choices=(129, 257, 513)):
    """Nodes per axis of each batched instance, drawn from `choices`."""
    rng = np.random.default_rng(seed)
    return [int(c) for c in rng.choice(np.asarray(choices), count)]


def unet_init(shapes, seed=0, head_scale=0.0):
    """Initial U-Net parameters (FP32 flat vector, layer order of the library):
    weights of a conv with c_in inputs and a k x k kernel ~ N(0, 2 / (k^2 c_in))
    (He), zero biases; the head's weights scaled by head_scale (0: the initial
    network predicts no change).  shapes: (c_in, c_out, k) per layer."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co, k) in enumerate(shapes):
        std = np.sqrt(2.0 / (k * k * ci))
        if li == len(shapes) - 1:
            std *= head_scale
        parts.append(rng.standard_normal(co * k * k * ci) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def sweep_mus(mu_end=2.0, step=0.01, jitter=0.002, seed=0):
    """Field values of a training sweep: 0, then steps of step + U(-jitter, jitter)
    up to mu_end."""
    rng = np.random.default_rng(seed)
    mus = [0.0]
    while mus[-1] < mu_end - 1e-12:
        mus.append(min(mu_end, mus[-1] + step + rng.uniform(-jitter, jitter)))
    return mus
