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
