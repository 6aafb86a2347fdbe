"""Helmholtz fundamental solution (eq. (G)) and its target-normal
derivative (used in eq. (ringkernelderiv) and the Neumann rows)."""
from __future__ import annotations

import math

import numpy as np


def G(k: float, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """G_k(x, y) = exp(i k |x-y|) / (4 pi |x-y|); x, y broadcast over [..., 3]."""
    d = x - y
    R = np.sqrt(np.sum(d * d, axis=-1))
    return np.exp(1j * k * R) / (4 * math.pi * R)


def grad_x_G(k: float, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Gradient of G_k with respect to the target x:
    grad G = G (i k - 1/R) (x - y)/R, shape [..., 3]."""
    d = x - y
    R = np.sqrt(np.sum(d * d, axis=-1))
    g = np.exp(1j * k * R) / (4 * math.pi * R)
    return (g * (1j * k - 1.0 / R) / R)[..., None] * d


def dG_dnx(k: float, x: np.ndarray, nx: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Target-normal derivative n_x . grad_x G_k(x, y)."""
    return np.sum(grad_x_G(k, x, y) * nx, axis=-1)
