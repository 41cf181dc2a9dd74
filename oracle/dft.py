"""Brute-force discrete Fourier transform (O(N^2) matrix form), FP64.

Test infrastructure: pins the FFT primitive used by the oracle.  The transform
follows Sec. 2.2: forward kernel exp(-i k.x), unnormalised; inverse 1/N.
"""
import numpy as np


def dft_matrix(n: int, inverse: bool = False) -> np.ndarray:
    j = np.arange(n)
    sign = 1.0 if inverse else -1.0
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


def dft2(f: np.ndarray) -> np.ndarray:
    """Full 2D forward DFT of an (ny, nx) array by explicit matrix products."""
    ny, nx = f.shape
    return dft_matrix(ny) @ f.astype(np.complex128) @ dft_matrix(nx).T


def idft2(F: np.ndarray) -> np.ndarray:
    ny, nx = F.shape
    return dft_matrix(ny, True) @ F @ dft_matrix(nx, True).T / (nx * ny)
