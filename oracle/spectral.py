"""Exact solution of u_tt = c0^2 Lap u on the periodic box (constant c0).

Test infrastructure: the reference the paper's method approximates in a
constant medium.  u(t) = F^-1[ F f0 cos(c0|xi|t) + F f1 sin(c0|xi|t)/(c0|xi|) ].
"""
import numpy as np


def solve(f0, f1, grid, c0: float, t: float) -> np.ndarray:
    xi1 = 2 * np.pi * np.fft.fftfreq(grid.n1, d=grid.d1)
    xi2 = 2 * np.pi * np.fft.fftfreq(grid.n2, d=grid.d2)
    w = c0 * np.sqrt(xi1[None, :] ** 2 + xi2[:, None] ** 2)
    F0 = np.fft.fft2(f0)
    out = F0 * np.cos(w * t)
    if f1 is not None:
        F1 = np.fft.fft2(f1)
        s = np.where(w > 0, np.sin(w * t) / np.where(w > 0, w, 1.0), t)
        out = out + F1 * s
    return np.real(np.fft.ifft2(out))
