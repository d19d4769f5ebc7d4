"""Closed forms of the diagonals of B by Poisson summation (Lemmas 4.2, 4.3).

Lemma 4.2: the diagonal d_i of block i of B is the DFT of the periodized
kernel sampled on the i-th shifted grid.  With the paper's unitary F, block
i of B is F* A^c_i F, whose diagonal is the standard DFT (kernel exp(-2 pi i
kn/N)) of the first column of the circulant block A^c_i, i.e. of
v_i[n] = phi_per((i-1) h_L + n h).

As in the proof of Lemma 4.3, the sum over all samples of the Gaussian
equals a periodic sum of its Fourier transform (Poisson summation).  For
phase r = i-1 (0-based) and frequency k:
    d_r[k] = (1/h) sum_m exp(2 pi i (k/N + m) r/s) ghat(2 pi (k/N + m)/h)
with ghat(w) = (sqrt(pi)/eps) exp(-w^2/(4 eps^2)) the Fourier transform
of exp(-eps^2 x^2).  The second-derivative kernel phi'' has transform
-w^2 ghat(w).
"""
import numpy as np


def ghat(w, eps):
    return (np.sqrt(np.pi) / eps) * np.exp(-(w * w) / (4.0 * eps * eps))


def diag_closed_form(n, s, T, eps, r, deriv=0, mmax=12):
    """d_r[k], k = 0..n-1, for the kernel phi (deriv=0) or phi'' (deriv=2)."""
    h = 2.0 * T / n
    k = np.arange(n, dtype=np.float64)
    out = np.zeros(n, dtype=np.complex128)
    for m in range(-mmax, mmax + 1):
        nu = k / n + m
        w = 2.0 * np.pi * nu / h
        g = ghat(w, eps)
        if deriv == 2:
            g = -(w * w) * g
        out += np.exp(2j * np.pi * nu * r / s) * g
    return out / h


def nyquist_minimum(n, T, eps):
    """(d_1)_{N/2+1} of Lemma 4.3, the smallest entry of the first diagonal."""
    return diag_closed_form(n, 1, T, eps, 0)[n // 2].real
