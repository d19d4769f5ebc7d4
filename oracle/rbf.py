"""Gaussian RBF and its periodization (section 2.1).

phi(r) = exp(-eps^2 r^2)                       eq. (rbf)
phi_per(x) = sum_m phi(x - 2 m T)              eq. (periodic_rbf)
phi''(r) = -2 eps^2 exp(-eps^2 r^2)(1 - 2 eps^2 r^2)   (section 6.1, Example)
phi'(r) = -2 eps^2 r exp(-eps^2 r^2)                  (Neumann rows, section 6.3)

The infinite image sum is truncated: for |x| <= 2T every omitted image lies
at distance > 6.8/eps, where the Gaussian is below exp(-46.24) < 1e-20.
"""
import math

import numpy as np


def phi(r, eps):
    r = np.asarray(r, dtype=np.float64)
    return np.exp(-(eps * r) ** 2)


def phi1(r, eps):
    """First derivative of the Gaussian with respect to its argument."""
    r = np.asarray(r, dtype=np.float64)
    e2 = eps * eps
    return -2.0 * e2 * r * np.exp(-e2 * r * r)


def phi2(r, eps):
    """Second derivative of the Gaussian with respect to its argument."""
    r = np.asarray(r, dtype=np.float64)
    e2 = eps * eps
    return -2.0 * e2 * np.exp(-e2 * r * r) * (1.0 - 2.0 * e2 * r * r)


def shape_parameter(tau0, n, T):
    """eps = c N with c = pi / (2 T sqrt(2 log(1 + tau0^-2))), eq. (constant_shapeparam)."""
    c = math.pi / (2.0 * T * math.sqrt(2.0 * math.log1p(tau0 ** -2)))
    return c * n


def n_images(eps, T):
    """Images m = -m*..m* suffice for arguments |x| <= 2T."""
    return int(math.ceil(6.8 / (2.0 * eps * T))) + 2


def periodize(f, x, eps, T):
    """sum_m f(x - 2 m T, eps) over the images that matter for |x| <= 2T."""
    x = np.asarray(x, dtype=np.float64)
    m = n_images(eps, T)
    out = np.zeros_like(x)
    for k in range(-m, m + 1):
        out += f(x - 2.0 * k * T, eps)
    return out


def phi_per(x, eps, T):
    return periodize(phi, x, eps, T)


def phi1_per(x, eps, T):
    return periodize(phi1, x, eps, T)


def phi2_per(x, eps, T):
    return periodize(phi2, x, eps, T)
