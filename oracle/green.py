"""Periodic Green operator of the oracle (test infrastructure only).

The stress is found by a spectral method in which FFTs turn the Green-function
convolution into a product per frequency (Sec. 2.1). For a homogeneous
reference medium C0 and unit wave direction n the Green operator is built by
the general route, valid for any C0:

    K_ik = C0_ijkl n_j n_l            (acoustic tensor)
    N    = K^-1
    Gamma_ijkl = 1/4 (N_ik n_j n_l + N_jk n_i n_l + N_il n_j n_k + N_jl n_i n_k)

Frequencies are those of the discrete grid, ``xi_a = k_a / n_a`` with
``k_a`` in ``[-n_a/2, n_a/2)``. Where any index equals ``n_a/2`` (a Nyquist
frequency of an even grid) the operator is replaced by ``C0^-1``, which makes
the stress vanish there at the fixed point. FFTs are numpy's (a library
primitive): forward unnormalised, inverse scaled by 1/N^3.
"""
from __future__ import annotations

import numpy as np

from .tensors import c4_to_mandel


def frequencies(shape):
    """Integer frequency indices (kx, ky, kz) broadcastable to [z][y][x]."""
    n0, n1, n2 = shape
    kx = np.fft.fftfreq(n0) * n0
    ky = np.fft.fftfreq(n1) * n1
    kz = np.fft.fftfreq(n2) * n2
    return kx, ky, kz


def gamma_mandel(nvec, C0):
    """Mandel 6x6 Green operator for unit directions ``nvec`` (..., 3)."""
    K = np.einsum("ijkl,...j,...l->...ik", C0, nvec, nvec)
    N = np.linalg.inv(K)
    G = 0.25 * (np.einsum("...ik,...j,...l->...ijkl", N, nvec, nvec)
                + np.einsum("...jk,...i,...l->...ijkl", N, nvec, nvec)
                + np.einsum("...il,...j,...k->...ijkl", N, nvec, nvec)
                + np.einsum("...jl,...i,...k->...ijkl", N, nvec, nvec))
    return c4_to_mandel(G)


def gamma_field(shape, C0, C0inv_mandel):
    """Mandel Green operator at every frequency, shape (n2, n1, n0, 6, 6).

    It depends only on the grid and C0, so a solver builds it once.
    """
    n0, n1, n2 = shape
    kx, ky, kz = frequencies(shape)
    G = np.empty((n2, n1, n0, 6, 6))
    KY, KX = np.meshgrid(ky, kx, indexing="ij")          # (n1, n0)
    for z in range(n2):
        xi = np.stack([KX / n0, KY / n1, np.full_like(KX, kz[z] / n2)], axis=-1)
        norm = np.linalg.norm(xi, axis=-1)
        nyq = (np.abs(KX) == n0 / 2) | (np.abs(KY) == n1 / 2) | (abs(kz[z]) == n2 / 2)
        zero = norm == 0
        nvec = xi / np.where(zero, 1.0, norm)[..., None]
        nvec[zero] = (1.0, 0.0, 0.0)        # xi = 0 is overwritten by the mean strain
        Gz = gamma_mandel(nvec, C0)
        Gz[nyq] = C0inv_mandel
        G[z] = Gz
    return G


def green_apply(tau_hat, G, E_mandel):
    """e_hat = -Gamma0(xi) : tau_hat(xi) for every frequency; e_hat(0) = N^3 E.

    ``tau_hat``: complex (6, n2, n1, n0) Mandel components of the full 3D FFT;
    ``G``: the operator from ``gamma_field``.
    """
    t = np.moveaxis(tau_hat, 0, -1)[..., None]            # (n2, n1, n0, 6, 1)
    out = np.moveaxis(-(G @ t)[..., 0], -1, 0).copy()
    out[:, 0, 0, 0] = tau_hat[0].size * E_mandel
    return out
