"""Plain FP64 kernel spectrum: the 2-D DFT of Eq. 10 (test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The point-spread matrix K (ky x kx, centre ((ky-1)//2, (kx-1)//2)) is placed in
a Py x Px zero array with its centre at index (0, 0) -- entry K(a, b) goes to
((a - cy) mod Py, (b - cx) mod Px) -- so that the circular convolution of the
zero-padded map with it yields the centre-aligned "same" window at the origin
(Sec. 2.5: zero padding turns the circular convolution into a linear one).
The spectrum is then Eq. 10 written with 0-based indices,

    Khat(u, v) = sum_n sum_m kw(n, m) exp(-i 2 pi (u n / Py + v m / Px)),

evaluated as two products with DFT matrices.  The exponent index u*n is
reduced modulo the length in integers before the angle is formed, so every
twiddle is cos/sin of an angle in [0, 2 pi).
"""
import numpy as np


def wrap_centre(K, Py, Px):
    """Zero-padded Py x Px array with K's centre moved to index (0, 0)."""
    K = np.asarray(K, np.float64)
    ky, kx = K.shape
    if Py < ky or Px < kx:
        raise ValueError("padding smaller than the kernel")
    cy, cx = (ky - 1) // 2, (kx - 1) // 2
    kw = np.zeros((Py, Px), np.float64)
    for a in range(ky):
        for b in range(kx):
            kw[(a - cy) % Py, (b - cx) % Px] = K[a, b]
    return kw


def dft_matrix(N, sign=-1):
    """F[u, n] = exp(sign * i 2 pi (u n mod N) / N)."""
    n = np.arange(N, dtype=np.int64)
    m = np.outer(n, n) % N
    return np.exp(sign * 2j * np.pi * (m.astype(np.float64) / N))


def kernel_spectrum(K, Py, Px):
    """Unscaled FP64 DFT (Eq. 10) of the wrap-centred, zero-padded kernel."""
    kw = wrap_centre(K, Py, Px)
    return dft_matrix(Py) @ kw @ dft_matrix(Px).T
