"""FP64 oracle for the night-sky-brightness convolution (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library and the library never imports it.

`direct.c` holds the plain FP64 direct sums of Eq. 7 (Sec. 2.3) on the pixel
grid with zero padding (Sec. 2.5); this module loads it with ctypes and
converts arguments.  `spectrum.py` holds the plain DFT of Eq. 10 used to check
the stored kernel spectrum.

Conventions (the readings every caller shares): the kernel centre is
((ky-1)//2, (kx-1)//2); the "same" output is the input-sized window of the full
linear convolution aligned on that centre; no area element is applied.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB_PATH: another build of direct.c (the sanitizer build)
_LIB_PATH = os.environ.get("ORACLE_LIB_PATH") or os.path.join(_HERE, "liboracle.so")
_lib = None

_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b

        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "orc_conv_full": [_c_dbl_p, _i64, _i64, _c_dbl_p, _i64, _i64, _c_dbl_p],
        "orc_conv_same": [_c_dbl_p, _i64, _i64, _c_dbl_p, _i64, _i64, _c_dbl_p],
        "orc_conv_same_pixels": [_c_dbl_p, _i64, _i64, _c_dbl_p, _i64, _i64,
                                 _c_i64_p, _i64, _c_dbl_p],
        "orc_adjoint_same": [_c_dbl_p, _i64, _i64, _c_dbl_p, _i64, _i64, _c_dbl_p],
        "orc_adjoint_same_pixels": [_c_dbl_p, _i64, _i64, _c_dbl_p, _i64, _i64,
                                    _c_i64_p, _i64, _c_dbl_p],
        "orc_adjoint_sparse": [_c_i64_p, _c_dbl_p, _i64, _i64, _i64, _c_dbl_p,
                               _i64, _i64, _c_dbl_p],
        "orc_conv_same_separable": [_c_dbl_p, _i64, _i64, _c_dbl_p, _i64,
                                    _c_dbl_p, _i64, _c_dbl_p, _c_dbl_p],
        "orc_conv_same_separable_pixels": [_c_dbl_p, _i64, _i64, _c_dbl_p, _i64,
                                           _c_dbl_p, _i64, _c_i64_p, _i64,
                                           _c_dbl_p],
        "orc_num_threads": [],
        "orc_set_num_threads": [ctypes.c_int],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _d(a):
    """Contiguous FP64 copy (FP32 inputs are promoted exactly)."""
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_c_dbl_p):
    return a.ctypes.data_as(t)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name}: bad argument")


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> int:
    """Threads for the oracle's OpenMP loops from now on; returns the number
    in effect."""
    return int(_load().orc_set_num_threads(int(n)))


def conv_full(R, K):
    """Full linear convolution (Eq. 7 on the grid), (ny+ky-1) x (nx+kx-1)."""
    R, K = _d(R), _d(K)
    ny, nx = R.shape
    ky, kx = K.shape
    S = np.empty((ny + ky - 1, nx + kx - 1), np.float64)
    _check(_load().orc_conv_full(_p(R), ny, nx, _p(K), ky, kx, _p(S)), "conv_full")
    return S


def conv_same(R, K):
    """Input-sized window of the full convolution, aligned on the kernel centre."""
    R, K = _d(R), _d(K)
    ny, nx = R.shape
    ky, kx = K.shape
    S = np.empty((ny, nx), np.float64)
    _check(_load().orc_conv_same(_p(R), ny, nx, _p(K), ky, kx, _p(S)), "conv_same")
    return S


def conv_same_pixels(R, K, idx):
    """"Same" convolution at flat pixel indices idx (i*nx + j)."""
    R, K = _d(R), _d(K)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    ny, nx = R.shape
    ky, kx = K.shape
    out = np.empty(idx.shape[0], np.float64)
    _check(_load().orc_conv_same_pixels(_p(R), ny, nx, _p(K), ky, kx,
                                        _p(idx, _c_i64_p), idx.shape[0], _p(out)),
           "conv_same_pixels")
    return out


def adjoint_same(G, K):
    """Transpose of the "same" operator applied to an ny x nx map."""
    G, K = _d(G), _d(K)
    ny, nx = G.shape
    ky, kx = K.shape
    A = np.empty((ny, nx), np.float64)
    _check(_load().orc_adjoint_same(_p(G), ny, nx, _p(K), ky, kx, _p(A)), "adjoint_same")
    return A


def adjoint_same_pixels(G, K, idx):
    """Transposed operator at flat pixel indices."""
    G, K = _d(G), _d(K)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    ny, nx = G.shape
    ky, kx = K.shape
    out = np.empty(idx.shape[0], np.float64)
    _check(_load().orc_adjoint_same_pixels(_p(G), ny, nx, _p(K), ky, kx,
                                           _p(idx, _c_i64_p), idx.shape[0], _p(out)),
           "adjoint_same_pixels")
    return out


def adjoint_sparse(sites, g, shape, K):
    """Transposed operator applied to a map that is g at `sites`, 0 elsewhere."""
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    g = _d(g)
    K = _d(K)
    ny, nx = shape
    ky, kx = K.shape
    A = np.empty((ny, nx), np.float64)
    _check(_load().orc_adjoint_sparse(_p(sites, _c_i64_p), _p(g), sites.shape[0],
                                      ny, nx, _p(K), ky, kx, _p(A)), "adjoint_sparse")
    return A


def conv_same_separable(R, u, v):
    """"Same" convolution with K = outer(u, v), as row then column 1-D sums."""
    R, u, v = _d(R), _d(u), _d(v)
    ny, nx = R.shape
    T = np.empty((ny, nx), np.float64)
    S = np.empty((ny, nx), np.float64)
    _check(_load().orc_conv_same_separable(_p(R), ny, nx, _p(u), u.shape[0],
                                           _p(v), v.shape[0], _p(T), _p(S)),
           "conv_same_separable")
    return S


def conv_same_separable_pixels(R, u, v, idx):
    """Separable "same" convolution at flat pixel indices."""
    R, u, v = _d(R), _d(u), _d(v)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    ny, nx = R.shape
    out = np.empty(idx.shape[0], np.float64)
    _check(_load().orc_conv_same_separable_pixels(_p(R), ny, nx, _p(u), u.shape[0],
                                                  _p(v), v.shape[0],
                                                  _p(idx, _c_i64_p), idx.shape[0],
                                                  _p(out)),
           "conv_same_separable_pixels")
    return out


def conv_same_classes(Rs, Ks):
    """Several factorable source classes (Sec. 2.2, Eq. 4): class t has its
    own radiance map R_t and kernel K_t (its angular-spectral pattern folded
    into the kernel as in Eq. 6), and the sky brightness is the sum over
    classes of the "same" convolutions K_t (*) R_t."""
    assert len(Rs) == len(Ks) and len(Rs) >= 1
    S = conv_same(Rs[0], Ks[0])
    for R, K in zip(Rs[1:], Ks[1:]):
        S += conv_same(R, K)
    return S


def conv_same_classes_pixels(Rs, Ks, idx):
    """Class sum of Eq. 4 at flat pixel indices."""
    assert len(Rs) == len(Ks) and len(Rs) >= 1
    out = conv_same_pixels(Rs[0], Ks[0], idx)
    for R, K in zip(Rs[1:], Ks[1:]):
        out += conv_same_pixels(R, K, idx)
    return out


def rel_l2(x, ref):
    """||x - ref||_2 / ||ref||_2 in FP64."""
    x = np.asarray(x, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def max_err_frac(x, ref):
    """max|x - ref| / max|ref| in FP64."""
    x = np.asarray(x, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
