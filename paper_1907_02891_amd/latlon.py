"""Steps either side of the convolution on longitude-latitude data.

Sec. 2.4: radiance composites come on a uniform longitude-latitude grid whose
ground scale varies with latitude, so the paper reprojects them onto a
transverse Mercator (UTM) grid, nearest neighbour, before convolving; the
gather runs on the GPU (`lp.reproject_nn`, C entry point lp_reproject_nn),
with the scale factor of Eq. 11 for an optional ground-area weight.

Sec. 4 outlines an alternative it does not develop: stay on the native
longitude-latitude grid and use a kernel that is held constant within narrow
latitude bands.  `band_kernel` samples a radial PSF on that grid for a band's
centre latitude (one pixel step is R dphi north-south and R cos(phi) dlambda
east-west), and `LatitudeBands` runs the bands as overlap-save slabs: slab t
holds its band's rows plus the kernel's reach above and below, all slabs go
through one batched call (lp_convolve_batched, one launch per stage and
padding class), and each slab writes only its band's rows of the output
(lp_batch_set_output_rows), so the stitched map needs no copy.  With whole
halos a slab's kept rows need only as many padded rows as the slab has.
"""
from __future__ import annotations

import math

import numpy as np

from . import lp

EARTH_RADIUS_KM = 6367.0  # the sphere radius the paper uses with Eq. 11
UTM_K0 = 0.9996           # the usual UTM central scale (Sec. 2.4)


def band_kernel(radial, lat_c_deg, dlat_deg, dlon_deg, half_y, half_x, radius_km=EARTH_RADIUS_KM):
    """(2 half_y + 1) x (2 half_x + 1) kernel of one latitude band: the radial
    PSF `radial(d_km)` at the ground distance of each pixel offset from the
    centre, for a band centred at latitude lat_c_deg (FP64)."""
    rad = math.pi / 180.0
    step_ns = radius_km * dlat_deg * rad
    step_ew = radius_km * math.cos(lat_c_deg * rad) * dlon_deg * rad
    dy = step_ns * np.arange(-half_y, half_y + 1, dtype=np.float64)
    dx = step_ew * np.arange(-half_x, half_x + 1, dtype=np.float64)
    d = np.hypot(dy[:, None], dx[None, :])
    return np.asarray(radial(d), dtype=np.float64)


def band_centres(band_edges, lat_first_deg, dlat_deg):
    """Centre latitude of each band [e_t, e_{t+1}) of a grid whose row r lies
    at lat_first - r dlat."""
    e = np.asarray(band_edges, dtype=np.float64)
    return lat_first_deg - dlat_deg * 0.5 * (e[:-1] + e[1:] - 1.0)


class LatitudeBands:
    """Convolution of an ny x nx longitude-latitude map where output rows
    [band_edges[t], band_edges[t+1]) use kernels[t] (all kernels the same
    odd or even shape); each output pixel equals the "same" convolution of
    the whole map with its band's kernel."""

    def __init__(self, ny, nx, band_edges, kernels, *, pitch_km=1.0, device=None, stream=None):
        edges = [int(e) for e in band_edges]
        if edges[0] != 0 or edges[-1] != ny or any(b <= a for a, b in zip(edges, edges[1:])):
            raise ValueError("band edges must rise strictly from 0 to ny")
        kernels = [np.ascontiguousarray(k, dtype=np.float64) for k in kernels]
        if len(kernels) != len(edges) - 1 or any(k.shape != kernels[0].shape for k in kernels):
            raise ValueError("one kernel per band, all of one shape")
        ky, kx = kernels[0].shape
        cy = (ky - 1) // 2
        above, below = ky - 1 - cy, cy  # input rows an output row reaches up / down
        self.ny, self.nx, self.edges = int(ny), int(nx), edges
        self.slabs = [(max(0, a - above), min(ny, b + below)) for a, b in zip(edges, edges[1:])]
        shapes = [(s1 - s0, nx) for s0, s1 in self.slabs]
        self.batch = lp.Batch(shapes, list(range(len(kernels))), [k.shape for k in kernels], pitch_km=pitch_km)
        # windows before bind: each slab is padded only as far as its kept
        # rows need (Py >= slab rows when the halos are whole)
        for t, ((s0, _), a, b) in enumerate(zip(self.slabs, edges, edges[1:])):
            self.batch.set_output_rows(t, a - s0, b - a)
        self.batch.bind(device=device, stream=stream)
        self.batch.set_kernels(kernels)

    def convolve(self, x, out=None):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
                and tuple(x.shape) == (self.ny, self.nx)):
            raise ValueError("x must be a contiguous CUDA float32 tensor of the map's shape")
        if out is None:
            out = torch.empty_like(x)
        if out.data_ptr() == x.data_ptr():
            raise ValueError("the output must not alias the input (slabs overlap)")
        maps = [x[s0:s1] for s0, s1 in self.slabs]
        outs = [out[a:b] for a, b in zip(self.edges, self.edges[1:])]
        self.batch.convolve(maps, outs)
        return out
