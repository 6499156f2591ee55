"""Python binding of the C ABI in include/lp.h (argument marshalling only).

Every step of the computation runs in the HIP library liblp.so; this module
loads it with ctypes, hands it torch device pointers and the current HIP
stream, and turns error codes into exceptions.  If the library is missing the
import fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: its bundled HIP runtime (soname libamdhip64.so.7) must be the
# one liblp.so binds to, so that both share one runtime and one device context.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# LP_LIB_PATH: another build of the same library (the host-sanitizer build of
# the CPU test suite); the default is the in-tree liblp.so
LIB_PATH = os.environ.get("LP_LIB_PATH") or os.path.join(_HERE, "liblp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1907_02891_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

LP_OK, LP_E_INVALID, LP_E_SIZE, LP_E_STATE, LP_E_NOMEM, LP_E_DEVICE = 0, -1, -2, -3, -4, -5
FORM_NONE, FORM_REAL_QUADRANT, FORM_COMPLEX = 0, 1, 2
KERNELS_AUTO, KERNELS_GENERIC, KERNELS_SPECIALISED = 0, 1, 2
STAGE_ROWS, STAGE_COLUMNS, STAGE_ROWS_INVERSE = 0, 1, 2
PRECISION_FP32, PRECISION_SPLIT_FP16, PRECISION_SPLIT_BF16 = 0, 1, 2
MAX_CLASSES = 16
MAX_PY, MAX_PX = 131072, 40958
MAX_COLUMN_TILE = 20480  # longer padded columns take the four-step column stage
NOALLOC_MAX_BYTES = 128 << 20  # scratch array of lp_convolve_noalloc

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)

class LatLonGrid(ctypes.Structure):
    """lp_latlon_grid: row r at latitude lat_first - r dlat, column c at
    longitude lon_first + c dlon (degrees)."""
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("lat_first_deg", ctypes.c_double), ("lon_first_deg", ctypes.c_double),
                ("dlat_deg", ctypes.c_double), ("dlon_deg", ctypes.c_double)]


class TMGrid(ctypes.Structure):
    """lp_tm_grid: row i at northing y_first - i pitch, column j at easting
    x_first + j pitch (km from the equator / central meridian)."""
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("x_first_km", ctypes.c_double), ("y_first_km", ctypes.c_double),
                ("pitch_km", ctypes.c_double), ("lon0_deg", ctypes.c_double),
                ("k0", ctypes.c_double), ("radius_km", ctypes.c_double)]


_SIGS = {
    "lp_last_error": ([], ctypes.c_char_p),
    "lp_version": ([], ctypes.c_char_p),
    "lp_last_status": ([], ctypes.c_int),
    "lp_plan_create": ([_i64, _i64, _i64, _i64, ctypes.c_double], _vp),
    "lp_plan_destroy": ([_vp], None),
    "lp_plan_set_padding": ([_vp, _i64, _i64], ctypes.c_int),
    "lp_plan_get_padding": ([_vp, _i64p, _i64p], ctypes.c_int),
    "lp_plan_workspace_bytes": ([_vp], ctypes.c_size_t),
    "lp_plan_bind": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "lp_kernel_spectrum": ([_vp, _dp], ctypes.c_int),
    "lp_plan_spectrum_form": ([_vp], ctypes.c_int),
    "lp_plan_read_spectrum": ([_vp, _fp], ctypes.c_int),
    "lp_convolve": ([_vp, _vp, _vp], ctypes.c_int),
    "lp_adjoint": ([_vp, _vp, _vp], ctypes.c_int),
    "lp_convolve_noalloc": ([_vp, _vp, _vp], ctypes.c_int),
    "lp_plan_timing": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_plan_set_poison": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_plan_stage_ms": ([_vp, _dp, ctypes.c_int, _ip], ctypes.c_int),
    "lp_plan_shape": ([_vp, _ip, _ip], ctypes.c_int),
    "lp_plan_column_split": ([_vp, _i64p, _i64p], ctypes.c_int),
    "lp_plan_set_kernels": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_plan_kernels": ([_vp], ctypes.c_int),
    "lp_plan_set_precision": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_plan_set_classes": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_reproject_nn": ([ctypes.POINTER(LatLonGrid), _vp, ctypes.POINTER(TMGrid), _vp, ctypes.c_int, _vp],
                        ctypes.c_int),
    "lp_plan_classes": ([_vp], ctypes.c_int),
    "lp_kernel_spectra": ([_vp, ctypes.POINTER(_dp)], ctypes.c_int),
    "lp_convolve_classes": ([_vp, ctypes.POINTER(_vp), _vp], ctypes.c_int),
    "lp_adjoint_class": ([_vp, ctypes.c_int, _vp, _vp], ctypes.c_int),
    "lp_plan_precision": ([_vp], ctypes.c_int),
    "lp_plan_variant_count": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_plan_get_variant": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_plan_set_variant": ([_vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "lp_plan_variant_info": ([_vp, ctypes.c_int, ctypes.c_int, _ip, ctypes.c_int], ctypes.c_int),
    "lp_batch_create": ([ctypes.c_int, _i64p, _i64p, _ip, ctypes.c_int, _i64p, _i64p, ctypes.c_double], _vp),
    "lp_batch_create_padded": ([ctypes.c_int, _i64p, _i64p, _ip, ctypes.c_int, _i64p, _i64p, ctypes.c_double,
                                _i64p, ctypes.c_int, _i64p, ctypes.c_int], _vp),
    "lp_batch_spec_lengths": ([ctypes.c_int, _i64p, ctypes.c_int], ctypes.c_int),
    "lp_batch_destroy": ([_vp], None),
    "lp_batch_workspace_bytes": ([_vp], ctypes.c_size_t),
    "lp_batch_bind": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "lp_batch_kernel_spectra": ([_vp, ctypes.POINTER(_dp)], ctypes.c_int),
    "lp_convolve_batched": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)], ctypes.c_int),
    "lp_batch_use_graph": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_batch_set_output_rows": ([_vp, ctypes.c_int, _i64, _i64], ctypes.c_int),
    "lp_batch_group_count": ([_vp], ctypes.c_int),
    "lp_batch_group_info": ([_vp, ctypes.c_int, _i64p, ctypes.c_int], ctypes.c_int),
    "lp_batch_tile_group": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_batch_set_variant": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "lp_batch_set_graph_branches": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_batch_set_poison": ([_vp, ctypes.c_int], ctypes.c_int),
    "lp_batch_get_variant": ([_vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class LPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def last_error() -> str:
    return _lib.lp_last_error().decode()


def version() -> str:
    return _lib.lp_version().decode()


def _check(rc):
    if rc != LP_OK:
        raise LPError(rc, last_error())
    return rc


def raw():
    """The ctypes library handle (for tests of the C ABI itself)."""
    return _lib


def _ordered(bound, tensors, launch):
    """Run `launch` (which enqueues on the plan's bound stream) ordered with
    torch's current stream: when the two differ, the bound stream first waits
    for the work already queued on the current one (which may still be
    writing the inputs), the current stream then waits for the bound one (so
    the outputs are complete for whatever the caller queues next), and every
    tensor is marked as used on the bound stream so that the caching
    allocator does not hand its memory out again before that stream is done
    with it."""
    import torch
    cur = torch.cuda.current_stream(tensors[0].device)
    if bound is None or cur == bound:
        return launch()
    bound.wait_stream(cur)
    try:
        return launch()
    finally:
        cur.wait_stream(bound)
        for t in tensors:
            t.record_stream(bound)


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """One map shape and one kernel (lp_plan_*).  Host-only until bind()."""

    def __init__(self, ny, nx, ky, kx, pitch_km=0.5, padding=None):
        self._p = _lib.lp_plan_create(int(ny), int(nx), int(ky), int(kx), float(pitch_km))
        if not self._p:
            raise LPError(_lib.lp_last_status(), last_error())
        self.ny, self.nx, self.ky, self.kx = int(ny), int(nx), int(ky), int(kx)
        self.workspace = None
        self.stream = None
        if padding is not None:
            self.set_padding(*padding)

    def close(self):
        # _lib is None when the interpreter tears the module down first
        if getattr(self, "_p", None) and _lib is not None:
            _lib.lp_plan_destroy(self._p)
            self._p = None

    __del__ = close

    @property
    def handle(self):
        return self._p

    def set_padding(self, py, px):
        _check(_lib.lp_plan_set_padding(self._p, int(py), int(px)))

    @property
    def padding(self):
        py, px = _i64(), _i64()
        _check(_lib.lp_plan_get_padding(self._p, ctypes.byref(py), ctypes.byref(px)))
        return py.value, px.value

    @property
    def workspace_bytes(self):
        return int(_lib.lp_plan_workspace_bytes(self._p))

    @property
    def shape(self):
        c, b = ctypes.c_int(), ctypes.c_int()
        _check(_lib.lp_plan_shape(self._p, ctypes.byref(c), ctypes.byref(b)))
        return c.value, b.value

    @property
    def column_split(self):
        """(P1, P2): (1, Py) when a padded column fits one workgroup, else the
        four-step factors Py = P1 * P2."""
        p1, p2 = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.lp_plan_column_split(self._p, ctypes.byref(p1), ctypes.byref(p2)))
        return p1.value, p2.value

    def bind(self, device=None, stream=None, workspace=None):
        """Allocate (or take) a torch uint8 device workspace and bind it with
        `stream` (default: torch's current stream)."""
        import torch
        if workspace is None:
            dev = torch.device("cuda") if device is None else torch.device(device)
            workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        elif not (isinstance(workspace, torch.Tensor) and workspace.is_cuda and workspace.dtype == torch.uint8
                  and workspace.is_contiguous()):
            raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
        ptr = workspace.data_ptr()
        off = (-ptr) % 256
        self.workspace = workspace
        self.stream = torch.cuda.current_stream(workspace.device) if stream is None else stream
        _check(_lib.lp_plan_bind(self._p, ctypes.c_void_p(ptr + off),
                                 workspace.numel() - off, _stream_ptr(self.stream)))
        return self

    def set_kernel(self, psf):
        psf = np.ascontiguousarray(psf, dtype=np.float64)
        if psf.shape != (self.ky, self.kx):
            raise ValueError(f"kernel shape {psf.shape} != ({self.ky}, {self.kx})")
        _check(_lib.lp_kernel_spectrum(self._p, psf.ctypes.data_as(_dp)))
        return self

    def set_classes(self, n):
        """Number of source classes summed by convolve_classes (before bind)."""
        _check(_lib.lp_plan_set_classes(self._p, int(n)))

    @property
    def classes(self):
        return int(_lib.lp_plan_classes(self._p))

    def set_kernels_classes(self, psfs):
        """One kernel per class (lp_kernel_spectra)."""
        arrs = [np.ascontiguousarray(k, dtype=np.float64) for k in psfs]
        if len(arrs) != self.classes:
            raise ValueError(f"{len(arrs)} kernels for {self.classes} classes")
        for k in arrs:
            if k.shape != (self.ky, self.kx):
                raise ValueError(f"kernel shape {k.shape} != ({self.ky}, {self.kx})")
        ptrs = (_dp * len(arrs))(*[k.ctypes.data_as(_dp) for k in arrs])
        _check(_lib.lp_kernel_spectra(self._p, ptrs))
        return self

    @property
    def form(self):
        return int(_lib.lp_plan_spectrum_form(self._p))

    def read_spectrum(self):
        """Stored spectrum (scaled by 1/(Py Px)) as complex64 Py x (Px/2+1)."""
        py, px = self.padding
        out = np.empty((py, px // 2 + 1, 2), np.float32)
        _check(_lib.lp_plan_read_spectrum(self._p, out.ctypes.data_as(_fp)))
        return out[..., 0] + 1j * out[..., 1]

    def _io(self, x, out):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
                and x.is_contiguous() and tuple(x.shape) == (self.ny, self.nx)):
            raise ValueError(f"expected a contiguous float32 CUDA tensor of shape ({self.ny}, {self.nx})")
        if out is None:
            out = torch.empty_like(x)
        elif not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
                  and tuple(out.shape) == (self.ny, self.nx)):
            raise ValueError("bad output tensor")
        return out

    def convolve(self, radiance, out=None):
        """S = K (*) R, "same" size, on the bound stream (lp_convolve),
        ordered with torch's current stream."""
        out = self._io(radiance, out)
        _ordered(self.stream, [radiance, out],
                 lambda: _check(_lib.lp_convolve(self._p, ctypes.c_void_p(radiance.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()))))
        return out

    def convolve_noalloc(self, radiance, out):
        """lp_convolve_noalloc: as convolve, with the intermediate in the
        library's own device scratch array (the call allocates nothing; `out`
        must be given).  Calls that overlap on one GPU race."""
        out = self._io(radiance, out)
        _ordered(self.stream, [radiance, out],
                 lambda: _check(_lib.lp_convolve_noalloc(self._p, ctypes.c_void_p(radiance.data_ptr()),
                                                         ctypes.c_void_p(out.data_ptr()))))
        return out

    def adjoint(self, grad_out, out=None):
        """Transposed operator (lp_adjoint), ordered as convolve."""
        out = self._io(grad_out, out)
        _ordered(self.stream, [grad_out, out],
                 lambda: _check(_lib.lp_adjoint(self._p, ctypes.c_void_p(grad_out.data_ptr()),
                                                ctypes.c_void_p(out.data_ptr()))))
        return out

    def convolve_classes(self, maps, out=None):
        """B = sum_t K_t (*) L_t over the plan's classes (lp_convolve_classes)."""
        if len(maps) != self.classes:
            raise ValueError(f"{len(maps)} maps for {self.classes} classes")
        out = self._io(maps[0], out)
        for m in maps[1:]:
            self._io(m, out)
        ptrs = (_vp * len(maps))(*[m.data_ptr() for m in maps])
        _ordered(self.stream, list(maps) + [out],
                 lambda: _check(_lib.lp_convolve_classes(self._p, ptrs, ctypes.c_void_p(out.data_ptr()))))
        return out

    def adjoint_class(self, cls, grad_out, out=None):
        """C_cls^T grad_out (lp_adjoint_class)."""
        out = self._io(grad_out, out)
        _ordered(self.stream, [grad_out, out],
                 lambda: _check(_lib.lp_adjoint_class(self._p, int(cls), ctypes.c_void_p(grad_out.data_ptr()),
                                                      ctypes.c_void_p(out.data_ptr()))))
        return out

    def set_kernels(self, which):
        """KERNELS_AUTO (specialised column kernel where available) or
        KERNELS_GENERIC."""
        _check(_lib.lp_plan_set_kernels(self._p, int(which)))

    @property
    def kernels(self):
        return int(_lib.lp_plan_kernels(self._p))

    def set_precision(self, mode):
        """PRECISION_FP32, PRECISION_SPLIT_FP16 or PRECISION_SPLIT_BF16
        (radix-16 passes on matrix cores); before bind."""
        _check(_lib.lp_plan_set_precision(self._p, int(mode)))

    @property
    def precision(self):
        return int(_lib.lp_plan_precision(self._p))

    def variant_count(self, stage):
        return int(_lib.lp_plan_variant_count(self._p, int(stage)))

    def variant(self, stage):
        return int(_lib.lp_plan_get_variant(self._p, int(stage)))

    def set_variant(self, stage, k):
        _check(_lib.lp_plan_set_variant(self._p, int(stage), int(k)))

    def variant_info(self, stage, k):
        """dict(radices, threads per transform, transforms per workgroup,
        min waves per SIMD, tiles per workgroup (0: persistent loop), length,
        half exchange, staged, matrix core)."""
        v = (ctypes.c_int * 11)()
        _check(_lib.lp_plan_variant_info(self._p, int(stage), int(k), v, 11))
        return {"radices": (v[0], v[1], v[2]), "threads": v[3], "per_group": v[4],
                "min_waves": v[5], "tiles_per_group": v[6], "length": v[7], "half_exchange": bool(v[8]),
                "staged": bool(v[9]), "matrix_core": bool(v[10])}

    def set_poison(self, enable=True):
        """NaN-fill the intermediates before every call (lp_plan_set_poison)."""
        _check(_lib.lp_plan_set_poison(self._p, int(bool(enable))))

    def timing(self, enable=True, every=1):
        """Stage events on every `every`-th call from the next one
        (lp_plan_timing); enable=False stops."""
        _check(_lib.lp_plan_timing(self._p, int(every) if enable else 0))

    def stage_ms(self):
        """(per-stage summed ms [rows fwd, columns, rows inv], calls)."""
        ms = (ctypes.c_double * 3)()
        calls = ctypes.c_int()
        _check(_lib.lp_plan_stage_ms(self._p, ms, 3, ctypes.byref(calls)))
        return list(ms), calls.value


class Batch:
    """Many maps with a few kernels (lp_batch_*): tiles x bands."""

    def __init__(self, shapes, psf_ids, psf_shapes, pitch_km=0.5, lengths=None):
        """lengths: optional (column lengths, row lengths) the padding classes
        may use (subsets of spec_lengths())."""
        n = len(shapes)
        ny = (ctypes.c_int64 * n)(*[int(s[0]) for s in shapes])
        nx = (ctypes.c_int64 * n)(*[int(s[1]) for s in shapes])
        ids = (ctypes.c_int * n)(*[int(i) for i in psf_ids])
        npsf = len(psf_shapes)
        ky = (ctypes.c_int64 * npsf)(*[int(s[0]) for s in psf_shapes])
        kx = (ctypes.c_int64 * npsf)(*[int(s[1]) for s in psf_shapes])
        if lengths is None:
            self._b = _lib.lp_batch_create(n, ny, nx, ids, npsf, ky, kx, float(pitch_km))
        else:
            ly = (ctypes.c_int64 * max(1, len(lengths[0])))(*lengths[0])
            lx = (ctypes.c_int64 * max(1, len(lengths[1])))(*lengths[1])
            self._b = _lib.lp_batch_create_padded(n, ny, nx, ids, npsf, ky, kx, float(pitch_km),
                                                  ly, len(lengths[0]), lx, len(lengths[1]))
        if not self._b:
            raise LPError(_lib.lp_last_status(), last_error())
        self.shapes = [(int(a), int(b)) for a, b in shapes]
        self.psf_shapes = [tuple(p) for p in psf_shapes]
        self.workspace = None
        self.stream = None

    def close(self):
        if getattr(self, "_b", None) and _lib is not None:
            _lib.lp_batch_destroy(self._b)
            self._b = None

    __del__ = close

    @property
    def workspace_bytes(self):
        return int(_lib.lp_batch_workspace_bytes(self._b))

    def bind(self, device=None, stream=None):
        import torch
        dev = torch.device("cuda") if device is None else torch.device(device)
        ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        ptr = ws.data_ptr()
        off = (-ptr) % 256
        self.workspace = ws
        self.stream = torch.cuda.current_stream(dev) if stream is None else stream
        _check(_lib.lp_batch_bind(self._b, ctypes.c_void_p(ptr + off), ws.numel() - off,
                                  _stream_ptr(self.stream)))
        return self

    def set_kernels(self, psfs):
        arrs = [np.ascontiguousarray(p, dtype=np.float64) for p in psfs]
        for a, sh in zip(arrs, self.psf_shapes):
            if a.shape != sh:
                raise ValueError(f"kernel shape {a.shape} != {sh}")
        ptrs = (_dp * len(arrs))(*[a.ctypes.data_as(_dp) for a in arrs])
        _check(_lib.lp_batch_kernel_spectra(self._b, ptrs))
        self._psfs = arrs
        return self

    def set_output_rows(self, tile, first, count):
        """Keep only rows [first, first + count) of map `tile`'s output
        (lp_batch_set_output_rows); its output tensor is then count x nx."""
        _check(_lib.lp_batch_set_output_rows(self._b, int(tile), int(first), int(count)))
        if not hasattr(self, "_out_rows"):
            self._out_rows = {}
        self._out_rows[int(tile)] = int(count)

    def convolve(self, maps, outs=None):
        """maps: list of contiguous float32 CUDA tensors (shape per map)."""
        import torch
        rows = getattr(self, "_out_rows", {})
        oshapes = [(rows.get(t, sh[0]), sh[1]) for t, sh in enumerate(self.shapes)]
        n = len(self.shapes)
        if len(maps) != n:
            raise ValueError(f"{len(maps)} maps for a batch of {n}")
        if outs is None:
            outs = [torch.empty(osh, dtype=torch.float32, device=m.device) for m, osh in zip(maps, oshapes)]
        elif len(outs) != n:
            raise ValueError(f"{len(outs)} outputs for a batch of {n}")
        for t, (m, o, sh, osh) in enumerate(zip(maps, outs, self.shapes, oshapes)):
            for x, want, what in ((m, sh, "map"), (o, osh, "output")):
                if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
                        and x.is_contiguous() and tuple(x.shape) == want):
                    raise ValueError(f"{what} {t}: expected a contiguous float32 CUDA tensor of shape {want}")
        ins = (_vp * n)(*[m.data_ptr() for m in maps])
        ous = (_vp * n)(*[o.data_ptr() for o in outs])
        _ordered(self.stream, list(maps) + list(outs),
                 lambda: _check(_lib.lp_convolve_batched(self._b, ins, ous)))
        return outs

    def use_graph(self, enable=True):
        _check(_lib.lp_batch_use_graph(self._b, int(bool(enable))))

    @property
    def groups(self):
        out = []
        for g in range(_lib.lp_batch_group_count(self._b)):
            v = (ctypes.c_int64 * 6)()
            _check(_lib.lp_batch_group_info(self._b, g, v, 6))
            out.append({"padding": (v[0], v[1]), "maps": v[2], "row_variants": v[3],
                        "column_variants": v[4], "max_ny": v[5]})
        return out

    def tile_group(self, t):
        return int(_lib.lp_batch_tile_group(self._b, int(t)))

    def set_variant(self, g, stage, k):
        _check(_lib.lp_batch_set_variant(self._b, int(g), int(stage), int(k)))

    def set_poison(self, enable=True):
        """NaN-fill every map's intermediate before each call (lp_batch_set_poison)."""
        _check(_lib.lp_batch_set_poison(self._b, int(bool(enable))))

    def set_graph_branches(self, n):
        """Classes captured on n parallel graph branches (1 to 4)."""
        _check(_lib.lp_batch_set_graph_branches(self._b, int(n)))

    def variant(self, g, stage):
        return int(_lib.lp_batch_get_variant(self._b, int(g), int(stage)))


def spec_lengths():
    """(column lengths, row lengths) that have specialised kernels."""
    out = []
    for axis in (0, 1):
        n = _lib.lp_batch_spec_lengths(axis, None, 0)
        v = (ctypes.c_int64 * n)()
        _lib.lp_batch_spec_lengths(axis, v, n)
        out.append(list(v))
    return tuple(out)


def reproject_nn(src, src_grid, dst_grid, *, ground_area=False, out=None, stream=None):
    """Nearest-neighbour reprojection of a longitude-latitude map onto a
    transverse Mercator grid (lp_reproject_nn).  src: CUDA float32
    (rows, cols) tensor; src_grid: LatLonGrid; dst_grid: TMGrid."""
    import torch
    if not (isinstance(src, torch.Tensor) and src.is_cuda and src.dtype == torch.float32
            and src.is_contiguous() and tuple(src.shape) == (src_grid.rows, src_grid.cols)):
        raise ValueError("src must be a contiguous CUDA float32 tensor of the source grid's shape")
    if out is None:
        out = torch.empty((dst_grid.rows, dst_grid.cols), dtype=torch.float32, device=src.device)
    elif not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
              and tuple(out.shape) == (dst_grid.rows, dst_grid.cols)):
        raise ValueError("bad output tensor")
    st = torch.cuda.current_stream(src.device) if stream is None else stream
    _check(_lib.lp_reproject_nn(ctypes.byref(src_grid), ctypes.c_void_p(src.data_ptr()),
                                ctypes.byref(dst_grid), ctypes.c_void_p(out.data_ptr()),
                                int(bool(ground_area)), _stream_ptr(st)))
    return out


def next_5smooth(n, even=False):
    """Smallest 2^a 3^b 5^c >= n (even if asked)."""
    m = max(1, int(n))
    while True:
        r = m
        for f in (2, 3, 5):
            while r % f == 0:
                r //= f
        if r == 1 and (not even or m % 2 == 0):
            return m
        m += 1


def window_padding(ny, nx, ky, kx):
    """Smallest padded size that still gives the exact input-sized window:
    5-smooth, >= n + floor(k/2) per axis, even along x (lp_plan_set_padding)."""
    return next_5smooth(ny + ky // 2), next_5smooth(nx + kx // 2, even=True)


def make_plan(psf, ny, nx, *, pitch_km=0.5, padding=None, device=None, kernels=KERNELS_AUTO,
              precision=PRECISION_FP32):
    """Plan + workspace + kernel spectrum in one call."""
    psf = np.asarray(psf)
    p = Plan(ny, nx, psf.shape[0], psf.shape[1], pitch_km, padding)
    p.set_kernels(kernels)
    p.set_precision(precision)
    p.bind(device=device)
    p.set_kernel(psf)
    return p


def make_plan_classes(psfs, ny, nx, *, pitch_km=0.5, padding=None, device=None,
                      kernels=KERNELS_AUTO, precision=PRECISION_FP32):
    """Plan for a sum over source classes (Eq. 4), one kernel per class."""
    psfs = [np.asarray(k) for k in psfs]
    p = Plan(ny, nx, psfs[0].shape[0], psfs[0].shape[1], pitch_km, padding)
    p.set_classes(len(psfs))
    p.set_kernels(kernels)
    p.set_precision(precision)
    p.bind(device=device)
    p.set_kernels_classes(psfs)
    return p


def _autograd():
    import torch

    class LPConvolve(torch.autograd.Function):
        """S = conv(R) with gradient grad_R = conv^T(grad_S) (lp_adjoint)."""

        @staticmethod
        def forward(ctx, radiance, plan):
            ctx.plan = plan
            return plan.convolve(radiance.contiguous())

        @staticmethod
        def backward(ctx, grad_s):
            return ctx.plan.adjoint(grad_s.contiguous()), None

    class LPConvolveClasses(torch.autograd.Function):
        """B = sum_t C_t(L_t); grad L_t = C_t^T(grad B) (lp_adjoint_class)."""

        @staticmethod
        def forward(ctx, plan, *maps):
            ctx.plan = plan
            return plan.convolve_classes([m.contiguous() for m in maps])

        @staticmethod
        def backward(ctx, grad_b):
            g = grad_b.contiguous()
            return (None,) + tuple(ctx.plan.adjoint_class(t, g) for t in range(ctx.plan.classes))

    return LPConvolve, LPConvolveClasses


_LPConvolve = None
_LPConvolveClasses = None


def convolve(radiance, plan):
    """Differentiable "same" convolution through the plan."""
    global _LPConvolve, _LPConvolveClasses
    if _LPConvolve is None:
        _LPConvolve, _LPConvolveClasses = _autograd()
    return _LPConvolve.apply(radiance, plan)


def convolve_classes(maps, plan):
    """Differentiable class sum of Eq. 4 through a plan of len(maps) classes."""
    global _LPConvolve, _LPConvolveClasses
    if _LPConvolve is None:
        _LPConvolve, _LPConvolveClasses = _autograd()
    return _LPConvolveClasses.apply(plan, *maps)
