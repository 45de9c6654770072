"""Python binding of the C ABI in include/simradar.h (ctypes).

Argument marshalling only: every step of the fast-mode path runs in the HIP
library.  The module raises ImportError when the library is not built; there
is no other implementation behind it.

Low-level functions keep the C names (``sim_create``, ``sim_surface_update``,
...) and take raw device pointers; :class:`Simulator` wraps a context and its
workspace and accepts torch tensors.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsimradar.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                      "(run python -m paper_2408_11472_amd.build)")

_lib = ctypes.CDLL(LIB_PATH)

SIM_OK = 0
SIM_ERR_ARG = 1
SIM_ERR_SHAPE = 2
SIM_ERR_UNSUPPORTED = 3
SIM_ERR_WORKSPACE = 4
SIM_ERR_DEVICE = 5

SIM_PREC_FP64 = 0
SIM_PREC_FP32_PHASE64 = 1

SIM_CODE_NONFINITE = -1
SIM_CODE_FOLDED = -2
SIM_CODE_OUT_OF_WINDOW = -3
SIM_CODE_BACKFACING = -4

COUNTER_NAMES = ("illuminated", "out_of_window", "folded", "backfacing",
                 "nonfinite", "window_overflow")
FACET_FIELDS = ("disp_x", "disp_y", "h", "sx", "sy", "jac",
                "ddisp_x", "ddisp_y", "dh")

EXPORTED = ("sim_abi_version", "sim_status_string", "sim_create", "sim_destroy",
            "sim_get_precision", "sim_workspace_size", "sim_set_workspace",
            "sim_surface_update", "sim_range_doppler_accumulate",
            "sim_update_and_accumulate", "sim_segments_to_iq",
            "sim_profile_enable", "sim_profile_read")

KERNEL_KINDS = ("surface_colpass", "surface_rowpass", "fused_rowpass", "accumulate_facets",
                "reduce_partials", "segments_to_iq")


class sim_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("cwm", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("x_origin", ctypes.c_double), ("y_origin", ctypes.c_double),
                ("gravity", ctypes.c_double)]


class sim_radar(ctypes.Structure):
    _fields_ = [("altitude", ctypes.c_double), ("velocity", ctypes.c_double),
                ("sat_x", ctypes.c_double), ("sat_y0", ctypes.c_double),
                ("carrier_hz", ctypes.c_double), ("prf_hz", ctypes.c_double),
                ("gate_spacing", ctypes.c_double), ("window_start", ctypes.c_double),
                ("beamwidth_3db", ctypes.c_double), ("fresnel_sq", ctypes.c_double),
                ("mss", ctypes.c_double),
                ("n_gates", ctypes.c_int32), ("n_doppler", ctypes.c_int32),
                ("n_fast", ctypes.c_int32), ("window", ctypes.c_int32)]


class sim_facets(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in FACET_FIELDS]


class sim_kernel_times(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 6), ("launches", ctypes.c_uint64 * 6)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double

_sig = {
    "sim_abi_version": (ctypes.c_int, []),
    "sim_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sim_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int]),
    "sim_destroy": (ctypes.c_int, [_P]),
    "sim_get_precision": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "sim_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid),
                                          ctypes.POINTER(sim_radar),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "sim_set_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "sim_surface_update": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid), _P, _D, _D,
                                          ctypes.POINTER(sim_facets), _P]),
    "sim_range_doppler_accumulate": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid),
                                                    ctypes.POINTER(sim_facets),
                                                    ctypes.POINTER(sim_radar), _D, _I, _P,
                                                    _I, _P, _P, _P]),
    "sim_update_and_accumulate": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid), _P,
                                                 ctypes.POINTER(sim_radar), _D, _I, _P, _I,
                                                 _P, _P, _P]),
    "sim_segments_to_iq": (ctypes.c_int, [_P, ctypes.POINTER(sim_radar), _P, _I, _P, _P]),
    "sim_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "sim_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(sim_kernel_times)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class SimError(RuntimeError):
    def __init__(self, call, status):
        self.status = status
        msg = _lib.sim_status_string(status).decode()
        super().__init__(f"{call} failed: {msg} (status {status})")


def _check(call, status):
    if status != SIM_OK:
        raise SimError(call, status)


# ---- low-level: same names as the C ABI --------------------------------

def sim_abi_version() -> int:
    return _lib.sim_abi_version()


def sim_status_string(status: int) -> str:
    return _lib.sim_status_string(status).decode()


def sim_create(device: int, precision: int) -> int:
    ctx = _P()
    _check("sim_create", _lib.sim_create(ctypes.byref(ctx), device, precision))
    return ctx.value


def sim_destroy(ctx) -> None:
    _check("sim_destroy", _lib.sim_destroy(ctx))


def sim_workspace_size(ctx, grid: sim_grid, radar: sim_radar) -> int:
    n = ctypes.c_size_t()
    _check("sim_workspace_size",
           _lib.sim_workspace_size(ctx, ctypes.byref(grid), ctypes.byref(radar), ctypes.byref(n)))
    return n.value


def sim_set_workspace(ctx, ptr, nbytes) -> None:
    _check("sim_set_workspace", _lib.sim_set_workspace(ctx, ptr, nbytes))


def sim_surface_update(ctx, grid, spec0_ptr, t, dt_pair, facets: sim_facets, stream) -> None:
    _check("sim_surface_update",
           _lib.sim_surface_update(ctx, ctypes.byref(grid), spec0_ptr, t, dt_pair,
                                   ctypes.byref(facets), stream))


def sim_range_doppler_accumulate(ctx, grid, facets: sim_facets, radar, t, j, t_fast_ptr,
                                 n_spec, counters_ptr, code_ptr, stream) -> None:
    _check("sim_range_doppler_accumulate",
           _lib.sim_range_doppler_accumulate(ctx, ctypes.byref(grid), ctypes.byref(facets),
                                             ctypes.byref(radar), t, j, t_fast_ptr, n_spec,
                                             counters_ptr, code_ptr, stream))


def sim_update_and_accumulate(ctx, grid, spec0_ptr, radar, t, j, t_fast_ptr, n_spec,
                              counters_ptr, code_ptr, stream) -> None:
    _check("sim_update_and_accumulate",
           _lib.sim_update_and_accumulate(ctx, ctypes.byref(grid), spec0_ptr,
                                          ctypes.byref(radar), t, j, t_fast_ptr, n_spec,
                                          counters_ptr, code_ptr, stream))


def sim_segments_to_iq(ctx, radar, t_fast_ptr, n_spec, y_ptr, stream) -> None:
    _check("sim_segments_to_iq",
           _lib.sim_segments_to_iq(ctx, ctypes.byref(radar), t_fast_ptr, n_spec, y_ptr, stream))


def sim_profile_enable(ctx, enable: bool) -> None:
    _check("sim_profile_enable", _lib.sim_profile_enable(ctx, 1 if enable else 0))


def sim_profile_read(ctx) -> dict:
    out = sim_kernel_times()
    _check("sim_profile_read", _lib.sim_profile_read(ctx, ctypes.byref(out)))
    return {k: (out.ms[i], int(out.launches[i])) for i, k in enumerate(KERNEL_KINDS)}


# ---- conversions ---------------------------------------------------------

def grid_struct(g) -> sim_grid:
    """sim_grid from any object with the grid attributes."""
    return sim_grid(int(g.nx), int(g.ny), int(bool(g.cwm)), 0, float(g.dx), float(g.dy),
                    float(g.x_origin), float(g.y_origin), float(g.gravity))


def radar_struct(r) -> sim_radar:
    return sim_radar(float(r.altitude), float(r.velocity), float(r.sat_x), float(r.sat_y0),
                     float(r.carrier_hz), float(r.prf_hz), float(r.gate_spacing),
                     float(r.window_start), float(r.beamwidth_3db), float(r.fresnel_sq),
                     float(r.mss), int(r.n_gates), int(r.n_doppler), int(r.n_fast),
                     int(r.window))


# ---- tensor-level wrapper -------------------------------------------------

class Simulator:
    """A context with its workspace, sized for one (grid, radar) pair.

    ``precision`` is SIM_PREC_FP32_PHASE64 (float facets, complex64 spectra)
    or SIM_PREC_FP64 (double, complex128)."""

    def __init__(self, grid, radar, precision=SIM_PREC_FP32_PHASE64, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.precision = precision
        self.real_dtype = torch.float64 if precision == SIM_PREC_FP64 else torch.float32
        self.complex_dtype = torch.complex128 if precision == SIM_PREC_FP64 else torch.complex64
        self.grid = grid_struct(grid)
        self.radar = radar_struct(radar)
        self.ctx = sim_create(device, precision)
        nbytes = sim_workspace_size(self.ctx, self.grid, self.radar)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        sim_set_workspace(self.ctx, self._ws_ptr, nbytes)

    def close(self):
        if self.ctx:
            sim_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # helpers
    def _stream(self, stream=None):
        s = stream if stream is not None else self.torch.cuda.current_stream(self.device)
        return s.cuda_stream

    def _need(self, t, dtype, shape=None, name="tensor"):
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous {dtype} CUDA tensor")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t.data_ptr()

    def empty_facets(self):
        g = self.grid
        return {n: self.torch.empty((g.ny, g.nx), dtype=self.real_dtype, device=self.device)
                for n in FACET_FIELDS}

    def _facets_struct(self, fac):
        g = self.grid
        ptrs = [self._need(fac[n], self.real_dtype, (g.ny, g.nx), n) for n in FACET_FIELDS]
        return sim_facets(*ptrs)

    def empty_spectra(self, n_spec):
        r = self.radar
        return self.torch.zeros((n_spec, r.n_gates, r.n_doppler), dtype=self.complex_dtype,
                                device=self.device)

    def counters(self):
        return self.torch.zeros(6, dtype=self.torch.int64, device=self.device)

    # the hot-path calls
    def surface_update(self, spec0, t, dt_pair, out=None, stream=None):
        g = self.grid
        out = out if out is not None else self.empty_facets()
        sim_surface_update(self.ctx, self.grid,
                           self._need(spec0, self.complex_dtype, (g.ny, g.nx), "spec0"),
                           float(t), float(dt_pair), self._facets_struct(out),
                           self._stream(stream))
        return out

    def range_doppler_accumulate(self, facets, t, j, t_fast, counters=None, facet_code=None,
                                 stream=None):
        n_spec = t_fast.shape[0]
        r = self.radar
        g = self.grid
        sim_range_doppler_accumulate(
            self.ctx, self.grid, self._facets_struct(facets), self.radar, float(t), int(j),
            self._need(t_fast, self.complex_dtype, (n_spec, r.n_gates, r.n_doppler), "t_fast"),
            n_spec,
            None if counters is None else self._need(counters, self.torch.int64, (6,), "counters"),
            None if facet_code is None else self._need(facet_code, self.torch.int32,
                                                       (g.ny, g.nx), "facet_code"),
            self._stream(stream))

    def update_and_accumulate(self, spec0, t, j, t_fast, counters=None, facet_code=None,
                              stream=None):
        n_spec = t_fast.shape[0]
        r = self.radar
        g = self.grid
        sim_update_and_accumulate(
            self.ctx, self.grid, self._need(spec0, self.complex_dtype, (g.ny, g.nx), "spec0"),
            self.radar, float(t), int(j),
            self._need(t_fast, self.complex_dtype, (n_spec, r.n_gates, r.n_doppler), "t_fast"),
            n_spec,
            None if counters is None else self._need(counters, self.torch.int64, (6,), "counters"),
            None if facet_code is None else self._need(facet_code, self.torch.int32,
                                                       (g.ny, g.nx), "facet_code"),
            self._stream(stream))

    def segments_to_iq(self, t_fast, y=None, stream=None):
        r = self.radar
        n_spec = t_fast.shape[0]
        if y is None:
            y = self.torch.empty(((n_spec - 1) * r.n_fast, r.n_gates), dtype=self.complex_dtype,
                                 device=self.device)
        sim_segments_to_iq(self.ctx, self.radar,
                           self._need(t_fast, self.complex_dtype,
                                      (n_spec, r.n_gates, r.n_doppler), "t_fast"),
                           n_spec,
                           self._need(y, self.complex_dtype,
                                      ((n_spec - 1) * r.n_fast, r.n_gates), "y"),
                           self._stream(stream))
        return y

    def profile(self, enable: bool = True):
        """Start (clearing) or stop per-kernel event timing."""
        sim_profile_enable(self.ctx, enable)

    def profile_read(self) -> dict:
        """{kernel kind: (summed ms, launches)} since profiling was enabled."""
        return sim_profile_read(self.ctx)

    def run(self, spec0, n_updates, t_fast=None, y=None, counters=None, stream=None):
        """Algorithm 1 and post-processing: U + 1 spectra, then Y."""
        t_fast = t_fast if t_fast is not None else self.empty_spectra(n_updates + 1)
        r = self.radar
        for j in range(n_updates + 1):
            t = (j * r.n_fast) / r.prf_hz
            self.update_and_accumulate(spec0, t, j, t_fast, counters=counters, stream=stream)
        return t_fast, self.segments_to_iq(t_fast, y, stream=stream)
