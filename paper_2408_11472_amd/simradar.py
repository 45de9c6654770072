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
# SIMRADAR_LIB selects another build of the same library (for instance one
# compiled with other launch constants); the default is the in-tree build.
LIB_PATH = os.environ.get("SIMRADAR_LIB") or os.path.join(HERE, "libsimradar.so")

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
            "sim_range_doppler_accumulate_noalloc", "sim_update_and_accumulate", "sim_prepared_spectrum_size", "sim_prepare_spectrum",
            "sim_update_and_accumulate_prepared", "sim_run_updates", "sim_segments_to_iq",
            "sim_waveform_loss", "sim_waveform_loss_adjoint", "sim_segments_to_iq_adjoint",
            "sim_range_doppler_accumulate_adjoint", "sim_range_doppler_accumulate_run",
            "sim_range_doppler_accumulate_adjoint_run",
            "sim_batch_create", "sim_batch_destroy", "sim_batch_workspace_size",
            "sim_batch_run", "sim_set_tuning", "sim_delay_doppler", "sim_set_tables",
            "sim_streamer_create", "sim_streamer_destroy", "sim_streamer_cache_size",
            "sim_streamer_run", "sim_batch_set_mode", "sim_batch_set_tuning",
            "sim_profile_enable", "sim_profile_read")

SIM_TUNE_ROW_BANDS = 0
SIM_TUNE_ROW_PATH = 1
SIM_TUNE_UPDATE_LANES = 2
SIM_TUNE_ACC_BANDS = 3
SIM_ROW_PATH_AUTO, SIM_ROW_PATH_FUSED, SIM_ROW_PATH_SPLIT = 0, 1, 2

KERNEL_KINDS = ("surface_colpass", "surface_rowpass", "fused_rowpass", "accumulate_facets",
                "reduce_partials", "segments_to_iq", "adjoint", "prepare", "delay_doppler",
                "batched_update")
SIM_DD_CENTROID_GIVEN, SIM_DD_CENTROID_ESTIMATE = 0, 1


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
    _fields_ = [("ms", ctypes.c_double * len(KERNEL_KINDS)),
                ("launches", ctypes.c_uint64 * len(KERNEL_KINDS)),
                ("dropped", ctypes.c_uint64)]


class sim_tables(ctypes.Structure):
    _fields_ = [("antenna", ctypes.c_void_p), ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("u0", ctypes.c_double), ("du", ctypes.c_double), ("v0", ctypes.c_double),
                ("dv", ctypes.c_double), ("nrcs", ctypes.c_void_p),
                ("n_theta", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("dtheta", ctypes.c_double)]


class sim_dd_params(ctypes.Structure):
    _fields_ = [("burst", ctypes.c_int32), ("centroid_mode", ctypes.c_int32),
                ("centroid", ctypes.c_double), ("migration", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


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
    "sim_range_doppler_accumulate_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid),
                                                            ctypes.POINTER(sim_facets),
                                                            ctypes.POINTER(sim_radar), _D, _I,
                                                            _P, _I, _P, _P, _P]),
    "sim_update_and_accumulate": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid), _P,
                                                 ctypes.POINTER(sim_radar), _D, _I, _P, _I,
                                                 _P, _P, _P]),
    "sim_prepared_spectrum_size": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid),
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "sim_prepare_spectrum": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid), _P, _P, _P]),
    "sim_update_and_accumulate_prepared": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid), _P,
                                                          ctypes.POINTER(sim_radar), _D, _I, _P,
                                                          _I, _P, _P, _P]),
    "sim_run_updates": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid), _P, ctypes.POINTER(sim_radar),
                                       _I, _I, ctypes.POINTER(ctypes.c_double), _P, _I, _P, _P]),
    "sim_segments_to_iq": (ctypes.c_int, [_P, ctypes.POINTER(sim_radar), _P, _I, _P, _P]),
    "sim_waveform_loss": (ctypes.c_int, [_P, ctypes.POINTER(sim_radar), _P, _I, _P, _P, _P, _P]),
    "sim_waveform_loss_adjoint": (ctypes.c_int, [_P, ctypes.POINTER(sim_radar), _P, _I, _P, _P,
                                                 _P, _P, _P]),
    "sim_segments_to_iq_adjoint": (ctypes.c_int, [_P, ctypes.POINTER(sim_radar), _P, _I, _P,
                                                  _P]),
    "sim_range_doppler_accumulate_adjoint": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid),
                                                            ctypes.POINTER(sim_facets),
                                                            ctypes.POINTER(sim_radar), _D, _I,
                                                            _P, _I, _P, _P, _P, _P]),
    "sim_range_doppler_accumulate_run": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid),
                                                        ctypes.POINTER(sim_facets),
                                                        ctypes.POINTER(sim_radar), _I, _I,
                                                        ctypes.POINTER(ctypes.c_double), _P, _I,
                                                        _P, _P]),
    "sim_range_doppler_accumulate_adjoint_run": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid),
                                                                ctypes.POINTER(sim_facets),
                                                                ctypes.POINTER(sim_radar), _I, _I,
                                                                ctypes.POINTER(ctypes.c_double),
                                                                _P, _I, _P, _P, _P, _P]),
    "sim_batch_create": (ctypes.c_int, [_P, _I, ctypes.POINTER(sim_grid),
                                        ctypes.POINTER(sim_radar), ctypes.POINTER(_I),
                                        ctypes.POINTER(_P)]),
    "sim_batch_destroy": (ctypes.c_int, [_P]),
    "sim_batch_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "sim_batch_run": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                     ctypes.POINTER(_P), ctypes.c_int, _P]),
    "sim_set_tuning": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "sim_set_tables": (ctypes.c_int, [_P, ctypes.POINTER(sim_tables)]),
    "sim_batch_set_mode": (ctypes.c_int, [_P, ctypes.c_int]),
    "sim_batch_set_tuning": (ctypes.c_int, [_P, _I, ctypes.c_int, ctypes.c_int]),
    "sim_streamer_create": (ctypes.c_int, [_P, ctypes.POINTER(sim_radar), _I,
                                           ctypes.POINTER(_P)]),
    "sim_streamer_destroy": (ctypes.c_int, [_P]),
    "sim_streamer_cache_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "sim_streamer_run": (ctypes.c_int, [_P, ctypes.POINTER(sim_grid), _P, _I, _P, _P, _P,
                                        ctypes.c_size_t, _P]),
    "sim_delay_doppler": (ctypes.c_int, [_P, ctypes.POINTER(sim_radar), _P, _I,
                                         ctypes.POINTER(sim_dd_params), _P, _P, _P, _P, _P]),
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


def sim_range_doppler_accumulate_noalloc(ctx, grid, facets: sim_facets, radar, t, j,
                                         t_fast_ptr, n_spec, counters_ptr, code_ptr,
                                         stream) -> None:
    _check("sim_range_doppler_accumulate_noalloc",
           _lib.sim_range_doppler_accumulate_noalloc(ctx, ctypes.byref(grid),
                                                     ctypes.byref(facets), ctypes.byref(radar),
                                                     t, j, t_fast_ptr, n_spec, counters_ptr,
                                                     code_ptr, stream))


def sim_update_and_accumulate(ctx, grid, spec0_ptr, radar, t, j, t_fast_ptr, n_spec,
                              counters_ptr, code_ptr, stream) -> None:
    _check("sim_update_and_accumulate",
           _lib.sim_update_and_accumulate(ctx, ctypes.byref(grid), spec0_ptr,
                                          ctypes.byref(radar), t, j, t_fast_ptr, n_spec,
                                          counters_ptr, code_ptr, stream))


def sim_prepared_spectrum_size(ctx, grid) -> int:
    n = ctypes.c_size_t(0)
    _check("sim_prepared_spectrum_size",
           _lib.sim_prepared_spectrum_size(ctx, ctypes.byref(grid), ctypes.byref(n)))
    return n.value


def sim_prepare_spectrum(ctx, grid, spec0_ptr, prepared_ptr, stream) -> None:
    _check("sim_prepare_spectrum",
           _lib.sim_prepare_spectrum(ctx, ctypes.byref(grid), spec0_ptr, prepared_ptr, stream))


def sim_update_and_accumulate_prepared(ctx, grid, prepared_ptr, radar, t, j, t_fast_ptr, n_spec,
                                       counters_ptr, code_ptr, stream) -> None:
    _check("sim_update_and_accumulate_prepared",
           _lib.sim_update_and_accumulate_prepared(ctx, ctypes.byref(grid), prepared_ptr,
                                                   ctypes.byref(radar), t, j, t_fast_ptr, n_spec,
                                                   counters_ptr, code_ptr, stream))


def sim_run_updates(ctx, grid, prepared_ptr, radar, j0, times, t_fast_ptr, n_spec, counters_ptr,
                    stream) -> None:
    """times: sequence of the pulse times of updates j0, j0 + 1, ..."""
    arr = (ctypes.c_double * len(times))(*[float(x) for x in times])
    _check("sim_run_updates",
           _lib.sim_run_updates(ctx, ctypes.byref(grid), prepared_ptr, ctypes.byref(radar), j0,
                                len(times), arr, t_fast_ptr, n_spec, counters_ptr, stream))


def sim_segments_to_iq(ctx, radar, t_fast_ptr, n_spec, y_ptr, stream) -> None:
    _check("sim_segments_to_iq",
           _lib.sim_segments_to_iq(ctx, ctypes.byref(radar), t_fast_ptr, n_spec, y_ptr, stream))


def sim_waveform_loss(ctx, radar, y_ptr, n_pulses, target_ptr, p_ptr, loss_ptr, stream) -> None:
    _check("sim_waveform_loss",
           _lib.sim_waveform_loss(ctx, ctypes.byref(radar), y_ptr, n_pulses, target_ptr, p_ptr,
                                  loss_ptr, stream))


def sim_waveform_loss_adjoint(ctx, radar, y_ptr, n_pulses, p_ptr, target_ptr, scale_ptr,
                              y_bar_ptr, stream) -> None:
    _check("sim_waveform_loss_adjoint",
           _lib.sim_waveform_loss_adjoint(ctx, ctypes.byref(radar), y_ptr, n_pulses, p_ptr,
                                          target_ptr, scale_ptr, y_bar_ptr, stream))


def sim_segments_to_iq_adjoint(ctx, radar, y_bar_ptr, n_spec, t_bar_ptr, stream) -> None:
    _check("sim_segments_to_iq_adjoint",
           _lib.sim_segments_to_iq_adjoint(ctx, ctypes.byref(radar), y_bar_ptr, n_spec, t_bar_ptr,
                                           stream))


def _times(times):
    return (ctypes.c_double * len(times))(*[float(x) for x in times])


def sim_range_doppler_accumulate_run(ctx, grid, facets, radar, j0, times, t_fast_ptr, n_spec,
                                     counters_ptr, stream) -> None:
    _check("sim_range_doppler_accumulate_run",
           _lib.sim_range_doppler_accumulate_run(ctx, ctypes.byref(grid), ctypes.byref(facets),
                                                 ctypes.byref(radar), j0, len(times),
                                                 _times(times), t_fast_ptr, n_spec, counters_ptr,
                                                 stream))


def sim_range_doppler_accumulate_adjoint_run(ctx, grid, facets, radar, j0, times, t_bar_ptr,
                                             n_spec, gh_ptr, gsx_ptr, gsy_ptr, stream) -> None:
    _check("sim_range_doppler_accumulate_adjoint_run",
           _lib.sim_range_doppler_accumulate_adjoint_run(ctx, ctypes.byref(grid),
                                                         ctypes.byref(facets), ctypes.byref(radar),
                                                         j0, len(times), _times(times), t_bar_ptr,
                                                         n_spec, gh_ptr, gsx_ptr, gsy_ptr, stream))


def sim_range_doppler_accumulate_adjoint(ctx, grid, facets, radar, t, j, t_bar_ptr, n_spec,
                                         gh_ptr, gsx_ptr, gsy_ptr, stream) -> None:
    _check("sim_range_doppler_accumulate_adjoint",
           _lib.sim_range_doppler_accumulate_adjoint(ctx, ctypes.byref(grid),
                                                     ctypes.byref(facets), ctypes.byref(radar),
                                                     t, j, t_bar_ptr, n_spec, gh_ptr, gsx_ptr,
                                                     gsy_ptr, stream))


def sim_delay_doppler(ctx, radar, y_ptr, n_pulses, params: sim_dd_params, beams_ptr,
                      centroid_ptr, beam_power_ptr, waveform_ptr, stream) -> None:
    _check("sim_delay_doppler",
           _lib.sim_delay_doppler(ctx, ctypes.byref(radar), y_ptr, n_pulses,
                                  ctypes.byref(params), beams_ptr, centroid_ptr,
                                  beam_power_ptr, waveform_ptr, stream))


SIM_BATCH_LANES, SIM_BATCH_PERSISTENT = 1, 2


def sim_batch_set_mode(batch, mode) -> None:
    _check("sim_batch_set_mode", _lib.sim_batch_set_mode(batch, int(mode)))


def sim_batch_set_tuning(batch, member, key, value) -> None:
    _check("sim_batch_set_tuning", _lib.sim_batch_set_tuning(batch, int(member), int(key),
                                                              int(value)))


def sim_set_tables(ctx, tables) -> None:
    _check("sim_set_tables",
           _lib.sim_set_tables(ctx, None if tables is None else ctypes.byref(tables)))


def sim_streamer_create(ctx, radar, chunk_updates) -> int:
    h = _P()
    _check("sim_streamer_create",
           _lib.sim_streamer_create(ctx, ctypes.byref(radar), chunk_updates, ctypes.byref(h)))
    return h.value


def sim_streamer_destroy(streamer) -> None:
    _check("sim_streamer_destroy", _lib.sim_streamer_destroy(streamer))


def sim_streamer_cache_size(streamer) -> int:
    n = ctypes.c_size_t(0)
    _check("sim_streamer_cache_size", _lib.sim_streamer_cache_size(streamer, ctypes.byref(n)))
    return n.value


def sim_streamer_run(streamer, grid, prepared_ptr, n_updates, t_host_ptr, y_host_ptr,
                     cache_ptr, cache_bytes, stream) -> None:
    _check("sim_streamer_run",
           _lib.sim_streamer_run(streamer, ctypes.byref(grid), prepared_ptr, n_updates,
                                 t_host_ptr, y_host_ptr, cache_ptr, cache_bytes, stream))


def sim_set_tuning(ctx, key, value) -> None:
    _check("sim_set_tuning", _lib.sim_set_tuning(ctx, key, value))


def sim_batch_create(ctx, grids, radars, n_updates) -> int:
    n = len(grids)
    ga = (sim_grid * n)(*grids)
    ra = (sim_radar * n)(*radars)
    ua = (_I * n)(*n_updates)
    b = _P()
    _check("sim_batch_create", _lib.sim_batch_create(ctx, n, ga, ra, ua, ctypes.byref(b)))
    return b.value


def sim_batch_destroy(batch) -> None:
    _check("sim_batch_destroy", _lib.sim_batch_destroy(batch))


def sim_batch_workspace_size(batch) -> int:
    n = ctypes.c_size_t()
    _check("sim_batch_workspace_size", _lib.sim_batch_workspace_size(batch, ctypes.byref(n)))
    return n.value


def sim_batch_run(batch, spec_ptrs, t_ptrs, y_ptrs, use_graph, stream) -> None:
    n = len(spec_ptrs)
    sa = (_P * n)(*spec_ptrs)
    ta = (_P * n)(*t_ptrs)
    ya = None if y_ptrs is None else (_P * n)(*y_ptrs)
    _check("sim_batch_run", _lib.sim_batch_run(batch, sa, ta, ya, 1 if use_graph else 0, stream))


def sim_profile_enable(ctx, enable: bool) -> None:
    _check("sim_profile_enable", _lib.sim_profile_enable(ctx, 1 if enable else 0))


def sim_profile_read(ctx) -> dict:
    """{kernel kind: (summed ms, launches)}; raises when launches went untimed
    (more than the event pool holds), since the sums would be partial."""
    out = sim_kernel_times()
    _check("sim_profile_read", _lib.sim_profile_read(ctx, ctypes.byref(out)))
    if out.dropped:
        raise RuntimeError(f"sim_profile_read: {int(out.dropped)} launches were not timed "
                           "(event pool exhausted); profile fewer launches at a time")
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
        self.lanes = 1
        self._alloc_workspace()

    def _alloc_workspace(self):
        """Workspace of the context's current lane count (sim_workspace_size)."""
        nbytes = sim_workspace_size(self.ctx, self.grid, self.radar)
        self.workspace = None
        self.workspace = self.torch.empty(nbytes + 256, dtype=self.torch.uint8,
                                          device=self.device)
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

    def _facets_struct(self, fac, count=None):
        """sim_facets of a facet set ([ny][nx] fields) or, with count, of a
        stacked run ([count][ny][nx] fields)."""
        g = self.grid
        shape = (g.ny, g.nx) if count is None else (count, g.ny, g.nx)
        ptrs = [self._need(fac[n], self.real_dtype, shape, n) for n in FACET_FIELDS]
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

    def range_doppler_accumulate_noalloc(self, facets, t, j, t_fast, counters=None,
                                         facet_code=None, stream=None):
        """range_doppler_accumulate through the entry point that uses the
        library's static scratch instead of the workspace (allocates
        nothing)."""
        n_spec = t_fast.shape[0]
        r = self.radar
        g = self.grid
        sim_range_doppler_accumulate_noalloc(
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

    def prepare_spectrum(self, spec0, stream=None):
        """The spectrum in the column-pass layout (a complex tensor of
        sim_prepared_spectrum_size bytes), for update_and_accumulate_prepared."""
        g = self.grid
        n = self._prepared_elems()
        out = self.torch.empty(n, dtype=self.complex_dtype, device=self.device)
        sim_prepare_spectrum(self.ctx, g,
                             self._need(spec0, self.complex_dtype, (g.ny, g.nx), "spec0"),
                             out.data_ptr(), self._stream(stream))
        return out

    def _prepared_elems(self):
        cs = 16 if self.precision == SIM_PREC_FP64 else 8
        return sim_prepared_spectrum_size(self.ctx, self.grid) // cs

    def update_and_accumulate_prepared(self, prepared, t, j, t_fast, counters=None,
                                       facet_code=None, stream=None):
        n_spec = t_fast.shape[0]
        r = self.radar
        g = self.grid
        sim_update_and_accumulate_prepared(
            self.ctx, self.grid,
            self._need(prepared, self.complex_dtype, (self._prepared_elems(),), "prepared"),
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

    def set_row_bands(self, n: int):
        """Blocks of the fused row pass (a power of two <= 512; 0 = default)."""
        sim_set_tuning(self.ctx, SIM_TUNE_ROW_BANDS, int(n))

    def set_row_path(self, path: int):
        """Row path of update_and_accumulate: SIM_ROW_PATH_AUTO, _FUSED or _SPLIT."""
        sim_set_tuning(self.ctx, SIM_TUNE_ROW_PATH, int(path))

    def set_acc_bands(self, n: int):
        """Most bands (blocks) of the facet accumulate (0 = default 512, else a
        power of two from 64 to 512)."""
        sim_set_tuning(self.ctx, SIM_TUNE_ACC_BANDS, int(n))

    def set_update_lanes(self, lanes: int):
        """Streams run_updates deals the updates to (1 .. 4); the workspace is
        re-made for that many lanes (work queued on the old one must be done:
        the device is synchronised first)."""
        lanes = int(lanes)
        if lanes == self.lanes:
            return
        self.torch.cuda.synchronize(self.device)
        sim_set_tuning(self.ctx, SIM_TUNE_UPDATE_LANES, lanes)
        self.lanes = lanes
        self._alloc_workspace()

    def profile(self, enable: bool = True):
        """Start (clearing) or stop per-kernel event timing."""
        sim_profile_enable(self.ctx, enable)

    def profile_read(self) -> dict:
        """{kernel kind: (summed ms, launches)} since profiling was enabled."""
        return sim_profile_read(self.ctx)

    # differentiable chain
    def waveform_loss(self, y, target=None, stream=None):
        """(P, loss) with P[g] = mean_x |y[x][g]|^2, loss = sum (P - target)^2
        (loss is None when target is None)."""
        r = self.radar
        n_pulses = y.shape[0]
        P = self.torch.empty(r.n_gates, dtype=self.real_dtype, device=self.device)
        L = None
        tptr = None
        if target is not None:
            L = self.torch.empty(1, dtype=self.real_dtype, device=self.device)
            tptr = self._need(target, self.real_dtype, (r.n_gates,), "target")
        sim_waveform_loss(self.ctx, self.radar,
                          self._need(y, self.complex_dtype, (n_pulses, r.n_gates), "y"),
                          n_pulses, tptr, P.data_ptr(), None if L is None else L.data_ptr(),
                          self._stream(stream))
        return P, (None if L is None else L[0])

    def waveform_loss_adjoint(self, y, P, target, scale=None, stream=None):
        r = self.radar
        n_pulses = y.shape[0]
        yb = self.torch.empty_like(y)
        sim_waveform_loss_adjoint(
            self.ctx, self.radar, self._need(y, self.complex_dtype, (n_pulses, r.n_gates), "y"),
            n_pulses, self._need(P, self.real_dtype, (r.n_gates,), "P"),
            self._need(target, self.real_dtype, (r.n_gates,), "target"),
            None if scale is None else self._need(scale, self.real_dtype, (1,), "scale"),
            yb.data_ptr(), self._stream(stream))
        return yb

    def segments_to_iq_adjoint(self, y_bar, n_spec, stream=None):
        r = self.radar
        tb = self.torch.empty((n_spec, r.n_gates, r.n_doppler), dtype=self.complex_dtype,
                              device=self.device)
        sim_segments_to_iq_adjoint(
            self.ctx, self.radar,
            self._need(y_bar, self.complex_dtype, ((n_spec - 1) * r.n_fast, r.n_gates), "y_bar"),
            n_spec, tb.data_ptr(), self._stream(stream))
        return tb

    def range_doppler_accumulate_run(self, facets, times, j0, t_fast, counters=None, stream=None):
        """range_doppler_accumulate of updates j0 .. j0 + len(times) - 1 in one
        call; every field of `facets` is [len(times)][ny][nx]."""
        n_spec = t_fast.shape[0]
        r = self.radar
        sim_range_doppler_accumulate_run(
            self.ctx, self.grid, self._facets_struct(facets, len(times)), self.radar, int(j0),
            times,
            self._need(t_fast, self.complex_dtype, (n_spec, r.n_gates, r.n_doppler), "t_fast"),
            n_spec,
            None if counters is None else self._need(counters, self.torch.int64, (6,), "counters"),
            self._stream(stream))

    def range_doppler_accumulate_adjoint_run(self, facets, times, j0, t_bar, out, stream=None):
        """range_doppler_accumulate_adjoint of updates j0 .. j0 + len(times) - 1
        in one call; the fields of `facets` and the three gradients of `out`
        (h, sx, sy) are [len(times)][ny][nx]."""
        g = self.grid
        r = self.radar
        n_spec = t_bar.shape[0]
        count = len(times)
        ptrs = [self._need(o, self.real_dtype, (count, g.ny, g.nx), "gradient") for o in out]
        sim_range_doppler_accumulate_adjoint_run(
            self.ctx, self.grid, self._facets_struct(facets, count), self.radar, int(j0), times,
            self._need(t_bar, self.complex_dtype, (n_spec, r.n_gates, r.n_doppler), "t_bar"),
            n_spec, ptrs[0], ptrs[1], ptrs[2], self._stream(stream))
        return {"h": out[0], "sx": out[1], "sy": out[2]}

    def range_doppler_accumulate_adjoint(self, facets, t, j, t_bar, out=None, stream=None):
        g = self.grid
        r = self.radar
        n_spec = t_bar.shape[0]
        if out is None:
            out = [self.torch.empty((g.ny, g.nx), dtype=self.real_dtype, device=self.device)
                   for _ in range(3)]
        for o in out:
            self._need(o, self.real_dtype, (g.ny, g.nx), "gradient")
        sim_range_doppler_accumulate_adjoint(
            self.ctx, self.grid, self._facets_struct(facets), self.radar, float(t), int(j),
            self._need(t_bar, self.complex_dtype, (n_spec, r.n_gates, r.n_doppler), "t_bar"),
            n_spec, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), self._stream(stream))
        return {"h": out[0], "sx": out[1], "sy": out[2]}

    def set_tables(self, antenna=None, u0=0.0, du=1.0, v0=0.0, dv=1.0, nrcs=None, dtheta=1.0):
        """Look-up tables of the facet amplitude (sim_set_tables): antenna
        [nv][nu] complex and/or nrcs [n_theta] real device tensors of the
        context's precision, kept referenced by this object; both None
        restores the closed forms."""
        if antenna is None and nrcs is None:
            sim_set_tables(self.ctx, None)
            self._tables = None
            return
        t = sim_tables(reserved=0)
        if antenna is not None:
            self._need(antenna, self.complex_dtype, None, "antenna")
            if antenna.dim() != 2:
                raise ValueError("antenna: expected a [nv][nu] tensor")
            t.antenna = antenna.data_ptr()
            t.nv, t.nu = int(antenna.shape[0]), int(antenna.shape[1])
            t.u0, t.du, t.v0, t.dv = float(u0), float(du), float(v0), float(dv)
        if nrcs is not None:
            self._need(nrcs, self.real_dtype, None, "nrcs")
            if nrcs.dim() != 1:
                raise ValueError("nrcs: expected a [n_theta] tensor")
            t.nrcs = nrcs.data_ptr()
            t.n_theta = int(nrcs.shape[0])
            t.dtheta = float(dtheta)
        sim_set_tables(self.ctx, t)
        self._tables = (antenna, nrcs)

    def run_streamed(self, prepared, n_updates, chunk_updates, t_host=None, y_host=None,
                     keep_spectra=True, stream=None):
        """A whole run with T_fast and Y in (pinned) host memory and device
        caches of chunk_updates update intervals (sim_streamer_*).  Returns
        (T_host or None, Y_host) once the stream has completed."""
        t = self.torch
        r = self.radar
        n_spec = n_updates + 1
        if y_host is None:
            y_host = t.empty((n_updates * r.n_fast, r.n_gates), dtype=self.complex_dtype,
                             pin_memory=True)
        if keep_spectra and t_host is None:
            t_host = t.empty((n_spec, r.n_gates, r.n_doppler), dtype=self.complex_dtype,
                             pin_memory=True)
        for name, x, shape in (("y_host", y_host, (n_updates * r.n_fast, r.n_gates)),
                               ("t_host", t_host, (n_spec, r.n_gates, r.n_doppler))):
            if x is None:
                continue
            if x.is_cuda or x.dtype != self.complex_dtype or not x.is_contiguous() or \
                    tuple(x.shape) != shape:
                raise ValueError(f"{name}: expected a contiguous host {self.complex_dtype} "
                                 f"tensor of shape {shape}")
        pptr = self._need(prepared, self.complex_dtype, (self._prepared_elems(),), "prepared")
        s = stream if stream is not None else t.cuda.current_stream(self.device)
        st = sim_streamer_create(self.ctx, self.radar, int(chunk_updates))
        try:
            nbytes = sim_streamer_cache_size(st)
            cache = t.empty(nbytes + 256, dtype=t.uint8, device=self.device)
            cptr = (cache.data_ptr() + 255) & ~255
            sim_streamer_run(st, self.grid, pptr, int(n_updates),
                             None if t_host is None else t_host.data_ptr(), y_host.data_ptr(),
                             cptr, nbytes, s.cuda_stream)
        finally:
            # the cache and the host buffers stay referenced until the stream is done
            s.synchronize()
            sim_streamer_destroy(st)
        return t_host, y_host

    def delay_doppler(self, y, burst=64, centroid=None, migration=True, stream=None):
        """Delay-Doppler processing of the IQ y [n_pulses][G] (sim_delay_doppler):
        returns dict(beams [n_bursts][burst][G] complex, centroid [n_bursts],
        beam_power [burst][G], waveform [G]).  centroid=None estimates it per
        burst, a number is used as given (cycles per pulse)."""
        r = self.radar
        n_pulses = y.shape[0]
        nb = n_pulses // burst
        t = self.torch
        out = {"beams": t.empty((nb, burst, r.n_gates), dtype=self.complex_dtype,
                                device=self.device),
               "centroid": t.empty(nb, dtype=self.real_dtype, device=self.device),
               "beam_power": t.empty((burst, r.n_gates), dtype=self.real_dtype,
                                     device=self.device),
               "waveform": t.empty(r.n_gates, dtype=self.real_dtype, device=self.device)}
        p = sim_dd_params(burst=int(burst),
                          centroid_mode=SIM_DD_CENTROID_ESTIMATE if centroid is None
                          else SIM_DD_CENTROID_GIVEN,
                          centroid=0.0 if centroid is None else float(centroid),
                          migration=1 if migration else 0, reserved=0)
        sim_delay_doppler(self.ctx, self.radar,
                          self._need(y, self.complex_dtype, (n_pulses, r.n_gates), "y"),
                          n_pulses, p, out["beams"].data_ptr(), out["centroid"].data_ptr(),
                          out["beam_power"].data_ptr(), out["waveform"].data_ptr(),
                          self._stream(stream))
        return out

    def run(self, spec0, n_updates, t_fast=None, y=None, counters=None, stream=None,
            prepared=None):
        """Algorithm 1 and post-processing: U + 1 spectra, then Y.  The
        spectrum is put in the column-pass layout once (or ``prepared`` is
        used as it is)."""
        t_fast = t_fast if t_fast is not None else self.empty_spectra(n_updates + 1)
        r = self.radar
        prep = prepared if prepared is not None else self.prepare_spectrum(spec0, stream=stream)
        self.run_updates(prep, [(j * r.n_fast) / r.prf_hz for j in range(n_updates + 1)], 0,
                         t_fast, counters=counters, stream=stream)
        return t_fast, self.segments_to_iq(t_fast, y, stream=stream)

    def run_updates(self, prepared, times, j0, t_fast, counters=None, stream=None):
        """Updates j0 .. j0 + len(times) - 1 (update j0 + i at times[i]) in
        one library call."""
        r = self.radar
        n_spec = t_fast.shape[0]
        sim_run_updates(
            self.ctx, self.grid,
            self._need(prepared, self.complex_dtype, (self._prepared_elems(),), "prepared"),
            self.radar, int(j0), times,
            self._need(t_fast, self.complex_dtype, (n_spec, r.n_gates, r.n_doppler), "t_fast"),
            n_spec,
            None if counters is None else self._need(counters, self.torch.int64, (6,), "counters"),
            self._stream(stream))
        return t_fast


def check_batch_buffers(grids, radars, updates, specs, T, Y, complex_dtype):
    """Validate the per-member buffers of a batch run before any launch: one
    spectrum, one T_fast and (when given) one Y per member, each a contiguous
    tensor of the batch's complex dtype with that member's shape (spectrum
    [ny][nx], T_fast [U + 1][G][N], Y [U n_fast][G]), on a GPU.  The C side
    reads R pointers and trusts every buffer's size, so a short list or a
    wrong shape must never reach it.  Raises ValueError."""
    R = len(grids)
    if len(specs) != R or len(T) != R or (Y is not None and len(Y) != R):
        raise ValueError(f"batch of {R} members: got {len(specs)} spectra, {len(T)} T_fast"
                         + ("" if Y is None else f", {len(Y)} Y") + " buffers")
    want = []
    for r in range(R):
        g, rr, u = grids[r], radars[r], int(updates[r])
        want += [(r, "spec", specs[r], (g.ny, g.nx)),
                 (r, "t_fast", T[r], (u + 1, rr.n_gates, rr.n_doppler))]
        if Y is not None:
            want.append((r, "y", Y[r], (u * rr.n_fast, rr.n_gates)))
    for r, name, x, shape in want:
        if x.dtype != complex_dtype or not x.is_contiguous():
            raise ValueError(f"member {r} {name}: expected a contiguous {complex_dtype} tensor")
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"member {r} {name}: expected shape {tuple(shape)}, got "
                             f"{tuple(x.shape)}")
    for r, name, x, _ in want:
        if not x.is_cuda:
            raise ValueError(f"member {r} {name}: expected a CUDA tensor")


class Batch:
    """Independent realisations run together on one context (update-major on
    one stream, optionally as one replayed HIP graph).  ``members`` is a list
    of (grid, radar, n_updates)."""

    def __init__(self, members, precision=SIM_PREC_FP32_PHASE64, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.precision = precision
        self.complex_dtype = torch.complex128 if precision == SIM_PREC_FP64 else torch.complex64
        self.grids = [grid_struct(g) for g, _, _ in members]
        self.radars = [radar_struct(r) for _, r, _ in members]
        self.updates = [int(u) for _, _, u in members]
        self.ctx = sim_create(device, precision)
        self.batch = sim_batch_create(self.ctx, self.grids, self.radars, self.updates)
        self.mode = SIM_BATCH_PERSISTENT          # the library's default
        nbytes = sim_batch_workspace_size(self.batch)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        sim_set_workspace(self.ctx, (self.workspace.data_ptr() + 255) & ~255, nbytes)
        self.stream = torch.cuda.Stream(self.device)

    def close(self):
        if getattr(self, "batch", None):
            sim_batch_destroy(self.batch)
            self.batch = None
        if getattr(self, "ctx", None):
            sim_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True):
        """Start (clearing) or stop per-kernel event timing of eager runs."""
        sim_profile_enable(self.ctx, enable)

    def profile_read(self) -> dict:
        """{kernel kind: (summed ms, launches)} since profiling was enabled."""
        return sim_profile_read(self.ctx)

    def set_mode(self, mode: int):
        """SIM_BATCH_LANES or SIM_BATCH_PERSISTENT (sim_batch_set_mode)."""
        sim_batch_set_mode(self.batch, mode)
        self.mode = mode

    def empty_outputs(self):
        T = [self.torch.empty((u + 1, r.n_gates, r.n_doppler), dtype=self.complex_dtype,
                              device=self.device) for r, u in zip(self.radars, self.updates)]
        Y = [self.torch.empty((u * r.n_fast, r.n_gates), dtype=self.complex_dtype,
                              device=self.device) for r, u in zip(self.radars, self.updates)]
        return T, Y

    def run(self, specs, T, Y=None, use_graph=False):
        """Run the batch on the batch's own stream (ordered after the current
        stream's work, and the current stream waits for it)."""
        check_batch_buffers(self.grids, self.radars, self.updates, specs, T, Y,
                            self.complex_dtype)
        cur = self.torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        sim_batch_run(self.batch, [x.data_ptr() for x in specs], [x.data_ptr() for x in T],
                      None if Y is None else [x.data_ptr() for x in Y], use_graph,
                      self.stream.cuda_stream)
        cur.wait_stream(self.stream)
        return T, Y
