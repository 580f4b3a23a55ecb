"""Thin ctypes binding of ``libnmdose.so`` (the C ABI in include/nmdose.h and
include/nmdose_nn.h).

Every ``nmd_*`` function here marshals its arguments and calls the C entry
point of the same name; all computation runs in the HIP kernels.  PyTorch is
used only to hold device memory and to supply the stream.  There is no CPU
fallback: if the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnmdose.so")

LEDGER_FIELDS = ("emitted", "dep_compton", "dep_pe", "dep_cutoff", "escaped", "discarded",
                 "dep_positron", "dep_beta")
STATS_FIELDS = ("histories", "photons", "steps", "nulls", "compton", "photoelectric",
                "rayleigh", "deposits", "merged", "max_merged", "escapes", "overflows",
                "claims", "rng_blocks", "list_merges", "gathers")
HREC_FIELDS = ("edep", "escaped", "n_compton", "n_pe", "n_rayleigh", "n_steps",
               "sum_voxel", "n_merged", "n_uniforms", "discarded")
STATUS = {0: "NMD_OK", -1: "NMD_E_INVALID", -2: "NMD_E_SHAPE", -3: "NMD_E_STATE",
          -4: "NMD_E_OOM", -5: "NMD_E_HIP", -6: "NMD_E_ABORTED", -7: "NMD_E_UNSUPPORTED"}


class NmdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class nmd_material(ctypes.Structure):
    _fields_ = [("z_eff", ctypes.c_double), ("z_over_a", ctypes.c_double)]


class nmd_run_opts(ctypes.Structure):
    _fields_ = [("photons_per_decay", ctypes.c_uint32), ("process_mask", ctypes.c_uint32),
                ("max_real_events", ctypes.c_uint32), ("photon_cutoff_mev", ctypes.c_float),
                ("source_kind", ctypes.c_uint32), ("pencil_origin_cm", ctypes.c_float * 3),
                ("pencil_dir", ctypes.c_float * 3), ("chunk", ctypes.c_uint32),
                ("grid_blocks", ctypes.c_uint32), ("abort_after_chunks", ctypes.c_uint32),
                ("history_records", ctypes.c_void_p)]


class nmd_nn_src(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_void_p), ("c0", ctypes.c_int32), ("up0", ctypes.c_int32),
                ("x1", ctypes.c_void_p), ("c1", ctypes.c_int32)]


NN_EXPORTS = ("nmd_conv3d_fwd", "nmd_conv3d_bwd_data", "nmd_conv3d_bwd_weight", "nmd_nn_pool2",
              "nmd_nn_combine", "nmd_nn_prepare", "nmd_nn_head_loss", "nmd_nn_head_infer",
              "nmd_nn_adam", "nmd_nn_cast_weight", "nmd_organ_mean_map",
              "nmd_organ_mean_map_noalloc", "nmd_debug_mfma")

INGEST_EXPORTS = ("nmd_resample_linear", "nmd_ct_to_phantom", "nmd_ct_ingest")

PROBE_EXPORTS = ("nmd_probe_ceiling", "nmd_probe_unit", "nmd_probe_lds")
CEILINGS = {"copy": 0, "atomic_f64": 1, "gather_u16": 2, "valu_fma": 3, "mul64": 4,
            "mfma_bf16": 5}
UNITS = ("loop", "philox", "uniform", "step", "compton", "rayleigh", "history", "merged")
# NMD_LDS_* lane patterns, in enum order
LDS_PATTERNS = ("contiguous", "halo48", "p48_same", "p48_far", "p80_g16", "p48_lane",
                "group_major", "p64_g16", "halo32", "p48_g16", "store48", "p96_g16")


class nmd_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("spacing_mm", ctypes.c_float * 3),
                ("origin_mm", ctypes.c_float * 3)]


class nmd_ct_table(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("hu", ctypes.c_float * 32),
                ("density", ctypes.c_float * 32), ("n_materials", ctypes.c_int32),
                ("hu_threshold", ctypes.c_float * 7), ("density_min", ctypes.c_float * 8),
                ("density_width", ctypes.c_float * 8), ("levels", ctypes.c_int32 * 8)]


EXPORTS = ("nmd_create", "nmd_destroy", "nmd_last_error", "nmd_set_stream",
           "nmd_run_opts_default", "nmd_set_phantom", "nmd_set_activity", "nmd_run_histories",
           "nmd_reset_tallies", "nmd_get_dose", "nmd_get_organ_dose", "nmd_get_organ_score",
           "nmd_get_ledger", "nmd_get_run_stats", "nmd_get_tallies", "nmd_set_tallies",
           "nmd_debug_sample", "nmd_debug_sample_source", "nmd_debug_xs",
           "nmd_read_organ_dose", "nmd_get_last_launch", "nmd_graph_create",
           "nmd_graph_launch", "nmd_graph_destroy", "nmd_save", "nmd_load",
           "nmd_set_electrons", "nmd_set_tracking", "nmd_set_positron",
           "nmd_set_emitter") + NN_EXPORTS + \
    INGEST_EXPORTS + PROBE_EXPORTS

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (torch first, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libnmdose.so is not built (run paper_2111_11687_amd/build.py)")
    import torch  # noqa: F401  (loads the HIP runtime the library will bind to)
    L = ctypes.CDLL(path)
    vp, i32, u64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "nmd_create": [ctypes.POINTER(vp), ctypes.c_int, vp],
        "nmd_destroy": [vp],
        "nmd_last_error": [vp],
        "nmd_set_stream": [vp, vp],
        "nmd_run_opts_default": [ctypes.POINTER(nmd_run_opts)],
        "nmd_set_phantom": [vp, i32, i32, i32, i32, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, vp, vp, vp, i32, ctypes.POINTER(nmd_material), i32],
        "nmd_set_activity": [vp, i32, vp, d],
        "nmd_run_histories": [vp, i32, u64, u64, ctypes.POINTER(nmd_run_opts)],
        "nmd_reset_tallies": [vp, i32],
        "nmd_get_dose": [vp, i32, vp, vp],
        "nmd_get_organ_dose": [vp, i32, i32, vp, vp, vp],
        "nmd_get_organ_score": [vp, i32, i32, vp],
        "nmd_get_ledger": [vp, i32, vp],
        "nmd_get_run_stats": [vp, i32, vp],
        "nmd_get_tallies": [vp, i32, vp, vp, ctypes.POINTER(u64)],
        "nmd_set_tallies": [vp, i32, vp, vp, u64],
        "nmd_debug_sample": [vp, i32, d, u64, u64, vp],
        "nmd_debug_sample_source": [vp, i32, u64, u64, vp],
        "nmd_debug_xs": [vp, i32, u64, vp, vp],
        "nmd_read_organ_dose": [vp, i32, i32, vp, vp, vp],
        "nmd_get_last_launch": [vp, ctypes.POINTER(ctypes.c_uint32),
                                ctypes.POINTER(ctypes.c_uint32)],
        "nmd_graph_create": [vp, i32, u64, u64, ctypes.POINTER(nmd_run_opts), vp, vp,
                             ctypes.POINTER(vp)],
        "nmd_graph_launch": [vp],
        "nmd_save": [vp, i32, ctypes.c_char_p],
        "nmd_set_electrons": [vp, i32, d, vp],
        "nmd_set_tracking": [vp, i32, i32],
        "nmd_set_positron": [vp, i32, i32, d, vp],
        "nmd_set_emitter": [vp, i32, i32, vp, vp, d],
        "nmd_load": [vp, i32, ctypes.c_char_p],
        "nmd_graph_destroy": [vp],
        "nmd_conv3d_fwd": [vp, i32, i32, i32, i32, ctypes.POINTER(nmd_nn_src), vp, vp, i32, i32,
                           vp, vp],
        "nmd_conv3d_bwd_data": [vp, i32, i32, i32, i32, vp, i32, vp, i32, vp, vp],
        "nmd_conv3d_bwd_weight": [vp, i32, i32, i32, i32, ctypes.POINTER(nmd_nn_src), vp, i32,
                                  vp, vp],
        "nmd_nn_pool2": [vp, i32, i32, i32, i32, i32, vp, vp],
        "nmd_nn_combine": [vp, i32, i32, i32, i32, i32, vp, vp, i32, i32, i32, vp, i32, i32, vp],
        "nmd_nn_prepare": [vp, i32, i32, i32, ctypes.POINTER(i32), vp, vp, vp, vp, vp, vp, vp,
                           vp],
        "nmd_nn_head_loss": [vp, ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_float, vp, vp],
        "nmd_nn_head_infer": [vp, i32, i32, i32, ctypes.POINTER(i32), vp, vp, vp, vp, vp, vp],
        "nmd_nn_adam": [vp, vp, vp, vp, vp, ctypes.c_int64, i32, ctypes.c_float,
                        ctypes.c_float, ctypes.c_float, ctypes.c_float, vp, vp, i32, i32],
        "nmd_nn_cast_weight": [vp, vp, i32, i32, vp, vp],
        "nmd_organ_mean_map": [vp, i32, vp, i32, vp],
        "nmd_organ_mean_map_noalloc": [vp, i32, vp, i32, vp],
        "nmd_debug_mfma": [vp, vp, vp, vp],
        "nmd_resample_linear": [vp, vp, ctypes.POINTER(nmd_grid), ctypes.POINTER(nmd_grid),
                                ctypes.c_float, vp],
        "nmd_ct_to_phantom": [vp, vp, ctypes.c_int64, ctypes.POINTER(nmd_ct_table), vp, vp],
        "nmd_ct_ingest": [vp, vp, ctypes.POINTER(nmd_grid), ctypes.POINTER(nmd_grid),
                          ctypes.POINTER(nmd_ct_table), vp, vp],
        "nmd_probe_ceiling": [vp, i32, u64, ctypes.c_uint32, ctypes.POINTER(d),
                              ctypes.POINTER(d)],
        "nmd_probe_unit": [vp, i32, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(d)],
        "nmd_probe_lds": [vp, i32, i32, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(d)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    L.nmd_destroy.restype = None
    L.nmd_graph_destroy.restype = None
    L.nmd_run_opts_default.restype = None
    L.nmd_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(ctx, status):
    if status != 0:
        msg = load_library().nmd_last_error(ctx)
        raise NmdError(status, msg.decode() if msg else "")


def _dptr(t):
    """Device address of a torch tensor (or None)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ---- one wrapper per C entry point -----------------------------------------
def nmd_create(device: int = 0, stream=None):
    L = load_library()
    h = ctypes.c_void_p()
    st = L.nmd_create(ctypes.byref(h), int(device), _stream_handle(stream))
    if st != 0:
        raise NmdError(st, "nmd_create failed on device %d" % device)
    return h


def nmd_destroy(ctx):
    load_library().nmd_destroy(ctx)


def nmd_last_error(ctx) -> str:
    m = load_library().nmd_last_error(ctx)
    return m.decode() if m else ""


def nmd_set_stream(ctx, stream=None):
    _check(ctx, load_library().nmd_set_stream(ctx, _stream_handle(stream)))


def nmd_run_opts_default() -> nmd_run_opts:
    o = nmd_run_opts()
    load_library().nmd_run_opts_default(ctypes.byref(o))
    return o


def nmd_set_phantom(ctx, phantom_id, density, material, organ_label, n_organs, materials,
                    voxel_mm):
    """density float32, material uint8, organ_label uint8 or None: torch
    device tensors of shape (nz, ny, nx); materials: [(z_eff, z_over_a)]."""
    nz, ny, nx = density.shape
    arr = (nmd_material * len(materials))(*[nmd_material(float(z), float(a))
                                            for z, a in materials])
    _check(ctx, load_library().nmd_set_phantom(
        ctx, int(phantom_id), nx, ny, nz, float(voxel_mm[0]), float(voxel_mm[1]),
        float(voxel_mm[2]), _dptr(density), _dptr(material), _dptr(organ_label), int(n_organs),
        arr, len(materials)))


def nmd_set_activity(ctx, phantom_id, activity, total_activity_bq=0.0):
    _check(ctx, load_library().nmd_set_activity(ctx, int(phantom_id), _dptr(activity),
                                                float(total_activity_bq)))


def nmd_run_histories(ctx, phantom_id, n_decays, seed, opts: nmd_run_opts | None = None):
    _check(ctx, load_library().nmd_run_histories(
        ctx, int(phantom_id), int(n_decays), int(seed),
        None if opts is None else ctypes.byref(opts)))


def nmd_reset_tallies(ctx, phantom_id):
    _check(ctx, load_library().nmd_reset_tallies(ctx, int(phantom_id)))


def nmd_get_dose(ctx, phantom_id, dose_rate, rel_uncertainty=None):
    _check(ctx, load_library().nmd_get_dose(ctx, int(phantom_id), _dptr(dose_rate),
                                            _dptr(rel_uncertainty)))


def nmd_get_organ_dose(ctx, phantom_id, n_organs, sigma=True):
    """Returns (Eq. 2 dose rate, Eq. 3 uncertainty, relative sigma of the
    organ mean, or None with sigma=False) as float64 numpy arrays of
    n_organs."""
    r = np.zeros(n_organs)
    e = np.zeros(n_organs)
    s = np.zeros(n_organs) if sigma else None
    p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    _check(ctx, load_library().nmd_get_organ_dose(ctx, int(phantom_id), int(n_organs), p(r),
                                                  p(e), p(s)))
    return r, e, s


def nmd_read_organ_dose(ctx, phantom_id, n_organs, sigma=True):
    """Results of the last organ reduction (e.g. one a graph ran)."""
    r = np.zeros(n_organs)
    e = np.zeros(n_organs)
    s = np.zeros(n_organs) if sigma else None
    p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    _check(ctx, load_library().nmd_read_organ_dose(ctx, int(phantom_id), int(n_organs), p(r),
                                                   p(e), p(s)))
    return r, e, s


def nmd_set_electrons(ctx, phantom_id, cutoff_mev, mean_excitation_ev=None):
    """cutoff_mev 0 turns electron transport off; else one mean excitation
    energy (eV) per material of the phantom."""
    arr = None
    if mean_excitation_ev is not None:
        arr = np.ascontiguousarray(mean_excitation_ev, dtype=np.float64)
    _check(ctx, load_library().nmd_set_electrons(
        ctx, int(phantom_id), float(cutoff_mev),
        None if arr is None else arr.ctypes.data_as(ctypes.c_void_p)))


def nmd_set_positron(ctx, phantom_id, on, noncol_fwhm_deg=0.5, mean_excitation_ev=None):
    """on: 18F positron range and the pair's non-collinearity (one mean
    excitation energy in eV per material of the phantom); off: none."""
    arr = None
    if mean_excitation_ev is not None:
        arr = np.ascontiguousarray(mean_excitation_ev, dtype=np.float64)
    _check(ctx, load_library().nmd_set_positron(
        ctx, int(phantom_id), int(bool(on)), float(noncol_fwhm_deg),
        None if arr is None else arr.ctypes.data_as(ctypes.c_void_p)))


def nmd_set_emitter(ctx, phantom_id, line_mev=(), line_yield=(), beta_mean_mev=0.0):
    """A gamma + beta emitter in place of the annihilation pair; no lines and
    no beta energy return to the pair."""
    e = np.ascontiguousarray(line_mev, dtype=np.float64)
    y = np.ascontiguousarray(line_yield, dtype=np.float64)
    if e.shape != y.shape:
        raise ValueError("one yield per line")
    _check(ctx, load_library().nmd_set_emitter(
        ctx, int(phantom_id), int(e.size), e.ctypes.data_as(ctypes.c_void_p) if e.size else None,
        y.ctypes.data_as(ctypes.c_void_p) if y.size else None, float(beta_mean_mev)))


TRACKING = {"global": 0, "regions": 1}


def nmd_set_tracking(ctx, phantom_id, mode):
    """mode: "global" / "regions" (or NMD_TRACK_* numbers)."""
    m = TRACKING[mode] if isinstance(mode, str) else int(mode)
    _check(ctx, load_library().nmd_set_tracking(ctx, int(phantom_id), m))


def nmd_save(ctx, phantom_id, path):
    _check(ctx, load_library().nmd_save(ctx, int(phantom_id), os.fsencode(path)))


def nmd_load(ctx, phantom_id, path):
    _check(ctx, load_library().nmd_load(ctx, int(phantom_id), os.fsencode(path)))


def nmd_get_last_launch(ctx):
    ch, gr = ctypes.c_uint32(), ctypes.c_uint32()
    _check(ctx, load_library().nmd_get_last_launch(ctx, ctypes.byref(ch), ctypes.byref(gr)))
    return int(ch.value), int(gr.value)


def nmd_graph_create(ctx, phantom_id, n_decays, seed, opts=None, dose_rate=None,
                     rel_uncertainty=None):
    g = ctypes.c_void_p()
    _check(ctx, load_library().nmd_graph_create(
        ctx, int(phantom_id), int(n_decays), int(seed),
        None if opts is None else ctypes.byref(opts), _dptr(dose_rate), _dptr(rel_uncertainty),
        ctypes.byref(g)))
    return g


def nmd_graph_launch(ctx, graph):
    _check(ctx, load_library().nmd_graph_launch(graph))


def nmd_graph_destroy(graph):
    load_library().nmd_graph_destroy(graph)


def nmd_get_organ_score(ctx, phantom_id, n_organs):
    r = np.zeros(n_organs)
    _check(ctx, load_library().nmd_get_organ_score(ctx, int(phantom_id), int(n_organs),
                                                   r.ctypes.data_as(ctypes.c_void_p)))
    return r


def nmd_get_ledger(ctx, phantom_id) -> dict:
    a = np.zeros(len(LEDGER_FIELDS))
    _check(ctx, load_library().nmd_get_ledger(ctx, int(phantom_id),
                                              a.ctypes.data_as(ctypes.c_void_p)))
    return dict(zip(LEDGER_FIELDS, a.tolist()))


def nmd_get_run_stats(ctx, phantom_id) -> dict:
    a = np.zeros(len(STATS_FIELDS), dtype=np.uint64)
    _check(ctx, load_library().nmd_get_run_stats(ctx, int(phantom_id),
                                                 a.ctypes.data_as(ctypes.c_void_p)))
    return dict(zip(STATS_FIELDS, [int(x) for x in a]))


def nmd_get_tallies(ctx, phantom_id, sum_dev, sum2_dev):
    n = ctypes.c_uint64()
    _check(ctx, load_library().nmd_get_tallies(ctx, int(phantom_id), _dptr(sum_dev),
                                               _dptr(sum2_dev), ctypes.byref(n)))
    return int(n.value)


def nmd_set_tallies(ctx, phantom_id, sum_dev, sum2_dev, n_decays):
    _check(ctx, load_library().nmd_set_tallies(ctx, int(phantom_id), _dptr(sum_dev),
                                               _dptr(sum2_dev), int(n_decays)))


def nmd_debug_sample(ctx, kind, e_mev, n, seed, out):
    _check(ctx, load_library().nmd_debug_sample(ctx, int(kind), float(e_mev), int(n), int(seed),
                                                _dptr(out)))


def nmd_debug_sample_source(ctx, phantom_id, n, seed, out):
    _check(ctx, load_library().nmd_debug_sample_source(ctx, int(phantom_id), int(n), int(seed),
                                                       _dptr(out)))


def nmd_debug_xs(ctx, phantom_id, energies, out):
    _check(ctx, load_library().nmd_debug_xs(ctx, int(phantom_id), int(energies.numel()),
                                            _dptr(energies), _dptr(out)))


# ---- denoiser entry points (include/nmdose_nn.h) ----------------------------
def _src(x0, c0=None, up0=False, x1=None, c1=0):
    """Convolution input [x0 | x1]; channel counts default to the tensors' last
    dim.  The structure keeps references to the tensors so that their memory
    outlives it."""
    c0 = int(x0.shape[-1]) if c0 is None else int(c0)
    if x1 is not None and not c1:
        c1 = int(x1.shape[-1])
    s = nmd_nn_src(x0.data_ptr(), c0, 1 if up0 else 0,
                   None if x1 is None else x1.data_ptr(), int(c1))
    s._keep = (x0, x1)
    return s


def _box(box):
    return (ctypes.c_int32 * 6)(*[int(b) for b in box])


def nmd_conv3d_fwd(ctx, dims, src: nmd_nn_src, weight, bias, c_out, relu, mask, y):
    n, d, h, w = dims
    _check(ctx, load_library().nmd_conv3d_fwd(ctx, n, d, h, w, ctypes.byref(src), _dptr(weight),
                                              _dptr(bias), int(c_out), 1 if relu else 0,
                                              _dptr(mask), _dptr(y)))


def nmd_conv3d_bwd_data(ctx, dims, dy, c_out, weight_t, c_in, mask, dx):
    n, d, h, w = dims
    _check(ctx, load_library().nmd_conv3d_bwd_data(ctx, n, d, h, w, _dptr(dy), int(c_out),
                                                   _dptr(weight_t), int(c_in), _dptr(mask),
                                                   _dptr(dx)))


def nmd_conv3d_bwd_weight(ctx, dims, src: nmd_nn_src, dy, c_out, dw, db=None):
    n, d, h, w = dims
    _check(ctx, load_library().nmd_conv3d_bwd_weight(ctx, n, d, h, w, ctypes.byref(src),
                                                     _dptr(dy), int(c_out), _dptr(dw),
                                                     _dptr(db)))


def nmd_nn_pool2(ctx, dims, c, x, y):
    n, d, h, w = dims
    _check(ctx, load_library().nmd_nn_pool2(ctx, n, d, h, w, int(c), _dptr(x), _dptr(y)))


def nmd_nn_combine(ctx, dims, c, mask, a, a_stride, a_off, b_mode, b, b_stride, b_off, out):
    n, d, h, w = dims
    _check(ctx, load_library().nmd_nn_combine(ctx, n, d, h, w, int(c), _dptr(mask), _dptr(a),
                                              int(a_stride), int(a_off), int(b_mode), _dptr(b),
                                              int(b_stride), int(b_off), _dptr(out)))


def nmd_nn_prepare(ctx, shape, box, dose_lo, dose_hi, density, activity, label, x0, target,
                   scale):
    nz, ny, nx = shape
    _check(ctx, load_library().nmd_nn_prepare(ctx, nz, ny, nx, _box(box), _dptr(dose_lo),
                                              _dptr(dose_hi), _dptr(density), _dptr(activity),
                                              _dptr(label), _dptr(x0), _dptr(target),
                                              _dptr(scale)))


def nmd_nn_head_loss(ctx, nvox, feat, x0, target, head_w, head_b, dfeat, grad,
                     weight_floor=0.0):
    _check(ctx, load_library().nmd_nn_head_loss(ctx, int(nvox), _dptr(feat), _dptr(x0),
                                                _dptr(target), _dptr(head_w), _dptr(head_b),
                                                float(weight_floor), _dptr(dfeat), _dptr(grad)))


def nmd_nn_head_infer(ctx, shape, box, feat, x0, head_w, head_b, scale, out):
    nz, ny, nx = shape
    _check(ctx, load_library().nmd_nn_head_infer(ctx, nz, ny, nx, _box(box), _dptr(feat),
                                                 _dptr(x0), _dptr(head_w), _dptr(head_b),
                                                 _dptr(scale), _dptr(out)))


def nmd_nn_adam(ctx, theta, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                w_bf16=None, w_t_bf16=None, c_out=0, c_in=0):
    _check(ctx, load_library().nmd_nn_adam(ctx, _dptr(theta), _dptr(m), _dptr(v), _dptr(grad),
                                           int(theta.numel()), int(step), float(lr),
                                           float(beta1), float(beta2), float(eps),
                                           _dptr(w_bf16), _dptr(w_t_bf16), int(c_out),
                                           int(c_in)))


def nmd_nn_cast_weight(ctx, theta, c_out, c_in, w_bf16=None, w_t_bf16=None):
    _check(ctx, load_library().nmd_nn_cast_weight(ctx, _dptr(theta), int(c_out), int(c_in),
                                                  _dptr(w_bf16), _dptr(w_t_bf16)))


def nmd_organ_mean_map(ctx, phantom_id, dose_map, n_organs):
    out = np.zeros(n_organs)
    _check(ctx, load_library().nmd_organ_mean_map(ctx, int(phantom_id), _dptr(dose_map),
                                                  int(n_organs),
                                                  out.ctypes.data_as(ctypes.c_void_p)))
    return out


def nmd_organ_mean_map_noalloc(ctx, phantom_id, dose_map, n_organs):
    out = np.zeros(n_organs)
    _check(ctx, load_library().nmd_organ_mean_map_noalloc(
        ctx, int(phantom_id), _dptr(dose_map), int(n_organs),
        out.ctypes.data_as(ctypes.c_void_p)))
    return out


def nmd_probe_ceiling(ctx, kind, nbytes=0, repeats=10):
    """(rate, ms) of ceiling `kind` (a CEILINGS name or number)."""
    k = CEILINGS[kind] if isinstance(kind, str) else int(kind)
    rate, ms = ctypes.c_double(), ctypes.c_double()
    _check(ctx, load_library().nmd_probe_ceiling(ctx, k, nbytes, repeats, ctypes.byref(rate),
                                                 ctypes.byref(ms)))
    return rate.value, ms.value


def nmd_probe_unit(ctx, kind, iters, blocks):
    """Launch time (ms) of the unit probe `kind` (a UNITS name or number)."""
    k = UNITS.index(kind) if isinstance(kind, str) else int(kind)
    ms = ctypes.c_double()
    _check(ctx, load_library().nmd_probe_unit(ctx, k, iters, blocks, ctypes.byref(ms)))
    return ms.value


def nmd_probe_lds(ctx, pattern, write=False, iters=256, blocks=1024):
    """Launch time (ms) of the LDS probe over `pattern` (an LDS_PATTERNS name
    or number), reads or writes."""
    k = LDS_PATTERNS.index(pattern) if isinstance(pattern, str) else int(pattern)
    ms = ctypes.c_double()
    _check(ctx, load_library().nmd_probe_lds(ctx, k, int(bool(write)), iters, blocks,
                                             ctypes.byref(ms)))
    return ms.value


def make_grid(g):
    """nmd_grid from a dict n=(nx, ny, nz), spacing=(sx, sy, sz), origin=(ox, oy, oz) (mm)."""
    out = nmd_grid()
    for a in range(3):
        out.n[a] = int(g["n"][a])
        out.spacing_mm[a] = float(g["spacing"][a])
        out.origin_mm[a] = float(g["origin"][a])
    return out


def make_ct_table(t):
    """nmd_ct_table from a dict with hu, density, threshold, density_min,
    density_width and levels."""
    out = nmd_ct_table()
    out.n_nodes = len(t["hu"])
    for i, (h, d) in enumerate(zip(t["hu"], t["density"])):
        out.hu[i] = float(h)
        out.density[i] = float(d)
    out.n_materials = len(t["levels"])
    for i, h in enumerate(t["threshold"]):
        out.hu_threshold[i] = float(h)
    for i in range(out.n_materials):
        out.density_min[i] = float(t["density_min"][i])
        out.density_width[i] = float(t["density_width"][i])
        out.levels[i] = int(t["levels"][i])
    return out


def nmd_resample_linear(ctx, src, src_grid, dst_grid, fill, dst):
    _check(ctx, load_library().nmd_resample_linear(ctx, _dptr(src), ctypes.byref(make_grid(src_grid)),
                                                   ctypes.byref(make_grid(dst_grid)), float(fill),
                                                   _dptr(dst)))


def nmd_ct_to_phantom(ctx, hu, table, density, material):
    _check(ctx, load_library().nmd_ct_to_phantom(ctx, _dptr(hu), int(hu.numel()),
                                                 ctypes.byref(make_ct_table(table)),
                                                 _dptr(density), _dptr(material)))


def nmd_ct_ingest(ctx, ct_hu, ct_grid, dose_grid, table, density, material):
    _check(ctx, load_library().nmd_ct_ingest(ctx, _dptr(ct_hu), ctypes.byref(make_grid(ct_grid)),
                                             ctypes.byref(make_grid(dose_grid)),
                                             ctypes.byref(make_ct_table(table)), _dptr(density),
                                             _dptr(material)))


def nmd_debug_mfma(ctx, a, b, d):
    _check(ctx, load_library().nmd_debug_mfma(ctx, _dptr(a), _dptr(b), _dptr(d)))


# ---- convenience layer used by the tests and the benchmark ------------------
class Engine:
    """Owns one context and the device copies of the inputs handed to it."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the engine has no CPU path")
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = nmd_create(device, torch.cuda.current_stream(self.device))
        self.problems = {}
        self.inputs = {}  # device copies: density, material, label, activity

    def close(self):
        if self.ctx is not None:
            nmd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_problem(self, phantom_id, prob, with_activity=True):
        t = self.torch
        dev = self.device
        rho = t.from_numpy(np.ascontiguousarray(prob.density, dtype=np.float32)).to(dev)
        mat = t.from_numpy(np.ascontiguousarray(prob.material, dtype=np.uint8)).to(dev)
        lab = t.from_numpy(np.ascontiguousarray(prob.label, dtype=np.uint8)).to(dev)
        nmd_set_phantom(self.ctx, phantom_id, rho, mat, lab, prob.n_organs, prob.materials,
                        prob.voxel_mm)
        act = None
        if with_activity:
            act = t.from_numpy(np.ascontiguousarray(prob.activity, dtype=np.float32)).to(dev)
            nmd_set_activity(self.ctx, phantom_id, act, prob.total_activity_bq)
        self.problems[phantom_id] = prob
        self.inputs[phantom_id] = {"density": rho, "material": mat, "label": lab, "activity": act}

    def run(self, phantom_id, n, seed, **kw):
        o = nmd_run_opts_default()
        for k, v in kw.items():
            if k in ("pencil_origin_cm", "pencil_dir"):
                for a in range(3):
                    getattr(o, k)[a] = float(v[a])
            elif k == "history_records":
                o.history_records = None if v is None else v.data_ptr()
            else:
                setattr(o, k, v)
        nmd_run_histories(self.ctx, phantom_id, n, seed, o)

    def dose(self, phantom_id):
        prob = self.problems[phantom_id]
        rate = self.torch.empty(prob.shape, dtype=self.torch.float64, device=self.device)
        rel = self.torch.empty_like(rate)
        nmd_get_dose(self.ctx, phantom_id, rate, rel)
        return rate, rel

    def tallies(self, phantom_id):
        prob = self.problems[phantom_id]
        s = self.torch.empty(prob.shape, dtype=self.torch.float64, device=self.device)
        s2 = self.torch.empty_like(s)
        n = nmd_get_tallies(self.ctx, phantom_id, s, s2)
        return s, s2, n

    def organs(self, phantom_id, sigma=True):
        return nmd_get_organ_dose(self.ctx, phantom_id, self.problems[phantom_id].n_organs,
                                  sigma)

    def ledger(self, phantom_id):
        return nmd_get_ledger(self.ctx, phantom_id)

    def stats(self, phantom_id):
        return nmd_get_run_stats(self.ctx, phantom_id)

    def sync(self):
        self.torch.cuda.synchronize(self.device)
