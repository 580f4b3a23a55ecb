"""CPU oracle for the dosimetry Monte Carlo -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``nmd_oracle.c``: a plain FP64 OpenMP Monte Carlo of
the method of Peng et al. (arXiv 2111.11687), Sections 2.1 (source, physics,
cutoffs, history-by-history uncertainty), Eq. 1 (dose rate) and Section 2.4
(Eq. 2 organ mean, Eq. 3 organ uncertainty).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nmd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

TRACK_EXACT, TRACK_WOODCOCK, TRACK_REGIONS = 0, 1, 2
KN_KAHN, KN_BUTCHER = 0, 1
RNG_PHILOX, RNG_XOSHIRO = 0, 1
SRC_ACTIVITY, SRC_PENCIL = 0, 1

LEDGER_FIELDS = ("emitted", "dep_compton", "dep_pe", "dep_cutoff", "escaped", "discarded",
                 "dep_positron", "dep_beta")
STATS_FIELDS = ("histories", "photons", "steps", "nulls", "compton", "photoelectric",
                "rayleigh", "deposits", "merged", "max_merged", "escapes", "uniforms")
HREC_FIELDS = ("edep", "escaped", "n_compton", "n_pe", "n_rayleigh", "n_steps",
               "sum_voxel", "n_merged", "n_uniforms", "discarded")

J_PER_MEV = 1.602176634e-13


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP) into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Phantom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("density", ctypes.c_void_p), ("material", ctypes.c_void_p),
                ("label", ctypes.c_void_p), ("n_organs", ctypes.c_int32),
                ("z_eff", ctypes.c_void_p), ("z_over_a", ctypes.c_void_p),
                ("n_mat", ctypes.c_int32), ("activity", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("n_hist", ctypes.c_uint64), ("first_hist", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("pid", ctypes.c_uint32),
                ("photons_per_decay", ctypes.c_int32), ("process_mask", ctypes.c_uint32),
                ("max_real_events", ctypes.c_int32), ("cutoff_mev", ctypes.c_double),
                ("tracking", ctypes.c_int32), ("kn_method", ctypes.c_int32),
                ("wide_uniforms", ctypes.c_int32), ("source_kind", ctypes.c_int32),
                ("pencil_origin", ctypes.c_double * 3), ("pencil_dir", ctypes.c_double * 3),
                ("n_threads", ctypes.c_int32), ("hist_out", ctypes.c_void_p),
                ("electron_cutoff_mev", ctypes.c_double),
                ("mean_excitation_ev", ctypes.c_void_p), ("rng", ctypes.c_int32),
                ("positron", ctypes.c_int32), ("noncol_fwhm_rad", ctypes.c_double),
                ("n_lines", ctypes.c_int32), ("line_mev", ctypes.c_void_p),
                ("line_yield", ctypes.c_void_p), ("beta_mean_mev", ctypes.c_double)]


class _Tally(ctypes.Structure):
    _fields_ = [("S", ctypes.c_void_p), ("S2", ctypes.c_void_p), ("O", ctypes.c_void_p),
                ("O2", ctypes.c_void_p), ("ledger", ctypes.c_double * 8),
                ("stats", ctypes.c_uint64 * 12)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        d, i32, u64, vp = ctypes.c_double, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p
        L.orc_sigma_kn.restype = d
        L.orc_sigma_kn.argtypes = [d]
        L.orc_grid_energy.restype = d
        L.orc_grid_energy.argtypes = [ctypes.c_int]
        L.orc_mass_atten_closed.restype = d
        L.orc_mass_atten_closed.argtypes = [ctypes.c_int, d, d, d]
        L.orc_mass_atten_interp.restype = d
        L.orc_mass_atten_interp.argtypes = [ctypes.c_int, d, d, d]
        L.orc_philox4x32_10.restype = None
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(_Phantom), ctypes.POINTER(_Opts),
                              ctypes.POINTER(_Tally)]
        L.orc_finalize.restype = None
        L.orc_finalize.argtypes = [vp, vp, vp, ctypes.c_int64, d, d, d, vp, vp]
        L.orc_organ_stats.restype = None
        L.orc_organ_stats.argtypes = [vp, vp, vp, ctypes.c_int64, i32, vp, vp]
        L.orc_sample.restype = ctypes.c_int
        L.orc_sample.argtypes = [ctypes.c_int, d, u64, u64, ctypes.c_int, ctypes.c_int, vp]
        L.orc_sample_source.restype = ctypes.c_int
        L.orc_sample_source.argtypes = [ctypes.POINTER(_Phantom), u64, u64, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, vp]
        L.orc_splitmix64.restype = u64
        L.orc_splitmix64.argtypes = [ctypes.POINTER(u64)]
        L.orc_xoshiro256ss.restype = u64
        L.orc_xoshiro256ss.argtypes = [ctypes.POINTER(u64 * 4)]
        L.orc_thomson_inverse.restype = d
        L.orc_thomson_inverse.argtypes = [d]
        L.orc_majorant.restype = d
        L.orc_majorant.argtypes = [ctypes.POINTER(_Phantom), d]
        L.orc_rotate.restype = None
        L.orc_rotate.argtypes = [vp, d, d]
        for name in ("orc_stopping_power",):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = [d, d, d]
        L.orc_beta_plus_shape.restype = d
        L.orc_beta_plus_shape.argtypes = [d]
        L.orc_csda_range.restype = d
        L.orc_csda_range.argtypes = [d, d, d, d]
        L.orc_energy_after.restype = d
        L.orc_energy_after.argtypes = [d, d, d, d, d]
        L.orc_electron_walk.restype = ctypes.c_int
        L.orc_electron_walk.argtypes = [ctypes.POINTER(_Phantom), vp, d, vp, vp, d, vp, vp,
                                        ctypes.c_int, ctypes.POINTER(d)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Primitives
# --------------------------------------------------------------------------
def sigma_kn(e_mev: float) -> float:
    """Klein-Nishina total cross section per electron (cm^2)."""
    return lib().orc_sigma_kn(float(e_mev))


def grid_energy(i: int) -> float:
    return lib().orc_grid_energy(int(i))


def mass_atten(process: int, z: float, z_over_a: float, e_mev: float,
               interp: bool = True) -> float:
    """Mass attenuation (cm^2/g): process 1 Compton, 2 photoelectric, 3 Rayleigh."""
    f = lib().orc_mass_atten_interp if interp else lib().orc_mass_atten_closed
    return f(int(process), float(z), float(z_over_a), float(e_mev))


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


_SAMPLE_WIDTH = {0: 4, 1: 1, 2: 3, 3: 2, 4: 2, 5: 1, 6: 1, 7: 1}


def sample(kind: str, n: int, seed: int = 1, e_mev: float = 0.511,
           wide: bool = False, rng: int = RNG_PHILOX) -> np.ndarray:
    """Draw n samples; kind in {'raw','uniform','marsaglia','kahn','butcher','thomson',
    'positron_energy','noncollinear'} (for 'noncollinear', e_mev is the FWHM in rad)."""
    k = {"raw": 0, "uniform": 1, "marsaglia": 2, "kahn": 3, "butcher": 4, "thomson": 5,
         "positron_energy": 6, "noncollinear": 7}[kind]
    out = np.zeros(n * _SAMPLE_WIDTH[k], dtype=np.float64)
    rc = lib().orc_sample(k, float(e_mev), int(n), int(seed), int(wide), int(rng), _ptr(out))
    if rc != 0:
        raise ValueError(kind)
    w = _SAMPLE_WIDTH[k]
    return out.reshape(n, w) if w > 1 else out


def sample_source(ph, n: int, seed: int = 1, tracking: int = TRACK_EXACT,
                  wide: bool | None = None, rng: int | None = None):
    """Decay points drawn as the transport draws them (Section 2.1: voxel
    probability proportional to the activity, position uniform in the
    voxel).  Returns (voxel index int64 [n], position cm [n, 3])."""
    if ph.activity is None:
        raise ValueError("phantom has no activity map")
    if wide is None:
        wide = tracking == TRACK_EXACT
    if rng is None:
        rng = RNG_XOSHIRO if tracking == TRACK_EXACT else RNG_PHILOX
    out = np.zeros((n, 4), dtype=np.float64)
    rc = lib().orc_sample_source(ctypes.byref(ph._c), int(n), int(seed), int(tracking),
                                 int(bool(wide)), int(rng), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the activity map (code %d)" % rc)
    return out[:, 0].astype(np.int64), out[:, 1:].copy()


def splitmix64(x: int):
    """One SplitMix64 step: (output, new state)."""
    st = ctypes.c_uint64(x)
    out = lib().orc_splitmix64(ctypes.byref(st))
    return int(out), int(st.value)


def xoshiro256ss(state, n: int):
    """n outputs of xoshiro256** from the 4-word state (the state is not
    modified)."""
    st = (ctypes.c_uint64 * 4)(*[int(v) for v in state])
    return [int(lib().orc_xoshiro256ss(ctypes.byref(st))) for _ in range(n)]


def thomson_inverse(u: float) -> float:
    return lib().orc_thomson_inverse(float(u))


def rotate(d, cost: float, uphi: float) -> np.ndarray:
    v = np.array(d, dtype=np.float64)
    lib().orc_rotate(_ptr(v), float(cost), float(uphi))
    return v


def stopping_power(t_mev: float, z_over_a: float, i_ev: float) -> float:
    """Electron collision stopping power, MeV cm^2/g (Bethe, no density effect)."""
    return lib().orc_stopping_power(t_mev, z_over_a, i_ev)


def csda_range(t_lo: float, t_hi: float, z_over_a: float, i_ev: float) -> float:
    """Mass path (g/cm^2) from t_hi down to t_lo."""
    return lib().orc_csda_range(t_lo, t_hi, z_over_a, i_ev)


def energy_after(t: float, mass_path: float, t_floor: float, z_over_a: float,
                 i_ev: float) -> float:
    return lib().orc_energy_after(t, mass_path, t_floor, z_over_a, i_ev)


def electron_walk(ph, mean_excitation_ev, cutoff_mev: float, r, d, t0: float, cap: int = 4096):
    """One straight-ahead CSDA electron walk; returns (deposits, escaped) with
    deposits a list of (flat voxel, MeV) in crossing order."""
    iev = np.ascontiguousarray(mean_excitation_ev, dtype=np.float64)
    rr = np.ascontiguousarray(r, dtype=np.float64)
    dd = np.ascontiguousarray(d, dtype=np.float64)
    vo = np.zeros(cap, dtype=np.int64)
    eo = np.zeros(cap, dtype=np.float64)
    esc = ctypes.c_double(0.0)
    n = lib().orc_electron_walk(ctypes.byref(ph._c), _ptr(iev), cutoff_mev, _ptr(rr), _ptr(dd),
                                t0, _ptr(vo), _ptr(eo), cap, ctypes.byref(esc))
    if n > cap:
        raise ValueError("more deposits than cap")
    return [(int(vo[k]), float(eo[k])) for k in range(n)], esc.value


# --------------------------------------------------------------------------
# Transport
# --------------------------------------------------------------------------
class Phantom:
    """Holds FP64/uint8 copies of a phantom in the oracle's layout
    ([nz][ny][nx], x fastest; voxel size in cm)."""

    def __init__(self, density, material, z_eff, z_over_a, voxel_cm, label=None,
                 n_organs=0, activity=None):
        self.density = np.ascontiguousarray(density, dtype=np.float64)
        nz, ny, nx = self.density.shape
        self.shape = (nz, ny, nx)
        self.material = np.ascontiguousarray(material, dtype=np.uint8)
        self.label = None if label is None else np.ascontiguousarray(label, dtype=np.uint8)
        self.n_organs = int(n_organs)
        self.z_eff = np.ascontiguousarray(z_eff, dtype=np.float64)
        self.z_over_a = np.ascontiguousarray(z_over_a, dtype=np.float64)
        self.voxel_cm = tuple(float(v) for v in voxel_cm)
        self.activity = (None if activity is None
                         else np.ascontiguousarray(activity, dtype=np.float64))
        self._c = _Phantom(nx, ny, nz, self.voxel_cm[0], self.voxel_cm[1], self.voxel_cm[2],
                           _ptr(self.density), _ptr(self.material), _ptr(self.label),
                           self.n_organs, _ptr(self.z_eff), _ptr(self.z_over_a),
                           len(self.z_eff), _ptr(self.activity))

    @property
    def nvox(self):
        nz, ny, nx = self.shape
        return nx * ny * nz

    @property
    def voxel_cm3(self):
        return self.voxel_cm[0] * self.voxel_cm[1] * self.voxel_cm[2]

    def majorant(self, e_mev: float) -> float:
        return lib().orc_majorant(ctypes.byref(self._c), float(e_mev))


class Tally:
    """Accumulated sums of one phantom: S_v, S2_v (MeV, MeV^2 per voxel),
    O_o, O2_o (per-history organ scores), ledger (MeV) and counters."""

    def __init__(self, ph: Phantom):
        self.S = np.zeros(ph.shape, dtype=np.float64)
        self.S2 = np.zeros(ph.shape, dtype=np.float64)
        self.O = np.zeros(ph.n_organs + 1, dtype=np.float64)
        self.O2 = np.zeros(ph.n_organs + 1, dtype=np.float64)
        self.n_decays = 0
        self._c = _Tally(_ptr(self.S), _ptr(self.S2), _ptr(self.O), _ptr(self.O2))

    @property
    def ledger(self) -> dict:
        return dict(zip(LEDGER_FIELDS, list(self._c.ledger)))

    @property
    def stats(self) -> dict:
        return dict(zip(STATS_FIELDS, [int(x) for x in self._c.stats]))


def run(ph: Phantom, n_hist: int, seed: int, tally: Tally | None = None, *,
        first_hist: int = 0, pid: int = 0, photons_per_decay: int = 2,
        process_mask: int = 7, max_real_events: int = 0, cutoff_mev: float = 0.010,
        tracking: int = TRACK_EXACT, kn_method: int | None = None, wide: bool | None = None,
        pencil=None, n_threads: int = 0, history_records: bool = False,
        electron_cutoff_mev: float = 0.0, mean_excitation_ev=None, rng: int | None = None,
        positron: bool = False, noncol_fwhm_deg: float = 0.5, emitter=None):
    """Run n_hist histories; returns (tally, per-history records or None).

    ``pencil=(origin_cm, direction)`` selects a pencil-beam source.  The
    defaults follow the tracking mode: exact traversal uses Kahn's sampler,
    53-bit uniforms and xoshiro256** streams (a generator family the device
    does not use); Woodcock replays the device draw order (Philox4x32-10,
    Butcher-Messel, 23-bit uniforms).  ``electron_cutoff_mev > 0`` walks Compton electrons
    above it straight ahead (CSDA; needs ``mean_excitation_ev`` per
    material); 0 deposits them on the spot.  ``positron=True`` gives each
    decay its 18F positron (kinetic energy from the beta+ spectrum, a
    straight CSDA walk, the pair born where it ends; needs
    ``mean_excitation_ev``) and tilts the second photon off back to back by
    a Rayleigh-distributed angle of FWHM ``noncol_fwhm_deg``.
    ``emitter=(line_mev, line_yield, beta_mean_mev)`` replaces the photon
    pair by a gamma + beta emitter: each decay emits at most one photon
    (line i with probability line_yield[i]) and leaves beta_mean_mev in its
    voxel.
    """
    if tally is None:
        tally = Tally(ph)
    if kn_method is None:
        kn_method = KN_KAHN if tracking == TRACK_EXACT else KN_BUTCHER
    if wide is None:
        wide = tracking == TRACK_EXACT
    if rng is None:
        rng = RNG_XOSHIRO if tracking == TRACK_EXACT else RNG_PHILOX
    rec = np.zeros((n_hist, len(HREC_FIELDS)), dtype=np.float64) if history_records else None
    o = _Opts()
    o.n_hist, o.first_hist, o.seed, o.pid = n_hist, first_hist, seed, pid
    o.photons_per_decay, o.process_mask = photons_per_decay, process_mask
    o.max_real_events, o.cutoff_mev = max_real_events, cutoff_mev
    o.tracking, o.kn_method, o.wide_uniforms = tracking, kn_method, int(bool(wide))
    o.rng = int(rng)
    if pencil is not None:
        o.source_kind = SRC_PENCIL
        for a in range(3):
            o.pencil_origin[a] = float(pencil[0][a])
            o.pencil_dir[a] = float(pencil[1][a])
    else:
        o.source_kind = SRC_ACTIVITY
        if ph.activity is None:
            raise ValueError("phantom has no activity map")
    o.n_threads = n_threads
    o.hist_out = _ptr(rec)
    iev = None
    if electron_cutoff_mev > 0.0 or positron:
        if mean_excitation_ev is None:
            raise ValueError("electron and positron transport need mean_excitation_ev per "
                             "material")
        iev = np.ascontiguousarray(mean_excitation_ev, dtype=np.float64)
        if iev.shape != (len(ph.z_eff),):
            raise ValueError("one mean excitation energy per material")
    o.electron_cutoff_mev = float(electron_cutoff_mev)
    o.mean_excitation_ev = _ptr(iev)
    o.positron = int(bool(positron))
    o.noncol_fwhm_rad = float(np.radians(noncol_fwhm_deg))
    if emitter is not None:
        le = np.ascontiguousarray(emitter[0], dtype=np.float64)
        ly = np.ascontiguousarray(emitter[1], dtype=np.float64)
        if le.shape != ly.shape:
            raise ValueError("one yield per line")
        o.n_lines, o.line_mev, o.line_yield = le.size, _ptr(le), _ptr(ly)
        o.beta_mean_mev = float(emitter[2])
    rc = lib().orc_run(ctypes.byref(ph._c), ctypes.byref(o), ctypes.byref(tally._c))
    if rc != 0:
        raise ValueError("oracle rejected the input (code %d)" % rc)
    tally.n_decays += n_hist
    return tally, rec


def finalize(ph: Phantom, tally: Tally, a_ts_bq: float | None = None):
    """Eq. 1: dose-rate map (Gy/s) and relative uncertainty map.  A(t_s)
    defaults to the map's total activity sum(A_v * V_v[mL])."""
    if a_ts_bq is None:
        a_ts_bq = float(ph.activity.sum() * ph.voxel_cm3)
    rate = np.zeros(ph.shape, dtype=np.float64)
    eps = np.zeros(ph.shape, dtype=np.float64)
    lib().orc_finalize(_ptr(tally.S), _ptr(tally.S2), _ptr(ph.density), ph.nvox, ph.voxel_cm3,
                       float(tally.n_decays), float(a_ts_bq), _ptr(rate), _ptr(eps))
    return rate, eps


def organ_stats(ph: Phantom, rate, eps):
    """Eq. 2 and Eq. 3 for labels 1..n_organs."""
    r = np.zeros(ph.n_organs, dtype=np.float64)
    e = np.zeros(ph.n_organs, dtype=np.float64)
    lib().orc_organ_stats(_ptr(np.ascontiguousarray(rate)), _ptr(np.ascontiguousarray(eps)),
                          _ptr(ph.label), ph.nvox, ph.n_organs, _ptr(r), _ptr(e))
    return r, e


def organ_mean_sigma(tally: Tally, a_ts_bq: float):
    """Organ dose rate from the per-history organ scores (A * O_o / N) and the
    relative standard error of that mean, for labels 1..n_organs."""
    n = float(tally.n_decays)
    m = tally.O[1:] / n
    var = np.maximum(tally.O2[1:] / n - m * m, 0.0) / (n - 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(m > 0, np.sqrt(var) / m, 0.0)
    return a_ts_bq * m, rel
