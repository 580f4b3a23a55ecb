"""Seeded synthetic inputs: phantoms, organ label maps and activity maps.

This module builds INPUTS only (geometry, densities, materials, labels and
activity concentrations).  It holds none of the transport or scoring
arithmetic, imports neither the HIP library nor the CPU oracle, and both
sides take their inputs from it.

The shapes follow the paper's workloads (Section 2.2): a centre-voxel point
photon source in a water cube, and a whole-body PET/CT patient with the four
materials of Section 2.1 (water/soft tissue, dry air, compact bone, lung) and
the 27 organs of Table 1.  The patient data are not available, so the
whole-body case is an analytic ellipsoid phantom with seeded jitter.

Layout of every 3-D array: C order [nz][ny][nx], x fastest.  Voxel sizes are
in mm.  Activity concentration is in Bq/mL.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Materials (Section 2.1 names four; the effective Z values and the
# electron fractions Z/A are the readings stated in the design notes).
#                 name           Z_eff  Z/A    density g/cm^3
MATERIALS = {
    "water":       (7.4, 0.5551, 1.0),
    "air":         (7.6, 0.499, 0.0012),
    "lung":        (7.5, 0.550, 0.26),
    "soft_tissue": (7.4, 0.551, 1.0),
    "bone":        (12.3, 0.515, 1.85),
}

# Mean excitation energies (eV) for electron stopping powers, ICRU Report 37
# values for liquid water, dry air, ICRP lung, ICRP soft tissue and ICRU
# compact bone.
MEAN_EXCITATION_EV = {"water": 75.0, "air": 85.7, "lung": 75.3, "soft_tissue": 72.3,
                      "bone": 91.9}

# The 27 organs of Table 1, in the table's order (labels 1..27); label 28 is
# the rest of the body, label 0 is outside the body.
ORGANS = (
    "Bladder", "Bowel", "Brain", "Brain_Stem", "Esophagus", "Eye_Left", "Eye_Right",
    "Heart", "Kidney_Left", "Kidney_Right", "Larynx", "Liver", "Lung_Left", "Lung_Right",
    "Optic_Chiasm", "Optical_Nerve_Left", "Optical_Nerve_Right", "Pancreas",
    "Parotid_Left", "Parotid_Right", "Pelvis", "Pituitary", "Rectum", "Spinal_Cord",
    "Spleen", "Stomach", "Thyroid_Gland",
)
BODY_LABEL = len(ORGANS) + 1  # 28

# Total activity of the synthetic patients: 8.0 mCi injected (Section 2.2)
# decayed over the 60 min uptake with the F-18 half-life of 109.77 min.
PATIENT_TOTAL_BQ = 8.0 * 3.7e7 * 0.5 ** (60.0 / 109.77)


@dataclass
class Problem:
    """One synthetic workload: a phantom, its activity and run settings."""
    name: str
    density: np.ndarray            # float32 [nz][ny][nx], g/cm^3
    material: np.ndarray           # uint8, index into `materials`
    label: np.ndarray              # uint8, 0 = none, 1..n_organs
    activity: np.ndarray           # float32 Bq/mL, >= 0
    voxel_mm: tuple                # (dx, dy, dz)
    materials: list                # [(z_eff, z_over_a)]
    n_organs: int
    organ_names: tuple
    photons_per_decay: int = 2
    n_decays: int = 10 ** 6
    seed: int = 1
    total_activity_bq: float = 0.0  # A(t_s); 0 -> sum(A_v V_v)
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.density.shape

    @property
    def nvox(self):
        return int(np.prod(self.density.shape))

    @property
    def voxel_cm(self):
        return tuple(v / 10.0 for v in self.voxel_mm)


def _material_table(names):
    return [(MATERIALS[n][0], MATERIALS[n][1]) for n in names]


def _shell_labels(n, centre):
    """Radial shells around the centre voxel: label k+1 for distance in
    [k, k+1) voxel widths, k < n_shells; 0 beyond."""
    nz, ny, nx = n
    cz, cy, cx = centre
    z, y, x = np.meshgrid(np.arange(nz) - cz, np.arange(ny) - cy, np.arange(nx) - cx,
                          indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    n_shells = min(cz, cy, cx, nz - 1 - cz, ny - 1 - cy, nx - 1 - cx) + 1
    k = np.floor(r).astype(np.int64)
    lab = np.where(k < n_shells, k + 1, 0).astype(np.uint8)
    return lab, int(n_shells)


def water_point_source(n=64, voxel_mm=2.0, n_decays=10 ** 6, seed=1, centre=None):
    """Water cube with a point photon source in the centre voxel, one
    0.511 MeV photon per history (the point-source experiment of Section 2.2).
    Labels are radial shells, giving a dose-distance curve."""
    shape = (n, n, n)
    c = n // 2 if centre is None else centre
    rho = np.full(shape, MATERIALS["water"][2], dtype=np.float32)
    mat = np.zeros(shape, dtype=np.uint8)
    act = np.zeros(shape, dtype=np.float32)
    act[c, c, c] = 1.0
    lab, n_shells = _shell_labels(shape, (c, c, c))
    return Problem("water_point_%d" % n, rho, mat, lab, act, (voxel_mm,) * 3,
                   _material_table(["water"]), n_shells,
                   tuple("shell_%d" % k for k in range(n_shells)),
                   photons_per_decay=1, n_decays=n_decays, seed=seed,
                   total_activity_bq=1.0, extra={"centre": (c, c, c)})


def slab_phantom(n=128, voxel_mm=3.0, n_decays=10 ** 8, geometry_seed=2, seed=102):
    """Heterogeneous slab phantom: a soft-tissue block in air with a lung slab
    and a bone cylinder (axis along y) placed by a seeded draw, and a point
    source of back-to-back photon pairs at the block centre.

    Labels: 1 lung slab, 2 bone cylinder, 3..10 soft-tissue octants around
    the source, 0 air."""
    rng = np.random.default_rng(geometry_seed)
    shape = (n, n, n)
    c = n // 2
    lo, hi = n // 16, n - n // 16          # block [8, 120) for n = 128
    mat = np.zeros(shape, dtype=np.uint8)  # 0 air, 1 lung, 2 soft, 3 bone
    mat[lo:hi, lo:hi, lo:hi] = 2
    t = int(rng.integers(15, 31)) * n // 128
    t = max(t, 2)
    gap = max(6 * n // 128, 2)
    z0 = int(rng.integers(c + gap, hi - t + 1))
    mat[z0:z0 + t, lo:hi, lo:hi] = 1
    r = float(rng.uniform(5.0, 10.0)) * n / 128.0
    zc = float(rng.uniform(z0 + 0.25 * t, z0 + 0.75 * t))
    xc = float(rng.uniform(lo + r + 1, hi - r - 1))
    zz, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    disc = (zz - zc) ** 2 + (xx - xc) ** 2 < r * r
    cyl = np.zeros(shape, dtype=bool)
    cyl[:, lo:hi, :] = disc[:, None, :]
    cyl &= mat > 0
    mat[cyl] = 3
    names = ["air", "lung", "soft_tissue", "bone"]
    dens = np.array([MATERIALS[k][2] for k in names], dtype=np.float32)
    rho = dens[mat]
    lab = np.zeros(shape, dtype=np.uint8)
    soft = mat == 2
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    octant = (z >= c).astype(np.uint8) * 4 + (y >= c).astype(np.uint8) * 2 + (x >= c)
    lab[soft] = 3 + octant[soft]
    lab[mat == 1] = 1
    lab[mat == 3] = 2
    act = np.zeros(shape, dtype=np.float32)
    act[c, c, c] = 1.0
    organ_names = ("lung_slab", "bone_cylinder") + tuple("soft_octant_%d" % k for k in range(8))
    return Problem("slab_%d" % n, rho, mat, lab, act, (voxel_mm,) * 3, _material_table(names),
                   10, organ_names, photons_per_decay=2, n_decays=n_decays, seed=seed,
                   total_activity_bq=1.0,
                   extra={"centre": (c, c, c), "slab_z": (z0, z0 + t), "cyl_xz": (xc, zc),
                          "cyl_r": r, "block": (lo, hi)})


# Organ templates of the reference adult body (cm, field of view
# 51.2 x 51.2 x 96): centre (x, y, z), semi-axes (a, b, c), material.
# x runs right->left of the image, y anterior->posterior, z feet->head.
_ORGAN_TEMPLATES = {
    "Lung_Left":           ((19.0, 26.0, 55.0), (5.5, 7.0, 10.0), "lung"),
    "Lung_Right":          ((32.2, 26.0, 55.0), (5.5, 7.0, 10.0), "lung"),
    "Pelvis":              ((25.6, 26.0, 18.0), (12.0, 7.0, 5.0), "bone"),
    "Liver":               ((32.0, 24.0, 44.0), (8.0, 6.0, 6.0), "soft_tissue"),
    "Bowel":               ((25.6, 21.0, 26.0), (9.0, 5.0, 5.5), "soft_tissue"),
    "Stomach":             ((19.6, 23.0, 46.0), (4.0, 3.0, 5.0), "soft_tissue"),
    "Spleen":              ((17.0, 30.0, 46.0), (3.0, 3.0, 5.0), "soft_tissue"),
    "Kidney_Left":         ((20.6, 30.0, 38.0), (2.5, 2.0, 5.0), "soft_tissue"),
    "Kidney_Right":        ((30.6, 30.0, 38.0), (2.5, 2.0, 5.0), "soft_tissue"),
    "Pancreas":            ((25.6, 27.0, 41.0), (5.0, 1.5, 1.5), "soft_tissue"),
    "Heart":               ((27.5, 22.0, 52.0), (5.0, 4.5, 5.0), "soft_tissue"),
    "Bladder":             ((25.6, 21.0, 15.0), (4.0, 3.5, 3.5), "soft_tissue"),
    "Rectum":              ((25.6, 29.0, 15.0), (1.5, 1.5, 4.0), "soft_tissue"),
    "Esophagus":           ((25.6, 30.0, 61.0), (1.0, 1.0, 8.0), "soft_tissue"),
    "Spinal_Cord":         ((25.6, 33.5, 45.0), (0.6, 0.6, 28.0), "soft_tissue"),
    "Brain":               ((25.6, 26.0, 87.0), (6.5, 8.0, 6.0), "soft_tissue"),
    "Brain_Stem":          ((25.6, 28.0, 79.5), (1.5, 1.5, 3.0), "soft_tissue"),
    "Thyroid_Gland":       ((25.6, 19.5, 68.0), (2.0, 1.0, 2.0), "soft_tissue"),
    "Larynx":              ((25.6, 19.5, 71.5), (1.5, 1.5, 2.0), "soft_tissue"),
    "Parotid_Left":        ((20.6, 25.0, 77.0), (1.5, 2.0, 2.5), "soft_tissue"),
    "Parotid_Right":       ((30.6, 25.0, 77.0), (1.5, 2.0, 2.5), "soft_tissue"),
    "Eye_Left":            ((22.6, 18.5, 83.0), (1.2, 1.2, 1.2), "soft_tissue"),
    "Eye_Right":           ((28.6, 18.5, 83.0), (1.2, 1.2, 1.2), "soft_tissue"),
    "Optical_Nerve_Left":  ((23.8, 20.5, 83.2), (0.4, 1.5, 0.4), "soft_tissue"),
    "Optical_Nerve_Right": ((27.4, 20.5, 83.2), (0.4, 1.5, 0.4), "soft_tissue"),
    "Optic_Chiasm":        ((25.6, 22.2, 83.5), (0.8, 0.5, 0.4), "soft_tissue"),
    "Pituitary":           ((25.6, 24.0, 82.0), (0.5, 0.5, 0.5), "soft_tissue"),
}
_REF_FOV = (51.2, 51.2, 96.0)
_HIGH_UPTAKE = ("Brain", "Heart", "Bladder")


def _ellipsoid_mask(shape, voxel_cm, centre, semi):
    """Boolean mask of voxel centres inside an axis-aligned ellipsoid, plus
    the bounding-box slices it was evaluated on."""
    nz, ny, nx = shape
    dx, dy, dz = voxel_cm
    sl = []
    for c, a, h, n in ((centre[2], semi[2], dz, nz), (centre[1], semi[1], dy, ny),
                       (centre[0], semi[0], dx, nx)):
        i0 = max(int(np.floor((c - a) / h)) - 1, 0)
        i1 = min(int(np.ceil((c + a) / h)) + 1, n)
        sl.append(slice(i0, max(i1, i0)))
    z = (np.arange(sl[0].start, sl[0].stop) + 0.5) * dz
    y = (np.arange(sl[1].start, sl[1].stop) + 0.5) * dy
    x = (np.arange(sl[2].start, sl[2].stop) + 0.5) * dx
    q = (((z - centre[2]) / semi[2]) ** 2)[:, None, None] \
        + (((y - centre[1]) / semi[1]) ** 2)[None, :, None] \
        + (((x - centre[0]) / semi[0]) ** 2)[None, None, :]
    return tuple(sl), q < 1.0


def patient_phantom(shape=(320, 256, 256), voxel_mm=(2.0, 2.0, 3.0), seed=3,
                    n_decays=10 ** 9, transport_seed=103, total_bq=PATIENT_TOTAL_BQ):
    """Synthetic PET/CT patient: a torso ellipsoid joined by a neck to a head
    ellipsoid, in soft tissue, with lungs (0.26 g/cm^3), a bone skeleton proxy
    (spine, skull and rib shells, pelvis; 1.85 g/cm^3) and the 27 organs of
    Table 1 at seeded positions (+-1 cm) and sizes (+-10 %).

    Activity: 1 in the body remainder; organ factor exp(N(0, 0.5^2)); brain,
    heart and bladder scaled by U(5, 20) (high FDG uptake, Section 3.2); voxel
    noise Poisson(400)/400; 0 in air.  Normalised so sum(A_v V_v) equals
    ``total_bq`` (A(t_s) of Eq. 1).  ``shape`` is (nz, ny, nx); the anatomy is
    scaled per axis to the field of view."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    nz, ny, nx = shape
    vcm = tuple(v / 10.0 for v in voxel_mm)
    fov = (nx * vcm[0], ny * vcm[1], nz * vcm[2])
    sc = tuple(fov[a] / _REF_FOV[a] for a in range(3))

    def place(c, s):
        return tuple(c[a] * sc[a] for a in range(3)), tuple(s[a] * sc[a] for a in range(3))

    names = ["air", "lung", "soft_tissue", "bone"]
    mid = {n: i for i, n in enumerate(names)}
    mat = np.zeros(shape, dtype=np.uint8)
    lab = np.zeros(shape, dtype=np.uint8)

    def paint(centre, semi, m, label, within=None, shell=None):
        sl, q = _ellipsoid_mask(shape, vcm, centre, semi)
        if shell is not None:
            # the inner mask is evaluated on its own (smaller) box: align it
            inner = np.zeros_like(q)
            sli, qi2 = _ellipsoid_mask(shape, vcm, centre, tuple(s * shell for s in semi))
            off = tuple(sli[a].start - sl[a].start for a in range(3))
            inner[off[0]:off[0] + qi2.shape[0], off[1]:off[1] + qi2.shape[1],
                  off[2]:off[2] + qi2.shape[2]] = qi2
            q = q & ~inner
        if within is not None:
            q = q & within[sl]
        if m is not None:
            mat[sl][q] = m
        if label is not None:
            lab[sl][q] = label
        return sl, q

    torso_semi = tuple(s * rng.uniform(0.9, 1.1) for s in (17.0, 11.0, 33.0))
    body = [place((25.6, 25.6, 40.0), torso_semi), place((25.6, 26.0, 72.0), (6.0, 6.0, 6.0)),
            place((25.6, 26.0, 84.0), (8.0, 9.5, 11.0))]
    for c, s in body:
        paint(c, s, mid["soft_tissue"], BODY_LABEL)
    inbody = mat > 0

    # skeleton proxy (label stays "body remainder")
    c, s = place((25.6, 26.0, 84.0), (8.0, 9.5, 11.0))
    paint(c, s, mid["bone"], None, within=inbody, shell=0.92)
    c, s = place((25.6, 33.5, 45.0), (1.6, 1.6, 31.0))
    paint(c, s, mid["bone"], None, within=inbody)
    tc, ts = place((25.6, 25.6, 40.0), torso_semi)
    rib_mask = np.zeros(shape, dtype=bool)
    sl, q = _ellipsoid_mask(shape, vcm, tc, ts)
    sli, qi = _ellipsoid_mask(shape, vcm, tc, (ts[0] * 0.93, ts[1] * 0.93, ts[2]))
    inner = np.zeros_like(q)
    off = tuple(sli[a].start - sl[a].start for a in range(3))
    inner[off[0]:off[0] + qi.shape[0], off[1]:off[1] + qi.shape[1],
          off[2]:off[2] + qi.shape[2]] = qi
    zc = (np.arange(sl[0].start, sl[0].stop) + 0.5) * vcm[2] / sc[2]
    band = (zc > 44.0) & (zc < 66.0) & (np.floor(zc / 1.5).astype(int) % 2 == 0)
    rib_mask[sl] = q & ~inner & band[:, None, None]
    mat[rib_mask & inbody] = mid["bone"]

    order = ["Lung_Left", "Lung_Right", "Pelvis", "Liver", "Bowel", "Stomach", "Spleen",
             "Kidney_Left", "Kidney_Right", "Pancreas", "Heart", "Bladder", "Rectum",
             "Esophagus", "Spinal_Cord", "Brain", "Brain_Stem", "Thyroid_Gland", "Larynx",
             "Parotid_Left", "Parotid_Right", "Eye_Left", "Eye_Right", "Optical_Nerve_Left",
             "Optical_Nerve_Right", "Optic_Chiasm", "Pituitary"]
    placed = {}
    for name in order:
        c0, s0, m = _ORGAN_TEMPLATES[name]
        jit = rng.uniform(-1.0, 1.0, size=3)
        if name in ("Optic_Chiasm", "Pituitary", "Optical_Nerve_Left", "Optical_Nerve_Right",
                    "Eye_Left", "Eye_Right", "Spinal_Cord", "Esophagus"):
            jit = jit * 0.2  # small midline structures keep their anatomy
        c = tuple(c0[a] + jit[a] for a in range(3))
        s = tuple(s0[a] * rng.uniform(0.9, 1.1) for a in range(3))
        c, s = place(c, s)
        shell = 0.75 if name == "Pelvis" else None
        paint(c, s, mid[m], ORGANS.index(name) + 1, within=inbody, shell=shell)
        placed[name] = (c, s)

    dens = np.array([MATERIALS[k][2] for k in names], dtype=np.float32)
    rho = dens[mat]

    # activity
    factor = np.zeros(BODY_LABEL + 1, dtype=np.float64)
    factor[BODY_LABEL] = 1.0
    for i, name in enumerate(ORGANS):
        f = float(np.exp(rng.normal(0.0, 0.5)))
        if name in _HIGH_UPTAKE:
            f *= float(rng.uniform(5.0, 20.0))
        factor[i + 1] = f
    base = factor[lab]
    noise = rng.poisson(400.0, size=shape).astype(np.float64) / 400.0
    act = np.where(lab > 0, base * noise, 0.0)
    vol_ml = vcm[0] * vcm[1] * vcm[2]
    act *= total_bq / (act.sum() * vol_ml)
    return Problem("patient_%dx%dx%d" % (nx, ny, nz), rho, mat, lab, act.astype(np.float32),
                   tuple(voxel_mm), _material_table(names), BODY_LABEL,
                   ORGANS + ("Body_Remainder",), photons_per_decay=2, n_decays=n_decays,
                   seed=transport_seed, total_activity_bq=float(total_bq),
                   extra={"organs": placed, "organ_factor": factor})


def batch_phantoms(n=64, first_seed=4000, n_decays=10 ** 7):
    """Uneven batch: per phantom nx, ny ~ U{64..192}, nz ~ U{64..256}, an
    isotropic voxel of 2, 3 or 4 mm, and the patient generator scaled to that
    field of view."""
    out = []
    for i in range(n):
        s = first_seed + i
        rng = np.random.default_rng(s)
        nx, ny = (int(v) for v in rng.integers(64, 193, size=2))
        nz = int(rng.integers(64, 257))
        h = float(rng.choice([2.0, 3.0, 4.0]))
        p = patient_phantom(shape=(nz, ny, nx), voxel_mm=(h, h, h), seed=s, n_decays=n_decays,
                            transport_seed=s + 100000)
        p.name = "batch_%d" % s
        out.append(p)
    return out


def pencil_line(problem: Problem, axis_y_cm: float, axis_z_cm: float):
    """Origin on the x = 0 face and direction +x for a pencil beam at (y, z)."""
    return (0.0, axis_y_cm, axis_z_cm), (1.0, 0.0, 0.0)


# ---------------------------------------------------------------------------
# Synthetic CT images (inputs of the CT ingestion)
# ---------------------------------------------------------------------------
# A stand-in HU-to-density curve with material thresholds: the paper cites
# Schneider et al. (2000) without giving its parameters.  The nodes put the
# four phantom materials at air -1000, lung -740, soft tissue 0 and bone
# +1100 HU.  Per material, densities are kept to a few levels (the engine
# holds at most 256 distinct material-density pairs): 8 for air, 32 for
# lung, 64 for soft tissue and 64 for bone, placed so that each nominal
# density is a level centre.
SYNTHETIC_CT_TABLE = dict(
    hu=[-1000.0, -740.0, 0.0, 1100.0, 3000.0],
    density=[0.0012, 0.26, 1.0, 1.85, 2.9],
    threshold=[-950.0, -200.0, 300.0],
    density_min=[0.0, 0.05, 0.7975, 1.0875],
    density_width=[0.0024, 0.02, 0.005, 0.025],
    levels=[8, 32, 64, 64],
)
# material order of the table: air, lung, soft tissue, bone
CT_MATERIAL_NAMES = ("air", "lung", "soft_tissue", "bone")
MATERIAL_HU = {"air": -1000.0, "lung": -740.0, "soft_tissue": 0.0, "water": 0.0, "bone": 1100.0}


def render_ct(problem: Problem, factor=(2, 2, 1), pad_mm=(8.0, 8.0, 6.0), noise_hu=5.0,
              seed=11):
    """A synthetic CT of ``problem``: a grid ``factor`` times finer than the
    phantom's (per axis x, y, z), extending ``pad_mm`` beyond it on each side,
    with the nominal HU of each voxel's material plus Gaussian noise of
    ``noise_hu``, and -1000 HU outside the phantom.  The material of a CT
    voxel is that of the phantom voxel holding its centre.  Returns
    ``(hu float32 [nz][ny][nx], ct_grid, phantom_grid)``; grids are dicts
    ``n=(nx, ny, nz), spacing=(sx, sy, sz), origin=(ox, oy, oz)`` in mm, with
    the phantom's outer corner at the origin."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = problem.shape
    vm = problem.voxel_mm
    ph_grid = dict(n=(nx, ny, nz), spacing=tuple(float(v) for v in vm), origin=(0.0, 0.0, 0.0))
    sp = tuple(float(vm[a]) / factor[a] for a in range(3))
    n = tuple(int(round((problem.shape[2 - a] * vm[a] + 2 * pad_mm[a]) / sp[a])) for a in range(3))
    ct_grid = dict(n=n, spacing=sp, origin=tuple(-float(p) for p in pad_mm))
    names = [None] * len(problem.materials)
    for name, (z, za, _) in MATERIALS.items():
        for i, (mz, mza) in enumerate(problem.materials):
            if names[i] is None and (mz, mza) == (z, za):
                names[i] = name
    mat_hu = np.array([MATERIAL_HU[n_] for n_ in names], dtype=np.float32)
    idx = []
    for a in range(3):
        c = ct_grid["origin"][a] + (np.arange(n[a]) + 0.5) * sp[a]
        i = np.floor(c / vm[a]).astype(np.int64)
        idx.append((i, (i >= 0) & (i < problem.shape[2 - a])))
    (ix, okx), (iy, oky), (iz, okz) = idx
    inside = okz[:, None, None] & oky[None, :, None] & okx[None, None, :]
    m = problem.material[np.clip(iz, 0, nz - 1)][:, np.clip(iy, 0, ny - 1)][:, :, np.clip(ix, 0, nx - 1)]
    hu = np.where(inside, mat_hu[m], np.float32(-1000.0)).astype(np.float32)
    hu += rng.normal(0.0, noise_hu, size=hu.shape).astype(np.float32)
    return hu, ct_grid, ph_grid
