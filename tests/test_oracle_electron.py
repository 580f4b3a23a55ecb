"""Pins of the oracle's electron model (oracle/electron.py): published
stopping powers and ranges, recoil kinematics from textbook relations, and
invariants of the straight-ahead CSDA walk."""
import math

import numpy as np
import pytest

from oracle import electron as El

WATER_ZA, WATER_I = 0.55508, 75.0  # H2O: Z/A and mean excitation energy (ICRU Report 37)


# ICRU Report 37 (1984), electrons in liquid water: collision stopping power
# (MeV cm^2/g) and CSDA range (g/cm^2); four significant digits as tabulated.
ICRU37_WATER_SCOL = {0.1: 4.115, 0.2: 2.793, 0.3: 2.355, 0.4: 2.148, 0.5: 2.034}
ICRU37_WATER_RANGE = {0.2: 4.488e-2, 0.3: 8.421e-2, 0.4: 1.288e-1, 0.5: 1.766e-1}


@pytest.mark.parametrize("t", sorted(ICRU37_WATER_SCOL))
def test_stopping_power_of_water_matches_icru37(t):
    # no density effect in water below 0.5 MeV, so the tabulated value is the
    # formula's: agreement to the table's last digit
    s = El.stopping_power(t, WATER_ZA, WATER_I)
    assert abs(s - ICRU37_WATER_SCOL[t]) <= 0.0006


@pytest.mark.parametrize("t", [0.3, 0.4, 0.5])
def test_range_differences_match_icru37(t):
    # the table's ranges include radiative loss (a few tenths of a percent
    # of the loss at these energies), which the collision-only range omits
    ref = ICRU37_WATER_RANGE[t] - ICRU37_WATER_RANGE[0.2]
    got = El.csda_range(0.2, t, WATER_ZA, WATER_I)
    assert abs(got - ref) <= 0.006 * ref


def test_stopping_power_scales_with_electron_fraction():
    s1 = El.stopping_power(0.3, 0.5, 80.0)
    s2 = El.stopping_power(0.3, 0.25, 80.0)
    assert s1 == pytest.approx(2.0 * s2, rel=1e-14, abs=0)
    # a higher mean excitation energy slows the loss
    assert El.stopping_power(0.3, 0.5, 100.0) < s1


def test_energy_after_inverts_the_range():
    t0 = 0.3407
    for frac in (1e-6, 0.1, 0.5, 0.99):
        path = frac * El.csda_range(0.2, t0, WATER_ZA, WATER_I)
        t1 = El.energy_after(t0, path, WATER_ZA, WATER_I)
        assert 0.2 < t1 < t0
        # the root finder stops at |dT| <= 1e-15 MeV: a mass-path error of
        # 1e-15 / S(T) < 1e-15 g/cm^2, which dominates for the shortest path
        assert El.csda_range(t1, t0, WATER_ZA, WATER_I) == pytest.approx(path, rel=1e-10,
                                                                          abs=1e-15)
    with pytest.raises(ValueError):
        El.energy_after(t0, 1.0, WATER_ZA, WATER_I)


def _perp(d):
    a = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    u = np.cross(d, a)
    return u / np.linalg.norm(u)


@pytest.mark.parametrize("e,cost", [(0.511, 0.3), (0.511, -1.0), (0.3, 0.7), (0.511, -0.2)])
def test_compton_electron_kinematics(e, cost):
    rng = np.random.default_rng(3)
    d_in = rng.normal(size=3)
    d_in /= np.linalg.norm(d_in)
    sint = math.sqrt(max(0.0, 1.0 - cost * cost))
    d_out = cost * d_in + sint * _perp(d_in)
    t, de = El.compton_electron(e, cost, d_in, d_out)
    k = e / El.MEC2_MEV
    # kinetic energy: the Compton formula E' = E / (1 + k (1 - cos theta))
    assert t == pytest.approx(e - e / (1 + k * (1 - cost)), rel=1e-14, abs=0)
    assert np.linalg.norm(de) == pytest.approx(1.0, rel=1e-14, abs=0)
    # recoil angle: cot(phi) = (1 + k) tan(theta / 2)
    theta = math.acos(cost)
    cosphi = float(np.dot(de, d_in))
    phi = math.acos(min(1.0, cosphi))
    if theta < math.pi:
        assert 1.0 / math.tan(phi) == pytest.approx((1 + k) * math.tan(theta / 2), rel=1e-9, abs=0)
    else:
        assert cosphi == pytest.approx(1.0, abs=1e-14)
    # the electron is emitted on the other side of d_in from the photon
    assert np.dot(np.cross(d_in, de), np.cross(d_in, d_out)) <= 1e-12
    # |p| c = sqrt(T (T + 2 m c^2)) for the momentum that conservation gives
    e1 = e - t
    p = np.linalg.norm(e * d_in - e1 * d_out)
    assert p == pytest.approx(math.sqrt(t * (t + 2 * El.MEC2_MEV)), rel=1e-12, abs=0)
    # the largest transfer at back-scatter: T_max = E 2k / (1 + 2k)
    if cost == -1.0:
        assert t == pytest.approx(e * 2 * k / (1 + 2 * k), rel=1e-14, abs=0)


def test_compton_electron_at_zero_angle_has_no_energy():
    d = np.array([0.0, 0.0, 1.0])
    t, _ = El.compton_electron(0.511, 1.0, d, d)
    assert t == 0.0


def _water_row(nx, h_cm, rho=1.0):
    density = np.full((1, 1, nx), rho)
    material = np.zeros((1, 1, nx), dtype=np.uint8)
    return density, material, (h_cm, 1.0, 1.0)


def test_walk_below_cutoff_deposits_locally():
    density, material, h = _water_row(4, 0.1)
    dep, esc = El.csda_walk(density, material, h, [WATER_ZA], [WATER_I], [0.25, 0.5, 0.5],
                            [1.0, 0.0, 0.0], 0.15)
    assert dep == [(2, 0.15)] and esc == 0.0


def test_walk_matches_brute_force_integration():
    """A 340.7 keV electron along a row of 0.1 mm water voxels: the energy
    left at each face from a fourth-order Runge-Kutta integration of
    dT/ds = -rho S(T) in 1e-6 cm steps."""
    h, t0, x0 = 0.01, 0.3407, 0.0037
    density, material, hv = _water_row(20, h)
    dep, esc = El.csda_walk(density, material, hv, [WATER_ZA], [WATER_I], [x0, 0.5, 0.5],
                            [1.0, 0.0, 0.0], t0)
    assert esc == 0.0
    assert sum(e for _, e in dep) == pytest.approx(t0, rel=1e-13, abs=0)

    def f(t):
        return -El.stopping_power(t, WATER_ZA, WATER_I)

    ds, s, t = 1e-6, 0.0, t0
    faces = [(i + 1) * h - x0 for i in range(20)]
    at_face = []
    while t > 0.2 and len(at_face) < len(faces):
        step = min(ds, faces[len(at_face)] - s)
        k1 = f(t)
        k2 = f(t + 0.5 * step * k1)
        k3 = f(t + 0.5 * step * k2)
        k4 = f(t + step * k3)
        t_new = t + step / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        s += step
        if t_new <= 0.2:
            break
        t = t_new
        if abs(s - faces[len(at_face)]) < 1e-15:
            at_face.append(t)
    # every voxel crossed whole loses the brute-force energy difference; the
    # voxel where the range runs out takes the rest
    assert [v for v, _ in dep] == list(range(len(at_face) + 1))
    edges = [t0] + at_face
    for i in range(len(at_face)):
        assert dep[i][1] == pytest.approx(edges[i] - edges[i + 1], rel=1e-8, abs=0)
    assert dep[-1][1] == pytest.approx(at_face[-1], rel=1e-8, abs=0)


def test_walk_depends_on_mass_path_only():
    """Twice the density in voxels half as long: the same deposits voxel by
    voxel (the CSDA loss depends on rho * s alone)."""
    rng = np.random.default_rng(5)
    za, ie = [WATER_ZA, 0.5], [WATER_I, 90.0]
    dens = rng.uniform(0.2, 1.8, size=(3, 4, 5))
    mat = rng.integers(0, 2, size=(3, 4, 5)).astype(np.uint8)
    d = np.array([0.6, -0.3, 0.2])
    d /= np.linalg.norm(d)
    r = np.array([0.011, 0.027, 0.013])
    a, ea = El.csda_walk(dens, mat, (0.006, 0.01, 0.008), za, ie, r, d, 0.34)
    b, eb = El.csda_walk(2 * dens, mat, (0.003, 0.005, 0.004), za, ie, r / 2, d, 0.34)
    assert [v for v, _ in a] == [v for v, _ in b]
    assert np.allclose([e for _, e in a], [e for _, e in b], rtol=1e-9, atol=1e-14)
    assert ea == pytest.approx(eb, rel=1e-9, abs=1e-14)


def test_walk_conserves_energy_and_crosses_face_neighbours():
    rng = np.random.default_rng(8)
    za, ie = [WATER_ZA, 0.49919, 0.53096], [WATER_I, 85.7, 91.9]
    dens = rng.uniform(0.001, 1.9, size=(6, 6, 6))
    mat = rng.integers(0, 3, size=(6, 6, 6)).astype(np.uint8)
    for trial in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = rng.uniform(0.0, 0.06, size=3)
        t0 = rng.uniform(0.2, 0.3407)
        dep, esc = El.csda_walk(dens, mat, (0.01, 0.01, 0.01), za, ie, r, d, t0)
        assert sum(e for _, e in dep) + esc == pytest.approx(t0, rel=1e-13, abs=0)
        assert all(e >= 0.0 for _, e in dep)
        for (v0, _), (v1, _) in zip(dep, dep[1:]):
            a = np.array(np.unravel_index(v0, (6, 6, 6))[::-1])
            b = np.array(np.unravel_index(v1, (6, 6, 6))[::-1])
            assert np.abs(a - b).sum() == 1


def test_walk_escape_carries_the_remaining_energy():
    """Air-like density over three 1 mm voxels: the electron leaves the grid
    with the energy its mass path leaves it."""
    density, material, hv = _water_row(3, 0.1, rho=0.0012)
    t0 = 0.3
    dep, esc = El.csda_walk(density, material, hv, [WATER_ZA], [WATER_I], [0.05, 0.5, 0.5],
                            [1.0, 0.0, 0.0], t0)
    assert [v for v, _ in dep] == [0, 1, 2]
    t_out = El.energy_after(t0, 0.0012 * 0.25, WATER_ZA, WATER_I)
    assert esc == pytest.approx(t_out, rel=1e-10, abs=0)
    assert sum(e for _, e in dep) + esc == pytest.approx(t0, rel=1e-13, abs=0)


# ---------------------------------------------------------------------------
# The C oracle's electron option (oracle/nmd_oracle.c), checked against the
# pinned model above and against run-level invariants.
# ---------------------------------------------------------------------------
from conftest import ledger_balance, oracle_phantom  # noqa: E402
from paper_2111_11687_amd import phantoms as P  # noqa: E402


def test_c_primitives_match_the_pinned_model(orc):
    for za, ie in [(WATER_ZA, WATER_I), (0.499, 85.7), (0.515, 91.9)]:
        for t in (0.2, 0.25, 0.3407, 0.5):
            assert orc.stopping_power(t, za, ie) == pytest.approx(
                El.stopping_power(t, za, ie), rel=1e-14, abs=0)
            assert orc.csda_range(0.2, t, za, ie) == pytest.approx(
                El.csda_range(0.2, t, za, ie), rel=1e-12, abs=1e-300)
        for frac in (1e-4, 0.3, 0.95):
            p = frac * El.csda_range(0.2, 0.3407, za, ie)
            assert orc.energy_after(0.3407, p, 0.2, za, ie) == pytest.approx(
                El.energy_after(0.3407, p, za, ie), rel=1e-12, abs=0)


def test_c_walk_matches_the_pinned_walk(orc):
    rng = np.random.default_rng(21)
    za, ie = [WATER_ZA, 0.499, 0.515], [WATER_I, 85.7, 91.9]
    dens = rng.uniform(0.001, 1.9, size=(5, 6, 7))
    mat = rng.integers(0, 3, size=(5, 6, 7)).astype(np.uint8)
    h = (0.012, 0.009, 0.015)
    ph = orc.Phantom(dens, mat, [7.4, 7.6, 12.3], za, h)
    for _ in range(25):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = rng.uniform(0.0, 1.0, size=3) * np.array([7, 6, 5]) * np.array(h)
        t0 = rng.uniform(0.2, 0.3407)
        a, ea = orc.electron_walk(ph, ie, 0.2, r, d, t0)
        b, eb = El.csda_walk(dens, mat, h, za, ie, r, d, t0)
        assert [v for v, _ in a] == [v for v, _ in b]
        assert np.allclose([e for _, e in a], [e for _, e in b], rtol=1e-10, atol=1e-15)
        assert ea == pytest.approx(eb, rel=1e-10, abs=1e-15)


def _patient(n=(40, 32, 32), seed=9):
    prob = P.patient_phantom(shape=n, voxel_mm=(8.0, 8.0, 12.0), seed=seed)
    iev = [P.MEAN_EXCITATION_EV[next(k for k in P.MATERIALS
                                     if tuple(P.MATERIALS[k][:2]) == tuple(m))]
           for m in prob.materials]
    return prob, iev


@pytest.mark.parametrize("tracking", ["exact", "woodcock"])
def test_electrons_keep_every_photon_draw_and_the_energy(orc, tracking):
    """The walk draws no random numbers: with the same seed every history has
    the same photon events and draws, and the energy it leaves plus the
    energy it sends out is the same."""
    prob, iev = _patient()
    ph = oracle_phantom(orc, prob)
    tr = orc.TRACK_EXACT if tracking == "exact" else orc.TRACK_WOODCOCK
    t0, r0 = orc.run(ph, 4000, 5, tracking=tr, history_records=True)
    t1, r1 = orc.run(ph, 4000, 5, tracking=tr, history_records=True,
                     electron_cutoff_mev=0.2, mean_excitation_ev=iev)
    assert np.array_equal(r0[:, [2, 3, 4, 5, 8]], r1[:, [2, 3, 4, 5, 8]])
    assert np.allclose(r0[:, 0] + r0[:, 1], r1[:, 0] + r1[:, 1], rtol=1e-12, atol=1e-12)
    assert abs(ledger_balance(t1.ledger)) < 1e-12
    # some electrons do walk: deposits spread over more voxels
    assert (r1[:, 7] >= r0[:, 7]).all() and (r1[:, 7] > r0[:, 7]).any()


def test_electron_cutoff_above_the_largest_transfer_changes_nothing(orc):
    prob, iev = _patient(n=(24, 20, 20))
    ph = oracle_phantom(orc, prob)
    # one thread: the tally's summation order is then fixed
    a, _ = orc.run(ph, 3000, 8, n_threads=1)
    b, _ = orc.run(ph, 3000, 8, n_threads=1, electron_cutoff_mev=0.35, mean_excitation_ev=iev)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.S2, b.S2)


def test_electron_option_rejects_missing_energies(orc):
    prob, iev = _patient(n=(24, 20, 20))
    ph = oracle_phantom(orc, prob)
    with pytest.raises(ValueError):
        orc.run(ph, 10, 1, electron_cutoff_mev=0.2)
    with pytest.raises(ValueError):
        orc.run(ph, 10, 1, electron_cutoff_mev=0.2, mean_excitation_ev=[0.0] * len(iev))
