"""Pins of the oracle's transport and scoring: energy conservation, narrow-beam
attenuation (homogeneous and along a heterogeneous line), first-collision
energy transfer, a total-absorption cell that fixes the dose units and the
history-by-history merge, Walters' variance on toy tallies, point-source
symmetry, and agreement of the independent tracking modes.  Tracking 2 is
Woodcock tracking with a majorant by region (the bounding box of the dense
voxels and the thin voxels around it): its pins are the same closed forms,
a beam that starts in the thin region and crosses the box, and agreement
with exact traversal."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2111_11687_amd import phantoms as P

MEC2 = 0.51099895
J_PER_MEV = 1.602176634e-13


def _oracle_phantom(orc, prob, activity=True):
    return orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                       [m[1] for m in prob.materials], prob.voxel_cm, label=prob.label,
                       n_organs=prob.n_organs, activity=prob.activity if activity else None)


def _mu(orc, z, zoa, rho, e=0.511):
    return rho * sum(orc.mass_atten(p, z, zoa, e) for p in (1, 2, 3))


def _balance(led):
    dep = led["dep_compton"] + led["dep_pe"] + led["dep_cutoff"] + led.get("dep_positron", 0.0)
    return (dep + led["escaped"] + led["discarded"]) / led["emitted"] - 1.0


@pytest.mark.parametrize("tracking", [0, 1, 2])
def test_energy_conservation(orc, tracking):
    prob = P.slab_phantom(n=48, voxel_mm=6.0)
    ph = _oracle_phantom(orc, prob)
    tal, _ = orc.run(ph, 20000, 3, tracking=tracking)
    assert abs(_balance(tal.ledger)) < 1e-9
    assert tal.ledger["emitted"] == pytest.approx(2 * 20000 * 0.511, rel=1e-12, abs=0)
    s = float(tal.S.sum())
    dep = tal.ledger["dep_compton"] + tal.ledger["dep_pe"] + tal.ledger["dep_cutoff"]
    assert s == pytest.approx(dep, rel=1e-12, abs=0)


@pytest.mark.parametrize("tracking", [0, 1, 2])
def test_narrow_beam_homogeneous_water(orc, tracking):
    n, h = 25, 4.0  # 10 cm of water
    prob = P.water_point_source(n=n, voxel_mm=h)
    ph = _oracle_phantom(orc, prob)
    y = z = n * h / 20.0
    N = 200000
    _, rec = orc.run(ph, N, 21, tracking=tracking,
                     pencil=((0.0, y, z), (1.0, 0.0, 0.0)), history_records=True)
    uncollided = (rec[:, 2] + rec[:, 3] + rec[:, 4] == 0).mean()
    p = math.exp(-_mu(orc, 7.4, 0.5551, 1.0) * n * h / 10.0)
    assert p == pytest.approx(0.3833, abs=2e-4)
    assert abs(uncollided - p) < 4 * math.sqrt(p * (1 - p) / N)


@pytest.mark.parametrize("tracking", [0, 1, 2])
def test_narrow_beam_through_lung_and_bone(orc, tracking):
    prob = P.slab_phantom()
    ex = prob.extra
    h = prob.voxel_cm[0]
    # a line along +x through the middle of the bone cylinder, which sits
    # inside the lung slab
    zc = ex["cyl_xz"][1]
    iz = int(zc)
    iy = prob.shape[1] // 2
    line_mat = prob.material[iz, iy, :]
    assert {1, 3} <= set(line_mat.tolist())  # crosses lung and bone
    mats = prob.materials
    mu = [_mu(orc, mats[m][0], mats[m][1], prob.density[iz, iy, i]) for i, m in
          enumerate(line_mat)]
    p = math.exp(-sum(mu) * h)
    ph = _oracle_phantom(orc, prob)
    N = 200000
    _, rec = orc.run(ph, N, 22, tracking=tracking,
                     pencil=((0.0, (iy + 0.5) * h, (iz + 0.5) * h), (1.0, 0.0, 0.0)),
                     history_records=True)
    uncollided = (rec[:, 2] + rec[:, 3] + rec[:, 4] == 0).mean()
    assert abs(uncollided - p) < 4 * math.sqrt(p * (1 - p) / N)


def test_first_collision_compton_energy_transfer(orc):
    """Compton only, one interaction then the photon is dropped: the mean
    deposit per photon is E0 <T/E>_KN (1 - exp(-mu_C L))."""
    n, h = 20, 5.0
    prob = P.water_point_source(n=n, voxel_mm=h)
    ph = _oracle_phantom(orc, prob)
    N = 400000
    tal, rec = orc.run(ph, N, 31, pencil=((0.0, 5.0, 5.0), (1.0, 0.0, 0.0)),
                       process_mask=1, max_real_events=1, history_records=True)
    k = 0.511 / MEC2

    def dsig(c):
        p = 1.0 / (1.0 + k * (1.0 - c))
        return p * p * (p + 1.0 / p - (1.0 - c * c))

    tot = integrate.quad(dsig, -1, 1, epsrel=1e-12)[0]
    mt = integrate.quad(lambda c: (1 - 1 / (1 + k * (1 - c))) * dsig(c), -1, 1,
                        epsrel=1e-12)[0] / tot
    mu_c = orc.mass_atten(1, 7.4, 0.5551, 0.511)
    want = 0.511 * mt * (1 - math.exp(-mu_c * n * h / 10.0))
    got = rec[:, 0]
    assert abs(got.mean() - want) < 4 * got.std() / math.sqrt(N)
    assert abs(_balance(tal.ledger)) < 1e-9


@pytest.mark.parametrize("tracking", [0, 1])
def test_total_absorption_cell_fixes_dose_units_and_merge(orc, tracking):
    """A photon started at the centre of one 1 m voxel of a dense high-Z
    medium (mu > 1.3 /cm at every energy, escape probability below 1e-18):
    every history deposits exactly E0, in several pieces merged into one
    per-history score, so S = N E0, S2 = N E0^2, dose E0 c / m and sigma 0."""
    rho = np.full((1, 1, 1), 20.0)
    ph = orc.Phantom(rho, np.zeros((1, 1, 1), np.uint8), [80.0], [0.4], (100.0,) * 3,
                     label=np.ones((1, 1, 1), np.uint8), n_organs=1)
    N = 20000
    tal, rec = orc.run(ph, N, 41, tracking=tracking, pencil=((50.0, 50.0, 50.0), (1.0, 0, 0)),
                       history_records=True)
    assert tal.ledger["escaped"] == 0.0
    assert (rec[:, 2] >= 1).mean() > 0.5  # most histories deposit in several pieces
    assert tal.S[0, 0, 0] == pytest.approx(N * 0.511, rel=1e-12, abs=0)
    assert tal.S2[0, 0, 0] == pytest.approx(N * 0.511 ** 2, rel=1e-12, abs=0)
    rate, eps = orc.finalize(ph, tal, a_ts_bq=1.0)
    m_kg = 20.0 * 1e6 * 1e-3
    assert rate[0, 0, 0] == pytest.approx(0.511 * J_PER_MEV / m_kg, rel=1e-12, abs=0)
    assert eps[0, 0, 0] < 1e-6
    # organ mean by per-history scores equals the map mean (Eq. 2)
    org_rate, rel = orc.organ_mean_sigma(tal, 1.0)
    assert org_rate[0] == pytest.approx(rate[0, 0, 0], rel=1e-12, abs=0)


def test_walters_variance_on_toy_tallies(orc):
    """Bernoulli(p) histories depositing c in one voxel: the relative standard
    error is sqrt((1-p) / (p (N-1)))."""
    shape = (1, 1, 3)
    rho = np.ones(shape)
    ph = orc.Phantom(rho, np.zeros(shape, np.uint8), [7.4], [0.55], (1.0, 1.0, 1.0),
                     label=np.ones(shape, np.uint8), n_organs=1, activity=np.ones(shape))
    tal = orc.Tally(ph)
    N, k, c = 1000, 250, 0.3
    tal.S[0, 0, 0], tal.S2[0, 0, 0] = k * c, k * c * c
    tal.S[0, 0, 1], tal.S2[0, 0, 1] = N * c, N * c * c  # constant deposit
    tal.n_decays = N
    rate, eps = orc.finalize(ph, tal, a_ts_bq=1.0)
    p = k / N
    assert eps[0, 0, 0] == pytest.approx(math.sqrt((1 - p) / (p * (N - 1))), rel=1e-12, abs=0)
    assert eps[0, 0, 1] < 1e-7
    assert eps[0, 0, 2] == 0.0 and rate[0, 0, 2] == 0.0
    # Eq. 2 and Eq. 3 on the toy map: mean of rates, RMS of relative errors
    r, e = orc.organ_stats(ph, rate, eps)
    assert r[0] == pytest.approx(rate.mean(), rel=1e-14, abs=0)
    assert e[0] == pytest.approx(math.sqrt((eps ** 2).mean()), rel=1e-14, abs=0)


def test_point_source_cube_symmetry(orc):
    """Centre-voxel source in an odd water cube: the dose map is invariant
    under the 48 symmetries of the cube (tested on a generating set)."""
    n = 15
    prob = P.water_point_source(n=n, voxel_mm=4.0)
    ph = _oracle_phantom(orc, prob)
    N = 400000
    tal, _ = orc.run(ph, N, 51, photons_per_decay=1)
    rate, eps = orc.finalize(ph, tal, a_ts_bq=1.0)
    sig = rate * eps
    ok = (eps > 0) & (eps < 0.2)
    for g in (lambda a: a[::-1], lambda a: a.transpose(1, 0, 2), lambda a: a.transpose(2, 1, 0),
              lambda a: a[:, :, ::-1]):
        m = ok & g(ok)
        m[n // 2, n // 2, n // 2] = False  # the source voxel maps to itself
        z = (rate - g(rate))[m] / np.sqrt(sig ** 2 + g(sig) ** 2)[m]
        # each pair counted twice: use half the voxels
        chi2 = (z ** 2).sum() / 2
        dof = m.sum() / 2
        assert stats.chi2.sf(chi2, dof) > 1e-3


def test_exact_and_woodcock_tracking_agree(orc):
    """The two tracking modes (independent free-flight and event algorithms,
    different uniforms and KN samplers) estimate the same dose."""
    prob = P.slab_phantom(n=48, voxel_mm=8.0)
    ph = _oracle_phantom(orc, prob)
    N = 400000
    ta, _ = orc.run(ph, N, 61, tracking=0)
    tb, _ = orc.run(ph, N, 62, tracking=1)
    ra, sa = orc.organ_mean_sigma(ta, 1.0)
    rb, sb = orc.organ_mean_sigma(tb, 1.0)
    z = (ra - rb) / np.sqrt((ra * sa) ** 2 + (rb * sb) ** 2)
    assert np.all(np.abs(z) < 4.0)
    da, ea = orc.finalize(ph, ta, 1.0)
    db, eb = orc.finalize(ph, tb, 1.0)
    m = (ea > 0) & (eb > 0) & (ea < 0.1) & (eb < 0.1) & (prob.density > 0.01)
    chi2 = (((da - db) ** 2)[m] / ((da * ea) ** 2 + (db * eb) ** 2)[m]).sum()
    assert stats.chi2.sf(chi2, m.sum()) > 1e-3
    assert abs(_balance(ta.ledger)) < 1e-9 and abs(_balance(tb.ledger)) < 1e-9


def test_exact_and_region_tracking_agree(orc):
    """Exact traversal and Woodcock tracking with region majorants estimate
    the same dose; the slab's tissue block sits in air, so photons cross the
    box both ways and interact in both regions."""
    prob = P.slab_phantom(n=48, voxel_mm=8.0)
    ph = _oracle_phantom(orc, prob)
    N = 400000
    ta, _ = orc.run(ph, N, 61, tracking=0)
    tb, _ = orc.run(ph, N, 64, tracking=2)
    ra, sa = orc.organ_mean_sigma(ta, 1.0)
    rb, sb = orc.organ_mean_sigma(tb, 1.0)
    z = (ra - rb) / np.sqrt((ra * sa) ** 2 + (rb * sb) ** 2)
    assert np.all(np.abs(z) < 4.0)
    da, ea = orc.finalize(ph, ta, 1.0)
    db, eb = orc.finalize(ph, tb, 1.0)
    m = (ea > 0) & (eb > 0) & (ea < 0.1) & (eb < 0.1) & (prob.density > 0.01)
    chi2 = (((da - db) ** 2)[m] / ((da * ea) ** 2 + (db * eb) ** 2)[m]).sum()
    assert stats.chi2.sf(chi2, m.sum()) > 1e-3
    # and the air: every voxel's dose there, pooled
    air = (prob.density < 0.01).ravel()
    sa_air = float(ta.S.reshape(-1)[air].sum())
    sb_air = float(tb.S.reshape(-1)[air].sum())
    va = float(ta.S2.reshape(-1)[air].sum())
    vb = float(tb.S2.reshape(-1)[air].sum())
    assert abs(sa_air - sb_air) < 4 * math.sqrt(va + vb)
    assert abs(_balance(tb.ledger)) < 1e-9
    # the point of the regions: fewer null collisions for the same histories
    tw, _ = orc.run(ph, N, 64, tracking=1)
    assert tb.stats["nulls"] < 0.9 * tw.stats["nulls"]
    assert tb.stats["histories"] == tw.stats["histories"] == N


def test_region_tracking_thin_surroundings(orc):
    """A pencil beam along a line of voxels: 80 cm of water at 0.009 g/cm^3
    (thinner than the box threshold, so outside the box), 10 cm of water at
    unit density (the box), 110 cm of the thin water again.  The beam starts
    in the thin region, enters the box, and leaves it; interactions in the
    thin region are real events at the thin density.  The uncollided
    fraction is exp(-sum mu L) for every tracking mode."""
    nx = 200
    density = np.full((1, 1, nx), 0.009)
    density[0, 0, 80:90] = 1.0
    material = np.zeros((1, 1, nx), dtype=np.int32)
    ph = orc.Phantom(density, material, [7.4], [0.5551], (1.0, 1.0, 1.0))
    mu = _mu(orc, 7.4, 0.5551, 1.0)
    p = math.exp(-mu * (10.0 + 0.009 * 190.0))
    N = 200000
    for tracking, seed in ((0, 71), (1, 72), (2, 73)):
        tal, rec = orc.run(ph, N, seed, tracking=tracking, photons_per_decay=1,
                           pencil=((1e-6, 0.5, 0.5), (1.0, 0.0, 0.0)), history_records=True)
        uncollided = (rec[:, 2] + rec[:, 3] + rec[:, 4] == 0).mean()
        assert abs(uncollided - p) < 4 * math.sqrt(p * (1 - p) / N), tracking
        assert abs(_balance(tal.ledger)) < 1e-9
        # energy deposited in the thin region before the box: first
        # collisions there happen at rate mu * 0.009 per cm
        if tracking == 2:
            first_thin = 1.0 - math.exp(-mu * 0.009 * 80.0)
            hit_thin = float(tal.S.reshape(-1)[:80].sum()) > 0.0
            assert hit_thin and first_thin > 0.05


def test_organ_score_equals_eq2(orc):
    prob = P.patient_phantom(shape=(40, 32, 32), voxel_mm=(16.0, 16.0, 24.0), seed=5)
    ph = _oracle_phantom(orc, prob)
    tal, _ = orc.run(ph, 50000, 71)
    a = prob.total_activity_bq
    rate, eps = orc.finalize(ph, tal, a)
    r2, _ = orc.organ_stats(ph, rate, eps)
    r_score, _ = orc.organ_mean_sigma(tal, a)
    nz = r2 > 0
    assert nz.sum() >= 10
    assert np.allclose(r_score[nz], r2[nz], rtol=1e-11, atol=0)


def test_invalid_inputs_rejected(orc):
    prob = P.water_point_source(n=8)
    ph = _oracle_phantom(orc, prob)
    ph.activity[:] = -1.0
    with pytest.raises(ValueError):
        orc.run(ph, 10, 1)
