"""Pins of the oracle's decay source, its second random-number family, the
per-history organ score behind the organ uncertainty, and the photon cutoff.

* Decay points (Section 2.1: the decay probability of a voxel follows the
  activity; position uniform in the voxel): pooled chi-square of the sampled
  voxels against A_v / sum(A) on a multi-voxel lognormal map with empty
  voxels, in both draw orders, and the moments and KS test of the in-voxel
  position.
* xoshiro256** / SplitMix64 (the family the exact-traversal mode draws
  from): SplitMix64's published first word from state 0, uniformity and lag
  correlation of the uniforms, and no correlation with the Philox stream of
  the same seed.
* Per-history organ score (history-by-history uncertainty of Section 2.1
  applied to the organ mean of Eq. 2): two photons of one history absorbed
  in different voxels of one organ must add before squaring, and a
  Bernoulli organ score gives the closed-form relative standard error.
* Photon cutoff (Section 2.1, 10 keV by default): with Compton only and the
  cutoff at the emission energy, the first Compton event ends every photon
  and leaves all of E0 in its voxel.
"""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2111_11687_amd import phantoms as P

MEC2 = 0.51099895
J_PER_MEV = 1.602176634e-13
# mean energy transfer <T/E> of Klein-Nishina at 511 keV (numerical
# integration of the differential cross section; also pinned in the
# primitive tests)
MEAN_T_OVER_E_511 = 0.344482


def _lognormal_map(shape, seed):
    rng = np.random.default_rng(seed)
    a = np.exp(rng.normal(0.0, 0.8, size=shape))
    a[rng.random(shape) < 0.3] = 0.0  # empty voxels must never be drawn
    return a


def _map_phantom(orc, shape, voxel_cm, activity):
    rho = np.ones(shape)
    return orc.Phantom(rho, np.zeros(shape, np.uint8), [7.4], [0.5551], voxel_cm,
                       activity=activity)


@pytest.mark.parametrize("tracking", [0, 1])
def test_decay_voxels_follow_the_activity(orc, tracking):
    shape = (9, 10, 12)
    act = _lognormal_map(shape, 11)
    ph = _map_phantom(orc, shape, (0.2, 0.3, 0.4), act)
    n = 2_000_000
    vox, _ = orc.sample_source(ph, n, seed=7, tracking=tracking)
    counts = np.bincount(vox, minlength=act.size)
    p = act.ravel() / act.sum()
    assert counts[p == 0].sum() == 0
    expect = n * p
    m = expect >= 5
    chi2 = float((((counts - expect) ** 2)[m] / expect[m]).sum())
    dof = int(m.sum()) - 1
    assert stats.chi2.sf(chi2, dof) > 1e-3, (chi2, dof)
    # the pooled tail (voxels with fewer than 5 expected) is consistent too
    tail_e, tail_c = expect[~m & (p > 0)].sum(), counts[~m & (p > 0)].sum()
    if tail_e > 0:
        assert abs(tail_c - tail_e) < 5 * math.sqrt(tail_e) + 5


@pytest.mark.parametrize("tracking", [0, 1])
def test_decay_position_uniform_in_voxel(orc, tracking):
    shape = (5, 6, 7)
    h = (0.2, 0.3, 0.4)
    ph = _map_phantom(orc, shape, h, _lognormal_map(shape, 12))
    n = 400_000
    vox, pos = orc.sample_source(ph, n, seed=9, tracking=tracking)
    nz, ny, nx = shape
    idx = np.stack([vox % nx, (vox // nx) % ny, vox // (nx * ny)], axis=1)
    frac = pos / np.asarray(h) - idx
    assert np.all(frac >= 0.0) and np.all(frac < 1.0)
    for a in range(3):
        f = frac[:, a]
        assert abs(f.mean() - 0.5) < 4 * math.sqrt(1 / 12 / n)
        assert abs(f.var() - 1 / 12) < 4 * math.sqrt(1 / 180 / n)
        assert stats.kstest(f, "uniform").pvalue > 1e-3
    # the three coordinates are independent of each other
    c = np.corrcoef(frac.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 4 / math.sqrt(n))


def test_splitmix64_published_first_word(orc):
    out, state = orc.splitmix64(0)
    assert out == 0xE220A8397B1DCDAF
    assert state == 0x9E3779B97F4A7C15


def test_xoshiro_uniforms(orc):
    n = 1_000_000
    u = orc.sample("uniform", n, seed=3, wide=True, rng=orc.RNG_XOSHIRO)
    assert np.all((u > 0) & (u < 1))
    counts = np.histogram(u, bins=100, range=(0, 1))[0]
    assert stats.chisquare(counts).pvalue > 1e-3
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 5 / math.sqrt(n)
    # 32-bit words: every bit is balanced
    w = orc.sample("raw", n // 4, seed=4, rng=orc.RNG_XOSHIRO).astype(np.uint64).ravel()
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint64)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / math.sqrt(w.size))
    # a family apart from the device's Philox streams of the same seed
    v = orc.sample("uniform", n, seed=3, wide=True, rng=orc.RNG_PHILOX)
    assert abs(np.corrcoef(u, v)[0, 1]) < 5 / math.sqrt(n)
    assert not np.any(u == v)


def test_xoshiro_state_update(orc):
    """Outputs from state (1, 2, 3, 4), worked by hand from the definition:
    rotl(5 * 2, 7) * 9 = 11520 first; the update leaves s1 = 0, so the
    second output is 0."""
    out = orc.xoshiro256ss((1, 2, 3, 4), 2)
    assert out == [11520, 0]


def _pe_cell(orc, n_side, rho, h_cm, label=True):
    """A cube of a dense high-Z medium, one organ everywhere: with the
    photoelectric effect alone each photon is absorbed at its first real
    event, whole, within about a voxel."""
    shape = (n_side,) * 3
    act = np.zeros(shape)
    c = n_side // 2
    act[c, c, c] = 1.0
    return orc.Phantom(np.full(shape, rho), np.zeros(shape, np.uint8), [100.0], [0.4],
                       (h_cm,) * 3, label=np.ones(shape, np.uint8) if label else None,
                       n_organs=1 if label else 0, activity=act)


@pytest.mark.parametrize("tracking", [0, 1])
def test_organ_score_squared_per_history(orc, tracking):
    """Two back-to-back photons absorbed in different voxels of one organ:
    the history's organ score q = (e1 + e2) c / (m N_o) is squared whole, so
    O2 = sum_h q_h^2 over the histories' total deposits, which differs from
    the per-voxel sum of squares whenever both photons are absorbed."""
    n_side, h = 3, 0.5
    ph = _pe_cell(orc, n_side, 40.0, h)
    mu = 40.0 * orc.mass_atten(2, 100.0, 0.4, 0.511)
    assert mu * h > 1.0  # absorbed within about a voxel
    N = 100_000
    tal, rec = orc.run(ph, N, 17, tracking=tracking, process_mask=2, history_records=True)
    w = J_PER_MEV / (40.0 * h ** 3 * 1e-3 * n_side ** 3)  # c / (m_v N_o)
    q = rec[:, 0] * w
    two = (rec[:, 7] >= 2).mean()  # histories depositing in two voxels
    assert two > 0.2
    assert tal.O[1] == pytest.approx(q.sum(), rel=1e-12, abs=0)
    assert tal.O2[1] == pytest.approx((q * q).sum(), rel=1e-12, abs=0)
    # squaring each voxel's deposit separately would book 2 a^2 instead of
    # (2 a)^2 for every history with the two photons in two voxels
    a = 0.511 * w
    split = rec[:, 7] == 2
    per_voxel = np.where(split, 2 * a * a, q * q).sum()
    assert tal.O2[1] - per_voxel == pytest.approx(2 * a * a * split.sum(), rel=1e-9, abs=0)
    assert tal.S.sum() == pytest.approx(rec[:, 0].sum(), rel=1e-12, abs=0)


@pytest.mark.parametrize("tracking", [0, 1])
def test_organ_sigma_bernoulli(orc, tracking):
    """A pencil beam through a photoelectric-only slab that is one organ: the
    organ score of a history is a (absorbed) or 0 (escaped), so the organ
    mean is a p_hat and its relative standard error is
    sqrt((1 - p_hat) / (p_hat (N - 1))); p_hat follows 1 - exp(-mu L)."""
    nx, h, rho = 8, 0.25, 2.0
    shape = (1, 1, nx)
    ph = orc.Phantom(np.full(shape, rho), np.zeros(shape, np.uint8), [100.0], [0.4],
                     (h,) * 3, label=np.ones(shape, np.uint8), n_organs=1)
    N = 200_000
    tal, rec = orc.run(ph, N, 19, tracking=tracking, process_mask=2,
                       pencil=((0.0, 0.5 * h, 0.5 * h), (1.0, 0.0, 0.0)), history_records=True)
    a = 0.511 * J_PER_MEV / (rho * h ** 3 * 1e-3 * nx)
    absorbed = rec[:, 3] > 0
    p_hat = absorbed.mean()
    assert tal.O[1] == pytest.approx(a * absorbed.sum(), rel=1e-12, abs=0)
    rate, rel = orc.organ_mean_sigma(tal, 1.0)
    assert rate[0] == pytest.approx(a * p_hat, rel=1e-12, abs=0)
    assert rel[0] == pytest.approx(math.sqrt((1 - p_hat) / (p_hat * (N - 1))), rel=1e-9, abs=0)
    mu = rho * orc.mass_atten(2, 100.0, 0.4, 0.511)
    p = 1.0 - math.exp(-mu * nx * h)
    assert abs(p_hat - p) < 4 * math.sqrt(p * (1 - p) / N)


@pytest.mark.parametrize("tracking", [0, 1])
def test_cutoff_at_emission_energy_ends_first_compton(orc, tracking):
    """Compton only, photon cutoff at 0.511 MeV: every scattered photon falls
    below it, so its E' is left where it scattered (the cutoff deposit) and
    the photon's whole E0 stays in the grid.  Deposit per photon =
    E0 (1 - exp(-mu_C L)); the cutoff share of it is 1 - <T/E> at 511 keV."""
    n, hmm = 20, 5.0
    prob = P.water_point_source(n=n, voxel_mm=hmm)
    ph = orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                     [m[1] for m in prob.materials], prob.voxel_cm)
    N = 200_000
    tal, rec = orc.run(ph, N, 23, tracking=tracking, process_mask=1, cutoff_mev=0.511,
                       pencil=((0.0, 5.0, 5.0), (1.0, 0.0, 0.0)), history_records=True)
    assert np.all(rec[:, 2] <= 1)  # one Compton event at most
    hit = rec[:, 2] == 1
    assert np.allclose(rec[hit, 0], 0.511, rtol=0, atol=1e-12)
    assert np.all(rec[~hit, 0] == 0.0)
    mu_c = orc.mass_atten(1, 7.4, 0.5551, 0.511)
    p = 1.0 - math.exp(-mu_c * n * hmm / 10.0)
    assert abs(hit.mean() - p) < 4 * math.sqrt(p * (1 - p) / N)
    led = tal.ledger
    share = led["dep_cutoff"] / (led["dep_cutoff"] + led["dep_compton"])
    # eps = E'/E has standard deviation below 0.25 at 511 keV
    assert abs(share - (1 - MEAN_T_OVER_E_511)) < 4 * 0.25 / math.sqrt(hit.sum())
    dep = led["dep_compton"] + led["dep_pe"] + led["dep_cutoff"]
    assert abs((dep + led["escaped"] + led["discarded"]) / led["emitted"] - 1) < 1e-9
