"""Pins of the oracle's positron model (18F positron range and the pair's
non-collinearity): the sampled kinetic energy against the evaluated mean and
endpoint of the 18F beta+ spectrum (tests/golden/f18_beta_plus.json), the
sampler against the spectrum shape it inverts, the deviation angle against
the Rayleigh law its FWHM defines (median = FWHM / 2), and the transport
with positrons on: all kinetic energy deposited near the decay point inside
water, the ledger closed, and positrons that leave the grid taking the pair
with them."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2111_11687_amd import phantoms as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "f18_beta_plus.json")))
WATER_I = 75.0
MEC2 = 0.51099895


def _balance(led):
    dep = led["dep_compton"] + led["dep_pe"] + led["dep_cutoff"] + led["dep_positron"]
    return (dep + led["escaped"] + led["discarded"]) / led["emitted"] - 1.0


def test_positron_energy_mean_and_endpoint(orc):
    t = orc.sample("positron_energy", 1_000_000, seed=3)
    t0 = GOLD["beta_plus_endpoint_kev"] * 1e-3
    assert t.max() < t0 and t.max() > 0.97 * t0 and t.min() > 0.0
    # the allowed shape with the Fermi function gives 250.4 keV; without the
    # Fermi function it would be 240.4 keV, with the electron's sign 227 keV
    mean = GOLD["beta_plus_mean_kev"] * 1e-3
    se = t.std() / math.sqrt(t.size)
    assert abs(t.mean() - mean) < 0.003 + 4 * se


def test_positron_energy_follows_the_shape(orc):
    """Chi-square of 10^6 sampled energies against the spectrum shape
    integrated afresh over 40 bins."""
    t0 = GOLD["beta_plus_endpoint_kev"] * 1e-3
    n = 1_000_000
    t = orc.sample("positron_energy", n, seed=5)
    edges = np.linspace(0.0, t0, 41)
    shape = lambda x: orc.lib().orc_beta_plus_shape(x)
    tot = integrate.quad(shape, 0.0, t0, limit=200)[0]
    p = np.array([integrate.quad(shape, a, b)[0] for a, b in zip(edges[:-1], edges[1:])]) / tot
    obs, _ = np.histogram(t, edges)
    m = p * n > 20
    chi2 = ((obs[m] - n * p[m]) ** 2 / (n * p[m])).sum()
    assert stats.chi2.sf(chi2, m.sum() - 1) > 1e-3


def test_noncollinearity_angle_is_rayleigh(orc):
    fwhm = math.radians(0.5)
    th = orc.sample("noncollinear", 400_000, seed=7, e_mev=fwhm)
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    # the median of a Rayleigh law is sigma sqrt(2 ln 2) = FWHM / 2
    assert abs(np.median(th) - fwhm / 2) < 0.01 * fwhm
    assert stats.kstest(th, lambda x: 1.0 - np.exp(-x * x / (2 * sigma * sigma))).pvalue > 1e-3


def _water_cube(n, voxel_mm):
    return P.water_point_source(n=n, voxel_mm=voxel_mm)


def test_positrons_deposit_their_energy_near_the_decay(orc):
    """A point source in a water cube far larger than the positron range,
    photons made to escape without interacting: every positron's kinetic
    energy stays in the cube, within the CSDA range of the endpoint energy
    of the source voxel, and the ledger closes."""
    prob = _water_cube(41, 0.5)
    ph = orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                     [m[1] for m in prob.materials], prob.voxel_cm, activity=prob.activity)
    n = 200_000
    tal, _ = orc.run(ph, n, 11, tracking=orc.TRACK_WOODCOCK, process_mask=0, positron=True,
                     mean_excitation_ev=[WATER_I])
    led = tal.ledger
    t_mean = integrate.quad(lambda x: x * orc.lib().orc_beta_plus_shape(x), 0, 0.6335)[0] / \
        integrate.quad(lambda x: orc.lib().orc_beta_plus_shape(x), 0, 0.6335)[0]
    assert led["dep_positron"] / n == pytest.approx(t_mean, rel=5e-3)
    assert led["escaped"] == pytest.approx(2 * 0.511 * n, rel=1e-12)
    assert abs(_balance(led)) < 1e-12
    s = tal.S.reshape(prob.shape)
    nz = np.argwhere(s > 0)
    c = np.array(prob.shape) // 2
    h = prob.voxel_cm[0]
    rmax = orc.lib().orc_csda_range(0.001, 0.6335, 0.5551, WATER_I)
    assert np.abs(nz - c).max() * h <= rmax + h
    assert rmax == pytest.approx(0.24, rel=0.05)


def test_positrons_leaving_the_grid_take_the_pair(orc):
    """Decays in a grid thinner than the positron range: a share of the
    positrons leave it, and with them both photons; the ledger closes."""
    prob = _water_cube(3, 0.3)
    ph = orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                     [m[1] for m in prob.materials], prob.voxel_cm, activity=prob.activity)
    n = 100_000
    tal, rec = orc.run(ph, n, 13, tracking=orc.TRACK_WOODCOCK, positron=True,
                       mean_excitation_ev=[WATER_I], history_records=True)
    led = tal.ledger
    assert abs(_balance(led)) < 1e-12
    gone = rec[:, 1] > 2 * 0.511  # the positron's energy escaped with the pair
    assert 0.05 < gone.mean() < 0.95
    assert led["dep_positron"] > 0.0


@pytest.mark.parametrize("tracking", [0, 1])
def test_energy_conservation_with_positrons_and_electrons(orc, tracking):
    prob = P.slab_phantom(n=48, voxel_mm=6.0)
    ph = orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                     [m[1] for m in prob.materials], prob.voxel_cm, label=prob.label,
                     n_organs=prob.n_organs, activity=prob.activity)
    iev = [P.MEAN_EXCITATION_EV[next(k for k in P.MATERIALS
                                     if tuple(P.MATERIALS[k][:2]) == tuple(m))]
           for m in prob.materials]
    tal, _ = orc.run(ph, 20_000, 17, tracking=tracking, positron=True, mean_excitation_ev=iev,
                     electron_cutoff_mev=0.2)
    assert abs(_balance(tal.ledger)) < 1e-9
    assert tal.ledger["dep_positron"] > 0.0
