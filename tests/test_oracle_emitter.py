"""Pins of the oracle's gamma + beta emitter (the other emitters that
Section 4 names, with the 177Lu and 131I data of tests/golden/*_decay.json): at
most one photon per decay, line i with probability y_i (a chi-square of the
emitted energies against the yields), the photons' escaped energy per decay
when nothing interacts (sum y_i E_i), the mean beta energy left exactly in
the decay voxel, and the ledger closed with every process on."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2111_11687_amd import phantoms as P

def _nuclide(name):
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", name + "_decay.json")))
    return ([e * 1e-3 for e in d["gamma_lines_kev"]], d["gamma_yields_per_decay"],
            d["beta_minus_mean_kev"] * 1e-3)


# 131I's lines reach 723 keV: its runs take the wide grid (1 keV to 1 MeV)
EMITTERS = {"lu177": _nuclide("lu177"), "i131": _nuclide("i131")}
LINES, YIELDS, BETA = EMITTERS["lu177"]
EMITTER = (LINES, YIELDS, BETA)


def _balance(led):
    dep = sum(led[k] for k in ("dep_compton", "dep_pe", "dep_cutoff", "dep_positron", "dep_beta"))
    return (dep + led["escaped"] + led["discarded"]) / led["emitted"] - 1.0


def _water(orc, n=21, mm=4.0):
    prob = P.water_point_source(n=n, voxel_mm=mm)
    return prob, orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                             [m[1] for m in prob.materials], prob.voxel_cm,
                             activity=prob.activity)


@pytest.mark.parametrize("nuclide", ["lu177", "i131"])
@pytest.mark.parametrize("tracking", [0, 1])
def test_emitter_lines_and_beta(orc, tracking, nuclide):
    """Photons that never interact (process mask 0) carry exactly their line
    energy out of the grid: the escaped energy of each history is 0 or one of
    the lines, with the yields' frequencies; the beta energy stays in the
    source voxel."""
    LINES, YIELDS, BETA = EMITTERS[nuclide]
    prob, ph = _water(orc)
    n = 400_000
    tal, rec = orc.run(ph, n, 31, tracking=tracking, process_mask=0,
                       emitter=EMITTERS[nuclide], history_records=True)
    esc = rec[:, 1]
    counts = [int(np.sum(np.isclose(esc, 0.0)))] + \
        [int(np.sum(np.isclose(esc, e, rtol=1e-12, atol=0))) for e in LINES]
    assert sum(counts) == n
    p = np.array([1.0 - sum(YIELDS)] + YIELDS)
    chi2 = float((((np.array(counts) - n * p) ** 2) / (n * p)).sum())
    assert stats.chi2.sf(chi2, len(p) - 1) > 1e-3
    led = tal.ledger
    mean_e = sum(y * e for y, e in zip(YIELDS, LINES))
    sd = math.sqrt(sum(y * e * e for y, e in zip(YIELDS, LINES)) - mean_e ** 2)
    assert abs(led["escaped"] / n - mean_e) < 4 * sd / math.sqrt(n)
    assert led["dep_beta"] == pytest.approx(n * BETA, rel=1e-10)
    assert tal.stats["photons"] == sum(counts[1:])
    s = tal.S.reshape(prob.shape)
    c = tuple(np.array(prob.shape) // 2)
    assert s[c] == pytest.approx(n * BETA, rel=1e-10)
    assert np.count_nonzero(s) == 1
    assert abs(_balance(led)) < 1e-12


@pytest.mark.parametrize("nuclide", ["lu177", "i131"])
@pytest.mark.parametrize("tracking", [0, 1])
def test_emitter_energy_conservation(orc, tracking, nuclide):
    prob = P.slab_phantom(n=48, voxel_mm=6.0)
    ph = orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                     [m[1] for m in prob.materials], prob.voxel_cm, label=prob.label,
                     n_organs=prob.n_organs, activity=prob.activity)
    tal, _ = orc.run(ph, 100_000, 37, tracking=tracking, emitter=EMITTERS[nuclide])
    led = tal.ledger
    assert abs(_balance(led)) < 1e-9
    assert led["dep_compton"] > 0 and led["dep_pe"] > 0


def test_emitter_rejects_bad_input(orc):
    prob, ph = _water(orc, n=9)
    for bad in (([1.2], [0.1], 0.1), ([0.1], [1.2], 0.1), ([0.1], [0.1], -1.0)):
        with pytest.raises(ValueError):
            orc.run(ph, 10, 1, emitter=bad)
    with pytest.raises(ValueError):
        orc.run(ph, 10, 1, emitter=EMITTER, positron=True, mean_excitation_ev=[75.0])
    # lines above 511 keV outrun the electron range tables
    with pytest.raises(ValueError):
        orc.run(ph, 10, 1, emitter=EMITTERS["i131"], electron_cutoff_mev=0.2,
                mean_excitation_ev=[75.0])
